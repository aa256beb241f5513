// RR-set generation on gfx950 (Algorithm 3's skeleton with one keyed coin per
// channel), stratified roots, and compaction into the RR-set CSR.
//
// RR sets are very uneven: most cost a few hundred incidences, while a set
// that reaches a hub vertex (a member of ~1e5 hyperedges) or grows into a
// giant component costs millions.  Generation therefore runs in two phases.
//
// Phase A (k_rr_light, persistent): wavefronts steal RR ids from a global
// counter; one wavefront owns one set at a time in a "slot" (member list that
// doubles as the BFS queue, plus a visited bitmap -- in LDS when every graph
// of the launch is small).  Each frontier batch (up to 64 queued vertices) is
// expanded in three load-balanced levels -- vertices -> incidences (v, he) ->
// runs of 4 member positions -- so lanes stay busy under degree and size skew
// and member ids are read contiguously; one Philox4x32-10 block gives the 4
// coins of a run; a live channel from an unvisited member sets its bit
// (atomic OR) and the winner appends it with a ballot-ranked store.  A set
// whose next batch holds a heavy vertex, or that has used up its incidence
// budget, is handed over intact (slot, queue head, size) to phase B and the
// wave takes a fresh slot.  Finished sets are written ascending to a staging
// area.
//
// Phase B (bulk-synchronous over the deferred sets): k_plan cuts every
// deferred set's current frontier into work items of bounded cost --
// segments of consecutive queue entries holding at most a few hundred
// incidences, or one heavy vertex's incidences in chunks -- and k_expand
// spreads the items over every wavefront of the GPU (several wavefronts per
// item when items are fewer than wavefronts), so a single giant set or hub
// expansion uses the whole chip; a wavefront that found only a few light
// members expands them itself right away (continuation) instead of leaving
// one more thin level to the next superstep.  Supersteps repeat until no frontier
// is left; k_finish sorts and stages each set.  No wave ever waits for
// another: items only refer to finished supersteps.
//
// A launch group covers several tasks -- (graph, key, pool, id range) -- back
// to back, described in device memory: both pools of a doubling round, or
// many IM instances on different graphs, share phase A and the supersteps.
//
// The other cascade models reuse this frame: under the gap models the same
// two phases run with level 3 replaced by one geometric-gap stream per
// incidence (expand_gaps); the linear-threshold walk (k_lt_walk) and the
// stratified setting's per-layer draws (k_layered) are one wave per set in
// phase A's slots.  A launch group holds graphs of one kind only.
//
// Compaction turns the per-id sizes into CSR offsets (device scan) and moves
// the staged members into the pools.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "dev_common.h"
#include "internal.h"
#include "plan_layout.h"

namespace hyperim {
namespace {

constexpr int kWG = 256;
constexpr int kWavesPerWG = kWG / kWave;
constexpr uint32_t kSortMax = 1024;          // phase A: sets up to this size are sorted in LDS
constexpr uint32_t kSortMaxWG = 4096;        // phase B: one workgroup sorts up to this size in LDS
constexpr uint32_t kLdsBitmapWords = 1024;   // visited bitmap in LDS when every |V| <= 32768
constexpr uint32_t kBigSet = 4096;           // compaction: one workgroup per larger set
constexpr uint32_t kItemCap = kPlanItemCap;      // phase B: work items per superstep
constexpr uint64_t kSlotBudget = 48ull << 30; // bytes of slot lists + bitmaps
// The remaining execution parameters (heavy-vertex threshold, per-set budget,
// chunk and segment sizes, prefilter threshold, supersteps per sync) are
// runtime values, see hyperim_tuning.

// Counters (uint64 each) in the workspace counter block.
// kItems and kItems + 1 alternate between supersteps: superstep s plans into
// counter s & 1 while its k_expand clears the other one for superstep s + 1.
// kPlanned counts the frontier entries k_plan has taken (summed queue heads),
// the progress measure of the host loop.
// kPhiloxA and kPhilox count the Philox4x32-10 blocks k_rr_light and k_expand
// drew (lane blocks whose coins were needed); kBytesMs and kPhiloxMs are
// bundled mode's algorithmic bytes and blocks.
enum Ctr {
    kWork = 0, kBump, kBigCount, kFreeNext, kDefCount, kItems, kItemsOther, kBytesA, kBytesB, kPlanned, kPhilox,
    kBytesMs, kPhiloxMs, kPhiloxA, kNumCtr
};

// One graph of a launch group.
// v_hbs[e] = (first member position, size) of hyperedge v_he[e], beside the
// incidence list so that an incidence's hyperedge needs no dependent load.
struct GraphDesc {
    const uint32_t *he_off, *he_mem, *v_off, *v_he, *thr, *P;
    const unsigned long long *v_hbs;   // low word: first position, high word: size
    uint32_t n, bm_words;
    // linear-threshold graphs: channels of the incidences before each one
    // (exclusive prefix of |he| - 1 over v_he, nnz + 1 entries); else null
    const unsigned long long *chan;
    // stratified-setting graphs: A(v) by layers and the count tables; else null
    const unsigned long long *lay_nb_off, *lay_ly_off;
    const uint32_t *lay_nb, *lay_ly_end, *l;
    const double *lay_ln, *lay_expm;
    // RR sets divided into R1 / R2 (Section 4.1): pool 0 draws its roots from
    // rP[0 .. rn1), pool 1 from rP[rn1 .. n), and a pool-0 set starts with
    // force[force_off[root] .. force_off[root + 1]) beside its root; else null
    const uint32_t *rP, *force;
    const unsigned long long *force_off;
    uint32_t rn1;
};

// The same arrays as global-memory pointers: descriptors are read from device
// memory, where the compiler cannot tell their address space and would emit
// flat loads.
#define HIM_GLOBAL __attribute__((address_space(1)))
struct GraphView {
    const HIM_GLOBAL uint32_t *he_off, *he_mem, *v_off, *v_he, *thr, *P, *rP;
    const HIM_GLOBAL unsigned long long *v_hbs;
    uint32_t n, bm_words, rn1;
};

// Descriptors are read at wave-uniform indices; their fields go to scalar
// registers.
__device__ __forceinline__ GraphView graph_view(const GraphDesc &d) {
    GraphView v;
    v.he_off = uni_ptr((const HIM_GLOBAL uint32_t *)d.he_off);
    v.he_mem = uni_ptr((const HIM_GLOBAL uint32_t *)d.he_mem);
    v.v_off = uni_ptr((const HIM_GLOBAL uint32_t *)d.v_off);
    v.v_he = uni_ptr((const HIM_GLOBAL uint32_t *)d.v_he);
    v.thr = uni_ptr((const HIM_GLOBAL uint32_t *)d.thr);
    v.P = uni_ptr((const HIM_GLOBAL uint32_t *)d.P);
    v.v_hbs = uni_ptr((const HIM_GLOBAL unsigned long long *)d.v_hbs);
    v.rP = uni_ptr((const HIM_GLOBAL uint32_t *)d.rP);
    v.n = uni(d.n);
    v.bm_words = uni(d.bm_words);
    v.rn1 = uni(d.rn1);
    return v;
}

// One task of a launch group: launch indices [previous end, end) are RR ids
// first_id, first_id + 1, ... of pool `pool` on graph `graph` with Philox key
// (key0, key1).
struct TaskDesc {
    uint64_t end, first_id;
    uint32_t pool, graph, key0, key1;
};

struct RRArgs {
    const GraphDesc *graphs;
    const TaskDesc *tasks;
    uint32_t ntasks, qlog;
    uint32_t heavy, budget, chunk, seg, prefilter_min;   // execution parameters
    uint32_t slot_n, slot_words;     // slot list length and bitmap words (largest graph)
    uint64_t count;                  // launch indices [0, count)
    uint64_t out_base;               // per-id array index of launch index 0
    unsigned long long *ctr;         // Ctr block
    uint32_t *lists;                 // per slot: slot_n entries
    uint32_t *bitmaps;               // per slot: slot_words (global mode)
    uint32_t slot_total;             // slots available (waves own the first ones)
    uint32_t *stage;
    uint64_t stage_cap;
    uint64_t *stage_off;             // per id
    uint32_t *sizes;                 // per id
    uint32_t *roots;                 // per id
    uint64_t *big_ids;               // per big set: per-id index
    // deferred sets (phase B)
    uint64_t *def_idx;
    uint32_t *def_root, *def_slot, *def_head, *def_size, *def_task;
    uint4 *items;
};

constexpr uint32_t kLiveCap = 256;   // live channels a wave holds before marking them (global marks)

struct WaveLdsCore {
    uint32_t fr_scan[kWave], fr_v[kWave], fr_e0[kWave];
    uint32_t in_scan[kWave], in_he[kWave], in_hb[kWave], in_hs[kWave], in_v[kWave], in_thr[kWave];
    uint32_t cont_u[kWave], cont_pos[kWave];   // phase B: members this wave appended, and where
};
// With visited bitmaps in global memory a wave also buffers live channels.
struct WaveLds : WaveLdsCore {
    uint32_t live[kLiveCap];                   // sources of live channels waiting to be marked
};

// The task of launch index idx (first task whose end exceeds idx); idx is
// wave-uniform.
__device__ __forceinline__ uint32_t task_of(const RRArgs &a, uint64_t idx) {
    uint32_t lo = 0, hi = a.ntasks - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (uni64(a.tasks[mid].end) > idx) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// What a set needs to know about where it comes from.
struct SetRef {
    GraphView G;
    uint64_t j;
    uint32_t pool;
    uint2 key;
};

// t and idx are wave-uniform.
__device__ __forceinline__ SetRef set_ref(const RRArgs &a, uint32_t t, uint64_t idx) {
    const TaskDesc &T = a.tasks[t];
    const uint64_t start = t ? uni64(a.tasks[t - 1].end) : 0ull;
    SetRef r;
    r.G = graph_view(a.graphs[uni(T.graph)]);
    r.j = uni64(T.first_id) + (idx - start);
    r.pool = uni(T.pool);
    r.key = make_uint2(uni(T.key0), uni(T.key1));
    return r;
}

// Stratified root of RR id j: block b of the ladder (Q = 2^qlog ids in block
// 0, Q 2^(b-1) in block b >= 1, so block sizes are powers of two), offset
// o_b = floor(x n / 2^64) from the block's Philox draw, root =
// P[floor((t n + o_b) / T_b)] computed in 128-bit arithmetic.  With the RR
// sets divided, P and n are the pool's own root list and its length.
__device__ __forceinline__ uint32_t rr_root(const GraphView &G, uint32_t qlog, uint64_t j, uint32_t pool, uint2 key) {
    const uint64_t Q = 1ull << qlog;
    uint32_t b, s;
    uint64_t J;
    if (j < Q) {
        b = 0;
        J = 0;
        s = qlog;
    } else {
        const uint32_t hb = 63u - (uint32_t)__clzll((long long)j);
        b = hb - qlog + 1u;
        J = 1ull << hb;
        s = hb;
    }
    const HIM_GLOBAL uint32_t *P = G.P;
    uint64_t n = G.n;
    if (G.rP != nullptr) {
        P = pool == 0u ? G.rP : G.rP + G.rn1;
        n = pool == 0u ? G.rn1 : G.n - G.rn1;
    }
    const uint4 r = philox4x32_10(root_counter(b, pool), key);
    const uint64_t x = (uint64_t)r.x | ((uint64_t)r.y << 32);
    const uint64_t o = __umul64hi(x, n);
    const uint64_t t = j - J;
    const uint64_t lo = t * n;
    uint64_t hi = __umul64hi(t, n);
    const uint64_t lo2 = lo + o;
    hi += lo2 < lo ? 1ull : 0ull;
    const uint64_t pos = s == 0 ? lo2 : ((lo2 >> s) | (hi << (64u - s)));
    return P[pos];
}

template <bool kLds>
__device__ __forceinline__ uint32_t bm_load(uint32_t *bm, uint32_t w) {
    if constexpr (kLds) return bm[w];
    else return __hip_atomic_load(bm + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Appends a wave's newly reached members to a list whose size lives in a
// register (phase A: one wave owns the set).
struct LocalAppend {
    uint32_t *list;
    uint32_t size, n;
    // Append the members u[t] of the set bits t of `mask` (this lane's newly
    // reached members), all lanes at once: one wave scan gives each lane its
    // place.  Every lane of the wave calls it.
    __device__ __forceinline__ void push8(uint32_t mask, const uint32_t (&u)[8]) {
        const uint32_t cnt = (uint32_t)__popc(mask);
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t total = uni(wave_bcast(incl, kWave - 1));
        if (total == 0) return;
        uint32_t at = size + incl - cnt;
#pragma unroll
        for (uint32_t t = 0; t < 8; ++t)
            if ((mask >> t) & 1u) {
                if (at < n) list[at] = u[t];   // at < n always holds: one bit per vertex
                ++at;
            }
        size = min(size + total, n);
    }
    // One member per lane at most (`fresh`): places from the wave's ballot.
    __device__ __forceinline__ void push1(bool fresh, uint32_t u) {
        const uint64_t bal = __ballot(fresh);
        if (bal == 0ull) return;
        if (fresh) {
            const uint32_t at = size + (uint32_t)__popcll(bal & ((1ull << lane_id()) - 1ull));
            if (at < n) list[at] = u;
        }
        size = min(size + (uint32_t)__popcll(bal), n);
    }
};

// Same with the size in global memory (phase B: many waves grow one set).
struct SharedAppend {
    uint32_t *list;
    uint32_t *size;
    uint32_t n;
    __device__ __forceinline__ void push8(uint32_t mask, const uint32_t (&u)[8]) {
        const uint32_t cnt = (uint32_t)__popc(mask);
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t total = uni(wave_bcast(incl, kWave - 1));
        if (total == 0) return;
        uint32_t base = 0;
        if (lane_id() == kWave - 1) base = atomicAdd(size, total);
        uint32_t at = uni(wave_bcast(base, kWave - 1)) + incl - cnt;
#pragma unroll
        for (uint32_t t = 0; t < 8; ++t)
            if ((mask >> t) & 1u) {
                if (at < n) list[at] = u[t];
                ++at;
            }
    }
};

// Member positions tested per lane and call: kQ Philox blocks of 4 coins.
// One block per lane and pass keeps every lane's Philox work useful (most
// hyperedges have few members, so the upper half of an 8-position run is
// often empty while its block would still cost the whole wave).
constexpr uint32_t kQ = 1;
constexpr uint32_t kRun = 4 * kQ;

// A queue entry of a deferred set with this bit set was expanded by the wave
// that appended it (continuation, below); readers of the queue mask it.
constexpr uint32_t kExpanded = 0x80000000u;

// SharedAppend that also records the first 64 members this wave appends, and
// their queue positions, in the wave's LDS.
struct ContAppend {
    uint32_t *list;
    uint32_t *size;
    uint32_t n;
    uint32_t *cu, *cp;
    uint32_t count;   // members appended so far (wave-uniform)
    __device__ __forceinline__ void push8(uint32_t mask, const uint32_t (&u)[8]) {
        const uint32_t cnt = (uint32_t)__popc(mask);
        const uint32_t incl = wave_incl_scan(cnt);
        const uint32_t total = uni(wave_bcast(incl, kWave - 1));
        if (total == 0) return;
        uint32_t base = 0;
        if (lane_id() == kWave - 1) base = atomicAdd(size, total);
        uint32_t at = uni(wave_bcast(base, kWave - 1)) + incl - cnt;
        uint32_t c = count + incl - cnt;
#pragma unroll
        for (uint32_t t = 0; t < 8; ++t)
            if ((mask >> t) & 1u) {
                if (at < n) list[at] = u[t];
                if (c < kWave) {
                    cu[c] = u[t];
                    cp[c] = at;
                }
                ++at;
                ++c;
            }
        count += total;
    }
};

// Marks the wave's buffered live-channel sources in the set's visited
// bitmap (global memory) and appends the ones not marked before.  Each lane
// issues up to four atomics before waiting for any, so a wave pays one
// memory round trip per 256 live channels rather than one per coin batch.
// Every lane of the wave calls it.
template <class App>
__device__ __forceinline__ void flush_live(uint32_t *bm, WaveLds &L, uint32_t &nlive, App &app) {
    wave_sync();
    const uint32_t lane = lane_id();
    for (uint32_t i0 = 0; i0 < nlive; i0 += 4 * kWave) {
        uint32_t uu[8], old[4];
#pragma unroll
        for (uint32_t r = 0; r < 8; ++r) uu[r] = 0u;
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
            const uint32_t i = i0 + r * kWave + lane;
            old[r] = ~0u;
            if (i < nlive) {
                uu[r] = L.live[i];
                old[r] = atomicOr(&bm[uu[r] >> 5], 1u << (uu[r] & 31));
            }
        }
        uint32_t fresh = 0;
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) fresh |= ((old[r] >> (uu[r] & 31)) & 1u) ? 0u : 1u << r;
        app.push8(fresh, uu);
    }
    nlive = 0;
    wave_sync();
}

// Test the channels (he, u -> ve) at member positions [p0, p0 + cm) of one
// hyperedge (cm <= kRun, p0 a multiple of 4) in this lane: the coins are the
// words of the Philox blocks of quads p0/4, p0/4 + 1, ...  Newly reached
// members go to `app`: at once when the visited bitmap is in LDS, else
// through the wave's buffer of live channels (L.live, nlive entries), marked
// in batches.  Every lane of the wave must call it (inactive lanes with
// active = false).
template <bool kLds, class App, class Lds>
__device__ __forceinline__ void test_run(const GraphView &G, uint64_t j, uint32_t pool, uint2 key, uint32_t *bm,
                                         bool prefilter, bool active, uint32_t he, uint32_t hb, uint32_t p0,
                                         uint32_t cm, uint32_t ve, uint32_t the, App &app, uint64_t &px,
                                         Lds &L, uint32_t &nlive) {
    uint32_t u[8];
#pragma unroll
    for (uint32_t t = 0; t < 8; ++t) u[t] = (t < kRun && active && t < cm) ? G.he_mem[hb + p0 + t] : ve;
    uint32_t seen[kRun];
#pragma unroll
    for (uint32_t t = 0; t < kRun; ++t) seen[t] = 0u;
    if (prefilter) {
        // all mark words in flight together (u[t] is always a vertex id)
#pragma unroll
        for (uint32_t t = 0; t < kRun; ++t) seen[t] = bm_load<kLds>(bm, u[t] >> 5);
    }
    bool cand[kRun];
    bool need[kQ];
#pragma unroll
    for (uint32_t q = 0; q < kQ; ++q) need[q] = false;
#pragma unroll
    for (uint32_t t = 0; t < kRun; ++t) {
        cand[t] = u[t] != ve && !(seen[t] & (1u << (u[t] & 31)));
        need[t / 4] |= cand[t];
    }
    bool any = false;
#pragma unroll
    for (uint32_t q = 0; q < kQ; ++q) any |= need[q];
    if (__ballot(any) == 0) return;
    uint32_t w[kRun];
#pragma unroll
    for (uint32_t q = 0; q < kQ; ++q) {
        uint4 c = make_uint4(0u, 0u, 0u, 0u);
        if (__ballot(need[q]) != 0 && need[q]) {
            c = philox4x32_10(coin_counter(j, he, ve, pool, (p0 >> 2) + q), key);
            ++px;
        }
        w[4 * q] = c.x;
        w[4 * q + 1] = c.y;
        w[4 * q + 2] = c.z;
        w[4 * q + 3] = c.w;
    }
    bool live[kRun];
    bool any_live = false;
#pragma unroll
    for (uint32_t t = 0; t < kRun; ++t) {
        live[t] = cand[t] && channel_live(w[t], the);
        any_live |= live[t];
    }
    // with small probabilities most runs have no live channel at all
    if (__ballot(any_live) == 0) return;
    if constexpr (kLds) {
        uint32_t fresh = 0;
#pragma unroll
        for (uint32_t t = 0; t < kRun; ++t) {
            if (live[t]) {
                const uint32_t bit = 1u << (u[t] & 31);
                if ((atomicOr(&bm[u[t] >> 5], bit) & bit) == 0u) fresh |= 1u << t;
            }
        }
        app.push8(fresh, u);
    } else {
        // placement from one ballot per position (as in ms_pair)
        static_assert(kRun == 4, "one ballot per run position");
        const uint64_t b0 = __ballot(live[0]), b1 = __ballot(live[1]), b2 = __ballot(live[2]), b3 = __ballot(live[3]);
        const uint32_t c0 = (uint32_t)__popcll(b0), c1 = (uint32_t)__popcll(b1), c2 = (uint32_t)__popcll(b2);
        const uint32_t tot = c0 + c1 + c2 + (uint32_t)__popcll(b3);
        if (nlive + tot > kLiveCap) flush_live(bm, L, nlive, app);
        const uint64_t below = (1ull << lane_id()) - 1ull;
        if (live[0]) L.live[nlive + (uint32_t)__popcll(b0 & below)] = u[0];
        if (live[1]) L.live[nlive + c0 + (uint32_t)__popcll(b1 & below)] = u[1];
        if (live[2]) L.live[nlive + c0 + c1 + (uint32_t)__popcll(b2 & below)] = u[2];
        if (live[3]) L.live[nlive + c0 + c1 + c2 + (uint32_t)__popcll(b3 & below)] = u[3];
        nlive += tot;
    }
}

// Independent cascade drawn by geometric gaps (models HYPERIM_MODEL_GAPS_*;
// the subset sampling of Section 2.2.1, Algorithm 2, on the IC channels):
// the stream of (RR id j, hyperedge he, target v) is he's positions in
// stored order, each live with p_v (a live position holding v itself is no
// channel and is dropped); the gaps of dead positions before the next live
// one, Geometric(p_v), come from word r mod 4 of the Philox block at
// counter (j_lo, he, v, pool << 31 | j_hi << 24 | r / 4) for gap r.  A gap
// drawn from word x with G positions left is the largest g <= G with
// Q(g) >= t, t = (2^32 - x) / 2^32: a descent over the bits of G, from the
// top, taking bit i when acc * S_i >= t (then acc = acc * S_i), with
// S_0 = q = 1 - p_v and S_{i+1} = S_i^2 -- IEEE double products in a fixed
// order, no logarithm, so any implementation of the same steps draws the
// same gaps.  g = G: no live position is left in the stream.
__device__ __forceinline__ uint32_t gap_draw(double q, uint32_t x, uint32_t G) {
#pragma clang fp contract(off)
    const double t = (double)((1ull << 32) - (uint64_t)x) * 0x1.0p-32;
    const uint32_t b = G ? 32u - (uint32_t)__clz(G) : 0u;
    uint32_t g = 0;
    double acc = 1.0;
    for (int i = (int)b - 1; i >= 0; --i) {
        double S = q;
        for (int k = 0; k < i; ++k) S = S * S;
        if ((uint64_t)g + (1ull << i) <= (uint64_t)G && acc * S >= t) {
            acc = acc * S;
            g += 1u << i;
        }
    }
    return g;
}

// The same draw from the stream's powers S_i = q^(2^i), i < kGapTab, kept in
// registers (each S_i is q squared i times in sequence, so the values and the
// descent's products are those of gap_draw); for G < 2^kGapTab.
constexpr uint32_t kGapTab = 8;
__device__ __forceinline__ uint32_t gap_draw_tab(const double (&S)[kGapTab], uint32_t x, uint32_t G) {
#pragma clang fp contract(off)
    const double t = (double)((1ull << 32) - (uint64_t)x) * 0x1.0p-32;
    uint32_t g = 0;
    double acc = 1.0;
#pragma unroll
    for (int i = (int)kGapTab - 1; i >= 0; --i) {
        const double a = acc * S[i];
        if (g + (1u << i) <= G && a >= t) {
            acc = a;
            g += 1u << i;
        }
    }
    return g;
}

// One candidate per lane (`live` with member u): marked and appended as in
// test_run.  Every lane of the wave calls it.
template <bool kLds, class App, class Lds>
__device__ __forceinline__ void push_live(uint32_t *bm, Lds &L, uint32_t &nlive, App &app, bool live, uint32_t u) {
    const uint64_t bal = __ballot(live);
    if (bal == 0ull) return;
    if constexpr (kLds) {
        bool fresh = false;
        if (live) {
            const uint32_t bit = 1u << (u & 31);
            fresh = (atomicOr(&bm[u >> 5], bit) & bit) == 0u;
        }
        app.push1(fresh, u);
    } else {
        const uint32_t tot = (uint32_t)__popcll(bal);
        if (nlive + tot > kLiveCap) flush_live(bm, L, nlive, app);
        if (live) L.live[nlive + (uint32_t)__popcll(bal & ((1ull << lane_id()) - 1ull))] = u;
        nlive += tot;
    }
}

// Levels 2 and 3 under the gap models: the call's incidences g in [0, D)
// (wave w of W takes g = w, w + W, ...) go to lanes as a queue -- a lane whose
// stream has ended takes the next incidence -- so lanes stay busy while
// streams of different lengths run (a stream is sequential: gap r + 1 starts
// where gap r ended).  Each step draws one gap per busy lane; a live position
// yields its member (the target itself excepted), which is marked and
// appended as in test_run.  Returns the algorithmic bytes (12 per incidence,
// 4 per member read), wave-uniform after the caller's sum.
template <bool kLds, bool kUniform, class App, class Lds>
__device__ __forceinline__ uint64_t expand_gaps(const GraphView &G, Lds &L, uint64_t j, uint32_t pool, uint2 key,
                                                uint32_t *bm, uint32_t v, uint32_t e0, uint32_t D,
                                                uint32_t th_uniform, App &app, uint64_t &px, uint32_t &nlive,
                                                uint32_t w, uint32_t W) {
#pragma clang fp contract(off)
    const uint32_t lane = lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t next = w;   // next incidence of this wave (wave-uniform)
    uint64_t bytes = 0;
    bool more = false;
    uint32_t he = 0, hb = 0, hs = 0, vv = v, cur = 0, r = 0;
    double q = 1.0;
    double S[kGapTab];   // q^(2^i) of the lane's stream, when hs < 2^kGapTab
#pragma unroll
    for (uint32_t i = 0; i < kGapTab; ++i) S[i] = 1.0;
    uint4 blk = make_uint4(0u, 0u, 0u, 0u);
    for (;;) {
        const uint64_t idle = __ballot(!more);
        if (idle != 0ull && next < D) {
            // refill: the idle lanes take the next incidences in lane order
            const uint64_t g = next + (uint64_t)__popcll(idle & below) * W;
            if (!more && g < D) {
                uint32_t e = e0 + (uint32_t)g, th = th_uniform;
                if constexpr (!kUniform) {
                    const uint32_t k = search64(L.fr_scan, (uint32_t)g);
                    const uint32_t start = k ? L.fr_scan[k - 1] : 0u;
                    vv = L.fr_v[k];
                    e = L.fr_e0[k] + ((uint32_t)g - start);
                    th = G.thr[vv];
                }
                he = G.v_he[e];
                const unsigned long long bs = G.v_hbs[e];
                hb = (uint32_t)bs;
                hs = (uint32_t)(bs >> 32);
                bytes += 12u;
                more = th != 0u && hs != 0u;   // threshold 0: no channel into vv is live
                cur = 0u;
                r = 0u;
                q = 1.0 - (th == kAlways ? 1.0 : (double)th * 0x1.0p-32);
                if (hs < (1u << kGapTab)) {
                    S[0] = q;
#pragma unroll
                    for (uint32_t i = 1; i < kGapTab; ++i) S[i] = S[i - 1] * S[i - 1];
                }
            }
            next += (uint64_t)__popcll(idle) * W;
        }
        if (__ballot(more) == 0ull) {
            if (next >= D) break;
            continue;
        }
        uint32_t u = vv;
        bool live = false;
        if (more) {
            if ((r & 3u) == 0u) {
                blk = philox4x32_10(coin_counter(j, he, vv, pool, r >> 2), key);
                ++px;
            }
            const uint32_t x = (r & 3u) == 0u ? blk.x : (r & 3u) == 1u ? blk.y : (r & 3u) == 2u ? blk.z : blk.w;
            ++r;
            const uint32_t left = hs - cur;
            const uint32_t gap = hs < (1u << kGapTab) ? gap_draw_tab(S, x, left) : gap_draw(q, x, left);
            if (gap >= left) {
                more = false;
            } else {
                const uint32_t pos = cur + gap;
                u = G.he_mem[hb + pos];
                bytes += 4u;
                live = u != vv;
                cur = pos + 1u;
                more = cur < hs;
            }
        }
        push_live<kLds>(bm, L, nlive, app, live, u);
    }
    return bytes;
}

// Levels 2 and 3 of a frontier expansion.  Each lane brings one vertex v with
// the incidence range [e0, e0 + d) of v_he to expand (d = 0 for none); with
// kUniform all lanes pass the same v and e0 and d is the wave's incidence
// count (one heavy vertex), which needs no owner search.  Every channel
// (he, u -> v) of those incidences is tested with its coin and newly reached
// members go to `app`.  Level 3 first tests the first run of kRun member
// positions of each lane's own incidence, then spreads the remaining runs of
// the longer hyperedges over the wave.  W waves (a power of two, wave w of them passing
// w) may share one call: they split the batches of 64 incidences between
// them, and when there are fewer batches than waves, each batch's runs too;
// every run is tested by exactly one of them.  Returns the algorithmic
// bytes of the incidences read (12 per incidence plus 4 per member
// position), each counted by one wave, wave-uniform.
template <bool kLds, bool kUniform, bool kGaps, class App, class Lds>
__device__ __forceinline__ uint64_t expand(const GraphView &G, Lds &L, uint64_t j, uint32_t pool, uint2 key,
                                           uint32_t *bm, bool prefilter, uint32_t v, uint32_t e0, uint32_t d,
                                           App &app, uint64_t &px, uint32_t w = 0, uint32_t W = 1) {
    const uint32_t lane = lane_id();
    uint32_t nlive = 0;   // live channels buffered in L.live (wave-uniform)
    uint32_t D = d;
    uint32_t th_uniform = 0;
    if constexpr (kUniform) {
        th_uniform = G.thr[v];
    } else {
        const uint32_t dscan = wave_incl_scan(d);
        D = wave_bcast(dscan, kWave - 1);
        wave_sync();
        L.fr_scan[lane] = dscan;
        L.fr_v[lane] = v;
        L.fr_e0[lane] = e0;
        wave_sync();
    }
    if constexpr (kGaps) {
        const uint64_t bytes = expand_gaps<kLds, kUniform>(G, L, j, pool, key, bm, v, e0, D, th_uniform, app, px,
                                                           nlive, w, W);
        if constexpr (!kLds) flush_live(bm, L, nlive, app);
        wave_sync();
        return wave_sum(bytes);
    }
    // batch share: batches b = boff, boff + bstride, ...; within a batch,
    // runs qb = sub_w * 64, (sub_w + sub) * 64, ...  (first runs: sub_w 0)
    const uint32_t nbatch = (D + kWave - 1) / kWave;
    uint32_t bstride = W, sub = 1;
    if (nbatch < W) {
        bstride = 1;
        while (bstride < nbatch) bstride <<= 1;
        sub = W / bstride;
    }
    const uint32_t boff = w & (bstride - 1), sub_w = w / bstride;
    uint64_t bytes = 0;
    for (uint32_t base = boff * kWave; base < D; base += bstride * kWave) {
        // level 2: one incidence (v, he) per lane
        const uint32_t g = base + lane;
        uint32_t he = 0, hb = 0, hs = 0, vv = v, th = th_uniform, no = 0;
        if (g < D) {
            uint32_t e = e0 + g;
            if constexpr (!kUniform) {
                const uint32_t k = search64(L.fr_scan, g);
                const uint32_t start = k ? L.fr_scan[k - 1] : 0u;
                vv = L.fr_v[k];
                e = L.fr_e0[k] + (g - start);
                th = G.thr[vv];
            }
            he = G.v_he[e];
            const unsigned long long bs = G.v_hbs[e];
            hb = (uint32_t)bs;
            hs = (uint32_t)(bs >> 32);
            no = th ? (hs + kRun - 1u) / kRun : 0u;   // threshold 0: no channel into vv is live
            if (sub_w == 0) bytes += 12u + 4u * hs;
        }
        // level 3, first pass: run 0 of the lane's own incidence
        if (sub_w == 0)
            test_run<kLds>(G, j, pool, key, bm, prefilter, no > 0, he, hb, 0u, min(kRun, hs), vv, th, app, px, L,
                           nlive);
        // second pass: runs 1.. of the longer hyperedges, flattened over the wave
        const uint32_t rem = no > 1 ? no - 1u : 0u;
        if (__ballot(rem > 0) == 0) continue;
        const uint32_t rscan = wave_incl_scan(rem);
        const uint32_t R = wave_bcast(rscan, kWave - 1);
        wave_sync();
        L.in_scan[lane] = rscan;
        L.in_he[lane] = he;
        L.in_hb[lane] = hb;
        L.in_hs[lane] = hs;
        if constexpr (!kUniform) {
            L.in_v[lane] = vv;
            L.in_thr[lane] = th;
        }
        wave_sync();
        for (uint32_t qb = sub_w * kWave; qb < R; qb += sub * kWave) {
            const uint32_t qg = qb + lane;
            const bool active = qg < R;
            uint32_t hee = 0, hbk = 0, p0 = 0, cm = 0, ve = v, the = th_uniform;
            if (active) {
                const uint32_t k = search64(L.in_scan, qg);
                const uint32_t start = k ? L.in_scan[k - 1] : 0u;
                p0 = (qg - start + 1u) * kRun;
                hee = L.in_he[k];
                hbk = L.in_hb[k];
                cm = min(kRun, L.in_hs[k] - p0);
                if constexpr (!kUniform) {
                    ve = L.in_v[k];
                    the = L.in_thr[k];
                }
            }
            test_run<kLds>(G, j, pool, key, bm, prefilter, active, hee, hbk, p0, cm, ve, the, app, px, L, nlive);
        }
    }
    if constexpr (!kLds) flush_live(bm, L, nlive, app);
    wave_sync();
    return wave_sum(bytes);
}

// Record a finished set's per-id outputs.
__device__ __forceinline__ void record_set(const RRArgs &a, uint64_t idx, uint64_t off, uint32_t size, uint32_t root) {
    const uint64_t o = a.out_base + idx;
    a.stage_off[o] = off;
    a.sizes[o] = size;
    a.roots[o] = root;
    if (size > kBigSet) a.big_ids[atomicAdd(&a.ctr[kBigCount], 1ull)] = o;
}

// ---- phase A ---------------------------------------------------------------
// A pool-0 set of a graph whose RR sets are divided (Section 4.1) starts
// with the members of its root's small layers beside the root: they are
// marked and appended before the traversal (every lane of the wave calls it).
__device__ __forceinline__ void seed_forced(const GraphDesc &D, uint32_t root, uint32_t *bm, LocalAppend &app) {
    const HIM_GLOBAL unsigned long long *fo = uni_ptr((const HIM_GLOBAL unsigned long long *)D.force_off);
    if (fo == nullptr) return;
    const HIM_GLOBAL uint32_t *fm = uni_ptr((const HIM_GLOBAL uint32_t *)D.force);
    const uint64_t f0 = uni64(fo[root]), f1 = uni64(fo[root + 1]);
    const uint32_t lane = lane_id();
    for (uint64_t f = f0; f < f1; f += kWave) {
        uint32_t u = 0;
        bool fresh = false;
        if (f + lane < f1) {
            u = fm[f + lane];
            const uint32_t bit = 1u << (u & 31);
            fresh = (atomicOr(&bm[u >> 5], bit) & bit) == 0u;
        }
        app.push1(fresh, u);
    }
}

template <bool kLdsBitmap, bool kGaps>
__global__ __launch_bounds__(kWG) void k_rr_light(RRArgs a) {
    using Lds = typename std::conditional<kLdsBitmap, WaveLdsCore, WaveLds>::type;
    __shared__ Lds lds[kWavesPerWG];
    __shared__ uint32_t sort_s[kWavesPerWG][kSortMax];
    __shared__ uint32_t lbm[kLdsBitmap ? kWavesPerWG : 1][kLdsBitmap ? kLdsBitmapWords : 1];
    const uint32_t lane = lane_id(), wv = uni(threadIdx.x / kWave);
    uint32_t slot = blockIdx.x * kWavesPerWG + wv;
    Lds &L = lds[wv];
    uint32_t *sortb = sort_s[wv];
    uint32_t *list = a.lists + (uint64_t)slot * a.slot_n;
    uint32_t *bm;
    if constexpr (kLdsBitmap) {
        bm = lbm[wv];
        for (uint32_t i = lane; i < kLdsBitmapWords; i += kWave) bm[i] = 0u;
    } else {
        bm = a.bitmaps + (uint64_t)slot * a.slot_words;
    }
    wave_sync();
    bool can_defer = !kLdsBitmap;
    uint64_t bytes_done = 0, px = 0;

    for (;;) {
        unsigned long long idx = 0;
        if (lane == 0) idx = atomicAdd(&a.ctr[kWork], 1ull);
        idx = uni64(wave_bcast64(idx, 0));
        if (idx >= a.count) break;
        const uint32_t task = task_of(a, idx);
        const SetRef S = set_ref(a, task, idx);
        const GraphView &G = S.G;
        const uint32_t root = rr_root(G, a.qlog, S.j, S.pool, S.key);
        if (lane == 0) {
            list[0] = root;
            atomicOr(&bm[root >> 5], 1u << (root & 31));
        }
        LocalAppend app{list, 1u, G.n};
        if (S.pool == 0u) seed_forced(a.graphs[uni(a.tasks[task].graph)], root, bm, app);
        uint32_t head = 0;
        uint64_t spent = 0;
        bool deferred = false;

        while (head < app.size) {
            // queue entries were stored by other lanes of this wave: wait for
            // the stores and drop stale L1 lines before reading them
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const uint32_t nb = min((uint32_t)kWave, app.size - head);
            uint32_t v = 0, e0 = 0, d = 0;
            if (lane < nb) {
                v = list[head + lane];
                e0 = G.v_off[v];
                d = G.v_off[v + 1] - e0;
            }
            if (can_defer && (spent > a.budget || __ballot(d > a.heavy) != 0)) {
                // hand the set over to phase B and continue with a fresh slot
                uint32_t fresh_slot = 0;
                if (lane == 0) fresh_slot = (uint32_t)atomicAdd(&a.ctr[kFreeNext], 1ull);
                fresh_slot = wave_bcast(fresh_slot, 0);
                if (fresh_slot < a.slot_total) {
                    if (lane == 0) {
                        const uint32_t dd = (uint32_t)atomicAdd(&a.ctr[kDefCount], 1ull);
                        a.def_idx[dd] = idx;
                        a.def_root[dd] = root;
                        a.def_slot[dd] = slot;
                        a.def_head[dd] = head;
                        a.def_size[dd] = app.size;
                        a.def_task[dd] = task;
                    }
                    slot = fresh_slot;
                    list = a.lists + (uint64_t)slot * a.slot_n;
                    bm = a.bitmaps + (uint64_t)slot * a.slot_words;
                    deferred = true;
                    break;
                }
                can_defer = false;   // no spare slot left: this wave finishes its sets itself
            }
            head += nb;
            spent += wave_bcast(wave_incl_scan(d), kWave - 1);
            bytes_done += 20ull * nb;
            bytes_done += expand<kLdsBitmap, false, kGaps>(G, L, S.j, S.pool, S.key, bm, false, v, e0, d, app, px);
        }
        if (deferred) continue;
        const uint32_t size = app.size;

        // ---- output: ascending members into the stage --------------------
        unsigned long long off = 0;
        if (lane == 0) off = atomicAdd(&a.ctr[kBump], (unsigned long long)size);
        off = wave_bcast64(off, 0);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (off + size <= a.stage_cap) {
            if (size <= kSortMax) {
                uint32_t P2 = kWave;
                while (P2 < size) P2 <<= 1;
                for (uint32_t i = lane; i < P2; i += kWave) sortb[i] = i < size ? list[i] : 0xFFFFFFFFu;
                wave_sync();
                for (uint32_t k = 2; k <= P2; k <<= 1) {
                    for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
                        for (uint32_t i = lane; i < P2; i += kWave) {
                            const uint32_t x = i ^ jj;
                            if (x > i) {
                                const uint32_t p = sortb[i], qv = sortb[x];
                                if ((p > qv) == ((i & k) == 0)) {
                                    sortb[i] = qv;
                                    sortb[x] = p;
                                }
                            }
                        }
                        wave_sync();
                    }
                }
                for (uint32_t i = lane; i < size; i += kWave) a.stage[off + i] = sortb[i];
                wave_sync();
            } else {
                uint32_t written = 0;
                for (uint32_t w0 = 0; w0 < G.bm_words; w0 += kWave) {
                    const uint32_t wi = w0 + lane;
                    uint32_t word = wi < G.bm_words ? bm_load<kLdsBitmap>(bm, wi) : 0u;
                    const uint32_t cnt = (uint32_t)__popc(word);
                    const uint32_t incl = wave_incl_scan(cnt);
                    uint64_t pos = off + written + incl - cnt;
                    while (word) {
                        const uint32_t bit = (uint32_t)__ffs(word) - 1u;
                        word &= word - 1u;
                        if (pos < off + size) a.stage[pos] = wi * 32u + bit;
                        ++pos;
                    }
                    written += wave_bcast(incl, kWave - 1);
                }
            }
        }
        if (lane == 0) record_set(a, idx, off, size, root);
        // clear this set's marks (the bitmap is all-zero again afterwards)
        if (kLdsBitmap && size * 4u > G.bm_words) {
            for (uint32_t i = lane; i < G.bm_words; i += kWave) bm[i] = 0u;
        } else {
            for (uint32_t i = lane; i < size; i += kWave) bm[list[i] >> 5] = 0u;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        wave_sync();
    }
    if (lane == 0 && bytes_done) atomicAdd(&a.ctr[kBytesA], bytes_done);
    px = wave_sum(px);
    if (lane == 0 && px) atomicAdd(&a.ctr[kPhiloxA], (unsigned long long)px);
}

// ---- linear-threshold model ------------------------------------------------
// RR sets of the live-edge form of LT (Section 2.1, LT bullet): every vertex v
// keeps at most one of its c(v) channels -- (hyperedge, member) pairs in
// ascending hyperedge order and stored member order, v skipped -- each with
// weight W / 2^32, W = min(thr[v], floor(2^32 / c(v))) (thr = always-live
// counting as 2^32), so the weights into v sum to at most 1.  The Philox word
// at hyperedge slot kLtSlot, position 0, of (RR id, v) picks channel
// floor(x / W) when x < W c(v), none otherwise.  An RR set is the reverse
// walk from its root along kept channels until no channel is kept or the
// walk meets a vertex already in the set.
//
// One wave per set (persistent over the launch group's ids, like phase A).
// c(v) and the incidence holding the picked channel come from the graph's
// channel prefix over v's incidences (a 64-way search: each round the lanes
// probe 64 evenly spaced incidences of the remaining range); the lanes then
// find v's position in that hyperedge.  Lane 0 keeps the walk's list and
// visited bitmap (a slot of the phase-A workspace), so the membership test
// reads what the same lane wrote.  The set leaves ascending through the
// phase-A output path.
constexpr uint32_t kLtSlot = 0xFFFFFFFEu;

template <bool kLdsBitmap>
__global__ __launch_bounds__(kWG) void k_lt_walk(RRArgs a) {
    __shared__ uint32_t sort_s[kWavesPerWG][kSortMax];
    __shared__ uint32_t lbm[kLdsBitmap ? kWavesPerWG : 1][kLdsBitmap ? kLdsBitmapWords : 1];
    const uint32_t lane = lane_id(), wv = uni(threadIdx.x / kWave);
    const uint32_t slot = blockIdx.x * kWavesPerWG + wv;
    uint32_t *sortb = sort_s[wv];
    uint32_t *list = a.lists + (uint64_t)slot * a.slot_n;
    uint32_t *bm;
    if constexpr (kLdsBitmap) {
        bm = lbm[wv];
        for (uint32_t i = lane; i < kLdsBitmapWords; i += kWave) bm[i] = 0u;
    } else {
        bm = a.bitmaps + (uint64_t)slot * a.slot_words;
    }
    wave_sync();
    uint64_t bytes_done = 0, px = 0;
    for (;;) {
        unsigned long long idx = 0;
        if (lane == 0) idx = atomicAdd(&a.ctr[kWork], 1ull);
        idx = uni64(wave_bcast64(idx, 0));
        if (idx >= a.count) break;
        const uint32_t task = task_of(a, idx);
        const SetRef S = set_ref(a, task, idx);
        const GraphView &G = S.G;
        const uint32_t root = rr_root(G, a.qlog, S.j, S.pool, S.key);
        const HIM_GLOBAL unsigned long long *chan =
            uni_ptr((const HIM_GLOBAL unsigned long long *)a.graphs[uni(a.tasks[task].graph)].chan);
        if (lane == 0) {
            list[0] = root;
            bm[root >> 5] |= 1u << (root & 31);
        }
        uint32_t size = 1, cur = root;
        for (;;) {
            const uint32_t e0 = uni(G.v_off[cur]), e1 = uni(G.v_off[cur + 1]);
            const uint64_t base = uni64(chan[e0]);
            const uint64_t C = uni64(chan[e1]) - base;   // c(v)
            bytes_done += 36ull;
            if (C == 0) break;
            const uint32_t thr = uni(G.thr[cur]);
            const uint64_t cap = (1ull << 32) / C;
            const uint64_t W = min(thr == kAlways ? (1ull << 32) : (uint64_t)thr, cap);
            const uint32_t x = uni(philox4x32_10(coin_counter(S.j, kLtSlot, cur, S.pool, 0u), S.key).x);
            ++px;
            if ((uint64_t)x >= W * C) break;   // W = 0 included: no channel is kept
            // the incidence e holding channel k: the last one in [e0, e1)
            // with chan[e] <= base + k (chan[e0] = base qualifies; the next
            // prefix exceeds it, so e has at least one channel)
            const uint64_t t = base + (uint64_t)x / W;
            uint32_t lo = e0, hi = e1;   // the answer lies in [lo, hi)
            while (hi - lo > (uint32_t)kWave) {
                const uint32_t step = (hi - lo + kWave - 1) / kWave;
                const uint32_t probe = lo + lane * step;
                const uint64_t ok = __ballot(probe < hi && chan[probe] <= t);
                const uint32_t l = 63u - (uint32_t)__clzll((long long)ok);   // lane 0 always qualifies
                lo += l * step;
                hi = min(hi, lo + step);
                bytes_done += 8ull;
            }
            const uint64_t ok = __ballot(lo + lane < hi && chan[lo + lane] <= t);
            const uint32_t e = lo + 63u - (uint32_t)__clzll((long long)ok);
            const unsigned long long bl = uni64(G.v_hbs[e]);
            const uint64_t k = t - uni64(chan[e]);   // rank among e's channels
            const uint32_t hb = (uint32_t)bl, hs = (uint32_t)(bl >> 32);
            // member k of the hyperedge with cur skipped
            uint32_t pc = hs;
            for (uint32_t p0 = 0; p0 < hs; p0 += kWave) {
                const uint64_t hit = __ballot(p0 + lane < hs && G.he_mem[hb + p0 + lane] == cur);
                if (hit) {
                    pc = p0 + (uint32_t)__ffsll((unsigned long long)hit) - 1u;
                    break;
                }
            }
            const uint32_t u = uni(G.he_mem[hb + ((uint32_t)k < pc ? (uint32_t)k : (uint32_t)k + 1u)]);
            bytes_done += 4ull * hs + 24ull;
            uint32_t seen = 0;
            if (lane == 0) {
                const uint32_t bit = 1u << (u & 31);
                seen = (bm_load<kLdsBitmap>(bm, u >> 5) & bit) != 0u;
                if (!seen) {
                    bm[u >> 5] |= bit;
                    list[size] = u;
                }
            }
            if (wave_bcast(seen, 0)) break;
            ++size;
            cur = u;
        }

        // ---- output: ascending members into the stage, as in phase A -----
        unsigned long long off = 0;
        if (lane == 0) off = atomicAdd(&a.ctr[kBump], (unsigned long long)size);
        off = wave_bcast64(off, 0);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // lane 0's list and bitmap stores
        if (off + size <= a.stage_cap) {
            if (size <= kSortMax) {
                uint32_t P2 = kWave;
                while (P2 < size) P2 <<= 1;
                for (uint32_t i = lane; i < P2; i += kWave) sortb[i] = i < size ? list[i] : 0xFFFFFFFFu;
                wave_sync();
                for (uint32_t kk = 2; kk <= P2; kk <<= 1) {
                    for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
                        for (uint32_t i = lane; i < P2; i += kWave) {
                            const uint32_t xx = i ^ jj;
                            if (xx > i) {
                                const uint32_t pv = sortb[i], qv = sortb[xx];
                                if ((pv > qv) == ((i & kk) == 0)) {
                                    sortb[i] = qv;
                                    sortb[xx] = pv;
                                }
                            }
                        }
                        wave_sync();
                    }
                }
                for (uint32_t i = lane; i < size; i += kWave) a.stage[off + i] = sortb[i];
                wave_sync();
            } else {
                uint32_t written = 0;
                for (uint32_t w0 = 0; w0 < G.bm_words; w0 += kWave) {
                    const uint32_t wi = w0 + lane;
                    uint32_t word = wi < G.bm_words ? bm_load<kLdsBitmap>(bm, wi) : 0u;
                    const uint32_t cnt = (uint32_t)__popc(word);
                    const uint32_t incl = wave_incl_scan(cnt);
                    uint64_t pos = off + written + incl - cnt;
                    while (word) {
                        const uint32_t bit = (uint32_t)__ffs(word) - 1u;
                        word &= word - 1u;
                        if (pos < off + size) a.stage[pos] = wi * 32u + bit;
                        ++pos;
                    }
                    written += wave_bcast(incl, kWave - 1);
                }
            }
        }
        if (lane == 0) record_set(a, idx, off, size, root);
        for (uint32_t i = lane; i < size; i += kWave) bm[list[i] >> 5] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        wave_sync();
    }
    if (lane == 0 && bytes_done) atomicAdd(&a.ctr[kBytesA], bytes_done);
    if (lane == 0 && px) atomicAdd(&a.ctr[kPhiloxA], (unsigned long long)px);
}

// ---- stratified setting -------------------------------------------------------
// RR sets of the stratified setting (Section 3.1.1, "Activation probability"
// and "Sampling strategy"; Algorithm 3's per-layer draws).  For a popped
// vertex v with l layers and layer i of n members: the layer probability is
// P = 1 / (i ln(l + 1)), a member's p = min(1, P / n); the Philox blocks at
// counter (j_lo, i, v, pool << 31 | j_hi << 24 | r) give U from block 0's
// first two words and the selection draws from its last two and every word
// of the later blocks.  The count h inverts U: Binomial(n, p) for n <= 20,
// else Poisson(P) truncated at min(n, kMaxPick); then h members are picked
// one at a time, draw x picking index floor(x (n - r) / 2^32) among those not
// picked yet (ascending).  ln(l + 1) and e^-P come from the graph's
// host-evaluated tables; the count arithmetic is IEEE double with no fused
// multiply-adds, in the order the recursions state.
//
// One wave per set (persistent, phase A's slots, bitmaps and output path):
// the lanes take the set's queued vertices 64 at a time and each walks its
// vertex's layers; picked members go through the visited bitmap (atomic or:
// the lane that sets the bit appends the member at a wave counter in LDS).
// Picks of a layer of at most 32 members live in a bit mask; larger layers
// keep their picked indices, ascending, in a per-lane scratch list.
constexpr uint32_t kMaxPick = 64;

__device__ __forceinline__ uint32_t layer_count(uint32_t n, uint32_t i, uint32_t l, double U,
                                                const HIM_GLOBAL double *ln, const HIM_GLOBAL double *expm) {
#pragma clang fp contract(off)
    const double P = 1.0 / ((double)i * ln[l]);
    const double p = P / (double)n;
    if (n <= 20u) {
        if (p >= 1.0) return n;
        const double q = 1.0 - p;
        double prob = 1.0;
        for (uint32_t t = 0; t < n; ++t) prob = prob * q;
        const double ratio = p / q;
        double cdf = prob;
        uint32_t h = 0;
        while (U >= cdf && h < n) {
            prob = ((prob * (double)(n - h)) / (double)(h + 1)) * ratio;
            ++h;
            cdf = cdf + prob;
        }
        return h;
    }
    double prob = expm[(size_t)l * (l - 1) / 2 + i - 1];
    double cdf = prob;
    const uint32_t hmax = min(n, kMaxPick);
    uint32_t h = 0;
    while (U >= cdf && h < hmax) {
        prob = (prob * P) / (double)(h + 1);
        ++h;
        cdf = cdf + prob;
    }
    return h;
}

template <bool kLdsBitmap>
__global__ __launch_bounds__(kWG) void k_layered(RRArgs a, uint32_t *__restrict__ pick_scratch) {
    __shared__ uint32_t sort_s[kWavesPerWG][kSortMax];
    __shared__ uint32_t lbm[kLdsBitmap ? kWavesPerWG : 1][kLdsBitmap ? kLdsBitmapWords : 1];
    __shared__ uint32_t tail_s[kWavesPerWG];
    const uint32_t lane = lane_id(), wv = uni(threadIdx.x / kWave);
    const uint32_t slot = blockIdx.x * kWavesPerWG + wv;
    uint32_t *sortb = sort_s[wv];
    uint32_t *list = a.lists + (uint64_t)slot * a.slot_n;
    uint32_t *picks = pick_scratch + ((uint64_t)slot * kWave + lane) * kMaxPick;
    uint32_t *bm;
    if constexpr (kLdsBitmap) {
        bm = lbm[wv];
        for (uint32_t i = lane; i < kLdsBitmapWords; i += kWave) bm[i] = 0u;
    } else {
        bm = a.bitmaps + (uint64_t)slot * a.slot_words;
    }
    wave_sync();
    uint64_t bytes_done = 0, px = 0;
    for (;;) {
        unsigned long long idx = 0;
        if (lane == 0) idx = atomicAdd(&a.ctr[kWork], 1ull);
        idx = uni64(wave_bcast64(idx, 0));
        if (idx >= a.count) break;
        const uint32_t task = task_of(a, idx);
        const SetRef S = set_ref(a, task, idx);
        const GraphView &G = S.G;
        const GraphDesc &D = a.graphs[uni(a.tasks[task].graph)];
        const HIM_GLOBAL unsigned long long *nb_off = uni_ptr((const HIM_GLOBAL unsigned long long *)D.lay_nb_off);
        const HIM_GLOBAL unsigned long long *ly_off = uni_ptr((const HIM_GLOBAL unsigned long long *)D.lay_ly_off);
        const HIM_GLOBAL uint32_t *nb = uni_ptr((const HIM_GLOBAL uint32_t *)D.lay_nb);
        const HIM_GLOBAL uint32_t *ly_end = uni_ptr((const HIM_GLOBAL uint32_t *)D.lay_ly_end);
        const HIM_GLOBAL uint32_t *lv_of = uni_ptr((const HIM_GLOBAL uint32_t *)D.l);
        const HIM_GLOBAL double *ln = uni_ptr((const HIM_GLOBAL double *)D.lay_ln);
        const HIM_GLOBAL double *expm = uni_ptr((const HIM_GLOBAL double *)D.lay_expm);
        const uint32_t root = rr_root(G, a.qlog, S.j, S.pool, S.key);
        if (lane == 0) {
            list[0] = root;
            if constexpr (kLdsBitmap) bm[root >> 5] |= 1u << (root & 31);
            else atomicOr(&bm[root >> 5], 1u << (root & 31));
            tail_s[wv] = 1u;
        }
        wave_sync();
        uint32_t head = 0, size = 1;
        while (head < size) {
            // queue entries were stored by other lanes of this wave
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const uint32_t nbq = min((uint32_t)kWave, size - head);
            if (lane < nbq) {
                const uint32_t v = list[head + lane];
                const uint32_t l = lv_of[v];
                const uint64_t base = nb_off[v], lb = ly_off[v];
                uint32_t lo = 0;
                bytes_done += 20ull + 4ull * l;
                for (uint32_t i = 1; i <= l; ++i) {
                    const uint32_t hi = ly_end[lb + i - 1], n = hi - lo;
                    uint4 w = philox4x32_10(make_uint4((uint32_t)S.j, i, v,
                                                       (S.pool << 31) | ((uint32_t)(S.j >> 32) << 24)),
                                            S.key);
                    ++px;
                    const double U = (double)((uint64_t)(w.x >> 11) | ((uint64_t)w.y << 21)) * 0x1.0p-53;
                    const uint32_t h = layer_count(n, i, l, U, ln, expm);
                    uint32_t mask = 0, np = 0, word = 2, blk = 0;
                    for (uint32_t r = 0; r < h; ++r) {
                        if (word == 4) {
                            w = philox4x32_10(make_uint4((uint32_t)S.j, i, v,
                                                         (S.pool << 31) | ((uint32_t)(S.j >> 32) << 24) | ++blk),
                                              S.key);
                            ++px;
                            word = 0;
                        }
                        const uint32_t x = word == 0 ? w.x : word == 1 ? w.y : word == 2 ? w.z : w.w;
                        ++word;
                        const uint32_t aidx = (uint32_t)(((uint64_t)x * (uint64_t)(n - r)) >> 32);
                        uint32_t pi;
                        if (n <= 32u) {
                            // the aidx-th clear bit of the mask
                            uint32_t c = aidx;
                            pi = 0;
                            for (uint32_t t = 0; t < n; ++t) {
                                if ((mask >> t) & 1u) continue;
                                if (c == 0) {
                                    pi = t;
                                    break;
                                }
                                --c;
                            }
                            mask |= 1u << pi;
                        } else {
                            pi = aidx;
                            uint32_t t = 0;
                            for (; t < np; ++t) {
                                const uint32_t q = picks[t];
                                if (q <= pi) ++pi;
                                else break;
                            }
                            for (uint32_t z = np; z > t; --z) picks[z] = picks[z - 1];
                            picks[t] = pi;
                            ++np;
                        }
                        const uint32_t u = nb[base + lo + pi];
                        const uint32_t bit = 1u << (u & 31);
                        if ((atomicOr(&bm[u >> 5], bit) & bit) == 0u) {
                            const uint32_t pos = atomicAdd(&tail_s[wv], 1u);
                            list[pos] = u;
                        }
                    }
                    bytes_done += 8ull + 4ull * h;
                    lo = hi;
                }
            }
            wave_sync();
            head += nbq;
            size = uni(tail_s[wv]);
        }

        // ---- output: ascending members into the stage, as in phase A -----
        unsigned long long off = 0;
        if (lane == 0) off = atomicAdd(&a.ctr[kBump], (unsigned long long)size);
        off = wave_bcast64(off, 0);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (off + size <= a.stage_cap) {
            if (size <= kSortMax) {
                uint32_t P2 = kWave;
                while (P2 < size) P2 <<= 1;
                for (uint32_t i = lane; i < P2; i += kWave) sortb[i] = i < size ? list[i] : 0xFFFFFFFFu;
                wave_sync();
                for (uint32_t kk = 2; kk <= P2; kk <<= 1) {
                    for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
                        for (uint32_t i = lane; i < P2; i += kWave) {
                            const uint32_t xx = i ^ jj;
                            if (xx > i) {
                                const uint32_t pv = sortb[i], qv = sortb[xx];
                                if ((pv > qv) == ((i & kk) == 0)) {
                                    sortb[i] = qv;
                                    sortb[xx] = pv;
                                }
                            }
                        }
                        wave_sync();
                    }
                }
                for (uint32_t i = lane; i < size; i += kWave) a.stage[off + i] = sortb[i];
                wave_sync();
            } else {
                uint32_t written = 0;
                for (uint32_t w0 = 0; w0 < G.bm_words; w0 += kWave) {
                    const uint32_t wi = w0 + lane;
                    uint32_t wd = wi < G.bm_words ? bm_load<kLdsBitmap>(bm, wi) : 0u;
                    const uint32_t cnt = (uint32_t)__popc(wd);
                    const uint32_t incl = wave_incl_scan(cnt);
                    uint64_t pos = off + written + incl - cnt;
                    while (wd) {
                        const uint32_t bit = (uint32_t)__ffs(wd) - 1u;
                        wd &= wd - 1u;
                        if (pos < off + size) a.stage[pos] = wi * 32u + bit;
                        ++pos;
                    }
                    written += wave_bcast(incl, kWave - 1);
                }
            }
        }
        if (lane == 0) record_set(a, idx, off, size, root);
        for (uint32_t i = lane; i < size; i += kWave) bm[list[i] >> 5] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        wave_sync();
    }
    bytes_done = wave_sum(bytes_done);
    px = wave_sum(px);
    if (lane == 0 && bytes_done) atomicAdd(&a.ctr[kBytesA], bytes_done);
    if (lane == 0 && px) atomicAdd(&a.ctr[kPhiloxA], (unsigned long long)px);
}

// ---- phase B ---------------------------------------------------------------
// Item: x = deferred set d | heavy << 31; light: y = first queue index,
// z = count (<= 64); heavy: y = vertex, z = first incidence, w = end.
// One atomicAdd per planning batch.  A reservation that crosses the cap is
// abandoned: its slots below the cap are filled with skip markers (x = ~0)
// by the reserving wave, so k_expand never reads an unwritten item.
constexpr uint32_t kSkipItem = 0xFFFFFFFFu;

// Owner lane of heavy-chunk slot q: binary search over the wave's inclusive
// scan of per-lane chunk counts, read through lane shuffles (every lane of
// the wave calls it).
__device__ __forceinline__ uint32_t owner_of(uint32_t hscan, uint32_t q) {
    return scan_owner([hscan](uint32_t k) { return (uint32_t)__shfl((int)hscan, (int)k, kWave); }, q);
}
constexpr uint32_t kShareMax = 16;   // waves that may share one item
constexpr uint32_t kContLevels = 8;  // levels a wave may expand past its item

// k_plan and k_expand read their arguments from device memory, so that a
// captured batch of supersteps serves every launch group.
__global__ __launch_bounds__(kWG) void k_plan(const RRArgs *__restrict__ ap, uint32_t parity) {
    const RRArgs a = *ap;
    const uint32_t lane = lane_id(), wv = uni(threadIdx.x / kWave);
    const uint32_t waves = gridDim.x * kWavesPerWG;
    const uint32_t ndef = uni((uint32_t)a.ctr[kDefCount]);   // sets phase A deferred
    uint64_t taken = 0;   // frontier entries this wave planned (progress count)
    for (uint32_t d = blockIdx.x * kWavesPerWG + wv; d < ndef; d += waves) {
        const uint32_t head0 = uni(a.def_head[d]);
        uint32_t head = head0;
        const uint32_t size = uni(a.def_size[d]);
        const uint32_t *list = a.lists + (uint64_t)uni(a.def_slot[d]) * a.slot_n;
        const GraphView G = graph_view(a.graphs[uni(a.tasks[uni(a.def_task[d])].graph)]);
        while (head < size) {
            uint32_t nb = min((uint32_t)kWave, size - head);
            uint32_t v = 0, e0 = 0, deg = 0, hv = 0, light = 0, cv = a.chunk;
            const uint32_t raw = lane < nb ? list[head + lane] : kExpanded;
            if (__ballot((raw & kExpanded) == 0u) == 0) {   // all expanded already
                head += nb;
                continue;
            }
            if ((raw & kExpanded) == 0u) {
                v = raw;
                e0 = G.v_off[v];
                deg = G.v_off[v + 1] - e0;
                // a heavy vertex is cut into chunks of cv incidences
                const HeavySplit hs = heavy_split(deg, a.chunk);
                cv = hs.len;
                hv = hs.count;
                light = hv ? 0u : deg;
            }
            // light vertices form segments of consecutive queue entries
            const uint32_t lscan = wave_incl_scan(light);
            const uint32_t seg = segment_of(lscan, light, a.seg);
            const uint32_t prev_seg = __shfl_up(seg, 1, kWave);
            const bool first = lane < nb && (lane == 0 || seg != prev_seg);
            uint64_t firsts = __ballot(first);
            uint32_t nseg = (uint32_t)__popcll(firsts);
            uint32_t hscan = wave_incl_scan(hv);
            uint32_t need = nseg + wave_bcast(hscan, kWave - 1);
            if (need > kItemCap) {   // too many heavy chunks at once: plan one vertex
                nb = 1;
                if (lane > 0) hv = 0;
                firsts = 1ull;
                nseg = 1;
                hscan = wave_incl_scan(hv);
                need = 1u + wave_bcast(hscan, kWave - 1);
            }
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(&a.ctr[kItems + parity], (unsigned long long)need);
            base = wave_bcast64(base, 0);
            if (base + need > kItemCap) {
                for (uint64_t x = base + lane; x < kItemCap; x += kWave) a.items[x].x = kSkipItem;
                break;
            }
            if (lane < nb && ((firsts >> lane) & 1ull)) {
                // segment = this lane up to the next first lane (or nb)
                const uint64_t above = lane + 1 < 64 ? (firsts >> (lane + 1)) << (lane + 1) : 0ull;
                const uint32_t next = above ? (uint32_t)__ffsll((unsigned long long)above) - 1u : nb;
                a.items[base + lane_rank(firsts)] = make_uint4(d, head + lane, min(next, nb) - lane, 0u);
            }
            // heavy chunks, spread over the wave (a hub has hundreds)
            const uint32_t H = wave_bcast(hscan, kWave - 1);
            for (uint32_t q0 = 0; q0 < H; q0 += kWave) {
                const uint32_t q = q0 + lane;
                const uint32_t k = owner_of(hscan, min(q, H - 1u));
                const uint32_t excl = (uint32_t)__shfl((int)(hscan - hv), (int)k, kWave);
                const uint32_t vk = (uint32_t)__shfl((int)v, (int)k, kWave);
                const uint32_t ek = (uint32_t)__shfl((int)e0, (int)k, kWave);
                const uint32_t ck = (uint32_t)__shfl((int)cv, (int)k, kWave);
                const uint32_t dk = (uint32_t)__shfl((int)deg, (int)k, kWave);
                if (q < H) {
                    const ChunkRange cr = chunk_range(ek, dk, ck, q - excl);
                    a.items[base + nseg + q] = make_uint4(d | 0x80000000u, vk, cr.lo, cr.hi);
                }
            }
            head += nb;
        }
        if (lane == 0) a.def_head[d] = head;
        taken += head - head0;
    }
    if (lane == 0 && taken) atomicAdd(&a.ctr[kPlanned], (unsigned long long)taken);
}

template <bool kGaps>
__global__ __launch_bounds__(kWG) void k_expand(const RRArgs *__restrict__ ap, uint32_t parity) {
    const RRArgs a = *ap;
    __shared__ WaveLds lds[kWavesPerWG];
    const uint32_t wv = uni(threadIdx.x / kWave);
    WaveLds &L = lds[wv];
    const uint64_t nitems = min(a.ctr[kItems + parity], (unsigned long long)kItemCap);
    if (blockIdx.x == 0 && threadIdx.x == 0) a.ctr[kItems + (parity ^ 1u)] = 0ull;   // next superstep's counter
    uint64_t bytes_done = 0, px = 0;
    // items have bounded cost (< seg + chunk incidences), so a static strided
    // assignment balances well and needs no shared counter.  With fewer items
    // than waves (the thin tail of a traversal), W waves share each item.
    const uint64_t waves = (uint64_t)gridDim.x * kWavesPerWG;
    uint32_t W = 1;
    while (W < kShareMax && 2ull * W * nitems <= waves) W <<= 1;
    const uint64_t gw = (uint64_t)blockIdx.x * kWavesPerWG + wv, groups = waves / W;
    const uint32_t w = (uint32_t)(gw & (W - 1));
    const uint32_t lane = lane_id();
    for (uint64_t it = gw / W; it < nitems && gw < groups * W; it += groups) {
        const uint4 ld = a.items[it];
        const uint4 item = make_uint4(uni(ld.x), uni(ld.y), uni(ld.z), uni(ld.w));
        if (item.x == kSkipItem) continue;
        const uint32_t d = item.x & 0x7FFFFFFFu;
        const bool heavy = (item.x >> 31) != 0u;
        const uint32_t slot = uni(a.def_slot[d]);
        const SetRef S = set_ref(a, uni(a.def_task[d]), uni64(a.def_idx[d]));
        const GraphView &G = S.G;
        uint32_t *list = a.lists + (uint64_t)slot * a.slot_n;
        uint32_t *bm = a.bitmaps + (uint64_t)slot * a.slot_words;
        uint32_t *size_p = &a.def_size[d];
        const bool prefilter =
            uni(__hip_atomic_load(size_p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >= a.prefilter_min;
        ContAppend app{list, size_p, G.n, L.cont_u, L.cont_pos, 0u};
        if (!heavy) {
            uint32_t v = 0, e0 = 0, deg = 0;
            const uint32_t raw = lane < item.z ? list[item.y + lane] : kExpanded;
            if ((raw & kExpanded) == 0u) {   // entries marked expanded are done
                v = raw;
                e0 = G.v_off[v];
                deg = G.v_off[v + 1] - e0;
                if (heavy_split(deg, a.chunk).count) deg = 0;   // expanded by its heavy items
            }
            if (w == 0) bytes_done += 20ull * (uint64_t)__popcll(__ballot((raw & kExpanded) == 0u));
            bytes_done += expand<false, false, kGaps>(G, L, S.j, S.pool, S.key, bm, prefilter, v, e0, deg, app, px, w, W);
        } else {
            // one heavy vertex: incidences [item.z, item.w) of vertex item.y
            bytes_done += expand<false, true, kGaps>(G, L, S.j, S.pool, S.key, bm, prefilter, item.y, item.z,
                                              item.w - item.z, app, px, w, W);
        }
        // Continuation: when this wave appended at most 64 members, all light
        // and together under seg incidences, it expands them itself (up to
        // kContLevels levels) and marks their queue entries expanded, so the
        // thin tail of a traversal does not take one superstep per level.
        // Nobody else reads those entries before the next superstep.
        for (uint32_t lev = 0; G.n <= kExpanded && lev < kContLevels; ++lev) {
            const uint32_t cn = app.count;
            if (cn == 0 || cn > kWave) break;
            wave_sync();
            uint32_t v = 0, e0 = 0, deg = 0, pos = 0;
            if (lane < cn) {
                v = L.cont_u[lane];
                pos = L.cont_pos[lane];
                e0 = G.v_off[v];
                deg = G.v_off[v + 1] - e0;
            }
            const uint32_t tot = wave_bcast(wave_incl_scan(deg), kWave - 1);
            if (__ballot(lane < cn && deg > a.chunk) != 0 || tot > a.seg) break;   // left to k_plan
            wave_sync();
            if (lane < cn) list[pos] = v | kExpanded;
            app.count = 0;
            bytes_done += 20ull * cn;
            bytes_done += expand<false, false, kGaps>(G, L, S.j, S.pool, S.key, bm, prefilter, v, e0, deg, app, px, 0u, 1u);
        }
    }
    if (lane == 0 && bytes_done) atomicAdd(&a.ctr[kBytesB], bytes_done);
    px = wave_sum(px);
    if (lane == 0 && px) atomicAdd(&a.ctr[kPhilox], (unsigned long long)px);
}

// One workgroup per deferred set: ascending members into the stage, per-id
// outputs, then the set's marks are cleared.
__global__ __launch_bounds__(kWG) void k_finish(RRArgs a, uint32_t ndef) {
    __shared__ uint32_t buf[kSortMaxWG];
    __shared__ uint32_t wave_tot[kWavesPerWG];
    __shared__ unsigned long long off_s;
    __shared__ uint32_t running;
    const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    for (uint32_t d = blockIdx.x; d < ndef; d += gridDim.x) {
        const uint32_t size = a.def_size[d];
        uint32_t *list = a.lists + (uint64_t)a.def_slot[d] * a.slot_n;
        uint32_t *bm = a.bitmaps + (uint64_t)a.def_slot[d] * a.slot_words;
        const uint32_t words = a.graphs[a.tasks[a.def_task[d]].graph].bm_words;
        if (threadIdx.x == 0) off_s = atomicAdd(&a.ctr[kBump], (unsigned long long)size);
        __syncthreads();
        const uint64_t off = off_s;
        if (off + size <= a.stage_cap) {
            if (size <= kSortMaxWG) {
                uint32_t P2 = kWG;
                while (P2 < size) P2 <<= 1;
                for (uint32_t i = threadIdx.x; i < P2; i += kWG) buf[i] = i < size ? (list[i] & ~kExpanded) : 0xFFFFFFFFu;
                __syncthreads();
                for (uint32_t k = 2; k <= P2; k <<= 1) {
                    for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
                        for (uint32_t i = threadIdx.x; i < P2; i += kWG) {
                            const uint32_t x = i ^ jj;
                            if (x > i) {
                                const uint32_t p = buf[i], qv = buf[x];
                                if ((p > qv) == ((i & k) == 0)) {
                                    buf[i] = qv;
                                    buf[x] = p;
                                }
                            }
                        }
                        __syncthreads();
                    }
                }
                for (uint32_t i = threadIdx.x; i < size; i += kWG) a.stage[off + i] = buf[i];
            } else {
                if (threadIdx.x == 0) running = 0;
                __syncthreads();
                for (uint32_t w0 = 0; w0 < words; w0 += kWG) {
                    const uint32_t wi = w0 + threadIdx.x;
                    uint32_t word = wi < words ? bm[wi] : 0u;
                    const uint32_t cnt = (uint32_t)__popc(word);
                    const uint32_t incl = wave_incl_scan(cnt);
                    if (lane == kWave - 1) wave_tot[wv] = incl;
                    __syncthreads();
                    uint32_t before = running;
                    for (uint32_t q = 0; q < wv; ++q) before += wave_tot[q];
                    uint64_t pos = off + before + incl - cnt;
                    while (word) {
                        const uint32_t bit = (uint32_t)__ffs(word) - 1u;
                        word &= word - 1u;
                        if (pos < off + size) a.stage[pos] = wi * 32u + bit;
                        ++pos;
                    }
                    __syncthreads();
                    if (threadIdx.x == kWG - 1) running = before + incl;
                    __syncthreads();
                }
            }
        }
        if (threadIdx.x == 0) record_set(a, a.def_idx[d], off, size, a.def_root[d]);
        __syncthreads();
        if (size > words) {
            for (uint32_t i = threadIdx.x; i < words; i += kWG) bm[i] = 0u;
        } else {
            for (uint32_t i = threadIdx.x; i < size; i += kWG) bm[(list[i] & ~kExpanded) >> 5] = 0u;
        }
        __syncthreads();
    }
}

// ---- bundled mode: 64 sets per bundle, bit-parallel over the sets ----------
// For graphs whose RR sets are large (supercritical cascades), the sets of a
// launch group -- one task, launch indices in bundles of 64 -- grow together,
// level by level.  Per bundle and vertex u, seen[u] has bit s when u is in
// set s of the bundle and nxt[u] the bits found in the current level.  A
// frontier entry (bundle, v, mask) expands v once for every set in mask: v's
// incidences and their members are read once, seen[u] removes the sets that
// already hold u, and only the remaining (set, quad) pairs draw their Philox
// block.  RR sets are reachability closures, so the sets equal those of the
// per-set traversal.
constexpr uint32_t kMsSets = 64;
constexpr uint32_t kMsOutVerts = 4096;   // vertices per output block (16 per thread)

// kMsFetch: next work item of the running expansion (waves fetch items one at
// a time; item costs vary with hyperedge sizes).
enum MsCtr {
    kMsCur = 0, kMsNext, kMsItems, kMsPending, kMsLevelDone, kMsDone, kMsEpoch, kMsOverflow, kMsFetch, kMsNumCtr
};

struct MsArgs {
    GraphDesc graph;
    const unsigned long long *bytesw;   // algorithmic bytes of each vertex as a member
    uint64_t first_id;                  // RR id of launch index 0
    uint32_t pool, key0, key1, qlog;
    uint32_t nbundles, chunk, seg;
    uint32_t filter;                    // entries with this many sets read seen masks before coins
    uint64_t count;                     // sets: launch indices [0, count)
    uint64_t stride;                    // words per bundle in seen / nxt (>= n)
    unsigned long long *seen, *nxt;
    uint32_t *cur_b, *cur_v;            // frontier entries (bundle, vertex) ...
    unsigned long long *cur_m;          // ... and their set masks
    uint32_t *nx_b, *nx_v;              // vertices reached in the current level
    uint32_t *batch_epoch;              // per 64 frontier entries: level in which they were planned
    uint64_t list_cap;                  // entries of each list
    unsigned long long *ctr;            // MsCtr
    unsigned long long *bytes;          // algorithmic bytes (RR counter block)
    unsigned long long *philox;         // Philox blocks drawn (RR counter block)
    uint4 *items;
    uint32_t *vcnt;                     // output: per (bundle, vertex block, set) counts
    uint32_t nvb;                       // vertex blocks per bundle
};

constexpr uint32_t kMsLiveCap = 512;   // live channels a wave holds before marking them

struct MsLds {
    // level 2: frontier entries of the wave
    uint32_t fr_scan[kWave], fr_v[kWave], fr_e0[kWave], fr_b[kWave], fr_thr[kWave];
    unsigned long long fr_m[kWave];
    // level 3: one incidence per lane (in_k: its frontier entry's lane)
    uint32_t in_scan[kWave], in_he[kWave], in_hb[kWave], in_hs[kWave], in_k[kWave];
    // live channels waiting to be marked: (member, bundle << 6 | set)
    uint2 live[kMsLiveCap];
};

// Position of the r-th set bit (r < popcount(m)) of m.
__device__ __forceinline__ uint32_t nth_bit(unsigned long long m, uint32_t r) {
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t w = 32; w > 0; w >>= 1) {
        const unsigned long long low = m & ((1ull << w) - 1ull);
        const uint32_t c = (uint32_t)__popcll(low);
        if (r >= c) {
            r -= c;
            m >>= w;
            pos += w;
        } else {
            m = low;
        }
    }
    return pos;
}

__device__ __forceinline__ void ms_append_next(const MsArgs &m, uint32_t b, uint32_t u) {
    const unsigned long long pos = atomicAdd(&m.ctr[kMsNext], 1ull);
    if (pos < m.list_cap) {
        m.nx_b[pos] = b;
        m.nx_v[pos] = u;
    } else {
        atomicOr(&m.ctr[kMsOverflow], 1ull);
    }
}

// Roots: set s of bundle b is launch index 64 b + s.
__global__ __launch_bounds__(kWG) void k_ms_roots(MsArgs m, RRArgs a) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.count) return;
    const GraphView G = graph_view(m.graph);
    const uint32_t root = rr_root(G, m.qlog, m.first_id + i, m.pool, make_uint2(m.key0, m.key1));
    a.roots[a.out_base + i] = root;
    const uint32_t b = (uint32_t)(i / kMsSets), s = (uint32_t)(i % kMsSets);
    const unsigned long long old = atomicOr(&m.nxt[(uint64_t)b * m.stride + root], 1ull << s);
    if (old == 0ull) ms_append_next(m, b, root);
    // divided RR sets (Section 4.1): a pool-0 set also starts from the
    // members of its root's small layers
    if (m.pool == 0u && m.graph.force_off != nullptr) {
        for (unsigned long long f = m.graph.force_off[root]; f < m.graph.force_off[root + 1]; ++f) {
            const uint32_t u = m.graph.force[f];
            const unsigned long long o2 = atomicOr(&m.nxt[(uint64_t)b * m.stride + u], 1ull << s);
            if (o2 == 0ull) ms_append_next(m, b, u);
        }
    }
}

// New level: the vertices reached in the last one, with the sets that did not
// hold them yet, become the frontier.  Runs only once the level's frontier
// is fully planned and expanded.
__global__ __launch_bounds__(kWG) void k_ms_advance(MsArgs m) {
    if (m.ctr[kMsLevelDone] == 0ull) return;
    const uint64_t cnt = min(m.ctr[kMsNext], (unsigned long long)m.list_cap);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t b = m.nx_b[i], u = m.nx_v[i];
        const uint64_t w = (uint64_t)b * m.stride + u;
        const unsigned long long found = m.nxt[w];
        m.nxt[w] = 0ull;
        const unsigned long long fresh = found & ~m.seen[w];
        if (fresh) {
            m.seen[w] |= fresh;   // each (bundle, vertex) appears once in the list
            const unsigned long long pos = atomicAdd(&m.ctr[kMsCur], 1ull);
            if (pos < m.list_cap) {
                m.cur_b[pos] = b;
                m.cur_v[pos] = u;
                m.cur_m[pos] = fresh;
            } else {
                atomicOr(&m.ctr[kMsOverflow], 1ull);
            }
        }
    }
}

// Level bookkeeping between the kernels of one step (a single thread).
// After expansion: the level is done once every frontier batch was planned.
__global__ void k_ms_ctl_expanded(unsigned long long *ctr) {
    if (ctr[kMsPending] == 0ull) {
        ctr[kMsLevelDone] = 1ull;
        ctr[kMsCur] = 0ull;
        ctr[kMsEpoch] += 1ull;
    } else {
        ctr[kMsLevelDone] = 0ull;
    }
    ctr[kMsItems] = 0ull;
    ctr[kMsFetch] = 0ull;
}

// After advancing: the new level's batches are pending; no frontier, done.
__global__ void k_ms_ctl_advanced(unsigned long long *ctr, uint64_t list_cap) {
    if (ctr[kMsLevelDone] != 0ull) {
        ctr[kMsNext] = 0ull;
        const unsigned long long cur = min(ctr[kMsCur], (unsigned long long)list_cap);
        ctr[kMsCur] = cur;
        ctr[kMsPending] = (cur + kWave - 1) / kWave;
        if (cur == 0ull) ctr[kMsDone] = 1ull;
    }
}

// Cut the frontier into work items, 64 entries per wave at a time: light
// vertices in segments of consecutive entries (< seg + chunk incidences),
// heavy ones in chunks of their incidences.  A batch whose items do not fit
// the item buffer stays pending for the next step of the same level.
__global__ __launch_bounds__(kWG) void k_ms_plan(MsArgs m) {
    const uint32_t lane = lane_id(), wv = uni(threadIdx.x / kWave);
    const uint64_t ncur = m.ctr[kMsCur];
    const uint32_t epoch = (uint32_t)m.ctr[kMsEpoch] + 1u;   // never 0: fresh entries read 0
    const uint64_t nbatch = (ncur + kWave - 1) / kWave;
    const GraphView G = graph_view(m.graph);
    unsigned long long bytes = 0;
    for (uint64_t bt = (uint64_t)blockIdx.x * kWavesPerWG + wv; bt < nbatch; bt += (uint64_t)gridDim.x * kWavesPerWG) {
        if (uni(m.batch_epoch[bt]) == epoch) continue;
        const uint64_t f = bt * kWave + lane;
        const uint32_t nb = (uint32_t)min((uint64_t)kWave, ncur - bt * kWave);
        uint32_t v = 0, e0 = 0, deg = 0, hv = 0, light = 0, cv = m.chunk, sets = 0;
        if (lane < nb) {
            v = m.cur_v[f];
            sets = (uint32_t)__popcll(m.cur_m[f]);
            e0 = G.v_off[v];
            deg = G.v_off[v + 1] - e0;
            // work grows with incidences times sets: heavy entries are cut
            // into chunks of about `chunk` (incidence, set) pairs
            const HeavySplit hs = ms_heavy_split(deg, sets, m.chunk);
            cv = hs.len;
            hv = hs.count;
            light = hv ? 0u : deg * sets;   // segment weight: (incidence, set) pairs
        }
        const uint32_t lscan = wave_incl_scan(light);
        const uint32_t seg = segment_of(lscan, light, m.seg);
        const uint32_t prev_seg = __shfl_up(seg, 1, kWave);
        const bool first = lane < nb && (lane == 0 || seg != prev_seg);
        const uint64_t firsts = __ballot(first);
        const uint32_t nseg = (uint32_t)__popcll(firsts);
        const uint32_t hscan = wave_incl_scan(hv);
        const uint32_t need = nseg + uni(wave_bcast(hscan, kWave - 1));
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(&m.ctr[kMsItems], (unsigned long long)need);
        base = uni64(wave_bcast64(base, 0));
        if (base + need > kItemCap) {
            for (uint64_t x = base + lane; x < kItemCap; x += kWave) m.items[x].x = kSkipItem;
            continue;
        }
        if (lane < nb && ((firsts >> lane) & 1ull)) {
            const uint64_t above = lane + 1 < 64 ? (firsts >> (lane + 1)) << (lane + 1) : 0ull;
            const uint32_t next = above ? (uint32_t)__ffsll((unsigned long long)above) - 1u : nb;
            m.items[base + lane_rank(firsts)] = make_uint4((uint32_t)f, min(next, nb) - lane, 0u, 0u);
        }
        // heavy chunks, spread over the wave
        const uint32_t H = uni(wave_bcast(hscan, kWave - 1));
        for (uint32_t q0 = 0; q0 < H; q0 += kWave) {
            const uint32_t q = q0 + lane;
            const uint32_t k = owner_of(hscan, min(q, H - 1u));
            const uint32_t excl = (uint32_t)__shfl((int)(hscan - hv), (int)k, kWave);
            const uint32_t fk = (uint32_t)__shfl((int)(uint32_t)f, (int)k, kWave);
            const uint32_t ek = (uint32_t)__shfl((int)e0, (int)k, kWave);
            const uint32_t ck = (uint32_t)__shfl((int)cv, (int)k, kWave);
            const uint32_t dk = (uint32_t)__shfl((int)deg, (int)k, kWave);
            if (q < H) {
                const ChunkRange cr = chunk_range(ek, dk, ck, q - excl);
                m.items[base + nseg + q] = make_uint4(fk | 0x80000000u, cr.lo, cr.hi, 0u);
            }
        }
        if (lane < nb) bytes += (unsigned long long)sets * m.bytesw[v];
        if (lane == 0) {
            m.batch_epoch[bt] = epoch;
            atomicSub(&m.ctr[kMsPending], 1ull);
        }
    }
    bytes = wave_sum(bytes);
    if (lane_id() == 0 && bytes) atomicAdd(m.bytes, bytes);
}

// Appends (bundle, vertex) pairs that just got their first bit in nxt to the
// next-level list: one counter reservation per wavefront.  Every lane of the
// wave calls it; lanes with `fresh` set contribute (b, u).
__device__ __forceinline__ void ms_append_wave(const MsArgs &m, bool fresh, uint32_t b, uint32_t u) {
    const uint64_t who = __ballot(fresh);
    if (who == 0) return;
    unsigned long long base = 0;
    if (lane_id() == (uint32_t)__ffsll((unsigned long long)who) - 1u)
        base = atomicAdd(&m.ctr[kMsNext], (unsigned long long)__popcll(who));
    base = wave_bcast64(base, (int)__ffsll((unsigned long long)who) - 1);
    if (fresh) {
        const unsigned long long pos = base + lane_rank(who);
        if (pos < m.list_cap) {
            m.nx_b[pos] = b;
            m.nx_v[pos] = u;
        } else {
            atomicOr(&m.ctr[kMsOverflow], 1ull);
        }
    }
}

// Marks the wave's buffered live channels in nxt and appends the (bundle,
// member) pairs that got their first bit to the next-level list.  A marking
// needs the old mask back, so each lane first issues up to four atomics and
// only then waits: one memory round trip per 256 channels instead of one per
// coin batch.  Every lane of the wave calls it.
__device__ __forceinline__ void ms_flush(const MsArgs &m, MsLds &L, uint32_t &nlive) {
    wave_sync();
    const uint32_t lane = lane_id();
    for (uint32_t i0 = 0; i0 < nlive; i0 += 4 * kWave) {
        unsigned long long old[4];
        uint32_t bb[4], uu[4];
        bool act[4];
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
            const uint32_t i = i0 + r * kWave + lane;
            act[r] = i < nlive;
            bb[r] = uu[r] = 0;
            old[r] = ~0ull;
            if (act[r]) {
                const uint2 e = L.live[i];
                uu[r] = e.x;
                bb[r] = e.y >> 6;
                old[r] = atomicOr(&m.nxt[(uint64_t)bb[r] * m.stride + uu[r]], 1ull << (e.y & 63u));
            }
        }
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) ms_append_wave(m, act[r] && old[r] == 0ull, bb[r], uu[r]);
    }
    nlive = 0;
    wave_sync();
}

// Coins of one (quad, set) pair: channels (he, u[t] -> v) for the candidate
// positions t of set s; live ones wait in the wave's buffer to be marked in
// nxt (sets already holding u are removed when the level advances).  Lanes
// with act = false only join the wave-wide steps.
__device__ __forceinline__ void ms_pair(const MsArgs &m, MsLds &L, uint32_t &nlive, bool act, uint32_t bnd,
                                        uint32_t s, uint32_t he, uint32_t q, uint32_t v, uint32_t thr,
                                        uint32_t cand4, const uint32_t (&u)[4], uint64_t &px) {
    uint4 c = make_uint4(0u, 0u, 0u, 0u);
    if (act) {
        c = philox4x32_10(coin_counter(m.first_id + (uint64_t)bnd * kMsSets + s, he, v, m.pool, q),
                          make_uint2(m.key0, m.key1));
        ++px;
    }
    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
    uint32_t lv = 0;
#pragma unroll
    for (uint32_t t = 0; t < 4; ++t)
        lv |= (act && ((cand4 >> t) & 1u) && channel_live(w[t], thr)) ? 1u << t : 0u;
    // placement from one ballot per position: the live channels of position
    // t follow those of positions < t, in lane order
    const uint64_t b0 = __ballot(lv & 1u), b1 = __ballot(lv & 2u), b2 = __ballot(lv & 4u), b3 = __ballot(lv & 8u);
    if ((b0 | b1 | b2 | b3) == 0ull) return;   // with small probabilities most pairs have no live channel
    const uint32_t c0 = (uint32_t)__popcll(b0), c1 = (uint32_t)__popcll(b1), c2 = (uint32_t)__popcll(b2);
    const uint32_t tot = c0 + c1 + c2 + (uint32_t)__popcll(b3);
    if (nlive + tot > kMsLiveCap) ms_flush(m, L, nlive);
    const uint64_t below = (1ull << lane_id()) - 1ull;
    const uint32_t tag = (bnd << 6) | s;
    if (lv & 1u) L.live[nlive + (uint32_t)__popcll(b0 & below)] = make_uint2(u[0], tag);
    if (lv & 2u) L.live[nlive + c0 + (uint32_t)__popcll(b1 & below)] = make_uint2(u[1], tag);
    if (lv & 4u) L.live[nlive + c0 + c1 + (uint32_t)__popcll(b2 & below)] = make_uint2(u[2], tag);
    if (lv & 8u) L.live[nlive + c0 + c1 + c2 + (uint32_t)__popcll(b3 & below)] = make_uint2(u[3], tag);
    nlive += tot;
}

// Levels 2-4 of a bundled expansion.  Each lane brings a frontier entry
// (bundle b, vertex v, set mask) and the incidence range [e0, e0 + d) of v to
// expand (d = 0 for none).  Level 2 spreads the incidences over the wave,
// level 3 the quads of member positions of those hyperedges, level 4 the
// (quad, set) pairs whose coins are drawn.  A quad whose entry carries at
// least m.filter sets first reads its members' seen masks and keeps
// only the sets that do not hold them; for smaller masks those scattered
// loads cost more than the coins they would save, so every set of the mask
// draws its coins and the level's advance drops what a set already holds.
// When the wave's pair counts are even (no lane has more than twice the
// mean), every lane walks its own quad's sets in registers; otherwise the
// pairs are spread over the wave through LDS.
__device__ __forceinline__ void ms_expand(const MsArgs &m, const GraphView &G, MsLds &L, uint32_t &nlive, uint32_t b,
                                          uint32_t v, unsigned long long mask, uint32_t e0, uint32_t d, uint64_t &px) {
    const uint32_t lane = lane_id();
    const uint32_t dscan = wave_incl_scan(d);
    const uint32_t D = uni(wave_bcast(dscan, kWave - 1));
    const uint32_t th = d ? G.thr[v] : 0u;
    wave_sync();
    L.fr_scan[lane] = dscan;
    L.fr_v[lane] = v;
    L.fr_e0[lane] = e0;
    L.fr_b[lane] = b;
    L.fr_thr[lane] = th;
    L.fr_m[lane] = mask;
    wave_sync();
    for (uint32_t base = 0; base < D; base += kWave) {
        // level 2: one incidence (v, he) per lane
        const uint32_t g = base + lane;
        uint32_t he = 0, hb = 0, hs = 0, nq = 0, fk = 0;
        if (g < D) {
            fk = search64(L.fr_scan, g);
            const uint32_t start = fk ? L.fr_scan[fk - 1] : 0u;
            const uint32_t e = L.fr_e0[fk] + (g - start);
            he = G.v_he[e];
            const unsigned long long bs = G.v_hbs[e];
            hb = (uint32_t)bs;
            hs = (uint32_t)(bs >> 32);
            nq = L.fr_thr[fk] ? (hs + 3u) >> 2 : 0u;   // threshold 0: no channel into the vertex is live
        }
        const uint32_t qscan = wave_incl_scan(nq);
        const uint32_t Q = uni(wave_bcast(qscan, kWave - 1));
        if (Q == 0) continue;
        wave_sync();
        L.in_scan[lane] = qscan;
        L.in_he[lane] = he;
        L.in_hb[lane] = hb;
        L.in_hs[lane] = hs;
        L.in_k[lane] = fk;
        wave_sync();
        for (uint32_t qb = 0; qb < Q; qb += kWave) {
            // level 3: one quad of member positions per lane
            const uint32_t qg = qb + lane;
            uint32_t pc = 0;
            uint32_t u[4] = {0u, 0u, 0u, 0u};
            unsigned long long cand[4] = {0ull, 0ull, 0ull, 0ull}, un = 0ull;
            uint32_t qhe = 0, qq = 0, qv = 0, qth = 0, qbnd = 0;
            if (qg < Q) {
                const uint32_t k = search64(L.in_scan, qg);
                const uint32_t start = k ? L.in_scan[k - 1] : 0u;
                const uint32_t f = L.in_k[k];
                qq = qg - start;
                qhe = L.in_he[k];
                qv = L.fr_v[f];
                qth = L.fr_thr[f];
                qbnd = L.fr_b[f];
                const unsigned long long qm = L.fr_m[f];
                const uint32_t p0 = 4u * qq, cnt = min(4u, L.in_hs[k] - p0);
                const uint32_t hbk = L.in_hb[k];
#pragma unroll
                for (uint32_t t = 0; t < 4; ++t) u[t] = t < cnt ? G.he_mem[hbk + p0 + t] : qv;
                uint32_t valid = 0;
#pragma unroll
                for (uint32_t t = 0; t < 4; ++t) valid |= (t < cnt && u[t] != qv) ? 1u << t : 0u;
                if ((uint32_t)__popcll(qm) >= m.filter) {
                    const uint64_t row = (uint64_t)qbnd * m.stride;
                    unsigned long long sm[4];
#pragma unroll
                    for (uint32_t t = 0; t < 4; ++t) sm[t] = ((valid >> t) & 1u) ? m.seen[row + u[t]] : ~0ull;
#pragma unroll
                    for (uint32_t t = 0; t < 4; ++t) cand[t] = qm & ~sm[t];
                } else {
#pragma unroll
                    for (uint32_t t = 0; t < 4; ++t) cand[t] = ((valid >> t) & 1u) ? qm : 0ull;
                }
#pragma unroll
                for (uint32_t t = 0; t < 4; ++t) un |= cand[t];
                pc = (uint32_t)__popcll(un);
            }
            const uint32_t pscan = wave_incl_scan(pc);
            const uint32_t PT = uni(wave_bcast(pscan, kWave - 1));
            if (PT == 0) continue;
            const uint32_t pmax = uni(wave_max(pc));
            if ((uint64_t)pmax * kWave <= 2ull * PT) {
                // level 4 in registers: lane walks the sets of its own quad
                unsigned long long rem = un;
                for (uint32_t r = 0; r < pmax; ++r) {
                    const bool act = rem != 0ull;
                    uint32_t s = 0, c4 = 0;
                    if (act) {
                        s = (uint32_t)__ffsll(rem) - 1u;
                        rem &= rem - 1ull;
#pragma unroll
                        for (uint32_t t = 0; t < 4; ++t) c4 |= (uint32_t)((cand[t] >> s) & 1ull) << t;
                    }
                    ms_pair(m, L, nlive, act, qbnd, s, qhe, qq, qv, qth, c4, u, px);
                }
                continue;
            }
            // level 4 over the wave: one (quad, set) pair per lane, the
            // quad's data read from its lane by shuffles
            for (uint32_t pb = 0; pb < PT; pb += kWave) {
                const uint32_t pg = pb + lane;
                const bool act = pg < PT;
                const uint32_t k = owner_of(pscan, act ? pg : PT - 1u);
                const uint32_t before = (uint32_t)__shfl((int)(pscan - pc), (int)k, kWave);
                const unsigned long long unk =
                    ((unsigned long long)(uint32_t)__shfl((int)(uint32_t)(un >> 32), (int)k, kWave) << 32) |
                    (uint32_t)__shfl((int)(uint32_t)un, (int)k, kWave);
                const uint32_t s = nth_bit(unk, act ? pg - before : 0u);
                const uint32_t bk = (uint32_t)__shfl((int)qbnd, (int)k, kWave);
                const uint32_t vk = (uint32_t)__shfl((int)qv, (int)k, kWave);
                const uint32_t thk = (uint32_t)__shfl((int)qth, (int)k, kWave);
                const uint32_t hek = (uint32_t)__shfl((int)qhe, (int)k, kWave);
                const uint32_t qk = (uint32_t)__shfl((int)qq, (int)k, kWave);
                uint32_t uk[4], c4 = 0;
#pragma unroll
                for (uint32_t t = 0; t < 4; ++t) {
                    uk[t] = (uint32_t)__shfl((int)u[t], (int)k, kWave);
                    // the set's bit of cand[t]: from the half that holds bit s
                    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)cand[t], (int)k, kWave);
                    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(cand[t] >> 32), (int)k, kWave);
                    c4 |= (((s < 32 ? lo >> s : hi >> (s - 32)) & 1u)) << t;
                }
                ms_pair(m, L, nlive, act, bk, s, hek, qk, vk, thk, c4, uk, px);
            }
        }
    }
    wave_sync();
}

__global__ __launch_bounds__(kWG) void k_ms_expand(MsArgs m) {
    __shared__ MsLds lds[kWavesPerWG];
    const uint32_t wv = uni(threadIdx.x / kWave);
    MsLds &L = lds[wv];
    const GraphView G = graph_view(m.graph);
    const uint64_t nitems = min(m.ctr[kMsItems], (unsigned long long)kItemCap);
    const uint32_t lane = lane_id();
    uint64_t px = 0;
    uint32_t nlive = 0;   // live channels buffered in L.live (wave-uniform)
    for (;;) {
        // items cost up to a few times each other (hyperedge sizes vary
        // inside a chunk), so waves take them one at a time
        unsigned long long it = 0;
        if (lane == 0) it = atomicAdd(&m.ctr[kMsFetch], 1ull);
        it = uni64(wave_bcast64(it, 0));
        if (it >= nitems) break;
        const uint4 ld = m.items[it];
        const uint4 item = make_uint4(uni(ld.x), uni(ld.y), uni(ld.z), uni(ld.w));
        if (item.x == kSkipItem) continue;
        if ((item.x >> 31) == 0u) {
            // light segment: entries [item.x, item.x + item.y)
            uint32_t b = 0, v = 0, e0 = 0, d = 0;
            unsigned long long mask = 0;
            if (lane < item.y) {
                const uint32_t f = item.x + lane;
                b = m.cur_b[f];
                v = m.cur_v[f];
                mask = m.cur_m[f];
                e0 = G.v_off[v];
                d = G.v_off[v + 1] - e0;
                if (ms_heavy_split(d, (uint32_t)__popcll(mask), m.chunk).count) d = 0;   // expanded by its heavy items
            }
            ms_expand(m, G, L, nlive, b, v, mask, e0, d, px);
        } else {
            // one heavy vertex: incidences [item.y, item.z) of entry item.x
            const uint32_t f = item.x & 0x7FFFFFFFu;
            const uint32_t b = uni(m.cur_b[f]), v = uni(m.cur_v[f]);
            const unsigned long long mask = uni64(m.cur_m[f]);
            // the chunk's incidences go to lanes in runs of up to 64 entries
            for (uint32_t e = item.y; e < item.z; e += kWave) {
                const uint32_t mine = e + lane < item.z ? 1u : 0u;
                ms_expand(m, G, L, nlive, b, v, mask, e + lane, mine, px);
            }
        }
    }
    ms_flush(m, L, nlive);
    px = wave_sum(px);
    if (lane == 0 && px) atomicAdd(m.philox, (unsigned long long)px);
}

// Output, pass 1: per (bundle, block of kMsOutVerts vertices) member counts
// of every set.
__global__ __launch_bounds__(kWG) void k_ms_count(MsArgs m) {
    __shared__ uint32_t cnt[kMsSets];
    const uint32_t b = blockIdx.x / m.nvb, blk = blockIdx.x % m.nvb;
    const uint32_t n = m.graph.n;
    if (threadIdx.x < kMsSets) cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t row = (uint64_t)b * m.stride;
    for (uint32_t i = 0; i < kMsOutVerts / kWG; ++i) {
        const uint32_t v = blk * kMsOutVerts + i * kWG + threadIdx.x;
        if (v >= n) break;
        unsigned long long w = m.seen[row + v];
        while (w) {
            const uint32_t s = (uint32_t)__ffsll(w) - 1u;
            w &= w - 1ull;
            atomicAdd(&cnt[s], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < kMsSets) m.vcnt[((uint64_t)b * m.nvb + blk) * kMsSets + threadIdx.x] = cnt[threadIdx.x];
}

// Pass 2, one thread per set: block counts become block offsets, the set
// gets its stage range and its per-id outputs.
__global__ __launch_bounds__(kWG) void k_ms_record(MsArgs m, RRArgs a) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.count) return;
    const uint32_t b = (uint32_t)(i / kMsSets), s = (uint32_t)(i % kMsSets);
    uint32_t total = 0;
    for (uint32_t blk = 0; blk < m.nvb; ++blk) {
        uint32_t *c = &m.vcnt[((uint64_t)b * m.nvb + blk) * kMsSets + s];
        const uint32_t x = *c;
        *c = total;
        total += x;
    }
    const unsigned long long off = atomicAdd(&a.ctr[kBump], (unsigned long long)total);
    record_set(a, i, off, total, a.roots[a.out_base + i]);
}

// Pass 3: members in ascending order.  Each thread owns 16 consecutive
// vertices of the block; per set, a workgroup scan of the threads' counts
// places them.
__global__ __launch_bounds__(kWG) void k_ms_write(MsArgs m, RRArgs a) {
    __shared__ uint32_t wsum[kWavesPerWG];
    constexpr uint32_t kPer = kMsOutVerts / kWG;
    const uint32_t b = blockIdx.x / m.nvb, blk = blockIdx.x % m.nvb;
    const uint32_t n = m.graph.n, lane = lane_id(), wv = threadIdx.x / kWave;
    const uint64_t row = (uint64_t)b * m.stride;
    const uint32_t v0 = blk * kMsOutVerts + threadIdx.x * kPer;
    unsigned long long w[kPer];
    unsigned long long any = 0;
#pragma unroll
    for (uint32_t t = 0; t < kPer; ++t) {
        w[t] = v0 + t < n ? m.seen[row + v0 + t] : 0ull;
        any |= w[t];
    }
    const uint64_t sets = min((uint64_t)kMsSets, m.count - (uint64_t)b * kMsSets);
    for (uint32_t s = 0; s < sets; ++s) {
        const unsigned long long bit = 1ull << s;
        uint32_t c = 0;
        if (any & bit) {
#pragma unroll
            for (uint32_t t = 0; t < kPer; ++t) c += (w[t] & bit) ? 1u : 0u;
        }
        const uint32_t incl = wave_incl_scan(c);
        if (lane == kWave - 1) wsum[wv] = incl;
        __syncthreads();
        uint32_t before = incl - c;
        for (uint32_t q = 0; q < wv; ++q) before += wsum[q];
        const uint64_t id = a.out_base + (uint64_t)b * kMsSets + s;
        const uint64_t off = a.stage_off[id];
        const uint32_t size = a.sizes[id];
        if (c && off + size <= a.stage_cap) {
            uint64_t pos = off + m.vcnt[((uint64_t)b * m.nvb + blk) * kMsSets + s] + before;
#pragma unroll
            for (uint32_t t = 0; t < kPer; ++t)
                if (w[t] & bit) a.stage[pos++] = v0 + t;
        }
        __syncthreads();
    }
}

// ---- compaction ------------------------------------------------------------
// Sets up to kBigSet members: each wave moves 64 consecutive ids, flattened
// over their members.
__global__ __launch_bounds__(kWG) void k_move_small(const uint64_t *__restrict__ stage_off,
                                                     const uint32_t *__restrict__ sizes,
                                                     const uint64_t *__restrict__ dst_off, uint64_t count,
                                                     const uint32_t *__restrict__ stage, uint32_t *__restrict__ mem) {
    __shared__ uint32_t scan_s[kWavesPerWG][kWave];
    __shared__ uint64_t src_s[kWavesPerWG][kWave], dst_s[kWavesPerWG][kWave];
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    const uint64_t waves = (uint64_t)gridDim.x * kWavesPerWG;
    for (uint64_t grp = (uint64_t)blockIdx.x * kWavesPerWG + wv; grp * kWave < count; grp += waves) {
        const uint64_t id = grp * kWave + lane;
        uint32_t sz = 0;
        uint64_t src = 0, dst = 0;
        if (id < count) {
            sz = sizes[id];
            if (sz > kBigSet) sz = 0;
            src = stage_off[id];
            dst = dst_off[id];
        }
        const uint32_t incl = wave_incl_scan(sz);
        const uint32_t total = wave_bcast(incl, kWave - 1);
        scan_s[wv][lane] = incl;
        src_s[wv][lane] = src;
        dst_s[wv][lane] = dst;
        wave_sync();
        for (uint32_t base = 0; base < total; base += kWave) {
            const uint32_t g = base + lane;
            if (g < total) {
                const uint32_t k = search64(scan_s[wv], g);
                const uint32_t e = g - (k ? scan_s[wv][k - 1] : 0u);
                mem[dst_s[wv][k] + e] = stage[src_s[wv][k] + e];
            }
        }
        wave_sync();
    }
}

// Sets above kBigSet members whose per-id index lies in [first, first + count):
// one workgroup each.
__global__ __launch_bounds__(kWG) void k_move_big(const uint64_t *__restrict__ big_ids,
                                                   const unsigned long long *__restrict__ big_count, uint64_t first,
                                                   uint64_t count, const uint64_t *__restrict__ stage_off,
                                                   const uint32_t *__restrict__ sizes,
                                                   const uint64_t *__restrict__ dst_off,
                                                   const uint32_t *__restrict__ stage, uint32_t *__restrict__ mem) {
    const uint64_t nbig = *big_count;
    for (uint64_t b = blockIdx.x; b < nbig; b += gridDim.x) {
        const uint64_t id = big_ids[b];
        if (id < first || id >= first + count) continue;
        const uint64_t src = stage_off[id], dst = dst_off[id - first];
        const uint32_t sz = sizes[id];
        for (uint32_t i = threadIdx.x; i < sz; i += blockDim.x) mem[dst + i] = stage[src + i];
    }
}

// Sums of four per-vertex weights over the members of a pool prefix.
__global__ __launch_bounds__(kWG) void k_weight_sum(const uint32_t *__restrict__ mem, uint64_t entries,
                                                     const unsigned long long *__restrict__ w0,
                                                     const unsigned long long *__restrict__ w1,
                                                     const unsigned long long *__restrict__ w2,
                                                     const unsigned long long *__restrict__ w3,
                                                     unsigned long long *__restrict__ out) {
    unsigned long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < entries;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = mem[i];
        a0 += w0[v];
        a1 += w1[v];
        a2 += w2[v];
        a3 += w3[v];
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    a2 = wave_sum(a2);
    a3 = wave_sum(a3);
    if (lane_id() == 0) {
        atomicAdd(out, a0);
        atomicAdd(out + 1, a1);
        atomicAdd(out + 2, a2);
        atomicAdd(out + 3, a3);
    }
}

// ---- host side -------------------------------------------------------------

// The descriptor of one graph in a launch group.
GraphDesc graph_desc(hyperim_graph g) {
    GraphDesc d{};   // fields of other models stay null
    d.he_off = g->he_off.as<uint32_t>();
    d.he_mem = g->he_mem.as<uint32_t>();
    d.v_off = g->v_off.as<uint32_t>();
    d.v_he = g->v_he.as<uint32_t>();
    d.thr = g->thr.as<uint32_t>();
    d.P = g->P.as<uint32_t>();
    d.v_hbs = g->v_hbs.as<unsigned long long>();
    d.n = g->n;
    d.bm_words = (uint32_t)(((uint64_t)g->n + 31u) / 32u);
    if (g->lt()) d.chan = g->chan.as<unsigned long long>();
    if (g->layered()) {
        d.lay_nb_off = g->lay_nb_off.as<unsigned long long>();
        d.lay_ly_off = g->lay_ly_off.as<unsigned long long>();
        d.lay_nb = g->lay_nb.as<uint32_t>();
        d.lay_ly_end = g->lay_ly_end.as<uint32_t>();
        d.l = g->l.as<uint32_t>();
        d.lay_ln = g->lay_ln.as<double>();
        d.lay_expm = g->lay_expm.as<double>();
    }
    if (g->routed) {
        d.rP = g->route_P.as<uint32_t>();
        d.force = g->force.as<uint32_t>();
        d.force_off = g->force_off.as<unsigned long long>();
        d.rn1 = g->route_n1;
    }
    return d;
}
struct LaunchShape {
    uint32_t grid;        // phase A workgroups at full occupancy (one slot per wave)
    uint32_t slots;       // total slots (phase A waves + spare slots for deferred sets)
    uint32_t grid_b;      // phase B workgroups at full occupancy
    uint32_t cus;         // compute units
    uint32_t slot_n, slot_words;
    bool lds;
};

// Slot layout for graphs of up to n_max vertices: phase A grid (from
// occupancy), slots (phase A waves plus spare slots for deferred sets, within
// kSlotBudget bytes) and the phase B grid.
struct SlotLayout {
    uint64_t grid, waves, slots, grid_b, bytes;
    uint32_t cus;
    bool lds;
};

int slot_layout(uint32_t n_max, SlotLayout *out) {
    int per_cu_lds = 0, per_cu_glb = 0, per_cu_b = 0, cus = 0, dev = 0;
    HIM_HIP(hipGetDevice(&dev));
    HIM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_lds, k_rr_light<true, false>, kWG, 0));
    HIM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_glb, k_rr_light<false, false>, kWG, 0));
    HIM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_b, k_expand<false>, kWG, 0));
    const bool lds = n_max <= kLdsBitmapWords * 32u;
    const uint64_t words = ((uint64_t)n_max + 31u) / 32u;
    const uint64_t per_slot = (uint64_t)n_max * 4u + (lds ? 0u : words * 4u);
    const uint64_t max_slots = std::max<uint64_t>(kSlotBudget / std::max<uint64_t>(per_slot, 1), 2 * kWavesPerWG);
    uint64_t grid = (uint64_t)cus * (uint64_t)std::max(lds ? per_cu_lds : per_cu_glb, 1);
    // phase A keeps at least half of the slots spare for deferred sets
    grid = std::min<uint64_t>(grid, max_slots / (2 * kWavesPerWG));
    grid = std::max<uint64_t>(grid, 1);
    const uint64_t waves = grid * kWavesPerWG;
    const uint64_t slots = lds ? waves : std::min<uint64_t>(max_slots, 4 * waves);
    out->grid = grid;
    out->waves = waves;
    out->slots = slots;
    out->grid_b = (uint64_t)cus * (uint64_t)std::max(per_cu_b, 1);
    out->bytes = slots * per_slot;
    out->cus = (uint32_t)cus;
    out->lds = lds;
    return HYPERIM_OK;
}

// Slots sized for graphs of up to n_max vertices (re-created when a larger
// graph arrives).
int ensure_workspace(RRWorkspace &ws, uint32_t n_max, hipStream_t s, LaunchShape *shape) {
    const bool lds = n_max <= kLdsBitmapWords * 32u;
    const uint32_t words = (uint32_t)(((uint64_t)n_max + 31u) / 32u);
    if (ws.grid != 0 && (ws.slot_n < n_max || ws.lds != lds)) {
        HIM_HIP(hipStreamSynchronize(s));
        ws.lists.release();
        ws.bitmaps.release();
        ws.grid = 0;
    }
    if (ws.grid == 0) {
        SlotLayout L;
        HIM_CHECK(slot_layout(n_max, &L));
        const uint64_t grid = L.grid, waves = L.waves, slots = L.slots;
        ws.grid = (uint32_t)grid;
        ws.waves = (uint32_t)waves;
        ws.slots = (uint32_t)slots;
        ws.grid_b = (uint32_t)L.grid_b;
        ws.cus = L.cus;
        ws.slot_n = std::max<uint32_t>(n_max, 1);
        ws.slot_words = words;
        ws.lds = lds;
        HIM_CHECK(ws.lists.reserve(sizeof(uint32_t) * (size_t)slots * ws.slot_n, s));
        if (!lds) {
            HIM_CHECK(ws.bitmaps.reserve(sizeof(uint32_t) * (size_t)slots * words, s));
            HIM_HIP(hipMemsetAsync(ws.bitmaps.ptr, 0, sizeof(uint32_t) * (size_t)slots * words, s));
        }
        HIM_CHECK(ws.counters.reserve(sizeof(unsigned long long) * kNumCtr, s));
        // deferred-set arrays for as many sets as there are slots (phase A may
        // run fewer waves than the occupancy allows, leaving more spare slots)
        const size_t ndef = slots;
        HIM_CHECK(ws.def_idx.reserve(sizeof(uint64_t) * ndef, s));
        HIM_CHECK(ws.def_u32.reserve(sizeof(uint32_t) * 5 * ndef, s));
        HIM_CHECK(ws.items.reserve(sizeof(uint4) * (size_t)kItemCap, s));
        HIM_CHECK(ws.args_dev.reserve(sizeof(RRArgs), s));
    }
    shape->grid = ws.grid;
    shape->slots = ws.slots;
    shape->grid_b = ws.grid_b;
    shape->cus = ws.cus;
    shape->slot_n = ws.slot_n;
    shape->slot_words = ws.slot_words;
    shape->lds = lds;
    return HYPERIM_OK;
}

// Id ranges of every (ladder block, stratum) pair inside [id_begin, id_end).
void stratum_ranges(hyperim_graph g, uint64_t seed, uint32_t instance, uint32_t qlog, uint32_t pool,
                    uint64_t id_begin, uint64_t id_end, std::vector<std::pair<uint64_t, uint64_t>> *out) {
    const uint64_t Q = 1ull << qlog;
    // with the RR sets divided, the pool's own root list and its strata
    const uint32_t n = g->routed ? (pool == 0 ? g->route_n1 : g->n - g->route_n1) : g->n;
    const uint32_t *B = g->routed ? g->route_B[pool ? 1 : 0] : g->info.B;
    uint64_t j = id_begin;
    while (j < id_end) {
        uint32_t b;
        uint64_t J, T;
        if (j < Q) {
            b = 0;
            J = 0;
            T = Q;
        } else {
            uint32_t hb = 63u - (uint32_t)__builtin_clzll(j);
            b = hb - qlog + 1u;
            J = 1ull << hb;
            T = J;
        }
        const uint4 r = philox4x32_10(root_counter(b, pool), make_uint2((uint32_t)seed, instance));
        const uint64_t x = (uint64_t)r.x | ((uint64_t)r.y << 32);
        const uint64_t o = (uint64_t)(((unsigned __int128)x * n) >> 64);
        uint64_t prev = 0;
        for (uint32_t h = 1; h <= kNStrata; ++h) {
            uint64_t th;
            if (h == kNStrata) {
                th = T;
            } else {
                // first t with floor((t n + o) / T) >= B_h
                unsigned __int128 need = (unsigned __int128)B[h] * T;
                th = need <= o ? 0 : (uint64_t)((need - o + n - 1) / n);
                th = std::min<uint64_t>(th, T);
            }
            const uint64_t lo = std::max<uint64_t>(J + prev, id_begin), hi = std::min<uint64_t>(J + th, id_end);
            if (lo < hi) out->push_back({lo, hi});
            prev = th;
        }
        j = J + T;
    }
}

int read_ctr(hipStream_t s, const unsigned long long *dev, int idx, uint64_t *out) {
    unsigned long long v = 0;
    HIM_HIP(hipMemcpyAsync(&v, dev + idx, sizeof(v), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    *out = v;
    return HYPERIM_OK;
}

// Wait for an event of the superstep loops, but not forever: a batch that has
// not finished after HYPERIM_WAIT_LIMIT_S seconds (default 600; a batch of
// the largest workloads takes a few seconds) ends the call with HYPERIM_EHIP
// naming the loop, instead of blocking the caller.
int wait_event(hipEvent_t e, const char *what) {
    static const double limit = [] {
        const char *v = getenv("HYPERIM_WAIT_LIMIT_S");
        const double x = v ? atof(v) : 0.0;
        return x > 0.0 ? x : 600.0;
    }();
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t q = hipEventQuery(e);
        if (q == hipSuccess) return HYPERIM_OK;
        if (q != hipErrorNotReady) {
            set_error_detail(std::string("waiting for ") + what + ": " + hipGetErrorString(q));
            return HYPERIM_EHIP;
        }
        const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (el > limit) {
            set_error_detail(std::string(what) + " did not finish within the wait limit");
            return HYPERIM_EHIP;
        }
        if (el > 2e-3) std::this_thread::sleep_for(std::chrono::microseconds(20));
        else std::this_thread::yield();
    }
}

// Events of the RR workspace: [0], [1] start and end of phase A, [2], [3] of
// the closing k_finish (bundled mode: of the whole group); superstep batch
// slot b (two batches in flight) owns kBatchEv events from 4 + b * kBatchEv:
// batch start, batch end (after its counter copy), then a start/end pair per
// k_expand launch when kernel times are asked for.  Events that time one
// kernel are stamped by its launch
// (hipExtLaunchKernelGGL): stream markers between dependent kernels would
// stall the device for several microseconds each.
constexpr int kMaxBatch = 64;
constexpr int kBatchEv = 2 + 2 * kMaxBatch;
constexpr int kNumEv = 4 + 2 * kBatchEv;

int event_pair(RRWorkspace &ws) {
    while (ws.events.size() < (size_t)kNumEv) {
        hipEvent_t e;
        HIM_HIP(hipEventCreate(&e));
        ws.events.push_back(e);
    }
    return HYPERIM_OK;
}

hipEvent_t *batch_events(RRWorkspace &ws, uint64_t k) { return &ws.events[4 + (size_t)(k & 1u) * kBatchEv]; }

// Pinned host staging of the RR workspace, in 64-bit words: counter-block
// copies (two superstep batches in flight, the end of a launch group), the
// spare-slot cursor, then per-call regions (graph and task descriptors, the
// pools' new totals).  Copies from and to it are asynchronous; the host
// touches a region only after waiting for the copy that uses it.
constexpr size_t kHostCtr = 16;
constexpr size_t kHostBatch = 0;   // + (k & 1) * kHostCtr for batch k
constexpr size_t kHostFinal = 2 * kHostCtr;
constexpr size_t kHostFreeNext = 3 * kHostCtr;
constexpr size_t kHostArgs = 4 * kHostCtr;   // the grid-wide phase's RRArgs on their way to the device
constexpr size_t kHostFixed = kHostArgs + (sizeof(RRArgs) + 7) / 8;
static_assert(kNumCtr <= kHostCtr, "counter block");

int ensure_host(RRWorkspace &ws, size_t words) {
    if (ws.host_words >= words) return HYPERIM_OK;
    const size_t w = std::max<size_t>(words, 2 * ws.host_words);
    if (ws.host) {
        HIM_HIP(hipDeviceSynchronize());   // no copy may still use the old buffer
        HIM_HIP(hipHostFree(ws.host));
    }
    ws.host = nullptr;
    ws.host_words = 0;
    HIM_HIP(hipHostMalloc((void **)&ws.host, w * sizeof(unsigned long long), hipHostMallocDefault));
    ws.host_words = w;
    ws.drop_graphs();   // captured batches copy into the old buffer
    return HYPERIM_OK;
}

// Captures the work `record` issues on the capture stream as one executable
// graph (record returns false when something it calls fails).  A device that
// cannot capture is remembered (graphs_off); *out is null then and the
// caller launches the kernels itself.
template <class Record>
int capture_graph(RRWorkspace &ws, Record &&record, hipGraphExec_t *out) {
    *out = nullptr;
    if (ws.graphs_off) return HYPERIM_OK;
    if (!ws.capture && hipStreamCreateWithFlags(&ws.capture, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        ws.graphs_off = true;
        return HYPERIM_OK;
    }
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(ws.capture, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        ok = record(ws.capture) && hipGetLastError() == hipSuccess;
        ok = hipStreamEndCapture(ws.capture, &g) == hipSuccess && ok && g;
    }
    hipGraphExec_t ex = nullptr;
    if (ok) ok = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
        (void)hipGetLastError();
        ws.graphs_off = true;
        return HYPERIM_OK;
    }
    *out = ex;
    return HYPERIM_OK;
}

// The captured superstep batch for `key` (everything the capture bakes in),
// captured on first use and kept in the workspace.
template <class Record>
int captured_batch(RRWorkspace &ws, const uint64_t (&key)[8], Record &&record, hipGraphExec_t *out) {
    *out = nullptr;
    for (const RRWorkspace::BatchGraph &b : ws.batch_graphs)
        if (std::equal(std::begin(key), std::end(key), std::begin(b.key))) {
            *out = b.exec;
            return HYPERIM_OK;
        }
    hipGraphExec_t ex = nullptr;
    HIM_CHECK(capture_graph(ws, record, &ex));
    if (!ex) return HYPERIM_OK;
    RRWorkspace::BatchGraph b;
    std::copy(std::begin(key), std::end(key), std::begin(b.key));
    b.exec = ex;
    ws.batch_graphs.push_back(b);
    *out = ex;
    return HYPERIM_OK;
}

// One launch group: phase A over `a`'s tasks, then phase B over the sets it
// deferred, then the deferred sets' output.  Per-id outputs land at
// a.out_base + launch index.  Supersteps go in batches of steps_per_sync, and
// the next batch is queued before the host reads the frontier count at the end
// of the last one, so the device never waits for the host between batches
// (the batch queued after the frontier ran out finds no work).  The closing
// counter block lands in ws.host + kHostFinal; `tail` may queue more work
// behind it, and the call returns after the stream has drained.  With
// `expect_defer` false the host first checks whether phase A deferred any set.
template <class Tail>
int run_launch(RRWorkspace &ws, RRStats &st, const hyperim_tuning &tune, RRArgs &a, const LaunchShape &shape,
               uint32_t grid, uint32_t grid_b, bool expect_defer, bool trace, bool time_kernels, bool graphs,
               bool gaps, hipStream_t s, Tail &&tail) {
    unsigned long long *ctr = a.ctr;
    unsigned long long *h = ws.host;
    // the grid-wide phase reads its arguments from the device
    *reinterpret_cast<RRArgs *>(h + kHostArgs) = a;
    HIM_HIP(hipMemcpyAsync(ws.args_dev.ptr, h + kHostArgs, sizeof(RRArgs), hipMemcpyHostToDevice, s));
    const RRArgs *ap = ws.args_dev.as<RRArgs>();
    // fresh work counter, deferred list and spare-slot cursor (spare slots
    // follow the launched waves' own slots)
    h[kHostFreeNext] = (unsigned long long)grid * kWavesPerWG;
    HIM_HIP(hipMemsetAsync(ctr + kWork, 0, sizeof(unsigned long long), s));
    HIM_HIP(hipMemsetAsync(ctr + kDefCount, 0, sizeof(unsigned long long), s));
    HIM_HIP(hipMemcpyAsync(ctr + kFreeNext, h + kHostFreeNext, sizeof(unsigned long long), hipMemcpyHostToDevice, s));
    HIM_CHECK(event_pair(ws));
    auto light = shape.lds ? (gaps ? k_rr_light<true, true> : k_rr_light<true, false>)
                           : (gaps ? k_rr_light<false, true> : k_rr_light<false, false>);
    auto expand_k = gaps ? k_expand<true> : k_expand<false>;
    hipExtLaunchKernelGGL(light, dim3(grid), dim3(kWG), 0, s, ws.events[0], ws.events[1], 0u, a);
    HIM_HIP(hipGetLastError());
    st.launches += 1;

    // phase B: supersteps over the deferred sets (LDS-bitmap launches defer none)
    bool phase_b = !shape.lds;
    uint64_t ndef = 0;
    if (phase_b && !expect_defer) {
        HIM_HIP(hipMemcpyAsync(h + kHostBatch, ctr, sizeof(unsigned long long) * kNumCtr, hipMemcpyDeviceToHost, s));
        HIM_HIP(hipStreamSynchronize(s));
        ndef = h[kHostBatch + kDefCount];
        phase_b = ndef != 0;
    }
    int batch = trace ? 1 : (int)std::min<uint32_t>(std::max<uint32_t>(tune.steps_per_sync, 1), kMaxBatch);
    // captured batches replay the same parities every time: an even batch
    // starts every replay on counter parity 0.  Launches timed one by one
    // (events stamped by the launch itself) are not captured: an event
    // recorded inside a graph does not time against one recorded outside.
    const bool use_graphs = graphs && !trace && !time_kernels && !ws.graphs_off;
    if (use_graphs && (batch & 1)) batch = std::min(batch + 1, kMaxBatch);
    auto account = [&](uint64_t k) -> int {
        hipEvent_t *E = batch_events(ws, k);
        float ms = 0.f;
        // first k_plan .. last k_expand (or the batch's counter copy)
        HIM_HIP(hipEventElapsedTime(&ms, E[0], time_kernels ? E[3 + 2 * (batch - 1)] : E[1]));
        st.ms_bfs += ms;
        st.ms_heavy += ms;
        for (int i = 0; time_kernels && i < batch; ++i) {
            float me = 0.f;
            HIM_HIP(hipEventElapsedTime(&me, E[2 + 2 * i], E[3 + 2 * i]));
            st.ms_expand += me;
        }
        st.expand_launches += batch;
        st.launches += 2 * batch;
        st.supersteps += batch;
        return HYPERIM_OK;
    };
    bool queued = false;   // a batch is queued but not yet accounted
    uint64_t k = 0;
    if (phase_b) {
        // planning waves: one per deferred set; until the count is known, the
        // spare slots bound it
        uint64_t plan_sets = ndef ? ndef : std::max<uint64_t>(shape.slots - (uint64_t)grid * kWavesPerWG, 1);
        // captured batches plan with one grid wide enough for any count of
        // deferred sets (planning waves stride over the sets)
        const uint32_t plan_grid_all = (uint32_t)std::max<uint64_t>(
            1, std::min<uint64_t>(div_up(std::max<uint64_t>(shape.slots - (uint64_t)grid * kWavesPerWG, 1),
                                         kWavesPerWG),
                                  4096));
        auto issue = [&](uint64_t kb) -> int {
            hipEvent_t *E = batch_events(ws, kb);
            unsigned long long *dst = h + kHostBatch + (kb & 1u) * kHostCtr;
            if (use_graphs) {
                // one replay: batch x (k_plan, k_expand) and the counter copy
                const uint64_t key[8] = {1u, (uint64_t)(kb & 1u), (uint64_t)batch, plan_grid_all,
                                         (uint64_t)grid_b, gaps ? 1u : 0u, (uint64_t)(uintptr_t)ap,
                                         (uint64_t)(uintptr_t)h ^ ((uint64_t)(uintptr_t)ctr << 1)};
                hipGraphExec_t ex = nullptr;
                HIM_CHECK(captured_batch(
                    ws, key,
                    [&](hipStream_t c) {
                        for (int i = 0; i < batch; ++i) {
                            const uint32_t parity = (uint32_t)(i & 1);
                            hipLaunchKernelGGL(k_plan, dim3(plan_grid_all), dim3(kWG), 0, c, ap, parity);
                            hipLaunchKernelGGL(expand_k, dim3(grid_b), dim3(kWG), 0, c, ap, parity);
                        }
                        return hipMemcpyAsync(dst, ctr, sizeof(unsigned long long) * kNumCtr, hipMemcpyDeviceToHost,
                                              c) == hipSuccess;
                    },
                    &ex));
                if (ex) {
                    HIM_HIP(hipEventRecord(E[0], s));
                    HIM_HIP(hipGraphLaunch(ex, s));
                    HIM_HIP(hipEventRecord(E[1], s));
                    return HYPERIM_OK;
                }
                // no capture on this device: launch directly (same parities)
            }
            const uint32_t plan_grid =
                (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(div_up(plan_sets, kWavesPerWG), 4096));
            for (int i = 0; i < batch; ++i) {
                const uint32_t parity = (uint32_t)((kb * (uint64_t)batch + (uint64_t)i) & 1u);
                hipExtLaunchKernelGGL(k_plan, dim3(plan_grid), dim3(kWG), 0, s, i == 0 ? E[0] : nullptr, nullptr,
                                      0u, ap, parity);
                // timed: the launch itself stamps its start and end events (no
                // stream markers between the kernels)
                if (time_kernels)
                    hipExtLaunchKernelGGL(expand_k, dim3(grid_b), dim3(kWG), 0, s, E[2 + 2 * i], E[3 + 2 * i], 0u,
                                          ap, parity);
                else
                    hipLaunchKernelGGL(expand_k, dim3(grid_b), dim3(kWG), 0, s, ap, parity);
            }
            HIM_HIP(hipGetLastError());
            HIM_HIP(hipMemcpyAsync(dst, ctr, sizeof(unsigned long long) * kNumCtr, hipMemcpyDeviceToHost, s));
            HIM_HIP(hipEventRecord(E[1], s));
            return HYPERIM_OK;
        };
        HIM_HIP(hipMemsetAsync(ctr + kItems, 0, 2 * sizeof(unsigned long long), s));
        HIM_CHECK(issue(0));
        uint64_t planned_before = 0;
        for (;;) {
            HIM_CHECK(issue(k + 1));   // queued before batch k is read
            HIM_CHECK(wait_event(batch_events(ws, k)[1], "a grid-wide superstep batch"));
            const unsigned long long *hb = h + kHostBatch + (k & 1u) * kHostCtr;
            ndef = hb[kDefCount];
            plan_sets = std::max<uint64_t>(ndef, 1);
            const uint32_t last = (uint32_t)(((k + 1) * (uint64_t)batch - 1) & 1u);
            const uint64_t items = hb[kItems + last];
            HIM_CHECK(account(k));
            if (trace)
                fprintf(stderr, "[hyperim] superstep %llu: %llu items, %llu entries planned\n",
                        (unsigned long long)((k + 1) * (uint64_t)batch), (unsigned long long)items,
                        (unsigned long long)hb[kPlanned]);
            // the deferred sets hold at most slot_n members each
            const int chk = phase_b_check(planned_before, hb[kPlanned], items,
                                          (uint64_t)a.slot_n * std::max<uint64_t>(ndef, 1));
            if (chk == kLoopDone) break;   // the last superstep found no frontier left
            if (chk != kLoopContinue) {
                HIM_HIP(hipStreamSynchronize(s));
                set_error_detail(chk == kLoopStalled
                                     ? "grid-wide phase stalled: a batch of supersteps with work planned no entry"
                                     : "grid-wide phase planned more entries than its sets can hold");
                return HYPERIM_EHIP;
            }
            planned_before = hb[kPlanned];
            ++k;
        }
        queued = true;   // batch k + 1, which finds no work
    }
    if (ndef) {
        hipExtLaunchKernelGGL(k_finish, dim3((uint32_t)std::min<uint64_t>(ndef, 4096)), dim3(kWG), 0, s,
                              ws.events[2], ws.events[3], 0u, a, (uint32_t)ndef);
        HIM_HIP(hipGetLastError());
        st.launches += 1;
    }
    HIM_HIP(hipMemcpyAsync(h + kHostFinal, ctr, sizeof(unsigned long long) * kNumCtr, hipMemcpyDeviceToHost, s));
    const int rc = tail();
    HIM_HIP(hipStreamSynchronize(s));
    HIM_CHECK(rc);
    float ms = 0.f;
    HIM_HIP(hipEventElapsedTime(&ms, ws.events[0], ws.events[1]));
    st.ms_bfs += ms;
    st.ms_light += ms;
    if (queued) HIM_CHECK(account(k + 1));
    if (ndef) {
        HIM_HIP(hipEventElapsedTime(&ms, ws.events[2], ws.events[3]));
        st.ms_bfs += ms;
        st.ms_heavy += ms;
    }
    st.deferred += h[kHostFinal + kDefCount];
    return HYPERIM_OK;
}

// One launch group of linear-threshold sets: one walk per set (k_lt_walk).
// Ends like run_launch: closing counter block in ws.host + kHostFinal,
// `tail` queued behind it, stream drained.
template <class Tail>
int run_lt_launch(RRWorkspace &ws, RRStats &st, const RRArgs &a, const LaunchShape &shape, uint32_t grid,
                  hipStream_t s, Tail &&tail) {
    unsigned long long *h = ws.host;
    HIM_CHECK(event_pair(ws));
    if (shape.lds)
        hipExtLaunchKernelGGL(k_lt_walk<true>, dim3(grid), dim3(kWG), 0, s, ws.events[0], ws.events[1], 0u, a);
    else
        hipExtLaunchKernelGGL(k_lt_walk<false>, dim3(grid), dim3(kWG), 0, s, ws.events[0], ws.events[1], 0u, a);
    HIM_HIP(hipGetLastError());
    st.launches += 1;
    HIM_HIP(hipMemcpyAsync(h + kHostFinal, a.ctr, sizeof(unsigned long long) * kNumCtr, hipMemcpyDeviceToHost, s));
    const int rc = tail();
    HIM_HIP(hipStreamSynchronize(s));
    HIM_CHECK(rc);
    float ms = 0.f;
    HIM_HIP(hipEventElapsedTime(&ms, ws.events[0], ws.events[1]));
    st.ms_bfs += ms;
    st.ms_light += ms;
    return HYPERIM_OK;
}

// One launch group of stratified-setting sets (k_layered), with the per-lane
// pick lists in the workspace.  Ends like run_launch.
template <class Tail>
int run_layered_launch(RRWorkspace &ws, RRStats &st, const RRArgs &a, const LaunchShape &shape, uint32_t grid,
                       hipStream_t s, Tail &&tail) {
    unsigned long long *h = ws.host;
    HIM_CHECK(ws.picks.reserve(sizeof(uint32_t) * (size_t)grid * kWavesPerWG * kWave * kMaxPick, s));
    HIM_CHECK(event_pair(ws));
    if (shape.lds)
        hipExtLaunchKernelGGL(k_layered<true>, dim3(grid), dim3(kWG), 0, s, ws.events[0], ws.events[1], 0u, a,
                              ws.picks.as<uint32_t>());
    else
        hipExtLaunchKernelGGL(k_layered<false>, dim3(grid), dim3(kWG), 0, s, ws.events[0], ws.events[1], 0u, a,
                              ws.picks.as<uint32_t>());
    HIM_HIP(hipGetLastError());
    st.launches += 1;
    HIM_HIP(hipMemcpyAsync(h + kHostFinal, a.ctr, sizeof(unsigned long long) * kNumCtr, hipMemcpyDeviceToHost, s));
    const int rc = tail();
    HIM_HIP(hipStreamSynchronize(s));
    HIM_CHECK(rc);
    float ms = 0.f;
    HIM_HIP(hipEventElapsedTime(&ms, ws.events[0], ws.events[1]));
    st.ms_bfs += ms;
    st.ms_light += ms;
    return HYPERIM_OK;
}

// Bytes of the bundled-mode state per bundle for a graph of n vertices:
// seen and nxt masks, frontier and next-level lists, output counts, batch marks.
uint64_t ms_bytes_per_bundle(uint32_t n) {
    const uint64_t nvb = div_up(std::max<uint32_t>(n, 1), kMsOutVerts);
    return (uint64_t)n * (8 + 8 + 16 + 8) + nvb * kMsSets * 4 + div_up(n, kWave) * 4 + 4096;
}

// One bundled launch group: ids [0, a.count) of one task (all on graph g),
// bundles of 64 sets grown level by level, then written out in ascending
// order per set.  Ends like run_launch: closing counter block in
// ws.host + kHostFinal, `tail` queued behind it, stream drained.
template <class Tail>
int run_ms_launch(RRWorkspace &ws, RRStats &st, const hyperim_tuning &tune, RRArgs &a, const LaunchShape &shape,
                  hyperim_graph g, const TaskDesc &t, bool trace, bool time_kernels, bool graphs, hipStream_t s,
                  Tail &&tail) {
    const uint32_t n = g->n;
    const uint32_t nbundles = (uint32_t)div_up(a.count, kMsSets);
    const uint64_t stride = std::max<uint32_t>(n, 1);
    const uint64_t list_cap = (uint64_t)nbundles * stride;
    const uint32_t nvb = (uint32_t)div_up(stride, kMsOutVerts);
    if (list_cap >= (1ull << 31)) {
        set_error_detail("bundled launch group too large");
        return HYPERIM_EINVAL;
    }
    HIM_CHECK(ws.ms_seen.reserve(sizeof(unsigned long long) * nbundles * stride, s));
    HIM_CHECK(ws.ms_nxt.reserve(sizeof(unsigned long long) * nbundles * stride, s));
    HIM_CHECK(ws.ms_cur.reserve((sizeof(uint32_t) * 2 + sizeof(unsigned long long)) * list_cap, s));
    HIM_CHECK(ws.ms_next.reserve(sizeof(uint32_t) * 2 * list_cap, s));
    HIM_CHECK(ws.ms_batch.reserve(sizeof(uint32_t) * div_up(list_cap, kWave), s));
    HIM_CHECK(ws.ms_vcnt.reserve(sizeof(uint32_t) * (uint64_t)nbundles * nvb * kMsSets, s));
    HIM_CHECK(ws.ms_ctr.reserve(sizeof(unsigned long long) * kMsNumCtr, s));
    MsArgs m{};
    m.graph = graph_desc(g);
    m.bytesw = g->bytesw.as<unsigned long long>();
    m.first_id = t.first_id;
    m.pool = t.pool;
    m.key0 = t.key0;
    m.key1 = t.key1;
    m.qlog = a.qlog;
    m.nbundles = nbundles;
    m.chunk = a.chunk;
    m.seg = a.seg;
    m.filter = std::max<uint32_t>(tune.ms_filter, 1);
    m.count = a.count;
    m.stride = stride;
    m.seen = ws.ms_seen.as<unsigned long long>();
    m.nxt = ws.ms_nxt.as<unsigned long long>();
    m.cur_b = ws.ms_cur.as<uint32_t>();
    m.cur_v = m.cur_b + list_cap;
    m.cur_m = reinterpret_cast<unsigned long long *>(m.cur_v + list_cap);
    m.nx_b = ws.ms_next.as<uint32_t>();
    m.nx_v = m.nx_b + list_cap;
    m.batch_epoch = ws.ms_batch.as<uint32_t>();
    m.list_cap = list_cap;
    m.ctr = ws.ms_ctr.as<unsigned long long>();
    m.bytes = a.ctr + kBytesMs;
    m.philox = a.ctr + kPhiloxMs;
    m.items = a.items;
    m.vcnt = ws.ms_vcnt.as<uint32_t>();
    m.nvb = nvb;
    // clean state: no set holds anything, no vertex found, no batch planned
    HIM_HIP(hipMemsetAsync(m.seen, 0, sizeof(unsigned long long) * nbundles * stride, s));
    HIM_HIP(hipMemsetAsync(m.nxt, 0, sizeof(unsigned long long) * nbundles * stride, s));
    HIM_HIP(hipMemsetAsync(m.batch_epoch, 0, sizeof(uint32_t) * div_up(list_cap, kWave), s));
    HIM_HIP(hipMemsetAsync(m.ctr, 0, sizeof(unsigned long long) * kMsNumCtr, s));
    ws.host[kHostFreeNext + 1] = 1;
    HIM_HIP(hipMemcpyAsync(m.ctr + kMsLevelDone, ws.host + kHostFreeNext + 1, sizeof(unsigned long long),
                           hipMemcpyHostToDevice, s));
    HIM_CHECK(event_pair(ws));
    HIM_HIP(hipEventRecord(ws.events[0], s));
    const uint32_t grid_b = shape.grid_b;
    hipLaunchKernelGGL(k_ms_roots, dim3((uint32_t)div_up(a.count, kWG)), dim3(kWG), 0, s, m, a);
    hipLaunchKernelGGL(k_ms_advance, dim3(grid_b), dim3(kWG), 0, s, m);
    hipLaunchKernelGGL(k_ms_ctl_advanced, dim3(1), dim3(1), 0, s, m.ctr, list_cap);
    HIM_HIP(hipGetLastError());
    // levels: plan, expand, bookkeeping, advance, bookkeeping; a level whose
    // items overflow the buffer takes several steps
    const int per_sync = (int)std::min<uint32_t>(std::max<uint32_t>(tune.steps_per_sync, 1), kMaxBatch);
    hipEvent_t *E = batch_events(ws, 0);
    uint64_t steps = 0;
    float ms = 0.f;
    // progress: (level epoch, pending frontier batches) before this batch
    uint64_t epoch_before = 0, pending_before = ~0ull;
    const unsigned long long *hm = ws.host + kHostBatch;
    static_assert(kMsNumCtr <= kHostCtr, "bundled counter block");
    // a batch of steps and the counter copy, captured once for the group
    // (the arguments are the group's) and replayed until the sets are done
    struct ExecGuard {
        hipGraphExec_t ex = nullptr;
        ~ExecGuard() {
            if (ex) (void)hipGraphExecDestroy(ex);
        }
    } batch_exec;
    auto record_batch = [&](hipStream_t c, int batch) {
        for (int k = 0; k < batch; ++k) {
            hipLaunchKernelGGL(k_ms_plan, dim3(grid_b), dim3(kWG), 0, c, m);
            if (time_kernels) {
                hipExtLaunchKernelGGL(k_ms_expand, dim3(grid_b), dim3(kWG), 0, c, E[2 + 2 * k], E[3 + 2 * k], 0u, m);
            } else {
                hipLaunchKernelGGL(k_ms_expand, dim3(grid_b), dim3(kWG), 0, c, m);
            }
            hipLaunchKernelGGL(k_ms_ctl_expanded, dim3(1), dim3(1), 0, c, m.ctr);
            hipLaunchKernelGGL(k_ms_advance, dim3(grid_b), dim3(kWG), 0, c, m);
            hipLaunchKernelGGL(k_ms_ctl_advanced, dim3(1), dim3(1), 0, c, m.ctr, list_cap);
        }
        return hipMemcpyAsync(ws.host + kHostBatch, m.ctr, sizeof(unsigned long long) * kMsNumCtr,
                              hipMemcpyDeviceToHost, c) == hipSuccess;
    };
    // (launches timed one by one are not captured, as in run_launch)
    if (graphs && !trace && !time_kernels)
        HIM_CHECK(capture_graph(ws, [&](hipStream_t c) { return record_batch(c, per_sync); }, &batch_exec.ex));
    for (;;) {
        const int batch = trace ? 1 : per_sync;
        if (batch_exec.ex) {
            HIM_HIP(hipGraphLaunch(batch_exec.ex, s));
        } else if (!record_batch(s, batch)) {
            HIM_HIP(hipGetLastError());
            set_error_detail("bundled superstep batch: a launch or copy failed");
            return HYPERIM_EHIP;
        }
        HIM_HIP(hipGetLastError());
        steps += batch;
        HIM_HIP(hipEventRecord(E[1], s));
        HIM_CHECK(wait_event(E[1], "a bundled superstep batch"));
        const uint64_t done = hm[kMsDone];
        // a level adds at least one new (set, member) pair, so levels are
        // bounded by the members of the group's sets
        const int chk = bundled_check(epoch_before, pending_before, hm[kMsEpoch], hm[kMsPending], done,
                                      (uint64_t)nbundles * kMsSets * stride + 2);
        if (chk == kLoopStalled || chk == kLoopOverBound) {
            set_error_detail(chk == kLoopStalled ? "bundled generation stalled: a batch of steps changed no level"
                                                 : "bundled generation ran more levels than its sets can have");
            return HYPERIM_EHIP;
        }
        epoch_before = hm[kMsEpoch];
        pending_before = hm[kMsPending];
        for (int k = 0; time_kernels && k < batch; ++k) {
            float me = 0.f;
            HIM_HIP(hipEventElapsedTime(&me, E[2 + 2 * k], E[3 + 2 * k]));
            st.ms_bundled += me;
        }
        st.bundled_launches += batch;
        st.supersteps += batch;
        st.launches += 5 * batch;
        if (trace) {
            uint64_t cur = 0;
            HIM_CHECK(read_ctr(s, m.ctr, kMsCur, &cur));
            fprintf(stderr, "[hyperim] bundled step %llu: frontier %llu\n", (unsigned long long)steps,
                    (unsigned long long)cur);
        }
        if (done) break;
    }
    uint64_t overflow = 0;
    HIM_CHECK(read_ctr(s, m.ctr, kMsOverflow, &overflow));
    if (overflow) {
        set_error_detail("bundled frontier list overflow");
        return HYPERIM_EHIP;
    }
    // output: counts per vertex block, set ranges, members in ascending order
    const uint32_t out_grid = nbundles * nvb;
    hipLaunchKernelGGL(k_ms_count, dim3(out_grid), dim3(kWG), 0, s, m);
    hipLaunchKernelGGL(k_ms_record, dim3((uint32_t)div_up(a.count, kWG)), dim3(kWG), 0, s, m, a);
    hipLaunchKernelGGL(k_ms_write, dim3(out_grid), dim3(kWG), 0, s, m, a);
    HIM_HIP(hipGetLastError());
    HIM_HIP(hipMemcpyAsync(ws.host + kHostFinal, a.ctr, sizeof(unsigned long long) * kNumCtr, hipMemcpyDeviceToHost,
                           s));
    HIM_HIP(hipEventRecord(ws.events[3], s));
    const int rc = tail();
    HIM_HIP(hipStreamSynchronize(s));
    HIM_CHECK(rc);
    HIM_HIP(hipEventElapsedTime(&ms, ws.events[0], ws.events[3]));
    st.ms_bfs += ms;
    st.ms_heavy += ms;
    st.launches += 6;
    return HYPERIM_OK;
}

}  // namespace

namespace {

// Appending the staged sets with group-local indices [first, first + count)
// to pool p takes two steps around a wait for the stream.  compact_scan
// queues the offsets (an exclusive scan of the sizes from p's total) and the
// copy of the new total into *total_host.
int compact_scan(RRWorkspace &ws, hyperim_pool p, uint64_t first, uint64_t count, unsigned long long *total_host,
                 hipStream_t s) {
    if (count == 0) return HYPERIM_OK;
    HIM_CHECK(pool_reserve(p, count, 0, s));
    uint64_t *dst_off = p->off + p->count;
    HIM_CHECK(scan_u32_to_u64(ws.sizes.as<uint32_t>() + first, dst_off, count, p->total, ws.scan_tmp, s));
    HIM_HIP(hipMemcpyAsync(total_host, dst_off + count, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    return HYPERIM_OK;
}

// compact_move, once the new total is on the host, grows p's storage and
// moves the members and roots (HYPERIM_ECAPACITY beyond max_entries or a
// caller buffer; the pool is then unchanged).
int compact_move(RRWorkspace &ws, hyperim_pool p, uint64_t first, uint64_t count, uint64_t new_total,
                 uint64_t max_entries, hipStream_t s) {
    if (count == 0) return HYPERIM_OK;
    if (max_entries && new_total > max_entries) {
        set_error_detail("pool would exceed max_entries");
        return HYPERIM_ECAPACITY;
    }
    HIM_CHECK(pool_reserve(p, count, new_total - p->total, s));
    uint64_t *dst_off = p->off + p->count;   // storage may have moved
    HIM_HIP(hipMemcpyAsync(p->roots + p->count, ws.roots.as<uint32_t>() + first, sizeof(uint32_t) * count,
                           hipMemcpyDeviceToDevice, s));
    const uint32_t grid = (uint32_t)std::min<uint64_t>(div_up(count, kWave * kWavesPerWG), 65535u);
    hipLaunchKernelGGL(k_move_small, dim3(std::max<uint32_t>(grid, 1)), dim3(kWG), 0, s,
                       ws.stage_off.as<uint64_t>() + first, ws.sizes.as<uint32_t>() + first, dst_off, count,
                       ws.stage.as<uint32_t>(), p->mem);
    hipLaunchKernelGGL(k_move_big, dim3(1024), dim3(kWG), 0, s, ws.big_ids.as<uint64_t>(),
                       ws.counters.as<unsigned long long>() + kBigCount, first, count, ws.stage_off.as<uint64_t>(),
                       ws.sizes.as<uint32_t>(), dst_off, ws.stage.as<uint32_t>(), p->mem);
    HIM_HIP(hipGetLastError());
    p->count += count;
    p->total = new_total;
    return HYPERIM_OK;
}

}  // namespace

size_t rr_slot_bytes(uint32_t n_max) {
    SlotLayout L;
    return slot_layout(n_max, &L) == HYPERIM_OK ? (size_t)L.bytes : 0;
}

int rr_generate_into(RRWorkspace &ws, RRStats &st, const std::vector<RRTask> &tasks,
                     const std::vector<hyperim_pool> &pools, uint32_t qlog, int form, uint64_t max_entries,
                     uint64_t stage_budget, hipStream_t s, std::vector<int> &pool_status, bool time_kernels,
                     bool graphs) {
    // HYPERIM_TRACE=1: synchronise after every grid-wide superstep and report
    // its item count and time on stderr (diagnostics; same results)
    static const bool trace = [] {
        const char *e = getenv("HYPERIM_TRACE");
        return e && e[0] == '1';
    }();
    pool_status.assign(tasks.size(), HYPERIM_OK);
    if (tasks.empty()) return HYPERIM_OK;
    // a launch group compacts its slices after one wait, so each task needs a
    // pool of its own
    std::vector<hyperim_pool> sorted(pools);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) {
        set_error_detail("two tasks of one generation call share a pool");
        return HYPERIM_EINVAL;
    }
    // execution parameters of the first task's graph
    const hyperim_tuning &tune = tasks[0].g->tune;
    // graph descriptors (one per distinct graph)
    std::map<hyperim_graph, uint32_t> gid;
    std::vector<GraphDesc> gdesc;
    uint32_t n_max = 1;
    for (const RRTask &t : tasks) {
        if (gid.count(t.g)) continue;
        gid[t.g] = (uint32_t)gdesc.size();
        hyperim_graph g = t.g;
        gdesc.push_back(graph_desc(g));
        n_max = std::max(n_max, g->n);
    }
    uint64_t count = 0;
    for (const RRTask &t : tasks) count += t.id_end - t.id_begin;
    if (count == 0) return HYPERIM_OK;
    LaunchShape shape;
    HIM_CHECK(ensure_workspace(ws, n_max, s, &shape));

    // launch shapes: the occupancy limits, capped per compute unit by the tuning
    auto capped = [&](uint32_t full, uint32_t per_cu) {
        return per_cu ? std::max<uint32_t>(1, std::min<uint32_t>(full, shape.cus * per_cu)) : full;
    };
    const uint32_t grid_a = capped(shape.grid, tune.blocks_a);
    const uint32_t grid_b = capped(shape.grid_b, tune.blocks_b);
    const size_t ndef_cap = shape.slots;   // stride of the deferred-set arrays
    const size_t spare = std::max<uint64_t>(shape.slots - (uint64_t)grid_a * kWavesPerWG, 1);

    // Launch groups are contiguous ranges of launch indices (the tasks laid
    // back to back), planned one at a time with what earlier groups taught.
    // A group's sets are staged, then compacted into their pools before the
    // next group runs, so the stage holds one group.  A group takes indices
    // while its predicted members fit the stage budget -- 1.3 x the graph's
    // members per set seen so far, or n (an upper bound) for a graph not
    // seen yet, whose first group then stops after kLearnIds of its sets
    // unless that bound fits for all of them and the graph has no bundled
    // mode to decide -- and (form 0) while the sets
    // it defers fit the spare slots at the
    // deferral rate seen so far (a set that finds no spare slot stays with
    // its wave).  The plain form (1) also ends a group at every (task, ladder
    // block, stratum) boundary.
    constexpr uint64_t kLearnIds = 2048;
    constexpr uint64_t kMsBudget = 8ull << 30;   // bytes of bundled-mode state per launch group
    // bundled mode for graphs whose sets are large on average (form 0 only;
    // the plain form keeps one traversal per set)
    // (a graph not seen yet starts bundled when its tuning enables the mode:
    // the first group's sets teach the estimate either way, and a graph tuned
    // for bundled mode has large sets, which the per-set mode grows slowly)
    auto bundled = [&](const RRTask &t) {
        return form == 0 && t.g->kind() == 0 && tune.ms_min != 0xFFFFFFFFu &&
               (t.g->rr_members < 0.0 || t.g->rr_members >= (double)tune.ms_min);
    };
    const double stage_words = (double)stage_budget / 4.0;
    auto per_set = [](hyperim_graph g) { return g->rr_members >= 0.0 ? 1.3 * g->rr_members + 1.0 : (double)g->n; };
    std::vector<uint64_t> tstart(tasks.size() + 1, 0);
    for (size_t i = 0; i < tasks.size(); ++i) tstart[i + 1] = tstart[i] + (tasks[i].id_end - tasks[i].id_begin);
    // unit boundaries: task ends (form 0), (task, block, stratum) ends (form 1)
    std::vector<uint64_t> unit_end;
    for (size_t i = 0; i < tasks.size(); ++i) {
        const RRTask &t = tasks[i];
        if (form == 1) {
            std::vector<std::pair<uint64_t, uint64_t>> ranges;
            stratum_ranges(t.g, t.seed, t.instance, qlog, t.pool, t.id_begin, t.id_end, &ranges);
            for (const auto &rg : ranges) unit_end.push_back(tstart[i] + (rg.second - t.id_begin));
        } else {
            unit_end.push_back(tstart[i + 1]);
        }
    }

    unsigned long long *ctr = ws.counters.as<unsigned long long>();
    RRArgs a{};
    a.qlog = qlog;
    a.heavy = tune.heavy;
    a.budget = tune.budget;
    a.chunk = tune.chunk;
    a.seg = std::max(tune.seg, tune.chunk);
    a.prefilter_min = tune.prefilter_min;
    a.slot_n = shape.slot_n;
    a.slot_words = shape.slot_words;
    a.ctr = ctr;
    a.lists = ws.lists.as<uint32_t>();
    a.bitmaps = ws.bitmaps.as<uint32_t>();
    a.slot_total = shape.slots;
    a.out_base = 0;
    a.def_idx = ws.def_idx.as<uint64_t>();
    a.def_root = ws.def_u32.as<uint32_t>();
    a.def_slot = a.def_root + ndef_cap;
    a.def_head = a.def_slot + ndef_cap;
    a.def_size = a.def_head + ndef_cap;
    a.def_task = a.def_size + ndef_cap;
    a.items = ws.items.as<uint4>();
    HIM_CHECK(ws.graph_desc.reserve(sizeof(GraphDesc) * gdesc.size(), s));
    HIM_CHECK(ws.task_desc.reserve(sizeof(TaskDesc) * tasks.size(), s));
    // pinned staging: fixed words, then the pools' new totals (one per
    // task), task descriptors, graph descriptors
    auto words = [](size_t bytes) { return (bytes + sizeof(unsigned long long) - 1) / sizeof(unsigned long long); };
    const size_t host_totals = kHostFixed;
    const size_t host_tasks = host_totals + tasks.size();
    const size_t host_graphs = host_tasks + words(sizeof(TaskDesc) * tasks.size());
    HIM_CHECK(ensure_host(ws, host_graphs + words(sizeof(GraphDesc) * gdesc.size())));
    GraphDesc *gstage = reinterpret_cast<GraphDesc *>(ws.host + host_graphs);
    std::copy(gdesc.begin(), gdesc.end(), gstage);
    HIM_HIP(hipMemcpyAsync(ws.graph_desc.ptr, gstage, sizeof(GraphDesc) * gdesc.size(), hipMemcpyHostToDevice, s));
    a.graphs = ws.graph_desc.as<GraphDesc>();

    struct Slice {
        size_t task;
        uint64_t lo, hi;   // launch indices
    };
    size_t unit = 0;
    for (uint64_t pos = 0; pos < count;) {
        // ---- plan the next group ---------------------------------------
        double rate = 0.0;
        for (const RRTask &t : tasks) rate = std::max(rate, t.g->rr_defer >= 0.0 ? t.g->rr_defer : 0.5);
        const uint64_t def_chunk =
            form == 0 ? std::max<uint64_t>((uint64_t)((double)spare / std::max(rate * 1.25, 1.0 / 64.0)), 4096)
                      : ~0ull;
        const uint64_t lo = pos;
        double acc = 0.0;
        size_t ti = std::upper_bound(tstart.begin(), tstart.end(), pos) - tstart.begin() - 1;
        while (unit_end[unit] <= pos) ++unit;
        const bool ms = bundled(tasks[ti]);
        if (ms) {
            // bundled mode: one task, as many sets as the stage and the
            // bundle memory allow
            const RRTask &t = tasks[ti];
            const uint64_t rest = tstart[ti + 1] - pos;
            const uint64_t max_sets =
                kMsSets * std::max<uint64_t>(1, kMsBudget / ms_bytes_per_bundle(t.g->n));
            const double m = per_set(t.g);
            uint64_t take = std::min<uint64_t>(rest, max_sets);
            take = std::min<uint64_t>(take, std::max<uint64_t>(1, (uint64_t)(stage_words / m)));
            acc = (double)take * m;
            pos += take;
        }
        for (; !ms;) {
            const RRTask &t = tasks[ti];
            const double m = per_set(t.g);
            const bool learn = t.g->rr_members < 0.0;
            const uint64_t rest = (form == 1 ? unit_end[unit] : tstart[ti + 1]) - pos;
            const double room = stage_words - acc;
            // a graph not seen yet stops its first group after kLearnIds sets,
            // unless the worst case of all its remaining sets fits already and
            // no bundled mode waits for what the group would teach
            const bool cap = learn && ((double)rest * m > room || t.g->tune.ms_min != 0xFFFFFFFFu);
            const uint64_t limit = cap ? std::min(rest, kLearnIds) : rest;
            uint64_t take = std::min<uint64_t>(limit, room > 0.0 ? (uint64_t)(room / m) : 0);
            take = std::min<uint64_t>(take, def_chunk - (pos - lo));
            if (take == 0 && pos == lo) take = 1;   // one set always fits
            acc += (double)take * m;
            pos += take;
            if (take < rest || pos == count || form == 1 || pos - lo >= def_chunk) break;
            ++ti;   // form 0: the group continues with the next task ...
            // ... unless that one runs bundled or has the other cascade model
            if (bundled(tasks[ti]) || tasks[ti].g->kind() != tasks[ti - 1].g->kind()) break;
        }
        const uint64_t hi = pos;
        // descriptors of the group's task slices
        std::vector<TaskDesc> tdesc;
        std::vector<Slice> slices;
        for (size_t i = 0; i < tasks.size(); ++i) {
            const uint64_t a0 = std::max(lo, tstart[i]), a1 = std::min(hi, tstart[i + 1]);
            if (a0 >= a1) continue;
            const RRTask &t = tasks[i];
            tdesc.push_back(TaskDesc{a1 - lo, t.id_begin + (a0 - tstart[i]), t.pool, gid[t.g], (uint32_t)t.seed,
                                     t.instance});
            slices.push_back(Slice{i, a0, a1});
        }
        const uint64_t n_ids = hi - lo;
        HIM_CHECK(ws.stage_off.reserve(sizeof(uint64_t) * n_ids, s, false));
        HIM_CHECK(ws.sizes.reserve(sizeof(uint32_t) * n_ids, s, false));
        HIM_CHECK(ws.roots.reserve(sizeof(uint32_t) * n_ids, s, false));
        HIM_CHECK(ws.big_ids.reserve(sizeof(uint64_t) * n_ids, s, false));
        // stage sized from the prediction (a miss re-runs the group)
        const uint64_t predicted = (uint64_t)acc + 4 * n_ids + (1u << 20);
        if (ws.stage.bytes < sizeof(uint32_t) * predicted)
            HIM_CHECK(ws.stage.reserve(sizeof(uint32_t) * predicted, s, false));
        // descriptors go through the pinned staging (the previous group has drained)
        TaskDesc *tstage = reinterpret_cast<TaskDesc *>(ws.host + host_tasks);
        std::copy(tdesc.begin(), tdesc.end(), tstage);
        HIM_HIP(hipMemcpyAsync(ws.task_desc.ptr, tstage, sizeof(TaskDesc) * tdesc.size(), hipMemcpyHostToDevice, s));
        a.tasks = ws.task_desc.as<TaskDesc>();
        a.ntasks = (uint32_t)tdesc.size();
        a.count = n_ids;
        a.stage_off = ws.stage_off.as<uint64_t>();
        a.sizes = ws.sizes.as<uint32_t>();
        a.roots = ws.roots.as<uint32_t>();
        a.big_ids = ws.big_ids.as<uint64_t>();
        const uint32_t grid =
            form == 0 ? grid_a : (uint32_t)std::min<uint64_t>(grid_a, div_up(a.count, kWavesPerWG));
        // a graph whose sets were never deferred before is checked after phase A
        bool expect_defer = false;
        for (const Slice &sl : slices) expect_defer |= tasks[sl.task].g->rr_defer != 0.0;
        // compaction offsets of every slice, queued behind the launch so that
        // one wait covers both (a launch whose stage overflowed discards them)
        std::vector<int> scan_rc(slices.size(), HYPERIM_OK);
        auto scans = [&]() -> int {
            for (size_t i = 0; i < slices.size(); ++i) {
                const Slice &sl = slices[i];
                scan_rc[i] = HYPERIM_OK;
                if (pool_status[sl.task] != HYPERIM_OK) continue;
                const int rc = compact_scan(ws, pools[sl.task], sl.lo - lo, sl.hi - sl.lo, ws.host + host_totals + i, s);
                if (rc == HYPERIM_ECAPACITY) scan_rc[i] = rc;
                else if (rc != HYPERIM_OK) return rc;
            }
            return HYPERIM_OK;
        };

        // ---- run it ----------------------------------------------------
        bool staged = false;
        for (int attempt = 0; attempt < 2 && !staged; ++attempt) {
            a.stage = ws.stage.as<uint32_t>();
            a.stage_cap = ws.stage.bytes / sizeof(uint32_t);
            HIM_HIP(hipMemsetAsync(ctr, 0, sizeof(unsigned long long) * kNumCtr, s));
            RRStats run{};
            if (ms)
                HIM_CHECK(run_ms_launch(ws, run, tune, a, shape, tasks[slices[0].task].g, tdesc[0], trace,
                                        time_kernels, graphs, s, scans));
            else if (tasks[slices[0].task].g->lt())
                HIM_CHECK(run_lt_launch(ws, run, a, shape, grid, s, scans));
            else if (tasks[slices[0].task].g->layered())
                HIM_CHECK(run_layered_launch(ws, run, a, shape, grid, s, scans));
            else
                HIM_CHECK(run_launch(ws, run, tune, a, shape, grid, grid_b, expect_defer, trace, time_kernels,
                                     graphs, tasks[slices[0].task].g->gaps(), s, scans));
            // time counts every attempt, work only the one that produced the output
            st.ms_bfs += run.ms_bfs;
            st.ms_light += run.ms_light;
            st.ms_heavy += run.ms_heavy;
            st.launches += run.launches;
            st.supersteps += run.supersteps;
            st.ms_expand += run.ms_expand;
            st.expand_launches += run.expand_launches;
            st.ms_bundled += run.ms_bundled;
            st.bundled_launches += run.bundled_launches;
            const unsigned long long *hf = ws.host + kHostFinal;
            const uint64_t bump = hf[kBump];
            for (const Slice &sl : slices) tasks[sl.task].g->rr_defer = (double)run.deferred / (double)a.count;
            if (bump <= a.stage_cap) {
                st.deferred += run.deferred;
                st.bytes_light += hf[kBytesA];
                st.bytes_heavy += hf[kBytesB];
                st.bytes_bundled += hf[kBytesMs];
                st.philox += hf[kPhiloxA] + hf[kPhilox] + hf[kPhiloxMs];
                st.philox_light += hf[kPhiloxA];
                st.philox_bundled += hf[kPhiloxMs];
                staged = true;
            } else {
                HIM_CHECK(ws.stage.reserve(sizeof(uint32_t) * (size_t)(bump + bump / 4 + 1024), s, false));
            }
        }
        if (!staged) {
            set_error_detail("RR stage overflow after resize");
            return HYPERIM_ENOMEM;
        }

        // ---- compact it ------------------------------------------------
        for (size_t i = 0; i < slices.size(); ++i) {
            const Slice &sl = slices[i];
            if (pool_status[sl.task] != HYPERIM_OK) continue;
            hyperim_pool p = pools[sl.task];
            const uint64_t before = p->total;
            int rc = scan_rc[i];
            if (rc == HYPERIM_OK)
                rc = compact_move(ws, p, sl.lo - lo, sl.hi - sl.lo, ws.host[host_totals + i], max_entries, s);
            if (rc == HYPERIM_ECAPACITY) {
                pool_status[sl.task] = rc;   // this pool is full; the others go on
            } else if (rc != HYPERIM_OK) {
                return rc;
            } else {
                // members per set of this graph, learned for later predictions
                hyperim_graph g = tasks[sl.task].g;
                g->rr_seen_sets += sl.hi - sl.lo;
                g->rr_seen_members += p->total - before;
                g->rr_members = (double)g->rr_seen_members / (double)g->rr_seen_sets;
            }
        }
    }
    return HYPERIM_OK;
}

int rr_incidences(hyperim_graph g, hyperim_pool p, uint64_t theta, hipStream_t s, RRWork *out) {
    uint64_t entries = 0;
    HIM_HIP(hipMemcpyAsync(&entries, p->off + theta, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    DevBuf acc;
    HIM_CHECK(acc.reserve(4 * sizeof(unsigned long long), s));
    HIM_HIP(hipMemsetAsync(acc.ptr, 0, 4 * sizeof(unsigned long long), s));
    if (entries) {
        const uint32_t grid = (uint32_t)std::min<uint64_t>(div_up(entries, kWG), 4096);
        hipLaunchKernelGGL(k_weight_sum, dim3(grid), dim3(kWG), 0, s, p->mem, entries,
                           g->weight.as<unsigned long long>(), g->bytesw.as<unsigned long long>(),
                           g->c.as<unsigned long long>(), g->phiw.as<unsigned long long>(),
                           acc.as<unsigned long long>());
    }
    unsigned long long v[4] = {0, 0, 0, 0};
    HIM_HIP(hipMemcpyAsync(v, acc.ptr, sizeof(v), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    acc.release();
    out->incidences = v[0];
    out->alg_bytes = v[1];
    out->coins = v[2];
    out->philox = v[3];
    return HYPERIM_OK;
}

}  // namespace hyperim
