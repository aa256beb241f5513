// RR-set generation on gfx950 (Algorithm 3's skeleton with one keyed coin per
// channel), stratified roots, and compaction into the RR-set CSR.
//
// Execution: a persistent launch whose wavefronts steal RR ids from a global
// counter.  One wavefront owns one RR set at a time:
//   - the set's member list doubles as the BFS queue (global, per wave slot);
//   - visited marks are a bitmap, in LDS when |V| is small, else global;
//   - each frontier batch (up to 64 queued vertices) is expanded cooperatively
//     in three load-balanced levels -- vertices -> incidences (v, he) ->
//     quads of 4 member positions -- so lanes stay busy whatever the degree
//     and hyperedge-size skew, and member ids are read contiguously;
//   - one Philox4x32-10 call yields the 4 coins of a quad; a live channel
//     from an unvisited member sets its bit (atomic OR) and the winner
//     appends it to the queue with a ballot-ranked store;
//   - the finished set is written ascending to a staging area, sorted in LDS
//     (small sets) or read back from the bitmap in id order (large sets).
// Compaction turns the per-id sizes into CSR offsets (device scan) and moves
// the staged members into the pool.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "dev_common.h"
#include "internal.h"

namespace hyperim {
namespace {

constexpr int kWG = 256;
constexpr int kWavesPerWG = kWG / kWave;
constexpr uint32_t kSortMax = 1024;          // sets up to this size are sorted in LDS
constexpr uint32_t kLdsBitmapWords = 1024;   // visited bitmap in LDS when |V| <= 32768
constexpr uint32_t kBigSet = 4096;           // compaction: one workgroup per larger set
constexpr uint64_t kSlotBudget = 16ull << 30; // bytes of per-wave lists + bitmaps

struct RRArgs {
    const uint32_t *__restrict__ he_off;
    const uint32_t *__restrict__ he_mem;
    const uint32_t *__restrict__ v_off;
    const uint32_t *__restrict__ v_he;
    const uint32_t *__restrict__ thr;
    const uint32_t *__restrict__ P;
    uint32_t n, key0, key1, pool, qlog, bm_words, prefilter;
    uint64_t id_begin, count;        // ids [id_begin, id_begin + count)
    uint64_t out_base;               // index of id_begin in the per-id arrays
    unsigned long long *work;        // next relative id to take
    unsigned long long *stage_bump;  // staged members so far
    unsigned long long *big_count;   // sets larger than kBigSet
    uint32_t *lists;                 // per wave slot: n entries
    uint32_t *bitmaps;               // per wave slot: bm_words (global mode)
    uint32_t *stage;
    uint64_t stage_cap;
    uint64_t *stage_off;             // per id
    uint32_t *sizes;                 // per id
    uint32_t *roots;                 // per id
    uint64_t *big_ids;               // per big set: relative id
};

struct WaveLds {
    uint32_t fr_scan[kWave], fr_v[kWave], fr_e0[kWave];
    uint32_t in_scan[kWave], in_he[kWave], in_hb[kWave], in_hs[kWave], in_v[kWave], in_thr[kWave];
    uint32_t sort[kSortMax];
};

// Stratified root of RR id j: block b of the ladder (Q = 2^qlog ids in block
// 0, Q 2^(b-1) in block b >= 1, so block sizes are powers of two), offset
// o_b = floor(x n / 2^64) from the block's Philox draw, root =
// P[floor((t n + o_b) / T_b)] computed in 128-bit arithmetic.
__device__ __forceinline__ uint32_t rr_root(const RRArgs &a, uint64_t j, uint2 key) {
    const uint64_t Q = 1ull << a.qlog;
    uint32_t b, s;
    uint64_t J;
    if (j < Q) {
        b = 0;
        J = 0;
        s = a.qlog;
    } else {
        const uint32_t hb = 63u - (uint32_t)__clzll((long long)j);
        b = hb - a.qlog + 1u;
        J = 1ull << hb;
        s = hb;
    }
    const uint4 r = philox4x32_10(root_counter(b, a.pool), key);
    const uint64_t x = (uint64_t)r.x | ((uint64_t)r.y << 32);
    const uint64_t o = __umul64hi(x, (uint64_t)a.n);
    const uint64_t t = j - J;
    const uint64_t lo = t * (uint64_t)a.n;
    uint64_t hi = __umul64hi(t, (uint64_t)a.n);
    const uint64_t lo2 = lo + o;
    hi += lo2 < lo ? 1ull : 0ull;
    const uint64_t pos = s == 0 ? lo2 : ((lo2 >> s) | (hi << (64u - s)));
    return a.P[pos];
}

template <bool kLds>
__device__ __forceinline__ uint32_t bm_load(uint32_t *bm, uint32_t w) {
    if constexpr (kLds) return bm[w];
    else return __hip_atomic_load(bm + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool kLdsBitmap>
__global__ __launch_bounds__(kWG) void k_rr_bfs(RRArgs a) {
    __shared__ WaveLds lds[kWavesPerWG];
    __shared__ uint32_t lbm[kLdsBitmap ? kWavesPerWG : 1][kLdsBitmap ? kLdsBitmapWords : 1];
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    const uint64_t slot = (uint64_t)blockIdx.x * kWavesPerWG + wv;
    WaveLds &L = lds[wv];
    uint32_t *list = a.lists + slot * a.n;
    uint32_t *bm;
    if constexpr (kLdsBitmap) {
        bm = lbm[wv];
        for (uint32_t i = lane; i < a.bm_words; i += kWave) bm[i] = 0u;
    } else {
        bm = a.bitmaps + slot * a.bm_words;
    }
    wave_sync();
    const uint2 key = make_uint2(a.key0, a.key1);

    for (;;) {
        unsigned long long idx = 0;
        if (lane == 0) idx = atomicAdd(a.work, 1ull);
        idx = wave_bcast64(idx, 0);
        if (idx >= a.count) break;
        const uint64_t j = a.id_begin + idx;
        const uint32_t root = rr_root(a, j, key);
        if (lane == 0) {
            list[0] = root;
            atomicOr(&bm[root >> 5], 1u << (root & 31));
        }
        uint32_t size = 1, head = 0;

        while (head < size) {
            // queue entries were stored by other lanes of this wave: wait for
            // the stores and drop stale L1 lines before reading them
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const uint32_t nb = min((uint32_t)kWave, size - head);
            uint32_t v = 0, e0 = 0, d = 0;
            if (lane < nb) {
                v = list[head + lane];
                e0 = a.v_off[v];
                d = a.v_off[v + 1] - e0;
            }
            head += nb;
            const uint32_t dscan = wave_incl_scan(d);
            const uint32_t D = wave_bcast(dscan, kWave - 1);
            L.fr_scan[lane] = dscan;
            L.fr_v[lane] = v;
            L.fr_e0[lane] = e0;
            wave_sync();
            for (uint32_t base = 0; base < D; base += kWave) {
                // level 2: one incidence (v, he) per lane
                const uint32_t g = base + lane;
                uint32_t he = 0, hb = 0, hs = 0, vv = 0, th = 0, nq = 0;
                if (g < D) {
                    const uint32_t k = search64(L.fr_scan, g);
                    const uint32_t start = k ? L.fr_scan[k - 1] : 0u;
                    vv = L.fr_v[k];
                    he = a.v_he[L.fr_e0[k] + (g - start)];
                    hb = a.he_off[he];
                    hs = a.he_off[he + 1] - hb;
                    th = a.thr[vv];
                    nq = th ? (hs + 3u) >> 2 : 0u;   // threshold 0: no channel into vv is live
                }
                const uint32_t qscan = wave_incl_scan(nq);
                const uint32_t Qn = wave_bcast(qscan, kWave - 1);
                wave_sync();
                L.in_scan[lane] = qscan;
                L.in_he[lane] = he;
                L.in_hb[lane] = hb;
                L.in_hs[lane] = hs;
                L.in_v[lane] = vv;
                L.in_thr[lane] = th;
                wave_sync();
                for (uint32_t qb = 0; qb < Qn; qb += kWave) {
                    // level 3: one quad of member positions per lane
                    const uint32_t qg = qb + lane;
                    uint32_t u[4];
                    uint32_t ve = 0, hee = 0, q = 0, the = 0;
                    bool need = false;
                    if (qg < Qn) {
                        const uint32_t k = search64(L.in_scan, qg);
                        const uint32_t start = k ? L.in_scan[k - 1] : 0u;
                        q = qg - start;
                        hee = L.in_he[k];
                        ve = L.in_v[k];
                        the = L.in_thr[k];
                        const uint32_t hbk = L.in_hb[k], hsk = L.in_hs[k];
                        const uint32_t p0 = q * 4u;
                        const uint32_t cm = min(4u, hsk - p0);
#pragma unroll
                        for (uint32_t t = 0; t < 4; ++t) u[t] = t < cm ? a.he_mem[hbk + p0 + t] : ve;
#pragma unroll
                        for (uint32_t t = 0; t < 4; ++t) {
                            bool cand = u[t] != ve;
                            if (cand && a.prefilter) cand = !(bm_load<kLdsBitmap>(bm, u[t] >> 5) & (1u << (u[t] & 31)));
                            need |= cand;
                        }
                    } else {
#pragma unroll
                        for (uint32_t t = 0; t < 4; ++t) u[t] = 0;
                    }
                    if (__ballot(need) == 0) continue;
                    uint4 c = make_uint4(0u, 0u, 0u, 0u);
                    if (need) c = philox4x32_10(coin_counter(j, hee, ve, a.pool, q), key);
                    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
                    for (uint32_t t = 0; t < 4; ++t) {
                        bool fresh = false;
                        if (need && u[t] != ve && channel_live(w[t], the)) {
                            const uint32_t bit = 1u << (u[t] & 31);
                            fresh = (atomicOr(&bm[u[t] >> 5], bit) & bit) == 0u;
                        }
                        const uint64_t bal = __ballot(fresh);
                        const uint32_t at = size + lane_rank(bal);
                        if (fresh && at < a.n) list[at] = u[t];   // at < n always holds: one bit per vertex
                        size = min(size + (uint32_t)__popcll(bal), a.n);
                    }
                }
            }
        }

        // ---- output: ascending members into the stage --------------------
        unsigned long long off = 0;
        if (lane == 0) off = atomicAdd(a.stage_bump, (unsigned long long)size);
        off = wave_bcast64(off, 0);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (off + size <= a.stage_cap) {
            if (size <= kSortMax) {
                uint32_t P2 = kWave;
                while (P2 < size) P2 <<= 1;
                for (uint32_t i = lane; i < P2; i += kWave) L.sort[i] = i < size ? list[i] : 0xFFFFFFFFu;
                wave_sync();
                for (uint32_t k = 2; k <= P2; k <<= 1) {
                    for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
                        for (uint32_t i = lane; i < P2; i += kWave) {
                            const uint32_t x = i ^ jj;
                            if (x > i) {
                                const uint32_t p = L.sort[i], qv = L.sort[x];
                                if ((p > qv) == ((i & k) == 0)) {
                                    L.sort[i] = qv;
                                    L.sort[x] = p;
                                }
                            }
                        }
                        wave_sync();
                    }
                }
                for (uint32_t i = lane; i < size; i += kWave) a.stage[off + i] = L.sort[i];
                wave_sync();
            } else {
                uint32_t written = 0;
                for (uint32_t w0 = 0; w0 < a.bm_words; w0 += kWave) {
                    const uint32_t wi = w0 + lane;
                    uint32_t word = wi < a.bm_words ? bm_load<kLdsBitmap>(bm, wi) : 0u;
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
        if (lane == 0) {
            const uint64_t o = a.out_base + idx;
            a.stage_off[o] = off;
            a.sizes[o] = size;
            a.roots[o] = root;
            if (size > kBigSet) a.big_ids[atomicAdd(a.big_count, 1ull)] = o;
        }
        // clear this set's marks (the bitmap is all-zero again afterwards)
        if (kLdsBitmap && size * 4u > a.bm_words) {
            for (uint32_t i = lane; i < a.bm_words; i += kWave) bm[i] = 0u;
        } else {
            for (uint32_t i = lane; i < size; i += kWave) bm[list[i] >> 5] = 0u;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        wave_sync();
    }
}

// Compaction of sets up to kBigSet members: each wave moves 64 consecutive
// ids, flattened over their members.
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

__global__ __launch_bounds__(kWG) void k_move_big(const uint64_t *__restrict__ big_ids,
                                                   const unsigned long long *__restrict__ big_count,
                                                   const uint64_t *__restrict__ stage_off,
                                                   const uint32_t *__restrict__ sizes,
                                                   const uint64_t *__restrict__ dst_off,
                                                   const uint32_t *__restrict__ stage, uint32_t *__restrict__ mem) {
    const uint64_t nbig = *big_count;
    for (uint64_t b = blockIdx.x; b < nbig; b += gridDim.x) {
        const uint64_t id = big_ids[b];
        const uint64_t src = stage_off[id], dst = dst_off[id];
        const uint32_t sz = sizes[id];
        for (uint32_t i = threadIdx.x; i < sz; i += blockDim.x) mem[dst + i] = stage[src + i];
    }
}

__global__ __launch_bounds__(kWG) void k_weight_sum(const uint32_t *__restrict__ mem, uint64_t entries,
                                                     const unsigned long long *__restrict__ w0,
                                                     const unsigned long long *__restrict__ w1,
                                                     unsigned long long *__restrict__ out) {
    unsigned long long a0 = 0, a1 = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < entries;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = mem[i];
        a0 += w0[v];
        a1 += w1[v];
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    if (lane_id() == 0) {
        atomicAdd(out, a0);
        atomicAdd(out + 1, a1);
    }
}

struct LaunchShape {
    uint32_t grid, waves;
    bool lds;
};

int ensure_workspace(hyperim_graph g, hipStream_t s, LaunchShape *shape) {
    RRWorkspace &ws = g->rr;
    const uint32_t n = g->n;
    const bool lds = n <= kLdsBitmapWords * 32u;
    const uint32_t words = (n + 31u) / 32u;
    if (ws.grid == 0) {
        int dev = 0;
        HIM_HIP(hipGetDevice(&dev));
        int cus = 0;
        HIM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        int per_cu = 0;
        if (lds)
            HIM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rr_bfs<true>, kWG, 0));
        else
            HIM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rr_bfs<false>, kWG, 0));
        per_cu = std::max(per_cu, 1);
        uint64_t grid = (uint64_t)cus * (uint64_t)per_cu;
        const uint64_t per_wave = (uint64_t)n * 4u + (lds ? 0u : (uint64_t)words * 4u);
        const uint64_t max_waves = std::max<uint64_t>(kSlotBudget / std::max<uint64_t>(per_wave, 1), kWavesPerWG);
        grid = std::min<uint64_t>(grid, max_waves / kWavesPerWG);
        grid = std::max<uint64_t>(grid, 1);
        ws.grid = (uint32_t)grid;
        ws.waves = ws.grid * kWavesPerWG;
        HIM_CHECK(ws.lists.reserve(sizeof(uint32_t) * (size_t)ws.waves * std::max<uint32_t>(n, 1), s));
        if (!lds) {
            HIM_CHECK(ws.bitmaps.reserve(sizeof(uint32_t) * (size_t)ws.waves * words, s));
            HIM_HIP(hipMemsetAsync(ws.bitmaps.ptr, 0, sizeof(uint32_t) * (size_t)ws.waves * words, s));
        }
        HIM_CHECK(ws.counters.reserve(sizeof(unsigned long long) * 8, s));
    }
    shape->grid = ws.grid;
    shape->waves = ws.waves;
    shape->lds = lds;
    return HYPERIM_OK;
}

// Id ranges of every (ladder block, stratum) pair inside [id_begin, id_end).
void stratum_ranges(hyperim_graph g, const RRKey &key, uint64_t id_begin, uint64_t id_end,
                    std::vector<std::pair<uint64_t, uint64_t>> *out) {
    const uint64_t Q = 1ull << key.qlog;
    const uint32_t n = g->n;
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
            b = hb - key.qlog + 1u;
            J = 1ull << hb;
            T = J;
        }
        const uint4 r = philox4x32_10(root_counter(b, key.pool), make_uint2((uint32_t)key.seed, key.instance));
        const uint64_t x = (uint64_t)r.x | ((uint64_t)r.y << 32);
        const uint64_t o = (uint64_t)(((unsigned __int128)x * n) >> 64);
        uint64_t prev = 0;
        for (uint32_t h = 1; h <= kNStrata; ++h) {
            uint64_t th;
            if (h == kNStrata) {
                th = T;
            } else {
                // first t with floor((t n + o) / T) >= B_h
                unsigned __int128 need = (unsigned __int128)g->info.B[h] * T;
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

}  // namespace

int rr_generate_stage(hyperim_graph g, const RRKey &key, uint64_t id_begin, uint64_t id_end, int form,
                      hipStream_t s, uint64_t *total) {
    RRWorkspace &ws = g->rr;
    const uint64_t count = id_end - id_begin;
    LaunchShape shape;
    HIM_CHECK(ensure_workspace(g, s, &shape));
    HIM_CHECK(ws.stage_off.reserve(sizeof(uint64_t) * std::max<uint64_t>(count, 1), s, false));
    HIM_CHECK(ws.sizes.reserve(sizeof(uint32_t) * std::max<uint64_t>(count, 1), s, false));
    HIM_CHECK(ws.roots.reserve(sizeof(uint32_t) * std::max<uint64_t>(count, 1), s, false));
    HIM_CHECK(ws.big_ids.reserve(sizeof(uint64_t) * std::max<uint64_t>(count, 1), s, false));  // big ids
    if (ws.stage.bytes < sizeof(uint32_t) * 4 * count)
        HIM_CHECK(ws.stage.reserve(sizeof(uint32_t) * std::max<uint64_t>(4 * count, 1 << 20), s, false));

    std::vector<std::pair<uint64_t, uint64_t>> ranges;
    if (form == 1) stratum_ranges(g, key, id_begin, id_end, &ranges);
    else ranges.push_back({id_begin, id_end});

    unsigned long long *ctr = ws.counters.as<unsigned long long>();
    while (ws.events.size() < 2 * ranges.size()) {
        hipEvent_t e;
        HIM_HIP(hipEventCreate(&e));
        ws.events.push_back(e);
    }
    for (int attempt = 0; attempt < 2; ++attempt) {
        HIM_HIP(hipMemsetAsync(ctr, 0, sizeof(unsigned long long) * 8, s));
        RRArgs a{};
        a.he_off = g->he_off.as<uint32_t>();
        a.he_mem = g->he_mem.as<uint32_t>();
        a.v_off = g->v_off.as<uint32_t>();
        a.v_he = g->v_he.as<uint32_t>();
        a.thr = g->thr.as<uint32_t>();
        a.P = g->P.as<uint32_t>();
        a.n = g->n;
        a.key0 = (uint32_t)key.seed;
        a.key1 = key.instance;
        a.pool = key.pool;
        a.qlog = key.qlog;
        a.bm_words = (g->n + 31u) / 32u;
        a.prefilter = 1;
        a.stage_bump = ctr + 1;
        a.big_count = ctr + 2;
        a.lists = ws.lists.as<uint32_t>();
        a.bitmaps = ws.bitmaps.as<uint32_t>();
        a.stage = ws.stage.as<uint32_t>();
        a.stage_cap = ws.stage.bytes / sizeof(uint32_t);
        a.stage_off = ws.stage_off.as<uint64_t>();
        a.sizes = ws.sizes.as<uint32_t>();
        a.roots = ws.roots.as<uint32_t>();
        a.big_ids = ws.big_ids.as<uint64_t>();
        for (size_t r = 0; r < ranges.size(); ++r) {
            a.id_begin = ranges[r].first;
            a.count = ranges[r].second - ranges[r].first;
            a.out_base = ranges[r].first - id_begin;
            a.work = ctr + 3 + (r & 1);
            if (r >= 1) HIM_HIP(hipMemsetAsync(a.work, 0, sizeof(unsigned long long), s));
            uint32_t grid = shape.grid;
            if (form == 1) grid = (uint32_t)std::min<uint64_t>(grid, div_up(a.count, kWavesPerWG));
            HIM_HIP(hipEventRecord(ws.events[2 * r], s));
            if (shape.lds)
                hipLaunchKernelGGL(k_rr_bfs<true>, dim3(grid), dim3(kWG), 0, s, a);
            else
                hipLaunchKernelGGL(k_rr_bfs<false>, dim3(grid), dim3(kWG), 0, s, a);
            HIM_HIP(hipGetLastError());
            HIM_HIP(hipEventRecord(ws.events[2 * r + 1], s));
        }
        unsigned long long bump = 0;
        HIM_HIP(hipMemcpyAsync(&bump, ctr + 1, sizeof(bump), hipMemcpyDeviceToHost, s));
        HIM_HIP(hipStreamSynchronize(s));
        for (size_t r = 0; r < ranges.size(); ++r) {
            float ms = 0.f;
            HIM_HIP(hipEventElapsedTime(&ms, ws.events[2 * r], ws.events[2 * r + 1]));
            ws.ms_bfs += ms;
            ws.launches += 1;
        }
        if (bump <= ws.stage.bytes / sizeof(uint32_t)) {
            *total = bump;
            return HYPERIM_OK;
        }
        HIM_CHECK(ws.stage.reserve(sizeof(uint32_t) * (size_t)(bump + bump / 4 + 1024), s, false));
    }
    set_error_detail("RR stage overflow after resize");
    return HYPERIM_ENOMEM;
}

int rr_compact_into(hyperim_graph g, hyperim_pool p, uint64_t count, hipStream_t s) {
    RRWorkspace &ws = g->rr;
    uint64_t *dst_off = p->off + p->count;
    HIM_CHECK(scan_u32_to_u64(ws.sizes.as<uint32_t>(), dst_off, count, p->total, ws.scan_tmp, s));
    if (count) {
        HIM_HIP(hipMemcpyAsync(p->roots + p->count, ws.roots.ptr, sizeof(uint32_t) * count,
                               hipMemcpyDeviceToDevice, s));
        const uint32_t grid = (uint32_t)std::min<uint64_t>(div_up(count, kWave * kWavesPerWG), 65535u);
        hipLaunchKernelGGL(k_move_small, dim3(std::max<uint32_t>(grid, 1)), dim3(kWG), 0, s,
                           ws.stage_off.as<uint64_t>(), ws.sizes.as<uint32_t>(), dst_off, count,
                           ws.stage.as<uint32_t>(), p->mem);
        hipLaunchKernelGGL(k_move_big, dim3(1024), dim3(kWG), 0, s, ws.big_ids.as<uint64_t>(),
                           ws.counters.as<unsigned long long>() + 2, ws.stage_off.as<uint64_t>(),
                           ws.sizes.as<uint32_t>(), dst_off, ws.stage.as<uint32_t>(), p->mem);
        HIM_HIP(hipGetLastError());
    }
    return HYPERIM_OK;
}

int rr_incidences(hyperim_graph g, hyperim_pool p, uint64_t theta, hipStream_t s, uint64_t *incidences,
                  uint64_t *alg_bytes) {
    uint64_t entries = 0;
    HIM_HIP(hipMemcpyAsync(&entries, p->off + theta, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    DevBuf acc;
    HIM_CHECK(acc.reserve(2 * sizeof(unsigned long long), s));
    HIM_HIP(hipMemsetAsync(acc.ptr, 0, 2 * sizeof(unsigned long long), s));
    if (entries) {
        const uint32_t grid = (uint32_t)std::min<uint64_t>(div_up(entries, kWG), 4096);
        hipLaunchKernelGGL(k_weight_sum, dim3(grid), dim3(kWG), 0, s, p->mem, entries,
                           g->weight.as<unsigned long long>(), g->bytesw.as<unsigned long long>(),
                           acc.as<unsigned long long>());
    }
    unsigned long long v[2] = {0, 0};
    HIM_HIP(hipMemcpyAsync(v, acc.ptr, sizeof(v), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    acc.release();
    *incidences = v[0];
    *alg_bytes = v[1];
    return HYPERIM_OK;
}

}  // namespace hyperim
