// Greedy max coverage over an RR-set pool (Algorithm 1 with the marginal
// coverage of Equation (2)) and the coverage count Lambda_R(S) of a seed set
// (Equation (1)'s estimator numerator).
//
// Coverage counts cnt[v] start as the number of sets containing v; an
// inverted index (counting sort by vertex) lists the sets of each vertex.
// Each round takes the argmax of the key (cnt+1, -v) over unchosen vertices
// -- largest marginal coverage, ties to the smallest id -- with a device-wide
// 64-bit max, then invalidates: every not-yet-covered set of the seed is
// marked covered and each of its members loses one count.  Every set is
// invalidated at most once, so all rounds together touch each pool entry at
// most once.  Each round is two kernels, the argmax and the invalidation; in
// the latter small sets are processed by wavefronts flattened over 64 sets,
// and sets above kBigSet members in chunks spread over the whole grid.  With
// Equation (8)'s bound the argmax pass also builds the first level of the
// prefix's top-k histogram (one more pass per further level).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "dev_common.h"
#include "internal.h"

namespace hyperim {
namespace {

constexpr int kWG = 256;
constexpr int kWavesPerWG = kWG / kWave;
constexpr uint32_t kBigSet = 4096;

__global__ void k_hist(const uint32_t *__restrict__ mem, uint64_t entries, uint32_t *__restrict__ cnt) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < entries;
         e += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[mem[e]], 1u);
}

__global__ void k_big_list(const uint64_t *__restrict__ off, uint64_t theta, uint64_t *__restrict__ list,
                           unsigned long long *__restrict__ count) {
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < theta;
         j += (uint64_t)gridDim.x * blockDim.x)
        if (off[j + 1] - off[j] > kBigSet) list[atomicAdd(count, 1ull)] = j;
}

// Per wave: 64 lane-owned segments mem[beg_k, beg_k + len_k), flattened.
struct FlatLds {
    uint32_t scan[kWave];
    uint64_t beg[kWave];
    uint64_t tag[kWave];
};

template <typename F>
__device__ __forceinline__ void wave_flat(FlatLds &L, uint32_t len, uint64_t beg, uint64_t tag, F &&body) {
    const uint32_t lane = lane_id();
    const uint32_t incl = wave_incl_scan(len);
    const uint32_t total = wave_bcast(incl, kWave - 1);
    wave_sync();
    L.scan[lane] = incl;
    L.beg[lane] = beg;
    L.tag[lane] = tag;
    wave_sync();
    for (uint32_t base = 0; base < total; base += kWave) {
        const uint32_t g = base + lane;
        if (g < total) {
            const uint32_t k = search64(L.scan, g);
            const uint32_t e = g - (k ? L.scan[k - 1] : 0u);
            body(k, L.beg[k] + e, L.tag[k]);
        }
    }
    wave_sync();
}

__global__ __launch_bounds__(kWG) void k_inv_small(const uint64_t *__restrict__ off, const uint32_t *__restrict__ mem,
                                                    uint64_t theta, const uint64_t *__restrict__ inv_off,
                                                    uint32_t *__restrict__ cursor, uint32_t *__restrict__ inv) {
    __shared__ FlatLds lds[kWavesPerWG];
    const uint32_t wv = threadIdx.x / kWave;
    const uint64_t waves = (uint64_t)gridDim.x * kWavesPerWG;
    for (uint64_t grp = (uint64_t)blockIdx.x * kWavesPerWG + wv; grp * kWave < theta; grp += waves) {
        const uint64_t j = grp * kWave + lane_id();
        uint32_t len = 0;
        uint64_t beg = 0;
        if (j < theta) {
            beg = off[j];
            const uint64_t sz = off[j + 1] - beg;
            len = sz > kBigSet ? 0u : (uint32_t)sz;
        }
        wave_flat(lds[wv], len, beg, j, [&](uint32_t, uint64_t e, uint64_t set) {
            const uint32_t u = mem[e];
            const uint32_t pos = atomicAdd(&cursor[u], 1u);
            inv[inv_off[u] + pos] = (uint32_t)set;
        });
    }
}

__global__ __launch_bounds__(kWG) void k_inv_big(const uint64_t *__restrict__ off, const uint32_t *__restrict__ mem,
                                                  const uint64_t *__restrict__ list,
                                                  const unsigned long long *__restrict__ count,
                                                  const uint64_t *__restrict__ inv_off, uint32_t *__restrict__ cursor,
                                                  uint32_t *__restrict__ inv) {
    // big sets fill each vertex's list from its end, so the list is the small
    // sets (the first cursor_small[u] entries) then the big ones
    const uint64_t nb = *count;
    for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const uint64_t j = list[b];
        for (uint64_t e = off[j] + threadIdx.x; e < off[j + 1]; e += blockDim.x) {
            const uint32_t u = mem[e];
            const uint32_t pos = atomicAdd(&cursor[u], 1u);
            inv[inv_off[u + 1] - 1u - pos] = (uint32_t)j;
        }
    }
}

// Arguments of the per-round kernels, in device memory so that one captured
// graph of all k rounds serves every pool and theta.
struct GreedyParams {
    const uint64_t *off;
    const uint32_t *mem;
    const uint64_t *inv_off;
    const uint32_t *inv;
    const uint32_t *nsmall;          // per vertex: small sets at the front of its list
    uint32_t *covered;               // per set: 0, or the round that covered it, plus one
    uint32_t *cnt;
    uint8_t *chosen;
    uint32_t *seeds;
    unsigned long long *gains;
    unsigned long long *best;        // k argmax keys
    uint32_t n;
    // Equation (8): before each round (and after the last) the sum of the k
    // largest counts, exact, selected by value-range histograms of kTkBins
    // bins over up to three levels of the counts' bits
    uint32_t *tk_cnt;                // kTkBins bin counts
    unsigned long long *tk_sum;      // kTkBins bin sums
    unsigned long long *tk_state;    // selected prefix, remaining count, sum so far
    unsigned long long *ub;          // k + 1 top-k sums, one per greedy prefix
    uint32_t *tk_done;               // workgroups that added their histogram (zero between passes)
    uint32_t k, tk_levels, tk_shift[3];
};

constexpr uint32_t kTkBins = 4096;
constexpr uint32_t kTkBits = 12;   // log2 kTkBins
static_assert(kTkBins == 1u << kTkBits, "bins");

// Equation (8)'s term for one greedy prefix: the sum of the k largest
// counts, by value-range histograms over the counts' bits.  At `level` a
// count x whose higher bits equal the prefix selected so far goes to bin
// (x >> tk_shift[level]) & (kTkBins - 1) (counts and sums).  Each workgroup
// builds its histogram in LDS and adds it to the global one; the workgroup
// that finishes last selects the bin holding the k-th largest count.

// Adds x (when `in`) to the LDS histogram; every lane of the wave calls it.
// Most counts fall into bin 0, which the wave adds up before one update.
__device__ __forceinline__ void tk_add(uint32_t *hc, unsigned long long *hs, uint32_t x, bool in, uint32_t shift) {
    const uint32_t bin = (x >> shift) & (kTkBins - 1u);
    const bool zero = in && bin == 0u;
    const uint64_t zb = __ballot(zero);
    const unsigned long long zs = wave_sum(zero ? (unsigned long long)x : 0ull);
    if (lane_id() == 0 && zb) {
        atomicAdd(&hc[0], (uint32_t)__popcll(zb));
        atomicAdd(&hs[0], zs);
    }
    if (in && bin != 0u) {
        atomicAdd(&hc[bin], 1u);
        atomicAdd(&hs[bin], (unsigned long long)x);
    }
}

// The whole (last) workgroup, after every workgroup's histogram is in: the
// bin that holds the k-th largest count among those the histogram took; the
// bins above it are added to the sum.  Each thread loads kTkBins / kWG
// consecutive bins at once; a suffix scan of the per-thread totals over the
// workgroup finds the thread whose range holds the boundary, which walks
// its bins from the top.  At the last level the bin is one exact value and
// ub[round] is complete; otherwise the prefix, the remaining count and the
// sum go to tk_state for the next level.  The histogram and the workgroup
// counter are cleared for the next pass.
constexpr uint32_t kTkPerThread = kTkBins / kWG;
static_assert(kTkBins % kWG == 0, "bins per thread");
__device__ void tk_select(const GreedyParams *__restrict__ P, uint32_t level, uint32_t round) {
    __shared__ unsigned long long sc[kWG], ss[kWG];
    const uint32_t t = threadIdx.x, b0 = t * kTkPerThread;
    unsigned long long c[kTkPerThread], v[kTkPerThread];
    unsigned long long tc = 0, ts = 0;
#pragma unroll
    for (uint32_t j = 0; j < kTkPerThread; ++j) {
        c[j] = __hip_atomic_load(&P->tk_cnt[b0 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v[j] = __hip_atomic_load(&P->tk_sum[b0 + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        tc += c[j];
        ts += v[j];
    }
    sc[t] = tc;
    ss[t] = ts;
    __syncthreads();
    // suffix sums: sc[t] = counts of bins >= b0
    for (uint32_t d = 1; d < (uint32_t)kWG; d <<= 1) {
        const unsigned long long yc = t + d < (uint32_t)kWG ? sc[t + d] : 0ull;
        const unsigned long long ys = t + d < (uint32_t)kWG ? ss[t + d] : 0ull;
        __syncthreads();
        sc[t] += yc;
        ss[t] += ys;
        __syncthreads();
    }
    const unsigned long long need = level ? P->tk_state[1] : (unsigned long long)P->k;
    unsigned long long above = sc[t] - tc, above_sum = ss[t] - ts;
    if (above < need && sc[t] >= need) {   // exactly one thread: the boundary is in its range
        const unsigned long long acc0 = level ? P->tk_state[2] : 0ull;
        const unsigned long long prefix = level ? P->tk_state[0] : 0ull;
        uint32_t found = b0;
        for (int j = (int)kTkPerThread - 1; j >= 0; --j) {
            if (above + c[j] >= need) {
                found = b0 + (uint32_t)j;
                break;
            }
            above += c[j];
            above_sum += v[j];
        }
        const unsigned long long rest = need - above, acc = acc0 + above_sum;
        const uint32_t shift = P->tk_shift[level];
        const uint32_t pshift = level ? P->tk_shift[level - 1] : shift;
        const unsigned long long sel = level ? (prefix << (pshift - shift)) | found : (unsigned long long)found;
        if (level + 1 == P->tk_levels) {
            P->ub[round] = acc + rest * sel;   // shift 0: the bin is the value itself
        } else {
            P->tk_state[0] = sel;
            P->tk_state[1] = rest;
            P->tk_state[2] = acc;
        }
    }
#pragma unroll
    for (uint32_t j = 0; j < kTkPerThread; ++j) {
        P->tk_cnt[b0 + j] = 0u;
        P->tk_sum[b0 + j] = 0ull;
    }
    if (t == 0) *P->tk_done = 0u;
}

// Adds the workgroup's LDS histogram to the global one; the workgroup that
// adds last (a device-scope counter, each workgroup's atomics fenced before
// its increment) runs tk_select.
__device__ void tk_flush(const GreedyParams *__restrict__ P, const uint32_t *hc, const unsigned long long *hs,
                         uint32_t level, uint32_t round) {
    __shared__ uint32_t last;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kTkBins; i += kWG)
        if (hc[i]) {
            atomicAdd(&P->tk_cnt[i], hc[i]);
            atomicAdd(&P->tk_sum[i], hs[i]);
        }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(P->tk_done, 1u) == gridDim.x - 1u ? 1u : 0u;
    __syncthreads();
    if (!last) return;
    __threadfence();
    tk_select(P, level, round);
}

__device__ __forceinline__ void tk_clear(uint32_t *hc, unsigned long long *hs) {
    for (uint32_t i = threadIdx.x; i < kTkBins; i += kWG) {
        hc[i] = 0u;
        hs[i] = 0ull;
    }
    __syncthreads();
}

// Level `level` > 0 of a prefix's top-k selection (level 0 runs inside
// k_argmax): the counts whose higher bits equal the prefix selected so far.
__global__ __launch_bounds__(kWG) void k_topk_hist(const GreedyParams *__restrict__ P, uint32_t level,
                                                   uint32_t round) {
    __shared__ uint32_t hc[kTkBins];
    __shared__ unsigned long long hs[kTkBins];
    tk_clear(hc, hs);
    const uint32_t n = P->n, shift = P->tk_shift[level], pshift = P->tk_shift[level - 1];
    const unsigned long long prefix = P->tk_state[0];
    for (uint64_t base = (uint64_t)blockIdx.x * kWG; base < n; base += (uint64_t)gridDim.x * kWG) {
        const uint64_t v = base + threadIdx.x;
        const uint32_t x = v < n ? P->cnt[v] : 0u;
        tk_add(hc, hs, x, v < n && (unsigned long long)(x >> pshift) == prefix, shift);
    }
    tk_flush(P, hc, hs, level, round);
}

// key = 0 for chosen vertices, else (cnt + 1) << 32 | (~v): the max is the
// largest count, then the smallest id.
__device__ __forceinline__ unsigned long long argmax_key(uint32_t c, uint8_t chosen, uint32_t v) {
    return chosen ? 0ull : (((unsigned long long)c + 1ull) << 32) | (unsigned long long)(0xFFFFFFFFu - v);
}

// Round `round`'s argmax (when `argmax` is set; the pass after the last
// round only takes the histogram) and, with kHist, level 0 of the prefix's
// top-k histogram over the same counts.  Each thread reads the counts and
// chosen flags of 4 consecutive vertices at a time (cnt and chosen are
// 256-byte aligned; the last quad may be partial); one atomic max per
// workgroup.
template <bool kHist>
__global__ __launch_bounds__(kWG) void k_argmax(const GreedyParams *__restrict__ P, uint32_t round,
                                                uint32_t argmax) {
    __shared__ unsigned long long part[kWavesPerWG];
    __shared__ uint32_t hc[kHist ? kTkBins : 1];
    __shared__ unsigned long long hs[kHist ? kTkBins : 1];
    if (kHist) tk_clear(hc, hs);
    const uint32_t n = P->n;
    const uint32_t shift = kHist ? P->tk_shift[0] : 0u;
    const uint4 *__restrict__ cnt4 = reinterpret_cast<const uint4 *>(P->cnt);
    const uchar4 *__restrict__ chosen4 = reinterpret_cast<const uchar4 *>(P->chosen);
    const uint32_t n4 = n / 4, nq = (n + 3u) / 4u, stride = gridDim.x * kWG;
    unsigned long long m = 0;
    // block-uniform trip count: every lane reaches the wave operations of tk_add
    for (uint32_t q0 = blockIdx.x * kWG; q0 < nq; q0 += stride) {
        const uint32_t q = q0 + threadIdx.x, v = 4 * q;
        uint32_t c[4] = {0u, 0u, 0u, 0u};
        uint8_t ch[4] = {1, 1, 1, 1};
        bool in[4] = {false, false, false, false};
        if (q < n4) {
            const uint4 cq = cnt4[q];
            const uchar4 hq = chosen4[q];
            c[0] = cq.x; c[1] = cq.y; c[2] = cq.z; c[3] = cq.w;
            ch[0] = hq.x; ch[1] = hq.y; ch[2] = hq.z; ch[3] = hq.w;
            in[0] = in[1] = in[2] = in[3] = true;
        } else if (q < nq) {
            for (uint32_t i = 0; i < 4; ++i)
                if (v + i < n) {
                    c[i] = P->cnt[v + i];
                    ch[i] = P->chosen[v + i];
                    in[i] = true;
                }
        }
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) {
            if (in[i]) {
                const unsigned long long key = argmax_key(c[i], ch[i], v + i);
                m = key > m ? key : m;
            }
            if (kHist) tk_add(hc, hs, c[i], in[i], shift);
        }
    }
    if (argmax) {
        m = wave_max(m);
        if (lane_id() == 0) part[threadIdx.x / kWave] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < kWavesPerWG; ++w) m = part[w] > m ? part[w] : m;
            m = part[0] > m ? part[0] : m;
            atomicMax(P->best + round, m);
        }
    }
    if (kHist) tk_flush(P, hc, hs, 0u, round);
}

// Members of a big set per work chunk in the invalidation.
constexpr uint32_t kBigChunk = 1024;

// Round `round`: record the argmax seed s, then invalidate every set of s
// not covered before this round.  Small sets (the front of s's list) go one
// per lane, flattened over the wave; big sets are cut into chunks of
// kBigChunk members spread over every wave of the grid.  A big set's chunks
// agree that it is new in this round through its stamp: covered[j] is 0 or
// round + 1 (set by the first chunk to look) for a set covered now, an older
// round otherwise.
__global__ __launch_bounds__(kWG) void k_invalidate(const GreedyParams *__restrict__ P, uint32_t round) {
    __shared__ FlatLds lds[kWavesPerWG];
    __shared__ uint32_t csum[kWavesPerWG][kWave];
    const unsigned long long key = P->best[round];
    const uint32_t s = 0xFFFFFFFFu - (uint32_t)key;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        P->seeds[round] = s;
        P->gains[round] = (key >> 32) - 1ull;
        P->chosen[s] = 1;
    }
    const uint64_t *__restrict__ off = P->off;
    const uint32_t *__restrict__ mem = P->mem;
    const uint32_t *__restrict__ inv = P->inv;
    uint32_t *__restrict__ covered = P->covered;
    uint32_t *__restrict__ cnt = P->cnt;
    const uint32_t stamp = round + 1u;
    const uint64_t x0 = P->inv_off[s], xs = x0 + P->nsmall[s], x1 = P->inv_off[s + 1];
    const uint32_t wv = threadIdx.x / kWave, lane = lane_id();
    const uint64_t gw = (uint64_t)blockIdx.x * kWavesPerWG + wv, waves = (uint64_t)gridDim.x * kWavesPerWG;
    // small sets: each appears once in s's list, so its lane owns it
    for (uint64_t grp = gw; x0 + grp * kWave < xs; grp += waves) {
        const uint64_t x = x0 + grp * kWave + lane;
        uint32_t len = 0;
        uint64_t beg = 0;
        if (x < xs) {
            const uint32_t j = inv[x];
            if (covered[j] == 0u) {
                covered[j] = stamp;
                beg = off[j];
                len = (uint32_t)(off[j + 1] - beg);
            }
        }
        wave_flat(lds[wv], len, beg, 0, [&](uint32_t, uint64_t e, uint64_t) { atomicSub(&cnt[mem[e]], 1u); });
    }
    // big sets, 64 at a time: every wave numbers their chunks the same way
    // and takes the chunks c with c = gw (mod waves)
    uint64_t run = 0;   // chunks of earlier batches
    for (uint64_t b0 = xs; b0 < x1; b0 += kWave) {
        const uint64_t x = b0 + lane;
        uint32_t nc = 0, j = 0;
        if (x < x1) {
            j = inv[x];
            const uint32_t c = __hip_atomic_load(&covered[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (c == 0u || c == stamp) nc = (uint32_t)div_up(off[j + 1] - off[j], kBigChunk);
        }
        const uint32_t incl = wave_incl_scan(nc);
        const uint32_t total = wave_bcast(incl, kWave - 1);
        wave_sync();
        csum[wv][lane] = incl;
        wave_sync();
        // first chunk index >= run owned by this wave
        uint64_t c = run + ((gw + waves - run % waves) % waves);
        for (; c < run + total; c += waves) {
            const uint32_t r = (uint32_t)(c - run);
            const uint32_t k = search64(csum[wv], r);
            const uint32_t first = k ? csum[wv][k - 1] : 0u;
            const uint32_t jk = (uint32_t)__shfl((int)j, (int)k, kWave);
            if (lane == 0) {
                const uint32_t old = atomicCAS(&covered[jk], 0u, stamp);
                (void)old;   // 0 or stamp: this chunk's set is new in this round
            }
            const uint64_t b = off[jk] + (uint64_t)(r - first) * kBigChunk;
            const uint64_t e1 = min(b + kBigChunk, off[jk + 1]);
            for (uint64_t e = b + lane; e < e1; e += kWave) atomicSub(&cnt[mem[e]], 1u);
        }
        run += total;
        wave_sync();
    }
}

// Seed flags; ids >= n are ignored.
__global__ void k_mark(const uint32_t *__restrict__ seeds, uint32_t k, uint32_t n, uint8_t *__restrict__ flags) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k && seeds[i] < n) flags[seeds[i]] = 1;
}

__global__ __launch_bounds__(kWG) void k_hits_small(const uint64_t *__restrict__ off, const uint32_t *__restrict__ mem,
                                                     uint64_t theta, const uint8_t *__restrict__ flags,
                                                     unsigned long long *__restrict__ hits) {
    __shared__ FlatLds lds[kWavesPerWG];
    __shared__ uint32_t hit[kWavesPerWG][kWave];
    const uint32_t wv = threadIdx.x / kWave, lane = lane_id();
    const uint64_t waves = (uint64_t)gridDim.x * kWavesPerWG;
    for (uint64_t grp = (uint64_t)blockIdx.x * kWavesPerWG + wv; grp * kWave < theta; grp += waves) {
        const uint64_t j = grp * kWave + lane;
        uint32_t len = 0;
        uint64_t beg = 0;
        if (j < theta) {
            beg = off[j];
            const uint64_t sz = off[j + 1] - beg;
            len = sz > kBigSet ? 0u : (uint32_t)sz;
        }
        hit[wv][lane] = 0;
        wave_flat(lds[wv], len, beg, 0, [&](uint32_t k, uint64_t e, uint64_t) {
            if (flags[mem[e]]) hit[wv][k] = 1;
        });
        const uint64_t bal = __ballot(hit[wv][lane] != 0);
        if (lane == 0 && bal) atomicAdd(hits, (unsigned long long)__popcll(bal));
        wave_sync();
    }
}

__global__ __launch_bounds__(kWG) void k_hits_big(const uint64_t *__restrict__ list,
                                                   const unsigned long long *__restrict__ count,
                                                   const uint64_t *__restrict__ off, const uint32_t *__restrict__ mem,
                                                   const uint8_t *__restrict__ flags,
                                                   unsigned long long *__restrict__ hits) {
    __shared__ int any;
    const uint64_t nb = *count;
    for (uint64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const uint64_t j = list[b];
        if (threadIdx.x == 0) any = 0;
        __syncthreads();
        for (uint64_t e = off[j] + threadIdx.x; e < off[j + 1]; e += blockDim.x)
            if (flags[mem[e]]) any = 1;
        __syncthreads();
        if (threadIdx.x == 0 && any) atomicAdd(hits, 1ull);
        __syncthreads();
    }
}

uint32_t grid_for(uint64_t items, uint64_t per_block, uint32_t cap) {
    uint64_t g = div_up(items, per_block);
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, cap));
}

int read_entries(hyperim_pool p, uint64_t theta, hipStream_t s, uint64_t *entries) {
    HIM_HIP(hipMemcpyAsync(entries, p->off + theta, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    return HYPERIM_OK;
}

// big-set list of the pool prefix; counter at ctr
int big_list(hyperim_pool p, uint64_t theta, uint64_t *list, unsigned long long *ctr, hipStream_t s) {
    HIM_HIP(hipMemsetAsync(ctr, 0, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_big_list, dim3(grid_for(theta, kWG, 4096)), dim3(kWG), 0, s, p->off, theta, list, ctr);
    return HYPERIM_OK;
}

}  // namespace

int greedy_device(GreedyWorkspace &w, hyperim_graph g, hyperim_pool p, uint64_t theta, uint32_t k, hipStream_t s,
                  uint32_t *seeds_host, uint64_t *gains_host, uint64_t *ub_host) {
    const uint32_t n = g->n;
    uint64_t entries = 0;
    HIM_CHECK(read_entries(p, theta, s, &entries));
    HIM_CHECK(w.cnt.reserve(sizeof(uint32_t) * n, s));
    HIM_CHECK(w.inv_off.reserve(sizeof(uint64_t) * ((size_t)n + 1), s));
    HIM_CHECK(w.cursor.reserve(sizeof(uint32_t) * n, s));
    HIM_CHECK(w.inv.reserve(sizeof(uint32_t) * std::max<uint64_t>(entries, 1), s));
    HIM_CHECK(w.covered.reserve(sizeof(uint32_t) * std::max<uint64_t>(theta, 1), s));
    HIM_CHECK(w.chosen.reserve(n, s));
    HIM_CHECK(w.best.reserve(sizeof(unsigned long long) * ((size_t)k + 1), s));
    HIM_CHECK(w.out.reserve(sizeof(uint32_t) * k + sizeof(uint64_t) * k, s));
    HIM_CHECK(w.big.reserve(sizeof(uint64_t) * std::max<uint64_t>(theta, 1), s));
    HIM_CHECK(w.cursor_big.reserve(sizeof(uint32_t) * n, s));
    unsigned long long *best = w.best.as<unsigned long long>();
    unsigned long long *nbig_all = best + k;   // big sets of the pool prefix
    uint32_t *seeds = w.out.as<uint32_t>();
    unsigned long long *gains = reinterpret_cast<unsigned long long *>(w.out.as<char>() + sizeof(uint32_t) * k);
    HIM_HIP(hipMemsetAsync(w.cnt.ptr, 0, sizeof(uint32_t) * n, s));
    HIM_HIP(hipMemsetAsync(w.cursor.ptr, 0, sizeof(uint32_t) * n, s));
    HIM_HIP(hipMemsetAsync(w.covered.ptr, 0, sizeof(uint32_t) * std::max<uint64_t>(theta, 1), s));
    HIM_HIP(hipMemsetAsync(w.cursor_big.ptr, 0, sizeof(uint32_t) * n, s));
    HIM_HIP(hipMemsetAsync(w.chosen.ptr, 0, n, s));
    HIM_HIP(hipMemsetAsync(best, 0, sizeof(unsigned long long) * ((size_t)k + 1), s));

    if (entries)
        hipLaunchKernelGGL(k_hist, dim3(grid_for(entries, kWG, 8192)), dim3(kWG), 0, s, p->mem, entries,
                           w.cnt.as<uint32_t>());
    HIM_CHECK(scan_u32_to_u64(w.cnt.as<uint32_t>(), w.inv_off.as<uint64_t>(), n, 0, w.scan_tmp, s));
    HIM_CHECK(big_list(p, theta, w.big.as<uint64_t>(), nbig_all, s));
    if (theta) {
        hipLaunchKernelGGL(k_inv_small, dim3(grid_for(theta, kWG, 8192)), dim3(kWG), 0, s, p->off, p->mem, theta,
                           w.inv_off.as<uint64_t>(), w.cursor.as<uint32_t>(), w.inv.as<uint32_t>());
        hipLaunchKernelGGL(k_inv_big, dim3(1024), dim3(kWG), 0, s, p->off, p->mem, w.big.as<uint64_t>(), nbig_all,
                           w.inv_off.as<uint64_t>(), w.cursor_big.as<uint32_t>(), w.inv.as<uint32_t>());
    }
    // the k rounds: one captured graph per (k, argmax grid), replayed with
    // this call's arguments in the device parameter block; the invalidation
    // grid is fixed (grid-stride over a seed's sets) so theta does not change
    // the graph
    const uint32_t argmax_grid = grid_for(n, 4 * 2 * kWG, 1024);   // two quads of vertices per thread
    const uint32_t inval_grid = 256;
    GreedyParams hp{};   // the top-k fields are set below
    hp.off = p->off;
    hp.mem = p->mem;
    hp.inv_off = w.inv_off.as<uint64_t>();
    hp.inv = w.inv.as<uint32_t>();
    hp.nsmall = w.cursor.as<uint32_t>();
    hp.covered = w.covered.as<uint32_t>();
    hp.cnt = w.cnt.as<uint32_t>();
    hp.chosen = w.chosen.as<uint8_t>();
    hp.seeds = seeds;
    hp.gains = gains;
    hp.best = best;
    hp.n = n;
    // Equation (8): levels of kTkBins-bin histograms over the counts' bits
    // (every count is at most theta)
    uint32_t levels = 0;
    if (ub_host) {
        const uint32_t bits = theta ? 64u - (uint32_t)__builtin_clzll(theta) : 1u;
        levels = bits <= kTkBits ? 1u : bits <= 2 * kTkBits ? 2u : 3u;
        hp.tk_shift[0] = levels == 1 ? 0u : bits - kTkBits;
        hp.tk_shift[1] = levels == 2 ? 0u : bits - 2 * kTkBits;
        hp.tk_shift[2] = 0u;
        const size_t tk_bytes = kTkBins * (sizeof(uint32_t) + sizeof(unsigned long long)) +
                                3 * sizeof(unsigned long long) + sizeof(unsigned long long) * ((size_t)k + 1) +
                                sizeof(uint32_t);
        HIM_CHECK(w.topk.reserve(tk_bytes, s));
        hp.tk_sum = w.topk.as<unsigned long long>();
        hp.tk_state = hp.tk_sum + kTkBins;
        hp.ub = hp.tk_state + 3;
        hp.tk_cnt = reinterpret_cast<uint32_t *>(hp.ub + k + 1);
        hp.tk_done = hp.tk_cnt + kTkBins;
        HIM_HIP(hipMemsetAsync(w.topk.ptr, 0, tk_bytes, s));
    }
    hp.k = k;
    hp.tk_levels = levels;
    HIM_CHECK(w.params.reserve(sizeof(GreedyParams), s));
    static_assert(sizeof(GreedyParams) <= sizeof(w.params_host), "parameter block");
    memcpy(w.params_host, &hp, sizeof(hp));
    HIM_HIP(hipMemcpyAsync(w.params.ptr, w.params_host, sizeof(GreedyParams), hipMemcpyHostToDevice, s));
    const GreedyParams *P = w.params.as<GreedyParams>();
    const uint32_t hist_grid = grid_for(n, 4 * kWG, 1024);
    if (!w.rounds_exec || w.graph_k != k || w.graph_grid[0] != argmax_grid || w.graph_grid[1] != inval_grid ||
        w.graph_params != w.params.ptr || w.graph_levels != levels) {
        if (w.rounds_exec) HIM_HIP(hipGraphExecDestroy(w.rounds_exec));
        w.rounds_exec = nullptr;
        if (!w.capture) HIM_HIP(hipStreamCreateWithFlags(&w.capture, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        HIM_HIP(hipStreamBeginCapture(w.capture, hipStreamCaptureModeThreadLocal));
        for (uint32_t i = 0; i <= k; ++i) {
            // round i's argmax with level 0 of Equation (8)'s term for the
            // first i seeds, the term's further levels, then the invalidation
            // (after the last round, the term alone)
            if (levels) {
                hipLaunchKernelGGL(k_argmax<true>, dim3(argmax_grid), dim3(kWG), 0, w.capture, P, i, i < k ? 1u : 0u);
                for (uint32_t l = 1; l < levels; ++l)
                    hipLaunchKernelGGL(k_topk_hist, dim3(hist_grid), dim3(kWG), 0, w.capture, P, l, i);
            } else if (i < k) {
                hipLaunchKernelGGL(k_argmax<false>, dim3(argmax_grid), dim3(kWG), 0, w.capture, P, i, 1u);
            }
            if (i == k) break;
            hipLaunchKernelGGL(k_invalidate, dim3(inval_grid), dim3(kWG), 0, w.capture, P, i);
        }
        HIM_HIP(hipStreamEndCapture(w.capture, &graph));
        const hipError_t e = hipGraphInstantiate(&w.rounds_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIM_HIP(e);
        w.graph_k = k;
        w.graph_grid[0] = argmax_grid;
        w.graph_grid[1] = inval_grid;
        w.graph_params = w.params.ptr;
        w.graph_levels = levels;
    }
    HIM_HIP(hipGraphLaunch(w.rounds_exec, s));
    HIM_HIP(hipGetLastError());
    if (seeds_host) HIM_HIP(hipMemcpyAsync(seeds_host, seeds, sizeof(uint32_t) * k, hipMemcpyDeviceToHost, s));
    if (gains_host) HIM_HIP(hipMemcpyAsync(gains_host, gains, sizeof(uint64_t) * k, hipMemcpyDeviceToHost, s));
    if (ub_host)
        HIM_HIP(hipMemcpyAsync(ub_host, hp.ub, sizeof(uint64_t) * ((size_t)k + 1), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    return HYPERIM_OK;
}

int coverage_device(GreedyWorkspace &w, hyperim_graph g, hyperim_pool p, uint64_t theta, const uint32_t *seeds_dev,
                    uint32_t k, hipStream_t s, uint64_t *covered_host) {
    const uint32_t n = g->n;
    HIM_CHECK(w.flags.reserve(n, s));
    HIM_CHECK(w.big.reserve(sizeof(uint64_t) * std::max<uint64_t>(theta, 1), s));
    HIM_CHECK(w.counters.reserve(4 * sizeof(unsigned long long), s));
    unsigned long long *ctr = w.counters.as<unsigned long long>();
    HIM_HIP(hipMemsetAsync(w.flags.ptr, 0, n, s));
    HIM_HIP(hipMemsetAsync(ctr, 0, 4 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_mark, dim3(grid_for(k, kWG, 65535)), dim3(kWG), 0, s, seeds_dev, k, n,
                       w.flags.as<uint8_t>());
    HIM_CHECK(big_list(p, theta, w.big.as<uint64_t>(), ctr + 1, s));
    if (theta) {
        hipLaunchKernelGGL(k_hits_small, dim3(grid_for(theta, kWG, 8192)), dim3(kWG), 0, s, p->off, p->mem, theta,
                           w.flags.as<uint8_t>(), ctr);
        hipLaunchKernelGGL(k_hits_big, dim3(1024), dim3(kWG), 0, s, w.big.as<uint64_t>(), ctr + 1, p->off, p->mem,
                           w.flags.as<uint8_t>(), ctr);
    }
    HIM_HIP(hipGetLastError());
    unsigned long long h = 0;
    HIM_HIP(hipMemcpyAsync(&h, ctr, sizeof(h), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    *covered_host = h;
    return HYPERIM_OK;
}

// ---- coverage without allocation ---------------------------------------------
// Scratch of hyperim_coverage_noalloc: the hit counters, the seed flags (n
// bytes) and the list of big sets (8 bytes per set), in one static device
// array.  Each device holds its own copy; host code uses the address that
// hipGetSymbolAddress returns on that device, never the array's name.
constexpr size_t kScratchBytes = 32ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
unsigned char *g_scratch[kMaxDevices] = {};

// The device address of `scratch` on `device` (the current device), looked
// up once per device.
int scratch_address(int device, unsigned char **out) {
    if (device < 0 || device >= kMaxDevices) {
        set_error_detail("device index beyond the scratch table");
        return HYPERIM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (!g_scratch[device]) {
        void *p = nullptr;
        HIM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch[device] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch[device];
    return HYPERIM_OK;
}

__global__ void k_zero_words(unsigned long long *__restrict__ p, uint64_t words) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void k_store_count(const unsigned long long *__restrict__ src, uint64_t *__restrict__ dst) { *dst = *src; }

inline size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

}  // namespace hyperim

using namespace hyperim;

extern "C" int hyperim_coverage_noalloc(hyperim_graph g, hyperim_pool pool, uint64_t theta, const uint32_t *seeds_dev,
                                        uint32_t k, void *stream, uint64_t *covered_dev) {
    if (!g || !pool || pool->g != g || !covered_dev || (k && !seeds_dev)) return HYPERIM_EINVAL;
    HIM_CHECK(check_device(g));
    if (theta > pool->count || k > g->n) {
        set_error_detail("need theta <= pool size and k <= n");
        return HYPERIM_EINVAL;
    }
    // layout: counters (256 B), flags (n bytes, 256-aligned), big-set list
    const size_t flags_at = 256, list_at = flags_at + round256(g->n);
    if (list_at + 8 * theta > kScratchBytes) {
        set_error_detail("coverage without allocation needs n + 8 theta bytes within its 32 MiB scratch");
        return HYPERIM_ECAPACITY;
    }
    unsigned char *base = nullptr;
    HIM_CHECK(scratch_address(g->device, &base));
    hipStream_t s = as_stream(stream);
    unsigned long long *ctr = reinterpret_cast<unsigned long long *>(base);
    uint8_t *flags = base + flags_at;
    uint64_t *list = reinterpret_cast<uint64_t *>(base + list_at);
    const uint64_t words = list_at / 8;   // counters and flags start at zero
    hipLaunchKernelGGL(k_zero_words, dim3(grid_for(words, kWG, 4096)), dim3(kWG), 0, s, ctr, words);
    if (k) hipLaunchKernelGGL(k_mark, dim3(grid_for(k, kWG, 65535)), dim3(kWG), 0, s, seeds_dev, k, g->n, flags);
    if (theta) {
        hipLaunchKernelGGL(k_big_list, dim3(grid_for(theta, kWG, 4096)), dim3(kWG), 0, s, pool->off, theta, list,
                           ctr + 1);
        hipLaunchKernelGGL(k_hits_small, dim3(grid_for(theta, kWG, 8192)), dim3(kWG), 0, s, pool->off, pool->mem,
                           theta, flags, ctr);
        hipLaunchKernelGGL(k_hits_big, dim3(1024), dim3(kWG), 0, s, list, ctr + 1, pool->off, pool->mem, flags, ctr);
    }
    hipLaunchKernelGGL(k_store_count, dim3(1), dim3(1), 0, s, ctr, covered_dev);
    HIM_HIP(hipGetLastError());
    return HYPERIM_OK;
}
