// Sample-set division (Section 3.1.1) on the device.  For every vertex v the
// co-membership weight w(v,u) (hyperedges shared with u) is counted in a
// global open-addressing table keyed by (v,u); the layers of A(v) are the
// distinct w values, layer 1 the largest.  Per vertex this yields l_v (number
// of layers), deg(v) = |A(v)| and top(v) = n(L_1).  Strata are log2 buckets
// of l_v, and P lists the vertices by (stratum, id) for stratified roots.
// Vertices are processed in batches whose pair count fits the table budget,
// so memory stays bounded for graphs with billions of co-member pairs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "block_table.h"
#include "dev_common.h"
#include "internal.h"

namespace hyperim {
namespace {

constexpr int kBlock = 256;
constexpr uint64_t kEmpty = ~0ull;
constexpr uint64_t kPairBudget = 1ull << 27;   // co-member pairs per batch

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBull;
    x ^= x >> 31;
    return x;
}

// Count one occurrence of `key`.
__device__ __forceinline__ void table_count(unsigned long long *keys, uint32_t *vals, uint64_t mask,
                                            uint64_t key) {
    uint64_t h = mix64(key) & mask;
    for (;;) {
        unsigned long long k = keys[h];
        if (k == key) {
            atomicAdd(&vals[h], 1u);
            return;
        }
        if (k == kEmpty) {
            unsigned long long prev = atomicCAS(&keys[h], kEmpty, (unsigned long long)key);
            if (prev == kEmpty || prev == key) {
                atomicAdd(&vals[h], 1u);
                return;
            }
        }
        h = (h + 1) & mask;
    }
}

// Insert `key` into a set; true when it was not there before.
__device__ __forceinline__ bool table_insert(unsigned long long *keys, uint64_t mask, uint64_t key) {
    uint64_t h = mix64(key) & mask;
    for (;;) {
        unsigned long long k = keys[h];
        if (k == key) return false;
        if (k == kEmpty) {
            unsigned long long prev = atomicCAS(&keys[h], kEmpty, (unsigned long long)key);
            if (prev == kEmpty) return true;
            if (prev == key) return false;
        }
        h = (h + 1) & mask;
    }
}

// Every co-member occurrence (v, he, u != v) of the batch's vertices.  Each
// wavefront takes 64 consecutive incidences (v, he) and spreads their member
// positions over its lanes, so a large hyperedge is not one lane's serial
// loop.
__global__ __launch_bounds__(kBlock) void k_pairs(const uint32_t *__restrict__ he_off,
                                                   const uint32_t *__restrict__ he_mem,
                                                   const uint32_t *__restrict__ v_off,
                                                   const uint32_t *__restrict__ v_he, uint32_t v0, uint32_t v1,
                                                   unsigned long long *keys, uint32_t *vals, uint64_t mask) {
    __shared__ uint32_t scan_s[kBlock / kWave][kWave], hb_s[kBlock / kWave][kWave], v_s[kBlock / kWave][kWave];
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    const uint32_t e_begin = v_off[v0], e_end = v_off[v1];
    const uint64_t waves = (uint64_t)gridDim.x * (kBlock / kWave);
    for (uint64_t g0 = (uint64_t)e_begin + ((uint64_t)blockIdx.x * (kBlock / kWave) + wv) * kWave; g0 < e_end;
         g0 += waves * kWave) {
        const uint64_t e = g0 + lane;
        uint32_t v = 0, hb = 0, hs = 0;
        if (e < e_end) {
            uint32_t lo = v0, hi = v1;  // v_off[lo] <= e < v_off[hi]
            while (hi - lo > 1) {
                const uint32_t mid = lo + (hi - lo) / 2;
                if (v_off[mid] <= (uint32_t)e) lo = mid; else hi = mid;
            }
            v = lo;
            const uint32_t he = v_he[e];
            hb = he_off[he];
            hs = he_off[he + 1] - hb;
        }
        const uint32_t incl = wave_incl_scan(hs);
        const uint32_t total = wave_bcast(incl, kWave - 1);
        wave_sync();
        scan_s[wv][lane] = incl;
        hb_s[wv][lane] = hb;
        v_s[wv][lane] = v;
        wave_sync();
        for (uint32_t b = 0; b < total; b += kWave) {
            const uint32_t q = b + lane;
            if (q < total) {
                const uint32_t k = search64(scan_s[wv], q);
                const uint32_t first = k ? scan_s[wv][k - 1] : 0u;
                const uint32_t vk = v_s[wv][k];
                const uint32_t u = he_mem[hb_s[wv][k] + (q - first)];
                if (u != vk) table_count(keys, vals, mask, ((uint64_t)vk << 32) | u);
            }
        }
        wave_sync();
    }
}

// Per table entry (v, u) with weight w: deg(v) += 1, wmax(v) = max, and l(v)
// += 1 when (v, w) is a new layer weight.  Entries of one vertex are spread
// over the table, so each workgroup aggregates per-vertex updates of a chunk
// in LDS and applies them once (hubs have ~1e5 entries).
constexpr uint32_t kAggPer = 4;
constexpr uint32_t kAggChunk = kBlock * kAggPer;
constexpr uint32_t kAggSlots = 2048;

__global__ __launch_bounds__(kBlock) void k_layers(const unsigned long long *__restrict__ keys,
                                                    const uint32_t *__restrict__ vals, uint64_t cap,
                                                    unsigned long long *keys2, uint64_t mask2,
                                                    uint32_t *__restrict__ deg, uint32_t *__restrict__ wmax,
                                                    uint32_t *__restrict__ l) {
    __shared__ BlockTable<kAggSlots> tab;
    __shared__ uint32_t tdeg[kAggSlots], tmax[kAggSlots], tl[kAggSlots];
    tab.clear_keys();
    for (uint32_t s = threadIdx.x; s < kAggSlots; s += kBlock) tdeg[s] = tmax[s] = tl[s] = 0;
    __syncthreads();
    for (uint64_t base = (uint64_t)blockIdx.x * kAggChunk; base < cap; base += (uint64_t)gridDim.x * kAggChunk) {
        for (uint32_t r = 0; r < kAggPer; ++r) {
            const uint64_t i = base + r * kBlock + threadIdx.x;
            if (i >= cap) break;
            const unsigned long long k = keys[i];
            if (k == kEmpty) continue;
            const uint32_t v = (uint32_t)(k >> 32), w = vals[i];
            const bool fresh = table_insert(keys2, mask2, ((uint64_t)v << 32) | w);
            const uint32_t sl = tab.slot(v);
            if (sl != kTableEmpty) {
                atomicAdd(&tdeg[sl], 1u);
                atomicMax(&tmax[sl], w);
                if (fresh) atomicAdd(&tl[sl], 1u);
            } else {
                atomicAdd(&deg[v], 1u);
                atomicMax(&wmax[v], w);
                if (fresh) atomicAdd(&l[v], 1u);
            }
        }
        __syncthreads();
        for (uint32_t s = threadIdx.x; s < kAggSlots; s += kBlock) {
            const uint32_t v = tab.key[s];
            if (v != kTableEmpty) {
                atomicAdd(&deg[v], tdeg[s]);
                atomicMax(&wmax[v], tmax[s]);
                if (tl[s]) atomicAdd(&l[v], tl[s]);
                tab.key[s] = kTableEmpty;
                tdeg[s] = tmax[s] = tl[s] = 0;
            }
        }
        __syncthreads();
    }
}

// top(v) = entries of v with the largest weight, aggregated the same way.
__global__ __launch_bounds__(kBlock) void k_top(const unsigned long long *__restrict__ keys,
                                                 const uint32_t *__restrict__ vals, uint64_t cap,
                                                 const uint32_t *__restrict__ wmax, uint32_t *__restrict__ top) {
    __shared__ BlockTable<kAggSlots> tab;
    __shared__ uint32_t tcnt[kAggSlots];
    tab.clear_keys();
    for (uint32_t s = threadIdx.x; s < kAggSlots; s += kBlock) tcnt[s] = 0;
    __syncthreads();
    for (uint64_t base = (uint64_t)blockIdx.x * kAggChunk; base < cap; base += (uint64_t)gridDim.x * kAggChunk) {
        for (uint32_t r = 0; r < kAggPer; ++r) {
            const uint64_t i = base + r * kBlock + threadIdx.x;
            if (i >= cap) break;
            const unsigned long long k = keys[i];
            if (k == kEmpty) continue;
            const uint32_t v = (uint32_t)(k >> 32);
            if (vals[i] != wmax[v]) continue;
            const uint32_t sl = tab.slot(v);
            if (sl != kTableEmpty) atomicAdd(&tcnt[sl], 1u);
            else atomicAdd(&top[v], 1u);
        }
        __syncthreads();
        for (uint32_t s = threadIdx.x; s < kAggSlots; s += kBlock) {
            const uint32_t v = tab.key[s];
            if (v != kTableEmpty) {
                atomicAdd(&top[v], tcnt[s]);
                tab.key[s] = kTableEmpty;
                tcnt[s] = 0;
            }
        }
        __syncthreads();
    }
}

// Stratum of each vertex, per-tile stratum counts (stratum-major layout),
// per-tile integer sums and the largest l_v.
__global__ __launch_bounds__(kBlock) void k_strata(uint32_t n, const uint32_t *__restrict__ l,
                                                    const uint32_t *__restrict__ deg, const uint32_t *__restrict__ top,
                                                    uint8_t *__restrict__ stratum, uint32_t *__restrict__ counts,
                                                    uint32_t tiles, unsigned long long *__restrict__ isums,
                                                    uint32_t *__restrict__ lmax) {
    __shared__ uint32_t cnt[kNStrata];
    __shared__ unsigned long long ps[3][kBlock / kWave];
    if (threadIdx.x < kNStrata) cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    uint64_t a = 0, b = 0, c = 0;
    if (v < n) {
        const uint32_t lv = l[v];
        uint32_t s = lv ? 32u - __clz(lv) : 0u;   // 1 + floor(log2 l_v)
        s = s < kNStrata - 1 ? s : kNStrata - 1;
        stratum[v] = (uint8_t)s;
        atomicAdd(&cnt[s], 1u);
        atomicMax(lmax, lv);
        a = top[v];
        b = deg[v];
        c = lv;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    if (lane == 0) {
        ps[0][wv] = a;
        ps[1][wv] = b;
        ps[2][wv] = c;
    }
    __syncthreads();
    if (threadIdx.x < kNStrata) counts[(uint64_t)threadIdx.x * tiles + blockIdx.x] = cnt[threadIdx.x];
    if (threadIdx.x == 0) {
        unsigned long long s0 = 0, s1 = 0, s2 = 0;
        for (int w = 0; w < kBlock / kWave; ++w) {
            s0 += ps[0][w];
            s1 += ps[1][w];
            s2 += ps[2][w];
        }
        isums[3 * (uint64_t)blockIdx.x + 0] = s0;
        isums[3 * (uint64_t)blockIdx.x + 1] = s1;
        isums[3 * (uint64_t)blockIdx.x + 2] = s2;
    }
}

// Histogram of the layer counts (Theorem 2's theta(l*) is a sum over it):
// counts below kLhistBins in LDS per workgroup, flushed once.
constexpr uint32_t kLhistBins = 1024;

__global__ __launch_bounds__(kBlock) void k_lhist(uint32_t n, const uint32_t *__restrict__ l,
                                                   unsigned long long *__restrict__ hist) {
    __shared__ uint32_t bins[kLhistBins];
    for (uint32_t b = threadIdx.x; b < kLhistBins; b += kBlock) bins[b] = 0;
    __syncthreads();
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const uint32_t x = l[v];
        if (x < kLhistBins) atomicAdd(&bins[x], 1u);
        else atomicAdd(&hist[x], 1ull);
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < kLhistBins; b += kBlock)
        if (bins[b]) atomicAdd(&hist[b], (unsigned long long)bins[b]);
}

// Stable placement of each vertex at its (stratum, id) rank.
__global__ __launch_bounds__(kBlock) void k_place(uint32_t n, const uint8_t *__restrict__ stratum,
                                                   const uint64_t *__restrict__ base, uint32_t tiles,
                                                   uint32_t *__restrict__ P) {
    __shared__ uint32_t wcount[kBlock / kWave][kNStrata];
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const uint32_t s = v < n ? stratum[v] : kNStrata;   // out-of-range lanes match nothing
    uint32_t rank = 0;
    for (uint32_t h = 0; h < kNStrata; ++h) {
        uint64_t mask = __ballot(s == h);
        if (lane == 0) wcount[wv][h] = (uint32_t)__popcll(mask);
        if (s == h) rank = lane_rank(mask);
    }
    __syncthreads();
    if (v < n) {
        uint64_t pos = base[(uint64_t)s * tiles + blockIdx.x] + rank;
        for (uint32_t w = 0; w < wv; ++w) pos += wcount[w][s];
        P[pos] = v;
    }
}

uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

uint32_t grid_for(uint64_t items) {
    uint64_t g = div_up(items, kBlock);
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, 65535ull * 16));
}

}  // namespace

int stratify_device(hyperim_graph g, PrepWorkspace &w, hipStream_t s) {
    const uint32_t n = g->n;
    const size_t nn = std::max<uint32_t>(n, 1);
    HIM_CHECK(g->l.reserve(sizeof(uint32_t) * nn, s));
    HIM_CHECK(g->deg.reserve(sizeof(uint32_t) * nn, s));
    HIM_CHECK(g->top.reserve(sizeof(uint32_t) * nn, s));
    HIM_CHECK(g->stratum.reserve(nn, s));
    HIM_CHECK(g->P.reserve(sizeof(uint32_t) * nn, s));
    DevBuf &wmax_b = w.wmax, &pc_b = w.pc, &tmp_b = w.tmp;
    HIM_CHECK(wmax_b.reserve(sizeof(uint32_t) * nn, s));
    for (DevBuf *b : {&g->l, &g->deg, &g->top, &wmax_b}) HIM_HIP(hipMemsetAsync(b->ptr, 0, sizeof(uint32_t) * nn, s));

    // pairs of vertex v = c(v); prefix sums pick the batches
    HIM_CHECK(pc_b.reserve(sizeof(uint64_t) * ((size_t)n + 1), s));
    HIM_CHECK(scan_u64(g->c.as<uint64_t>(), pc_b.as<uint64_t>(), n, 0, tmp_b, s));
    std::vector<uint64_t> pc((size_t)n + 1);
    HIM_HIP(hipMemcpyAsync(pc.data(), pc_b.ptr, sizeof(uint64_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));

    std::vector<std::pair<uint32_t, uint32_t>> batches;
    uint64_t max_pairs = 0;
    for (uint32_t v0 = 0; v0 < n;) {
        // largest v1 with pc[v1] - pc[v0] <= budget (at least one vertex)
        uint64_t limit = pc[v0] + kPairBudget;
        uint32_t v1 = (uint32_t)(std::upper_bound(pc.begin() + v0 + 1, pc.end(), limit) - pc.begin()) - 1;
        if (v1 <= v0) v1 = v0 + 1;
        batches.push_back({v0, v1});
        max_pairs = std::max(max_pairs, pc[v1] - pc[v0]);
        v0 = v1;
    }
    if (max_pairs) {
        const uint64_t cap = next_pow2(std::max<uint64_t>(2 * max_pairs, 1024));
        DevBuf &k1 = w.k1, &vals = w.vals, &k2 = w.k2;
        HIM_CHECK(k1.reserve(sizeof(uint64_t) * cap, s));
        HIM_CHECK(vals.reserve(sizeof(uint32_t) * cap, s));
        HIM_CHECK(k2.reserve(sizeof(uint64_t) * cap, s));
        for (auto [v0, v1] : batches) {
            const uint64_t pairs = pc[v1] - pc[v0];
            if (!pairs) continue;
            const uint64_t c = next_pow2(std::max<uint64_t>(2 * pairs, 1024));
            HIM_HIP(hipMemsetAsync(k1.ptr, 0xFF, sizeof(uint64_t) * c, s));
            HIM_HIP(hipMemsetAsync(vals.ptr, 0, sizeof(uint32_t) * c, s));
            HIM_HIP(hipMemsetAsync(k2.ptr, 0xFF, sizeof(uint64_t) * c, s));
            // one wave per 64 incidences (grid-stride; pairs bound the incidences of
            // hyperedges with two or more members)
            hipLaunchKernelGGL(k_pairs, dim3(std::min<uint32_t>(grid_for(std::max<uint64_t>(pairs, 1)), 8192)),
                               dim3(kBlock), 0, s,
                               g->he_off.as<uint32_t>(), g->he_mem.as<uint32_t>(), g->v_off.as<uint32_t>(),
                               g->v_he.as<uint32_t>(), v0, v1, k1.as<unsigned long long>(), vals.as<uint32_t>(),
                               c - 1);
            hipLaunchKernelGGL(k_layers, dim3(std::min<uint32_t>(grid_for(div_up(c, kAggPer)), 4096)), dim3(kBlock), 0, s, k1.as<unsigned long long>(),
                               vals.as<uint32_t>(), c, k2.as<unsigned long long>(), c - 1, g->deg.as<uint32_t>(),
                               wmax_b.as<uint32_t>(), g->l.as<uint32_t>());
            hipLaunchKernelGGL(k_top, dim3(std::min<uint32_t>(grid_for(div_up(c, kAggPer)), 4096)), dim3(kBlock), 0, s, k1.as<unsigned long long>(),
                               vals.as<uint32_t>(), c, wmax_b.as<uint32_t>(), g->top.as<uint32_t>());
        }
    }

    // strata, counts, statistics
    const uint32_t tiles = (uint32_t)std::max<uint64_t>(div_up(n, kBlock), 1);
    DevBuf &counts_b = w.counts, &base_b = w.base, &isum_b = w.isum, &lmax_b = w.lmax, &hist_b = w.hist;
    HIM_CHECK(counts_b.reserve(sizeof(uint32_t) * kNStrata * tiles, s));
    HIM_CHECK(base_b.reserve(sizeof(uint64_t) * (kNStrata * (size_t)tiles + 1), s));
    HIM_CHECK(isum_b.reserve(sizeof(uint64_t) * 3 * tiles, s));
    HIM_CHECK(lmax_b.reserve(sizeof(uint32_t), s));
    HIM_HIP(hipMemsetAsync(counts_b.ptr, 0, sizeof(uint32_t) * kNStrata * tiles, s));
    HIM_HIP(hipMemsetAsync(isum_b.ptr, 0, sizeof(uint64_t) * 3 * tiles, s));
    HIM_HIP(hipMemsetAsync(lmax_b.ptr, 0, sizeof(uint32_t), s));
    if (n)
        hipLaunchKernelGGL(k_strata, dim3(tiles), dim3(kBlock), 0, s, n, g->l.as<uint32_t>(), g->deg.as<uint32_t>(),
                           g->top.as<uint32_t>(), g->stratum.as<uint8_t>(), counts_b.as<uint32_t>(), tiles,
                           isum_b.as<unsigned long long>(), lmax_b.as<uint32_t>());
    uint32_t lmax = 0;
    HIM_HIP(hipMemcpyAsync(&lmax, lmax_b.ptr, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    HIM_CHECK(hist_b.reserve(sizeof(unsigned long long) * ((size_t)lmax + 1), s));
    HIM_HIP(hipMemsetAsync(hist_b.ptr, 0, sizeof(unsigned long long) * ((size_t)lmax + 1), s));
    if (n)
        hipLaunchKernelGGL(k_lhist, dim3(std::min<uint32_t>(tiles, 64)), dim3(kBlock), 0, s, n, g->l.as<uint32_t>(),
                           hist_b.as<unsigned long long>());
    HIM_CHECK(scan_u32_to_u64(counts_b.as<uint32_t>(), base_b.as<uint64_t>(), (uint64_t)kNStrata * tiles, 0, tmp_b,
                              s));
    if (n)
        hipLaunchKernelGGL(k_place, dim3(tiles), dim3(kBlock), 0, s, n, g->stratum.as<uint8_t>(),
                           base_b.as<uint64_t>(), tiles, g->P.as<uint32_t>());
    HIM_HIP(hipGetLastError());

    std::vector<uint64_t> base((size_t)kNStrata * tiles + 1);
    std::vector<uint64_t> isums((size_t)3 * tiles);
    std::vector<uint64_t> hist((size_t)lmax + 1);
    HIM_HIP(hipMemcpyAsync(base.data(), base_b.ptr, sizeof(uint64_t) * base.size(), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipMemcpyAsync(isums.data(), isum_b.ptr, sizeof(uint64_t) * isums.size(), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipMemcpyAsync(hist.data(), hist_b.ptr, sizeof(uint64_t) * hist.size(), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    hyperim_strata_info &info = g->info;
    for (uint32_t h = 0; h < kNStrata; ++h) info.B[h] = (uint32_t)base[(size_t)h * tiles];
    info.B[kNStrata] = n;
    info.sum_top = info.sum_deg = info.sum_l = 0;
    for (uint32_t t = 0; t < tiles; ++t) {
        info.sum_top += isums[3 * (size_t)t + 0];
        info.sum_deg += isums[3 * (size_t)t + 1];
        info.sum_l += isums[3 * (size_t)t + 2];
    }
    double tl = 0.0;   // sum over v with l_v > 0 of l_v / ln(l_v + 1), grouped by value
    for (uint32_t lv = 1; lv <= lmax; ++lv)
        if (hist[lv]) tl += (double)hist[lv] * ((double)lv / std::log((double)lv + 1.0));
    info.alpha = info.sum_deg ? (double)info.sum_top / (double)info.sum_deg : 0.0;
    info.beta = n ? (double)info.sum_l / (double)n : 0.0;
    info.theta_l = n ? tl / (double)n : 0.0;
    g->strat_lmax = lmax;
    if (g->layered()) HIM_CHECK(layers_build_device(g, lmax, s));
    g->stratified = true;
    // a divided graph keeps its division (the same strata give the same one)
    g->routed = false;
    if (g->route_on) {
        uint32_t n1 = 0;
        const int rc = route_build(g, s, &n1);
        if (rc != HYPERIM_OK) {
            g->route_on = false;   // left undivided, as after a failed hyperim_route
            return rc;
        }
    }
    return HYPERIM_OK;
}

}  // namespace hyperim
