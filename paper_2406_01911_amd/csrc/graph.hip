// Device-resident hypergraph (Section 2.1: G = (V, HE) with member lists
// V(he)).  Validates the caller's CSR, transposes it into vertex -> hyperedge
// incidence lists with ascending hyperedge ids, and derives the per-target
// coin thresholds of the IC channel model.  G_w is never materialised.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "block_table.h"
#include "dev_common.h"
#include "internal.h"

namespace hyperim {
namespace {

constexpr int kBlock = 256;
constexpr uint32_t kSmallSeg = 16;     // insertion sort by one thread
constexpr uint32_t kMidSeg = 4096;     // bitonic sort in LDS by one workgroup

enum Flag : uint32_t { kBadOffsets = 1, kBadId = 2, kDuplicate = 4 };

__global__ void k_check_offsets(const uint32_t *__restrict__ he_off, uint32_t m, uint32_t *flag) {
    uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0 && he_off[0] != 0u) atomicOr(flag, (uint32_t)kBadOffsets);
    if (e < m && he_off[e + 1] < he_off[e]) atomicOr(flag, (uint32_t)kBadOffsets);
}

// Incidences per vertex.  Each workgroup takes chunks of kChunk consecutive
// incidences and adds per-vertex totals to global memory once per chunk.
constexpr uint32_t kChunkPer = 8;                 // incidences per thread per chunk
constexpr uint32_t kChunk = kBlock * kChunkPer;
constexpr uint32_t kTableSlots = 4096;

__global__ __launch_bounds__(kBlock) void k_count(const uint32_t *__restrict__ he_mem, uint64_t nnz, uint32_t n,
                                                   uint32_t *__restrict__ cnt, uint32_t *flag) {
    __shared__ BlockTable<kTableSlots> tab;
    __shared__ uint32_t tval[kTableSlots];
    tab.clear_keys();
    for (uint32_t s = threadIdx.x; s < kTableSlots; s += kBlock) tval[s] = 0;
    __syncthreads();
    for (uint64_t base = (uint64_t)blockIdx.x * kChunk; base < nnz; base += (uint64_t)gridDim.x * kChunk) {
        for (uint32_t r = 0; r < kChunkPer; ++r) {
            const uint64_t i = base + r * kBlock + threadIdx.x;
            if (i >= nnz) break;
            const uint32_t v = he_mem[i];
            if (v >= n) {
                atomicOr(flag, (uint32_t)kBadId);
                continue;
            }
            const uint32_t sl = tab.slot(v);
            if (sl != kTableEmpty) atomicAdd(&tval[sl], 1u);
            else atomicAdd(&cnt[v], 1u);
        }
        __syncthreads();
        for (uint32_t sl = threadIdx.x; sl < kTableSlots; sl += kBlock) {
            const uint32_t v = tab.key[sl];
            if (v != kTableEmpty) {
                atomicAdd(&cnt[v], tval[sl]);
                tab.key[sl] = kTableEmpty;
                tval[sl] = 0;
            }
        }
        __syncthreads();
    }
}

__global__ void k_u64_to_u32(const uint64_t *__restrict__ in, uint32_t *__restrict__ out, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = (uint32_t)in[i];
}

// Scatter every incidence (he, position) into its vertex's segment (order
// inside a segment fixed afterwards by sorting) and accumulate c(v).  Per
// chunk, each workgroup ranks its incidences of one vertex in LDS, reserves
// the vertex's places with one global atomic and adds its c(v) share once.
constexpr uint32_t kFillPer = 4;
constexpr uint32_t kFillChunk = kBlock * kFillPer;
constexpr uint32_t kFillSlots = 2048;

__global__ __launch_bounds__(kBlock) void k_fill(const uint32_t *__restrict__ he_off,
                                                  const uint32_t *__restrict__ he_mem, uint32_t m, uint64_t nnz,
                                                  const uint32_t *__restrict__ v_off, uint32_t *__restrict__ cursor,
                                                  uint32_t *__restrict__ v_he, unsigned long long *__restrict__ c) {
    __shared__ BlockTable<kFillSlots> tab;
    __shared__ uint32_t tcnt[kFillSlots], tbase[kFillSlots];
    __shared__ unsigned long long tsum[kFillSlots];
    tab.clear_keys();
    for (uint32_t s = threadIdx.x; s < kFillSlots; s += kBlock) {
        tcnt[s] = 0;
        tsum[s] = 0;
    }
    __syncthreads();
    for (uint64_t base = (uint64_t)blockIdx.x * kFillChunk; base < nnz; base += (uint64_t)gridDim.x * kFillChunk) {
        uint32_t ev[kFillPer], vv[kFillPer], sl[kFillPer], rk[kFillPer];
#pragma unroll
        for (uint32_t r = 0; r < kFillPer; ++r) {
            sl[r] = kTableEmpty;
            vv[r] = kTableEmpty;
            const uint64_t i = base + r * kBlock + threadIdx.x;
            if (i >= nnz) continue;
            // owner hyperedge: largest e with he_off[e] <= i (skipping empty ones)
            uint32_t lo = 0, hi = m;  // he_off[lo] <= i < he_off[hi]
            while (hi - lo > 1) {
                const uint32_t mid = lo + (hi - lo) / 2;
                if (he_off[mid] <= (uint32_t)i) lo = mid; else hi = mid;
            }
            const uint32_t e = lo, v = he_mem[i];
            const unsigned long long cs = he_off[e + 1] - he_off[e] - 1u;
            ev[r] = e;
            vv[r] = v;
            sl[r] = tab.slot(v);
            if (sl[r] != kTableEmpty) {
                rk[r] = atomicAdd(&tcnt[sl[r]], 1u);
                atomicAdd(&tsum[sl[r]], cs);
            } else {
                const uint32_t pos = atomicAdd(&cursor[v], 1u);
                v_he[v_off[v] + pos] = e;
                atomicAdd(&c[v], cs);
            }
        }
        __syncthreads();
        for (uint32_t s = threadIdx.x; s < kFillSlots; s += kBlock) {
            const uint32_t v = tab.key[s];
            if (v != kTableEmpty) {
                tbase[s] = atomicAdd(&cursor[v], tcnt[s]);
                atomicAdd(&c[v], tsum[s]);
            }
        }
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < kFillPer; ++r)
            if (sl[r] != kTableEmpty) v_he[v_off[vv[r]] + tbase[sl[r]] + rk[r]] = ev[r];
        __syncthreads();
        for (uint32_t s = threadIdx.x; s < kFillSlots; s += kBlock) {
            tab.key[s] = kTableEmpty;
            tcnt[s] = 0;
            tsum[s] = 0;
        }
        __syncthreads();
    }
}

// Short segments: one thread, insertion sort; flags duplicates.
__global__ void k_sort_small(const uint32_t *__restrict__ v_off, uint32_t n, uint32_t *__restrict__ v_he,
                             uint32_t *__restrict__ mid_list, uint32_t *__restrict__ big_list,
                             uint32_t *__restrict__ counts, uint32_t *flag) {
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    uint32_t b = v_off[v], len = v_off[v + 1] - b;
    if (len > kMidSeg) {
        big_list[atomicAdd(&counts[1], 1u)] = v;
        return;
    }
    if (len > kSmallSeg) {
        mid_list[atomicAdd(&counts[0], 1u)] = v;
        return;
    }
    uint32_t a[kSmallSeg];
    for (uint32_t i = 0; i < len; ++i) a[i] = v_he[b + i];
    for (uint32_t i = 1; i < len; ++i) {
        uint32_t x = a[i];
        uint32_t k = i;
        while (k > 0 && a[k - 1] > x) {
            a[k] = a[k - 1];
            --k;
        }
        a[k] = x;
    }
    for (uint32_t i = 0; i < len; ++i) {
        if (i && a[i] == a[i - 1]) atomicOr(flag, (uint32_t)kDuplicate);
        v_he[b + i] = a[i];
    }
}

// Medium segments: one workgroup per vertex, bitonic sort in LDS.
__global__ __launch_bounds__(kBlock) void k_sort_mid(const uint32_t *__restrict__ v_off,
                                                     const uint32_t *__restrict__ list, const uint32_t *counts,
                                                     uint32_t *__restrict__ v_he, uint32_t *flag) {
    __shared__ uint32_t buf[kMidSeg];
    const uint32_t nlist = counts[0];
    for (uint32_t w = blockIdx.x; w < nlist; w += gridDim.x) {
        const uint32_t v = list[w];
        const uint32_t b = v_off[v], len = v_off[v + 1] - b;
        uint32_t P = 1;
        while (P < len) P <<= 1;
        for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) buf[i] = i < len ? v_he[b + i] : 0xFFFFFFFFu;
        __syncthreads();
        for (uint32_t k = 2; k <= P; k <<= 1) {
            for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
                for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) {
                    uint32_t x = i ^ jj;
                    if (x > i) {
                        uint32_t p = buf[i], q = buf[x];
                        bool up = (i & k) == 0;
                        if ((p > q) == up) {
                            buf[i] = q;
                            buf[x] = p;
                        }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
            uint32_t x = buf[i];
            if (i && buf[i - 1] == x) atomicOr(flag, (uint32_t)kDuplicate);
            v_he[b + i] = x;
        }
        __syncthreads();
    }
}

// Long segments (hub vertices): mark the hyperedge ids in a bitmap over all
// m hyperedges and read them back in ascending order.  A repeated id shows
// up as fewer set bits than the segment length.
__global__ __launch_bounds__(kBlock) void k_sort_big(const uint32_t *__restrict__ v_off,
                                                     const uint32_t *__restrict__ list, const uint32_t *counts,
                                                     uint32_t *__restrict__ v_he, uint32_t *__restrict__ bitmaps,
                                                     uint32_t words, uint32_t *flag) {
    __shared__ uint32_t wave_tot[kBlock / kWave];
    __shared__ uint32_t running;
    uint32_t *bm = bitmaps + (size_t)blockIdx.x * words;
    const uint32_t nlist = counts[1];
    const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    for (uint32_t w = blockIdx.x; w < nlist; w += gridDim.x) {
        const uint32_t v = list[w];
        const uint32_t b = v_off[v], len = v_off[v + 1] - b;
        for (uint32_t i = threadIdx.x; i < words; i += blockDim.x) bm[i] = 0u;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
            uint32_t e = v_he[b + i];
            atomicOr(&bm[e >> 5], 1u << (e & 31));
        }
        // the bits were set by L2 atomics: drop this CU's L1 copies before reading
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) running = 0;
        __syncthreads();
        for (uint32_t base = 0; base < words; base += blockDim.x) {
            uint32_t i = base + threadIdx.x;
            uint32_t word = i < words ? bm[i] : 0u;
            uint32_t c = __popc(word);
            uint32_t incl = wave_incl_scan(c);
            if (lane == kWave - 1) wave_tot[wv] = incl;
            __syncthreads();
            uint32_t before = running;
            for (uint32_t q = 0; q < wv; ++q) before += wave_tot[q];
            uint32_t pos = before + incl - c;
            while (word) {
                uint32_t bit = __ffs(word) - 1;
                word &= word - 1;
                if (pos < len) v_he[b + pos] = i * 32 + bit;
                ++pos;
            }
            __syncthreads();
            if (threadIdx.x == blockDim.x - 1) running = before + incl;
            __syncthreads();
        }
        if (threadIdx.x == 0 && running != len) atomicOr(flag, (uint32_t)kDuplicate);
        __syncthreads();
    }
}

// Coin thresholds and per-vertex incidence weights.
__global__ void k_thresholds(uint32_t n, uint32_t model, float p, const uint32_t *__restrict__ v_off,
                             const unsigned long long *__restrict__ c, uint32_t *__restrict__ thr,
                             unsigned long long *__restrict__ weight, unsigned long long *__restrict__ bytesw) {
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    float pv;
    if (model == HYPERIM_MODEL_CONST || model == HYPERIM_MODEL_LT_CONST || model == HYPERIM_MODEL_GAPS_CONST) {
        pv = p;
    } else {
        unsigned long long cv = c[v];
        pv = cv ? (float)(1.0 / (double)cv) : 0.0f;
    }
    uint32_t t;
    if (pv >= 1.0f) t = kAlways;
    else if (!(pv > 0.0f)) t = 0u;
    else t = (uint32_t)floor(ldexp((double)pv, 32));
    thr[v] = t;
    // d hyperedges of total size S = c + d: a member reads its offset pair (8 B),
    // d hyperedge ids and offset pairs (12 B each), S member ids (4 B each), and
    // costs 12 B of visited/queue/output traffic
    const unsigned long long d = v_off[v + 1] - v_off[v];
    weight[v] = 2ull * d + c[v];
    bytesw[v] = 20ull + 16ull * d + 4ull * c[v];
}

// Philox blocks of a vertex's expansion: sum over its hyperedges of
// ceil(|he| / 4).  One wavefront per vertex.
__global__ __launch_bounds__(kBlock) void k_philox_weight(uint32_t n, const uint32_t *__restrict__ v_off,
                                                          const uint32_t *__restrict__ v_he,
                                                          const uint32_t *__restrict__ he_off,
                                                          unsigned long long *__restrict__ phiw) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint64_t waves = (uint64_t)gridDim.x * (kBlock / kWave);
    for (uint64_t v = (uint64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; v < n; v += waves) {
        unsigned long long acc = 0;
        for (uint32_t e = v_off[v] + lane; e < v_off[v + 1]; e += kWave) {
            const uint32_t he = v_he[e];
            acc += (he_off[he + 1] - he_off[he] + 3u) / 4u;
        }
        acc = wave_sum(acc);
        if (lane == 0) phiw[v] = acc;
    }
}

// Per incidence: first member position and size of its hyperedge.
__global__ void k_incidence_spans(uint64_t nnz, const uint32_t *__restrict__ v_he, const uint32_t *__restrict__ he_off,
                                  uint2 *__restrict__ v_hbs) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t he = v_he[e];
        const uint32_t b = he_off[he];
        v_hbs[e] = make_uint2(b, he_off[he + 1] - b);
    }
}

// Channels of each incidence (v, he) under the linear-threshold model:
// |he| - 1 (the members of he other than v).
__global__ void k_channel_counts(uint64_t nnz, const uint2 *__restrict__ v_hbs, uint32_t *__restrict__ cnt) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (uint64_t)gridDim.x * blockDim.x)
        cnt[e] = v_hbs[e].y - 1u;
}

uint32_t grid_for(uint64_t items, uint32_t block = kBlock, uint32_t cap = 65535u * 8u) {
    uint64_t g = div_up(items, block);
    if (g == 0) g = 1;
    return (uint32_t)std::min<uint64_t>(g, cap);
}

}  // namespace

// Exclusive prefix over all incidences of their channel counts |he| - 1: the
// channels into v are chan[v_off[v]] .. chan[v_off[v + 1]] (needs v_hbs).
// cnt and tmp are scratch the caller keeps alive until the stream has run.
int channel_prefix(hyperim_graph g, DevBuf &cnt, DevBuf &tmp, hipStream_t s) {
    const uint64_t nnz = g->nnz;
    HIM_CHECK(g->chan.reserve(sizeof(uint64_t) * (nnz + 1), s));
    HIM_CHECK(cnt.reserve(sizeof(uint32_t) * std::max<uint64_t>(nnz, 1), s));
    if (nnz)
        hipLaunchKernelGGL(k_channel_counts, dim3(grid_for(nnz, kBlock, 8192)), dim3(kBlock), 0, s, nnz,
                           g->v_hbs.as<uint2>(), cnt.as<uint32_t>());
    HIM_HIP(hipGetLastError());
    return scan_u32_to_u64(cnt.as<uint32_t>(), g->chan.as<uint64_t>(), nnz, 0, tmp, s);
}

int graph_build_device(hyperim_graph g, PrepWorkspace &w, hipStream_t s) {
    const uint32_t n = g->n, m = g->m;
    const uint64_t nnz = g->nnz;
    DevBuf chan_cnt, chan_tmp;   // linear-threshold channel prefix (freed after the final wait)
    DevBuf &flag_b = w.flag, &cnt_b = w.cnt, &off64_b = w.off64, &tmp_b = w.tmp;
    HIM_CHECK(flag_b.reserve(4 * sizeof(uint32_t), s));
    uint32_t *flag = flag_b.as<uint32_t>();
    HIM_HIP(hipMemsetAsync(flag, 0, 4 * sizeof(uint32_t), s));

    hipLaunchKernelGGL(k_check_offsets, dim3(grid_for((uint64_t)m + 1)), dim3(kBlock), 0, s,
                       g->he_off.as<uint32_t>(), m, flag);
    HIM_CHECK(cnt_b.reserve(sizeof(uint32_t) * ((size_t)n + 1), s));
    HIM_HIP(hipMemsetAsync(cnt_b.ptr, 0, sizeof(uint32_t) * ((size_t)n + 1), s));
    hipLaunchKernelGGL(k_count, dim3(grid_for(nnz, kChunk, 4096)), dim3(kBlock), 0, s, g->he_mem.as<uint32_t>(), nnz, n,
                       cnt_b.as<uint32_t>(), flag);
    uint32_t hflag = 0;
    HIM_HIP(hipMemcpyAsync(&hflag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    if (hflag) {
        set_error_detail(hflag & kBadOffsets ? "hyperedge offsets decrease or do not start at 0"
                                             : "member id >= n");
        return HYPERIM_EINVAL;
    }

    HIM_CHECK(off64_b.reserve(sizeof(uint64_t) * ((size_t)n + 1), s));
    HIM_CHECK(scan_u32_to_u64(cnt_b.as<uint32_t>(), off64_b.as<uint64_t>(), n, 0, tmp_b, s));
    HIM_CHECK(g->v_off.reserve(sizeof(uint32_t) * ((size_t)n + 1), s));
    hipLaunchKernelGGL(k_u64_to_u32, dim3(grid_for((uint64_t)n + 1)), dim3(kBlock), 0, s,
                       off64_b.as<uint64_t>(), g->v_off.as<uint32_t>(), (uint64_t)n + 1);

    HIM_CHECK(g->v_he.reserve(sizeof(uint32_t) * std::max<uint64_t>(nnz, 1), s));
    HIM_CHECK(g->c.reserve(sizeof(uint64_t) * std::max<uint32_t>(n, 1), s));
    HIM_HIP(hipMemsetAsync(g->c.ptr, 0, sizeof(uint64_t) * std::max<uint32_t>(n, 1), s));
    HIM_HIP(hipMemsetAsync(cnt_b.ptr, 0, sizeof(uint32_t) * ((size_t)n + 1), s));
    if (nnz)
        hipLaunchKernelGGL(k_fill, dim3(grid_for(nnz, kFillChunk, 4096)), dim3(kBlock), 0, s, g->he_off.as<uint32_t>(),
                           g->he_mem.as<uint32_t>(), m, nnz, g->v_off.as<uint32_t>(), cnt_b.as<uint32_t>(),
                           g->v_he.as<uint32_t>(), g->c.as<unsigned long long>());

    // order every segment by hyperedge id
    DevBuf &lists_b = w.lists, &bm_b = w.bm;
    HIM_CHECK(lists_b.reserve(sizeof(uint32_t) * 2 * ((size_t)n + 1), s));
    uint32_t *mid_list = lists_b.as<uint32_t>();
    uint32_t *big_list = mid_list + n + 1;
    uint32_t *counts = flag + 1;  // [0] mid, [1] big
    if (n) {
        hipLaunchKernelGGL(k_sort_small, dim3(grid_for(n)), dim3(kBlock), 0, s, g->v_off.as<uint32_t>(), n,
                           g->v_he.as<uint32_t>(), mid_list, big_list, counts, flag);
        hipLaunchKernelGGL(k_sort_mid, dim3(std::min<uint32_t>(std::max<uint32_t>(n, 1), 4096)), dim3(kBlock), 0,
                           s, g->v_off.as<uint32_t>(), mid_list, counts, g->v_he.as<uint32_t>(), flag);
        const uint32_t words = (m + 31) / 32;
        const uint32_t big_grid = 128;
        HIM_CHECK(bm_b.reserve(sizeof(uint32_t) * (size_t)std::max<uint32_t>(words, 1) * big_grid, s));
        hipLaunchKernelGGL(k_sort_big, dim3(big_grid), dim3(kBlock), 0, s, g->v_off.as<uint32_t>(), big_list,
                           counts, g->v_he.as<uint32_t>(), bm_b.as<uint32_t>(), std::max<uint32_t>(words, 1),
                           flag);
    }
    HIM_HIP(hipMemcpyAsync(&hflag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    if (hflag & kDuplicate) {
        set_error_detail("a vertex appears twice in one hyperedge");
        return HYPERIM_EINVAL;
    }

    HIM_CHECK(g->thr.reserve(sizeof(uint32_t) * std::max<uint32_t>(n, 1), s));
    HIM_CHECK(g->weight.reserve(sizeof(uint64_t) * std::max<uint32_t>(n, 1), s));
    HIM_CHECK(g->bytesw.reserve(sizeof(uint64_t) * std::max<uint32_t>(n, 1), s));
    HIM_CHECK(g->phiw.reserve(sizeof(uint64_t) * std::max<uint32_t>(n, 1), s));
    HIM_CHECK(g->v_hbs.reserve(sizeof(uint2) * std::max<uint64_t>(nnz, 1), s));
    if (nnz)
        hipLaunchKernelGGL(k_incidence_spans, dim3(grid_for(nnz, kBlock, 8192)), dim3(kBlock), 0, s, nnz,
                           g->v_he.as<uint32_t>(), g->he_off.as<uint32_t>(), g->v_hbs.as<uint2>());
    if (g->lt() || g->layered()) HIM_CHECK(channel_prefix(g, chan_cnt, chan_tmp, s));
    if (n) {
        hipLaunchKernelGGL(k_thresholds, dim3(grid_for(n)), dim3(kBlock), 0, s, n, g->prob.model, g->prob.p,
                           g->v_off.as<uint32_t>(), g->c.as<unsigned long long>(), g->thr.as<uint32_t>(),
                           g->weight.as<unsigned long long>(), g->bytesw.as<unsigned long long>());
        hipLaunchKernelGGL(k_philox_weight, dim3(grid_for((uint64_t)n * kWave, kBlock, 8192)), dim3(kBlock), 0, s, n,
                           g->v_off.as<uint32_t>(), g->v_he.as<uint32_t>(), g->he_off.as<uint32_t>(),
                           g->phiw.as<unsigned long long>());
    }
    HIM_HIP(hipGetLastError());
    HIM_HIP(hipStreamSynchronize(s));
    return HYPERIM_OK;
}

}  // namespace hyperim
