// Sample-set division (Section 3.1.1) as tables, for the stratified-setting
// model: per vertex v the members of A(v) layer by layer (layer 1 = largest
// w(v,u)), ascending ids within a layer, plus the layer ends, and the host
// tables of ln(l + 1) and e^-P(L_i) that the RR kernel's count draws use.
//
// Built once per graph at stratify time, on the device:
//   1. every co-member occurrence (v, u) of incidence e is written, as the
//      key v << b | u (b = bits of a vertex id), at the incidence's channel
//      prefix chan[e] (the graph's exclusive prefix of |he| - 1 over v_he);
//   2. a device-wide radix sort orders the keys (rocPRIM), so each vertex's
//      occurrences are contiguous and ascending in u;
//   3. run heads give the distinct pairs (v, u) and their run lengths w(v,u);
//   4. a second, stable radix sort by the key v << 32 | ~w puts each vertex's
//      co-members in layers (descending w; equal w keep ascending u);
//   5. positions where the key changes are the layer ends.
// ln and e^-P are evaluated on the host with the C library's log and exp, so
// the device uses the same doubles as any host code that calls them.
#include <hip/hip_runtime.h>

#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cmath>
#include <vector>

#include "dev_common.h"
#include "internal.h"

namespace hyperim {
namespace {

constexpr uint32_t kBlock = 256;

uint32_t grid_for(uint64_t items, uint32_t cap = 8192) {
    const uint64_t g = std::max<uint64_t>(div_up(items, kBlock), 1);
    return (uint32_t)std::min<uint64_t>(g, cap);
}

// Owner vertex of incidence e: the last v with v_off[v] <= e.
__device__ __forceinline__ uint32_t owner(const uint32_t *__restrict__ v_off, uint32_t n, uint64_t e) {
    uint32_t lo = 0, hi = n;   // v_off[lo] <= e < v_off[hi]
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (v_off[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// 1. Occurrences: incidence e = (v, he) writes v << b | u for the members u
// of he other than v at chan[e] ...
__global__ void k_occ_emit(uint32_t n, uint64_t nnz, uint32_t b, const uint32_t *__restrict__ v_off,
                           const uint32_t *__restrict__ v_he, const uint32_t *__restrict__ he_off,
                           const uint32_t *__restrict__ he_mem, const unsigned long long *__restrict__ chan,
                           unsigned long long *__restrict__ occ) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = owner(v_off, n, e), he = v_he[e];
        uint64_t at = chan[e];
        for (uint32_t i = he_off[he]; i < he_off[he + 1]; ++i) {
            const uint32_t u = he_mem[i];
            if (u != v) occ[at++] = ((unsigned long long)v << b) | u;
        }
    }
}

// 3. Run heads of the sorted keys.
__global__ void k_heads(uint64_t total, const unsigned long long *__restrict__ key, uint32_t *__restrict__ head) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x)
        head[i] = (i == 0 || key[i] != key[i - 1]) ? 1u : 0u;
}

// Distinct pair k (at run head i): its key and its run's start.
__global__ void k_runs(uint64_t total, const unsigned long long *__restrict__ key, const uint32_t *__restrict__ head,
                       const unsigned long long *__restrict__ hscan, unsigned long long *__restrict__ ukey,
                       uint32_t *__restrict__ run_start) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x)
        if (head[i]) {
            const uint64_t k = hscan[i];
            ukey[k] = key[i];
            run_start[k] = (uint32_t)i;
        }
}

// Layer sort key of distinct pair k: v << 32 | ~w (ascending keys: v, then
// descending w); the value is u.
__global__ void k_wkeys(uint64_t uniq, uint64_t total, uint32_t b, const unsigned long long *__restrict__ ukey,
                        const uint32_t *__restrict__ run_start, unsigned long long *__restrict__ key2,
                        uint32_t *__restrict__ val) {
    const unsigned long long umask = (1ull << b) - 1ull;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < uniq; k += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t end = k + 1 < uniq ? run_start[k + 1] : (uint32_t)total;
        const uint32_t w = end - run_start[k];
        const unsigned long long v = ukey[k] >> b;
        key2[k] = (v << 32) | (unsigned long long)(~w);
        val[k] = (uint32_t)(ukey[k] & umask);
    }
}

// 5. Layer ends: entry k ends a layer when the next key differs (another
// weight or another vertex) or k is the last entry.
__global__ void k_layer_flags(uint64_t uniq, const unsigned long long *__restrict__ key2, uint32_t *__restrict__ flag) {
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < uniq; k += (uint64_t)gridDim.x * blockDim.x)
        flag[k] = (k + 1 == uniq || key2[k + 1] != key2[k]) ? 1u : 0u;
}

__global__ void k_layer_ends(uint64_t uniq, const unsigned long long *__restrict__ key2, const uint32_t *__restrict__ flag,
                             const unsigned long long *__restrict__ fscan, const unsigned long long *__restrict__ nb_off,
                             uint32_t *__restrict__ ly_end) {
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < uniq; k += (uint64_t)gridDim.x * blockDim.x)
        if (flag[k]) {
            const uint32_t v = (uint32_t)(key2[k] >> 32);
            ly_end[fscan[k]] = (uint32_t)(k + 1 - nb_off[v]);
        }
}

}  // namespace

int layers_build_device(hyperim_graph g, uint32_t lmax, hipStream_t s) {
    const uint32_t n = g->n;
    const uint64_t nnz = g->nnz;
    // occurrences: sum over v of c(v)
    uint64_t total = 0;
    HIM_HIP(hipMemcpyAsync(&total, g->chan.as<unsigned long long>() + nnz, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    const uint64_t uniq = g->info.sum_deg, nlay = g->info.sum_l;
    if (total >= (1ull << 32) || lmax > 16384u) {
        set_error_detail("stratified-setting tables: more than 2^32 co-member occurrences or 16384 layers");
        return HYPERIM_EINVAL;
    }
    const uint32_t b = n > 1 ? 32u - (uint32_t)__builtin_clz(n - 1u) : 1u;   // bits of a vertex id
    DevBuf occ, occ2, tmp, head, hscan, run_start, key2, key2s, val, flag, fscan, scan_tmp;
    HIM_CHECK(occ.reserve(sizeof(uint64_t) * std::max<uint64_t>(total, 1), s));
    HIM_CHECK(occ2.reserve(sizeof(uint64_t) * std::max<uint64_t>(total, 1), s));
    if (nnz)
        hipLaunchKernelGGL(k_occ_emit, dim3(grid_for(nnz)), dim3(kBlock), 0, s, n, nnz, b, g->v_off.as<uint32_t>(),
                           g->v_he.as<uint32_t>(), g->he_off.as<uint32_t>(), g->he_mem.as<uint32_t>(),
                           g->chan.as<unsigned long long>(), occ.as<unsigned long long>());
    HIM_HIP(hipGetLastError());
    // 2. all occurrences by (v, u)
    size_t tbytes = 0;
    HIM_HIP(rocprim::radix_sort_keys(nullptr, tbytes, occ.as<unsigned long long>(), occ2.as<unsigned long long>(),
                                     (size_t)total, 0u, 2u * b, s));
    HIM_CHECK(tmp.reserve(std::max<size_t>(tbytes, 1), s));
    if (total)
        HIM_HIP(rocprim::radix_sort_keys(tmp.ptr, tbytes, occ.as<unsigned long long>(), occ2.as<unsigned long long>(),
                                         (size_t)total, 0u, 2u * b, s));
    // 3. distinct pairs and their weights (occ is free again: it takes the
    // distinct keys)
    HIM_CHECK(head.reserve(sizeof(uint32_t) * std::max<uint64_t>(total, 1), s));
    HIM_CHECK(hscan.reserve(sizeof(uint64_t) * (total + 1), s));
    HIM_CHECK(run_start.reserve(sizeof(uint32_t) * std::max<uint64_t>(uniq, 1), s));
    HIM_CHECK(key2.reserve(sizeof(uint64_t) * std::max<uint64_t>(uniq, 1), s));
    HIM_CHECK(key2s.reserve(sizeof(uint64_t) * std::max<uint64_t>(uniq, 1), s));
    HIM_CHECK(val.reserve(sizeof(uint32_t) * std::max<uint64_t>(uniq, 1), s));
    HIM_CHECK(g->lay_nb.reserve(sizeof(uint32_t) * std::max<uint64_t>(uniq, 1), s));
    if (total) {
        hipLaunchKernelGGL(k_heads, dim3(grid_for(total)), dim3(kBlock), 0, s, total, occ2.as<unsigned long long>(),
                           head.as<uint32_t>());
        HIM_CHECK(scan_u32_to_u64(head.as<uint32_t>(), hscan.as<uint64_t>(), total, 0, scan_tmp, s));
    } else {
        HIM_HIP(hipMemsetAsync(hscan.ptr, 0, sizeof(uint64_t), s));
    }
    uint64_t uniq_dev = 0;
    HIM_HIP(hipMemcpyAsync(&uniq_dev, hscan.as<uint64_t>() + total, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    if (uniq_dev != uniq) {
        set_error_detail("stratified-setting tables: distinct co-members disagree with deg");
        return HYPERIM_EHIP;
    }
    if (total) {
        hipLaunchKernelGGL(k_runs, dim3(grid_for(total)), dim3(kBlock), 0, s, total, occ2.as<unsigned long long>(),
                           head.as<uint32_t>(), hscan.as<unsigned long long>(), occ.as<unsigned long long>(),
                           run_start.as<uint32_t>());
        hipLaunchKernelGGL(k_wkeys, dim3(grid_for(uniq)), dim3(kBlock), 0, s, uniq, total, b,
                           occ.as<unsigned long long>(), run_start.as<uint32_t>(), key2.as<unsigned long long>(),
                           val.as<uint32_t>());
    }
    // per-vertex ranges of the distinct co-members (deg prefix) and of the
    // layers (l prefix)
    HIM_CHECK(g->lay_nb_off.reserve(sizeof(uint64_t) * ((size_t)n + 1), s));
    HIM_CHECK(g->lay_ly_off.reserve(sizeof(uint64_t) * ((size_t)n + 1), s));
    HIM_CHECK(scan_u32_to_u64(g->deg.as<uint32_t>(), g->lay_nb_off.as<uint64_t>(), n, 0, scan_tmp, s));
    HIM_CHECK(scan_u32_to_u64(g->l.as<uint32_t>(), g->lay_ly_off.as<uint64_t>(), n, 0, scan_tmp, s));
    // 4. layers: stable sort of the distinct pairs by v << 32 | ~w, values u
    tbytes = 0;
    HIM_HIP(rocprim::radix_sort_pairs(nullptr, tbytes, key2.as<unsigned long long>(), key2s.as<unsigned long long>(),
                                      val.as<uint32_t>(), g->lay_nb.as<uint32_t>(), (size_t)uniq, 0u, 32u + b, s));
    HIM_CHECK(tmp.reserve(std::max<size_t>(tbytes, 1), s));
    if (uniq)
        HIM_HIP(rocprim::radix_sort_pairs(tmp.ptr, tbytes, key2.as<unsigned long long>(),
                                          key2s.as<unsigned long long>(), val.as<uint32_t>(),
                                          g->lay_nb.as<uint32_t>(), (size_t)uniq, 0u, 32u + b, s));
    // 5. layer ends
    HIM_CHECK(flag.reserve(sizeof(uint32_t) * std::max<uint64_t>(uniq, 1), s));
    HIM_CHECK(fscan.reserve(sizeof(uint64_t) * (uniq + 1), s));
    HIM_CHECK(g->lay_ly_end.reserve(sizeof(uint32_t) * std::max<uint64_t>(nlay, 1), s));
    if (uniq) {
        hipLaunchKernelGGL(k_layer_flags, dim3(grid_for(uniq)), dim3(kBlock), 0, s, uniq,
                           key2s.as<unsigned long long>(), flag.as<uint32_t>());
        HIM_CHECK(scan_u32_to_u64(flag.as<uint32_t>(), fscan.as<uint64_t>(), uniq, 0, scan_tmp, s));
        hipLaunchKernelGGL(k_layer_ends, dim3(grid_for(uniq)), dim3(kBlock), 0, s, uniq,
                           key2s.as<unsigned long long>(), flag.as<uint32_t>(), fscan.as<unsigned long long>(),
                           g->lay_nb_off.as<unsigned long long>(), g->lay_ly_end.as<uint32_t>());
    }
    HIM_HIP(hipGetLastError());
    // host tables: ln(l + 1) for l <= lmax, and e^-P(L_i) with
    // P(L_i) = 1 / (i ln(l + 1)) at index l (l - 1) / 2 + i - 1
    std::vector<double> ln((size_t)lmax + 1), expm(std::max<size_t>((size_t)lmax * (lmax + 1) / 2, 1));
    for (uint32_t l = 0; l <= lmax; ++l) ln[l] = std::log((double)l + 1.0);
    for (uint32_t l = 1; l <= lmax; ++l)
        for (uint32_t i = 1; i <= l; ++i) {
            const double P = 1.0 / ((double)i * std::log((double)l + 1.0));
            expm[(size_t)l * (l - 1) / 2 + i - 1] = std::exp(-P);
        }
    HIM_CHECK(g->lay_ln.reserve(sizeof(double) * ln.size(), s));
    HIM_CHECK(g->lay_expm.reserve(sizeof(double) * expm.size(), s));
    HIM_HIP(hipMemcpyAsync(g->lay_ln.ptr, ln.data(), sizeof(double) * ln.size(), hipMemcpyHostToDevice, s));
    HIM_HIP(hipMemcpyAsync(g->lay_expm.ptr, expm.data(), sizeof(double) * expm.size(), hipMemcpyHostToDevice, s));
    HIM_HIP(hipStreamSynchronize(s));   // the scratch buffers above are freed on return
    g->lay_lmax = lmax;
    return HYPERIM_OK;
}

}  // namespace hyperim
