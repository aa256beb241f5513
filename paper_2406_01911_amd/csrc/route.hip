// Division of the RR sets into R1 and R2 (Section 4.1, "Division of the RR
// sets"), an opt-in that biases the estimates (the design notes quantify it).
//
// alpha = F_cnt / T_cnt and beta = L_cnt / |V| come from stratify.  For a
// vertex v, layer i of A(v) with 1 <= i <= floor(beta) is small when
// |L_i| < alpha |A(v)|, tested exactly as |L_i| T_cnt < F_cnt |A(v)| on
// 128-bit products.  v's RR sets go to R1 when v has a small layer, and then
// start from v and every member of its small layers together; the other
// vertices' sets go to R2.  Pool 0 (R1) draws its roots, stratified as
// usual, from the R1 vertices in the stratum order of P, pool 1 (R2) from
// the others.  With either side empty the division is inert.
//
// On the device: the layer tables (layers.hip, built here for graphs that do
// not have them), one thread per vertex counting its forced members, and
// one writing them; the host splits P into the two root lists and their
// strata boundaries from the counts (O(n) host work, once per division).
#include <hip/hip_runtime.h>

#include <algorithm>
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

// a * b < c * d on full 128-bit products of 64-bit operands.
__device__ __forceinline__ bool prod_less(uint64_t a, uint64_t b, uint64_t c, uint64_t d) {
    const uint64_t h1 = __umul64hi(a, b), h2 = __umul64hi(c, d);
    return h1 < h2 || (h1 == h2 && a * b < c * d);
}

// Forced members of v (the members of its small layers among the first
// ilim), counted (out = null) or written at out + f_off[v].
__global__ void k_route_forced(uint32_t n, uint64_t ilim, uint64_t Fc, uint64_t Tc,
                               const unsigned long long *__restrict__ nb_off, const uint32_t *__restrict__ nb,
                               const unsigned long long *__restrict__ ly_off, const uint32_t *__restrict__ ly_end,
                               uint32_t *__restrict__ cnt, const unsigned long long *__restrict__ f_off,
                               uint32_t *__restrict__ out) {
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t base = nb_off[v], deg = nb_off[v + 1] - base;
        const uint64_t l0 = ly_off[v], nl = ly_off[v + 1] - l0;
        uint32_t prev = 0, c = 0;
        uint64_t at = out ? f_off[v] : 0;
        for (uint64_t i = 0; i < nl && i < ilim; ++i) {
            const uint32_t end = ly_end[l0 + i];
            if (prod_less(end - prev, Tc, Fc, deg)) {
                c += end - prev;
                if (out)
                    for (uint32_t k = prev; k < end; ++k) out[at++] = nb[base + k];
            }
            prev = end;
        }
        if (!out) cnt[v] = c;
    }
}

}  // namespace

int route_build(hyperim_graph g, hipStream_t s, uint32_t *n1) {
    *n1 = 0;
    g->routed = false;
    const uint32_t n = g->n;
    if (!g->lay_nb_off.ptr) {
        if (!g->chan.ptr) {
            DevBuf cnt, tmp;
            HIM_CHECK(channel_prefix(g, cnt, tmp, s));
            HIM_HIP(hipStreamSynchronize(s));
        }
        HIM_CHECK(layers_build_device(g, g->strat_lmax, s));
    }
    const uint64_t Fc = g->info.sum_top, Tc = g->info.sum_deg, ilim = n ? g->info.sum_l / n : 0;
    DevBuf cnt_b;
    HIM_CHECK(cnt_b.reserve(sizeof(uint32_t) * std::max<uint32_t>(n, 1), s));
    hipLaunchKernelGGL(k_route_forced, dim3(grid_for(n)), dim3(kBlock), 0, s, n, ilim, Fc, Tc,
                       g->lay_nb_off.as<unsigned long long>(), g->lay_nb.as<uint32_t>(),
                       g->lay_ly_off.as<unsigned long long>(), g->lay_ly_end.as<uint32_t>(), cnt_b.as<uint32_t>(),
                       (const unsigned long long *)nullptr, (uint32_t *)nullptr);
    HIM_HIP(hipGetLastError());
    std::vector<uint32_t> cnt(n), P(n);
    HIM_HIP(hipMemcpyAsync(cnt.data(), cnt_b.ptr, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s));
    HIM_HIP(hipMemcpyAsync(P.data(), g->P.ptr, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s));
    HIM_HIP(hipStreamSynchronize(s));
    uint32_t c1 = 0;
    for (uint32_t v = 0; v < n; ++v) c1 += cnt[v] != 0u;
    *n1 = c1;
    if (c1 == 0 || c1 == n) return HYPERIM_OK;   // inert: both pools over V
    // root lists: the R1 vertices in P's order, then the others; each
    // side's strata boundaries
    std::vector<uint32_t> rP(n);
    std::vector<uint64_t> f_off((size_t)n + 1, 0);
    for (uint32_t v = 0; v < n; ++v) f_off[v + 1] = f_off[v] + cnt[v];
    uint32_t a = 0, b = c1;
    uint32_t B[2][HYPERIM_NSTRATA + 1] = {};
    for (uint32_t h = 0; h < HYPERIM_NSTRATA; ++h) {
        B[0][h] = a;
        B[1][h] = b - c1;
        for (uint32_t i = g->info.B[h]; i < g->info.B[h + 1]; ++i) {
            const uint32_t v = P[i];
            if (cnt[v]) rP[a++] = v;
            else rP[b++] = v;
        }
    }
    B[0][HYPERIM_NSTRATA] = c1;
    B[1][HYPERIM_NSTRATA] = n - c1;
    const uint64_t total = f_off[n];
    HIM_CHECK(g->route_P.reserve(sizeof(uint32_t) * n, s));
    HIM_CHECK(g->force_off.reserve(sizeof(uint64_t) * ((size_t)n + 1), s));
    HIM_CHECK(g->force.reserve(sizeof(uint32_t) * std::max<uint64_t>(total, 1), s));
    HIM_HIP(hipMemcpyAsync(g->route_P.ptr, rP.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice, s));
    HIM_HIP(hipMemcpyAsync(g->force_off.ptr, f_off.data(), sizeof(uint64_t) * ((size_t)n + 1), hipMemcpyHostToDevice,
                           s));
    hipLaunchKernelGGL(k_route_forced, dim3(grid_for(n)), dim3(kBlock), 0, s, n, ilim, Fc, Tc,
                       g->lay_nb_off.as<unsigned long long>(), g->lay_nb.as<uint32_t>(),
                       g->lay_ly_off.as<unsigned long long>(), g->lay_ly_end.as<uint32_t>(), (uint32_t *)nullptr,
                       g->force_off.as<unsigned long long>(), g->force.as<uint32_t>());
    HIM_HIP(hipGetLastError());
    HIM_HIP(hipStreamSynchronize(s));   // the host vectors above are the copies' sources
    std::copy(&B[0][0], &B[0][0] + 2 * (HYPERIM_NSTRATA + 1), &g->route_B[0][0]);
    g->route_n1 = c1;
    g->routed = true;
    return HYPERIM_OK;
}

}  // namespace hyperim
