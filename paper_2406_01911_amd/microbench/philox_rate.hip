// Throughput of the library's Philox4x32-10 block function on the device:
// every lane draws `iters` blocks with distinct counters under a
// wave-uniform key (as the RR kernels do: the key lives in scalar
// registers), the outputs are folded into one word per lane so that no block
// is dead code.  The launch fills every compute unit at full occupancy.
// Built as its own small library (not part of libhyperim.so) and driven by
// the benchmark, which reports blocks/s beside the Philox work of the RR
// kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../csrc/dev_common.h"

using namespace hyperim;

__global__ __launch_bounds__(256) void k_philox_rate(uint32_t iters, uint32_t key0, uint32_t key1, uint32_t *out) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint2 key = make_uint2(uni(key0), uni(key1));
    uint32_t acc = 0;
    for (uint32_t i = 0; i < iters; ++i) {
        const uint4 r = philox4x32_10(make_uint4(tid, i, tid ^ 0x5bd1e995u, i >> 2), key);
        acc ^= r.x ^ r.y ^ r.z ^ r.w;
    }
    out[tid] = acc;
}

// Runs `reps` timed launches of blocks_per_cu workgroups of 256 lanes per
// compute unit, `iters` blocks per lane; *blocks_per_s receives the best
// rate, *ms the best launch time, *blocks the blocks of one launch.
// Returns 0 or a HIP error code.
extern "C" int philox_rate(uint32_t iters, uint32_t blocks_per_cu, uint32_t reps, double *blocks_per_s, double *ms,
                           double *blocks) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return (int)e;
    const uint32_t grid = (uint32_t)cus * blocks_per_cu;
    const size_t lanes = (size_t)grid * 256;
    uint32_t *out = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    if ((e = hipMalloc(&out, lanes * sizeof(uint32_t))) != hipSuccess) return (int)e;
    if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
        if (a) (void)hipEventDestroy(a);
        (void)hipFree(out);
        return (int)e;
    }
    hipLaunchKernelGGL(k_philox_rate, dim3(grid), dim3(256), 0, nullptr, 16u, 1u, 2u, out);   // warm-up
    float best = 0.f;
    for (uint32_t r = 0; r < reps && e == hipSuccess; ++r) {
        e = hipEventRecord(a, nullptr);
        hipLaunchKernelGGL(k_philox_rate, dim3(grid), dim3(256), 0, nullptr, iters, 1u + r, 2u, out);
        if (e == hipSuccess) e = hipEventRecord(b, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
        if (e == hipSuccess && (r == 0 || t < best)) best = t;
    }
    if (e == hipSuccess) e = hipGetLastError();
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(out);
    if (e != hipSuccess) return (int)e;
    *blocks = (double)lanes * (double)iters;
    *ms = best;
    *blocks_per_s = *blocks / (best * 1e-3);
    return 0;
}
