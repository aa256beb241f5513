// Device-wide exclusive prefix sums (three passes: tile sums, a single-block
// scan of the tile sums, tile-local scans plus the tile prefix).  Integer
// sums, so the result is independent of scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dev_common.h"
#include "internal.h"

namespace hyperim {
namespace {

constexpr int kBlock = 256;
constexpr int kItems = 8;                  // items per thread
constexpr int kTile = kBlock * kItems;     // 2048 items per tile

template <typename In>
__global__ __launch_bounds__(kBlock) void k_tile_sums(const In *__restrict__ in, uint64_t count,
                                                       uint64_t *__restrict__ sums) {
    __shared__ uint64_t part[kBlock / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    uint64_t acc = 0;
    for (int i = 0; i < kItems; ++i) {
        uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
        if (idx < count) acc += (uint64_t)in[idx];
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += part[w];
        sums[blockIdx.x] = t;
    }
}

// One workgroup scans the tile sums in place (exclusive, plus init).
__global__ __launch_bounds__(kBlock) void k_scan_sums(uint64_t *__restrict__ sums, uint64_t tiles, uint64_t init,
                                                       uint64_t *__restrict__ total_out) {
    __shared__ uint64_t part[kBlock / kWave];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = init;
    __syncthreads();
    const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    for (uint64_t base = 0; base < tiles; base += kBlock) {
        uint64_t idx = base + threadIdx.x;
        uint64_t x = idx < tiles ? sums[idx] : 0;
        uint64_t incl = wave_incl_scan(x);
        if (lane == kWave - 1) part[wv] = incl;
        __syncthreads();
        uint64_t before = carry;
        for (uint32_t w = 0; w < wv; ++w) before += part[w];
        if (idx < tiles) sums[idx] = before + incl - x;
        __syncthreads();
        if (threadIdx.x == kBlock - 1) carry = before + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total_out = carry;
}

template <typename In>
__global__ __launch_bounds__(kBlock) void k_tile_scan(const In *__restrict__ in, uint64_t count,
                                                       const uint64_t *__restrict__ sums,
                                                       uint64_t *__restrict__ out) {
    __shared__ uint64_t part[kBlock / kWave];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = sums[blockIdx.x];
    __syncthreads();
    const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const uint64_t base = (uint64_t)blockIdx.x * kTile;
    for (int i = 0; i < kItems; ++i) {
        uint64_t idx = base + (uint64_t)i * kBlock + threadIdx.x;
        uint64_t x = idx < count ? (uint64_t)in[idx] : 0;
        uint64_t incl = wave_incl_scan(x);
        if (lane == kWave - 1) part[wv] = incl;
        __syncthreads();
        uint64_t before = carry;
        for (uint32_t w = 0; w < wv; ++w) before += part[w];
        if (idx < count) out[idx] = before + incl - x;
        __syncthreads();
        if (threadIdx.x == kBlock - 1) carry = before + incl;
        __syncthreads();
    }
}

template <typename In>
int scan_impl(const In *in, uint64_t *out, uint64_t count, uint64_t init, DevBuf &tmp, hipStream_t s) {
    const uint64_t tiles = std::max<uint64_t>(div_up(count, kTile), 1);
    HIM_CHECK(tmp.reserve(sizeof(uint64_t) * (tiles + 1), s));
    uint64_t *sums = tmp.as<uint64_t>();
    if (count)
        hipLaunchKernelGGL(k_tile_sums<In>, dim3((uint32_t)tiles), dim3(kBlock), 0, s, in, count, sums);
    else
        HIM_HIP(hipMemsetAsync(sums, 0, sizeof(uint64_t), s));
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kBlock), 0, s, sums, tiles, init, out + count);
    if (count)
        hipLaunchKernelGGL(k_tile_scan<In>, dim3((uint32_t)tiles), dim3(kBlock), 0, s, in, count, sums, out);
    HIM_HIP(hipGetLastError());
    return HYPERIM_OK;
}

}  // namespace

int scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t count, uint64_t init, DevBuf &tmp,
                    hipStream_t s) {
    return scan_impl<uint32_t>(in, out, count, init, tmp, s);
}

int scan_u64(const uint64_t *in, uint64_t *out, uint64_t count, uint64_t init, DevBuf &tmp, hipStream_t s) {
    return scan_impl<uint64_t>(in, out, count, init, tmp, s);
}

}  // namespace hyperim
