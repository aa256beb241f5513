// Device-side building blocks shared by the gfx950 kernels of libhyperim:
// the counter-based Philox4x32-10 generator (Salmon et al., SC'11) used for
// every coin and root offset, the channel-coin keying, and 64-lane wavefront
// primitives (scan, ballot ranks, broadcasts).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hyperim {

constexpr int kWave = 64;                 // CDNA wavefront width
constexpr uint32_t kAlways = 0xFFFFFFFFu; // threshold meaning "channel always live"
constexpr uint32_t kNStrata = 8;

// Philox4x32-10 block function: ten S-P rounds over a 128-bit counter, the
// 64-bit key advanced by the Weyl increments between rounds.  Each round
// multiplies counter words 0 and 2 by the Philox constants, keeps both halves
// of the 64-bit products and mixes the high halves with the other words and
// the key.
__host__ __device__ __forceinline__ uint4 philox4x32_10(uint4 ctr, uint2 key) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * (uint64_t)ctr.x;
        const uint64_t m2 = (uint64_t)0xCD9E8D57u * (uint64_t)ctr.z;
        uint4 next;
        next.x = (uint32_t)(m2 >> 32) ^ ctr.y ^ key.x;
        next.y = (uint32_t)m2;
        next.z = (uint32_t)(m0 >> 32) ^ ctr.w ^ key.y;
        next.w = (uint32_t)m0;
        ctr = next;
        key.x += 0x9E3779B9u;
        key.y += 0xBB67AE85u;
    }
    return ctr;
}

// Counter of the four coins of channels (he, u -> v) in RR set j whose
// source positions pos in he satisfy pos >> 2 == quad.  Word (pos & 3) of the
// block is the coin; pool tag in bit 31, bits 32..38 of j in bits 24..30.
__host__ __device__ __forceinline__ uint4 coin_counter(uint64_t j, uint32_t he, uint32_t v,
                                                       uint32_t pool, uint32_t quad) {
    return make_uint4((uint32_t)j, he, v, (pool << 31) | ((uint32_t)(j >> 32) << 24) | quad);
}

// Counter of the random offset of ladder block b of a pool (he and v words
// hold ids no hyperedge or vertex can take).
__host__ __device__ __forceinline__ uint4 root_counter(uint32_t b, uint32_t pool) {
    return make_uint4(b, 0xFFFFFFFFu, 0xFFFFFFFFu, pool);
}

__device__ __forceinline__ bool channel_live(uint32_t coin, uint32_t thr) {
    return thr == kAlways || coin < thr;
}

// ---- wavefront primitives --------------------------------------------------
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T y = __shfl_up(x, d, kWave);
        if (lane >= (uint32_t)d) x += y;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_max(T x) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        T y = __shfl_xor(x, d, kWave);
        x = y > x ? y : x;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_bcast(uint32_t x, int src) { return __shfl(x, src, kWave); }
__device__ __forceinline__ uint64_t wave_bcast64(uint64_t x, int src) {
    return (uint64_t)__shfl((unsigned long long)x, src, kWave);
}

// Wave-uniform values kept in scalar registers: the value of the first active
// lane (callers pass values that are equal on every active lane).
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | (uint64_t)uni((uint32_t)x);
}
template <typename P>
__device__ __forceinline__ P uni_ptr(P p) {
    return (P)uni64((uint64_t)p);
}

// Make this wave's earlier LDS and global writes visible to its own later
// reads by other lanes, and keep the compiler from moving memory accesses
// across the point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Smallest k in [0, 64) with scan[k] > g, for a 64-entry nondecreasing array
// whose last entry exceeds g.
__device__ __forceinline__ uint32_t search64(const uint32_t *scan, uint32_t g) {
    uint32_t k = 0;
#pragma unroll
    for (uint32_t s = 32; s > 0; s >>= 1)
        if (scan[k + s - 1] <= g) k += s;
    return k;
}

__host__ __device__ __forceinline__ uint64_t div_up(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

}  // namespace hyperim
