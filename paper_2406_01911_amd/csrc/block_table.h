// Per-workgroup aggregation of keyed counter updates in LDS.
//
// Counting kernels over incidences or co-member pairs hit the same vertex
// many times (hubs are members of ~1e5 hyperedges), and global atomics on one
// address serialise.  Each workgroup instead accumulates into an
// open-addressing table in LDS, keyed by vertex id, and adds every key's
// total to global memory once per chunk.  A key that finds no slot within
// kProbe probes falls back to the caller's global update.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hyperim {

constexpr uint32_t kTableEmpty = 0xFFFFFFFFu;

template <uint32_t kSlots>
struct BlockTable {
    static_assert((kSlots & (kSlots - 1)) == 0, "power of two");
    static constexpr uint32_t kProbe = 16;
    uint32_t key[kSlots];

    __device__ __forceinline__ void clear_keys() {
        for (uint32_t s = threadIdx.x; s < kSlots; s += blockDim.x) key[s] = kTableEmpty;
    }

    // Slot of `k` (inserted if absent), or kTableEmpty when the probe
    // sequence is full.
    __device__ __forceinline__ uint32_t slot(uint32_t k) {
        uint32_t h = (k * 0x9E3779B1u) & (kSlots - 1);
        for (uint32_t p = 0; p < kProbe; ++p) {
            const uint32_t cur = __hip_atomic_load(&key[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (cur == k) return h;
            if (cur == kTableEmpty) {
                const uint32_t prev = atomicCAS(&key[h], kTableEmpty, k);
                if (prev == kTableEmpty || prev == k) return h;
            }
            h = (h + 1) & (kSlots - 1);
        }
        return kTableEmpty;
    }
};

}  // namespace hyperim
