// Work-item layout of the grid-wide RR-generation planners (k_plan and
// k_ms_plan) and the progress rules of the host loops that drive them.
//
// A planning wave takes up to 64 frontier entries.  Light entries (at most
// `chunk` incidences of work) form segments of consecutive entries; a heavy
// entry is cut into chunks of its incidence range.  The items of a batch are
// the segments first, then the heavy chunks in lane order.  These helpers are
// the arithmetic of that layout; the device planners call them with lane
// shuffles as the scan reader, and the host model the CPU tests exercise
// calls them with plain arrays.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hyperim {

constexpr uint32_t kPlanItemCap = 1u << 22;          // work items per superstep
constexpr uint32_t kPlanMaxItemsPerVertex = 1u << 20;  // per-set mode: chunks of one vertex at most

// ceil(a / b) without overflow for a near 2^32
__host__ __device__ __forceinline__ uint32_t plan_div_up(uint32_t a, uint32_t b) {
    return (uint32_t)(((uint64_t)a + b - 1u) / b);
}

// Per-set mode: a vertex of `deg` incidences is heavy when deg > chunk; its
// chunks are `len` incidences long (chunk, grown so that one vertex never
// needs more than kPlanMaxItemsPerVertex items) and there are `count` of them.
struct HeavySplit {
    uint32_t len, count;
};
__host__ __device__ __forceinline__ HeavySplit heavy_split(uint32_t deg, uint32_t chunk) {
    const uint32_t a = plan_div_up(deg, kPlanMaxItemsPerVertex);
    const uint32_t len = chunk > a ? chunk : a;
    HeavySplit h;
    h.len = len;
    h.count = deg > chunk ? plan_div_up(deg, len) : 0u;
    return h;
}

// Bundled mode: an entry's work is its incidences times the sets in its mask;
// chunks of about `chunk` (incidence, set) pairs, i.e. chunk / sets
// incidences (at least 1), and at most kPlanItemCap / 128 chunks per entry so
// that any batch of 64 entries fits an empty item buffer.  The entry is heavy
// when deg exceeds the chunk length.
__host__ __device__ __forceinline__ HeavySplit ms_heavy_split(uint32_t deg, uint32_t sets, uint32_t chunk) {
    const uint32_t per = chunk / (sets > 1u ? sets : 1u);
    const uint32_t c = per > 1u ? per : 1u;
    const uint32_t a = plan_div_up(deg, kPlanItemCap / 128u);
    HeavySplit h;
    h.len = c > a ? c : a;
    h.count = deg > h.len ? plan_div_up(deg, h.len) : 0u;
    return h;
}

// Segment of a light entry: floor(light incidences before it / seg).  With
// every light weight <= seg, segments have no gaps and each holds fewer than
// 2 seg incidences of work.
__host__ __device__ __forceinline__ uint32_t segment_of(uint32_t light_incl, uint32_t light, uint32_t seg) {
    return (light_incl - light) / seg;
}

// Owner of heavy-chunk slot q: lane k owns slots [scan(k) - count_k, scan(k))
// of the batch's heavy chunks, where scan(k) is the inclusive scan of the
// per-lane counts; the owner is the first lane whose scan exceeds q (q must
// be below scan(63)).  Binary search over the 64 scan values through the
// reader `at`.
template <class Reader>
__host__ __device__ __forceinline__ uint32_t scan_owner(Reader at, uint32_t q) {
    uint32_t k = 0;
    for (uint32_t s = 32; s > 0; s >>= 1)
        if (at(k + s - 1u) <= q) k += s;
    return k;
}

// Incidence range [lo, hi) of chunk r of a heavy vertex whose incidences are
// [e0, e0 + deg), cut into chunks of `len`.
struct ChunkRange {
    uint32_t lo, hi;
};
__host__ __device__ __forceinline__ ChunkRange chunk_range(uint32_t e0, uint32_t deg, uint32_t len, uint32_t r) {
    ChunkRange c;
    c.lo = e0 + r * len;
    const uint32_t end = e0 + deg;
    const uint64_t hi = (uint64_t)c.lo + len;   // no wrap near the end of a 2^32-incidence graph
    c.hi = hi < end ? (uint32_t)hi : end;
    return c;
}

// ---- progress of the host loops ---------------------------------------------
// Outcome of one check of a superstep loop.
enum LoopCheck : int { kLoopContinue = 0, kLoopDone = 1, kLoopStalled = 2, kLoopOverBound = 3 };

// Per-set mode, after a batch of supersteps.  `planned` is the device's
// running count of frontier entries the planner has taken (the sum of the
// deferred sets' queue heads), `items_last` the items planned by the batch's
// last superstep.  A superstep with items always takes at least one entry
// (the first reservation of a superstep fits the empty item buffer), so a
// batch whose last superstep still had items must have raised `planned`;
// `planned` can never exceed `entries_cap`, the members the deferred sets
// can hold.
__host__ __device__ __forceinline__ int phase_b_check(uint64_t planned_before, uint64_t planned, uint64_t items_last,
                                                      uint64_t entries_cap) {
    if (items_last == 0) return kLoopDone;
    if (planned > entries_cap) return kLoopOverBound;
    if (planned <= planned_before) return kLoopStalled;
    return kLoopContinue;
}

// Bundled mode, after a batch of steps.  Every step either plans at least
// one pending batch of the level's frontier or, when none is pending,
// finishes the level (its epoch advances); the loop ends once a level starts
// with no frontier (`done`).  So (epoch, pending) must change across a batch,
// and levels cannot outnumber `level_cap`.
__host__ __device__ __forceinline__ int bundled_check(uint64_t epoch_before, uint64_t pending_before, uint64_t epoch,
                                                      uint64_t pending, uint64_t done, uint64_t level_cap) {
    if (done) return kLoopDone;
    if (epoch > level_cap) return kLoopOverBound;
    if (epoch == epoch_before && pending >= pending_before) return kLoopStalled;
    return kLoopContinue;
}

}  // namespace hyperim
