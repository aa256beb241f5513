// Host-side internals of libhyperim: handle layouts, device workspaces and
// the launchers each kernel file exports to the API layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/hyperim.h"

namespace hyperim {

// Status plumbing -------------------------------------------------------------
void set_error_detail(const std::string &msg);

#define HIM_HIP(expr)                                                              \
    do {                                                                           \
        hipError_t _e = (expr);                                                    \
        if (_e != hipSuccess) {                                                    \
            ::hyperim::set_error_detail(std::string(#expr) + ": " + hipGetErrorString(_e)); \
            return HYPERIM_EHIP;                                                   \
        }                                                                          \
    } while (0)

#define HIM_CHECK(expr)                 \
    do {                                \
        int _rc = (expr);               \
        if (_rc != HYPERIM_OK) return _rc; \
    } while (0)

// Growable device buffer (never shrinks). ---------------------------------------
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int reserve(size_t need, hipStream_t s, bool keep = false);
    void release();
    template <typename T>
    T *as() const { return static_cast<T *>(ptr); }
};

// Workspace of RR generation, owned by a graph.
struct RRWorkspace {
    uint32_t waves = 0;          // phase A wavefronts (each starts with its own slot)
    uint32_t grid = 0;           // workgroups of the phase A launch
    uint32_t slots = 0;          // slots: phase A waves + spare slots for deferred sets
    uint32_t grid_b = 0;         // workgroups of a phase B expansion launch
    DevBuf lists;                // slots * n     : member list / BFS queue per slot
    DevBuf bitmaps;              // slots * words : visited bitmap per slot
    DevBuf def_idx;              // deferred sets: per-id index (uint64)
    DevBuf def_u32;              // deferred sets: root, slot, head, size (4 uint32 arrays)
    DevBuf items;                // phase B work items (uint4)
    double ms_light = 0.0, ms_heavy = 0.0;   // device time of phase A / phase B kernels
    hyperim_tuning tune{1024, 16384, 256, 512, 4096, 8, {0, 0}};  // execution parameters
    double members_per_id = 0.0;  // staged members per RR id in the last call (stage sizing)
    double defer_rate = 0.5;      // deferred sets per RR id in the last call (launch-group sizing)
    uint64_t supersteps = 0, deferred = 0;
    uint64_t bytes_light = 0, bytes_heavy = 0;  // algorithmic bytes expanded in each phase
    DevBuf counters;             // work counter, stage bump, misc
    DevBuf stage;                // unsorted->sorted members before compaction
    DevBuf stage_off;            // per id (uint64)
    DevBuf sizes;                // per id (uint32)
    DevBuf roots;                // per id (uint32)
    DevBuf scan_tmp;             // scan block sums
    DevBuf big_ids;              // per-id indices of sets compacted by whole workgroups
    std::vector<hipEvent_t> events;  // start/stop pairs around RR-generation launches
    double ms_bfs = 0.0;         // accumulated device time of those launches
    uint64_t launches = 0;
};

// Workspace of greedy / coverage, owned by a graph.
struct GreedyWorkspace {
    DevBuf cnt;       // n uint32  marginal coverage
    DevBuf inv_off;   // (n+1) uint64
    DevBuf cursor;    // n uint32
    DevBuf inv;       // entries uint32 (set ids)
    DevBuf covered;   // theta uint8
    DevBuf chosen;    // n uint8
    DevBuf best;      // k uint64 argmax keys + per-round counters
    DevBuf out;       // k seeds (uint32) then k gains (uint64)
    DevBuf big;       // sets above the big-set size (whole pool prefix)
    DevBuf round_big; // big sets covered in one round
    DevBuf flags;     // n uint8 seed marks (coverage)
    DevBuf counters;  // coverage counters
    DevBuf scan_tmp;
};

}  // namespace hyperim

struct hyperim_graph_s {
    int device = 0;
    uint32_t n = 0, m = 0;
    uint64_t nnz = 0;
    hyperim_prob prob{};
    // weight = d(v) + S(v) incidences read when v is expanded; bytesw = 20 + 12 d(v) + 4 S(v)
    // algorithmic bytes of v as an RR-set member (d = hyperedges of v, S = their total size)
    hyperim::DevBuf he_off, he_mem, v_off, v_he, thr, c, weight, bytesw;
    bool stratified = false;
    hyperim::DevBuf l, deg, top, stratum, P;
    hyperim_strata_info info{};
    hyperim::RRWorkspace rr;
    hyperim::GreedyWorkspace gr;
};

struct hyperim_pool_s {
    hyperim_graph g = nullptr;
    bool owned = true;
    char *buf = nullptr;       // caller buffer when !owned
    size_t bytes = 0;
    hyperim::DevBuf off_b, roots_b, mem_b;  // owned storage
    uint64_t *off = nullptr;   // count+1
    uint32_t *roots = nullptr; // count
    uint32_t *mem = nullptr;   // total
    uint64_t id_cap = 0, mem_cap = 0;
    uint64_t id_begin = 0, count = 0, total = 0;
    bool has_key = false;
    uint64_t seed = 0;
    uint32_t instance = 0, tag = 0;
    size_t required = 0;
};

namespace hyperim {

// ---- launchers (graph.hip) --------------------------------------------------
int graph_build_device(hyperim_graph g, hipStream_t s);

// ---- launchers (stratify.hip) -------------------------------------------------
int stratify_device(hyperim_graph g, hipStream_t s);

// ---- launchers (scan.hip) -----------------------------------------------------
// out[0..count] = exclusive prefix sums of in[0..count) plus init; out[count] = total.
int scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t count, uint64_t init, DevBuf &tmp,
                    hipStream_t s);
int scan_u64(const uint64_t *in, uint64_t *out, uint64_t count, uint64_t init, DevBuf &tmp, hipStream_t s);

// ---- launchers (rr.hip) -------------------------------------------------------
struct RRKey {
    uint64_t seed;
    uint32_t instance, qlog;
};
// RR ids [id_begin, id_end) of pool tag `pool`.
struct RRTask {
    uint32_t pool;
    uint64_t id_begin, id_end;
};
// Generate every task's RR sets into the workspace stage (per-id outputs laid
// out task after task); *total = members staged.  form 0 = all tasks in one
// launch group, form 1 = one launch group per (task, ladder block, stratum).
int rr_generate_stage(hyperim_graph g, const RRKey &key, const std::vector<RRTask> &tasks, int form, hipStream_t s,
                      uint64_t *total);
// Append the staged sets with per-id indices [first, first + count) to pool p
// (growing its storage; HYPERIM_ECAPACITY beyond max_entries or a caller buffer).
int rr_compact_into(hyperim_graph g, hyperim_pool p, uint64_t first, uint64_t count, uint64_t max_entries,
                    hipStream_t s);
// Make room in pool p for `ids` more ids and `entries` more members.
int pool_reserve(hyperim_pool p, uint64_t ids, uint64_t entries, hipStream_t s);
// Sums of weight[] (incidences) and bytesw[] (algorithmic bytes) over the
// members of the pool's first theta sets.
int rr_incidences(hyperim_graph g, hyperim_pool p, uint64_t theta, hipStream_t s, uint64_t *incidences,
                  uint64_t *alg_bytes);

// ---- launchers (greedy.hip) ---------------------------------------------------
int greedy_device(hyperim_graph g, hyperim_pool p, uint64_t theta, uint32_t k, hipStream_t s,
                  uint32_t *seeds_host, uint64_t *gains_host);
int coverage_device(hyperim_graph g, hyperim_pool p, uint64_t theta, const uint32_t *seeds_dev, uint32_t k,
                    hipStream_t s, uint64_t *covered_host);

// ---- host schedule (theta.cpp logic lives in api.hip) ---------------------------
uint32_t query_cu_count();

}  // namespace hyperim
