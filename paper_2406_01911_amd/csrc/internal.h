// Host-side internals of libhyperim: handle layouts, device workspaces and
// the launchers each kernel file exports to the API layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "hyperim.h"

namespace hyperim {

// Status plumbing -------------------------------------------------------------
void set_error_detail(const std::string &msg);
void clear_error_detail();

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

// Growable device buffer (never shrinks); frees its memory when destroyed.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    int reserve(size_t need, hipStream_t s, bool keep = false);
    void release();
    template <typename T>
    T *as() const { return static_cast<T *>(ptr); }
};

// Workspace of RR generation: one per device, shared by every graph on it
// (calls that use it hold its lock).
struct RRWorkspace {
    uint32_t waves = 0;          // phase A wavefronts (each starts with its own slot)
    uint32_t grid = 0;           // workgroups of the phase A launch
    uint32_t slots = 0;          // slots: phase A waves + spare slots for deferred sets
    uint32_t grid_b = 0;         // workgroups of a phase B expansion launch
    uint32_t cus = 0;            // compute units of the device
    uint32_t slot_n = 0, slot_words = 0;  // slot list length / bitmap words (largest graph so far)
    bool lds = false;            // phase A bitmaps in LDS (every graph small)
    DevBuf lists;                // slots * slot_n     : member list / BFS queue per slot
    DevBuf bitmaps;              // slots * slot_words : visited bitmap per slot
    DevBuf def_idx;              // deferred sets: launch index (uint64)
    DevBuf def_u32;              // deferred sets: root, slot, head, size, task (5 uint32 arrays)
    DevBuf graph_desc, task_desc;  // launch-group descriptors in device memory
    DevBuf items;                // phase B work items (uint4)
    // bundled mode: per-bundle seen / found masks, frontier and next-level
    // lists, batch marks, output counts, counters
    DevBuf ms_seen, ms_nxt, ms_cur, ms_next, ms_batch, ms_vcnt, ms_ctr;
    DevBuf picks;                // stratified setting: per-lane pick lists
    DevBuf counters;             // work counter, stage bump, misc
    DevBuf stage;                // unsorted->sorted members before compaction
    DevBuf stage_off;            // per id (uint64)
    DevBuf sizes;                // per id (uint32)
    DevBuf roots;                // per id (uint32)
    DevBuf scan_tmp;             // scan block sums
    DevBuf big_ids;              // per-id indices of sets compacted by whole workgroups
    std::vector<hipEvent_t> events;  // start/stop pairs around RR-generation launches
    DevBuf args_dev;             // arguments of the grid-wide phase kernels (device copy)
    // superstep batches captured as HIP graphs, replayed while a traversal
    // lasts; keyed by everything a capture bakes in
    struct BatchGraph {
        uint64_t key[8];
        hipGraphExec_t exec;
    };
    std::vector<BatchGraph> batch_graphs;
    hipStream_t capture = nullptr;   // stream the batches are captured on
    bool graphs_off = false;         // capture failed on this device: launch kernels directly
    void drop_graphs();
    unsigned long long *host = nullptr;  // pinned host staging: counter copies, descriptors, totals
    size_t host_words = 0;
    size_t bytes() const;        // device memory held
    void release();
};

// What one generation call did (device times from HIP events).
struct RRStats {
    double ms_bfs = 0.0, ms_light = 0.0, ms_heavy = 0.0;  // all / phase A / phase B kernels
    uint64_t launches = 0, supersteps = 0, deferred = 0;
    uint64_t bytes_light = 0, bytes_heavy = 0;   // algorithmic bytes expanded in each phase
    double ms_expand = 0.0;                      // k_expand launches alone
    uint64_t expand_launches = 0;
    double ms_bundled = 0.0;                     // k_ms_expand launches alone
    uint64_t bundled_launches = 0;
    uint64_t bytes_bundled = 0;                  // algorithmic bytes expanded in bundled mode
    uint64_t philox = 0;                         // Philox4x32-10 blocks drawn (all kernels)
    uint64_t philox_light = 0;                   // ... of which in the per-set phase
    uint64_t philox_bundled = 0;                 // ... of which in bundled mode
};

// Workspace of greedy / coverage: one per device, shared by every graph on it.
struct GreedyWorkspace {
    DevBuf cnt;       // n uint32  marginal coverage
    DevBuf inv_off;   // (n+1) uint64
    DevBuf cursor;    // n uint32
    DevBuf inv;       // entries uint32 (set ids)
    DevBuf covered;   // theta uint32: 0 or covering round + 1
    DevBuf chosen;    // n uint8
    DevBuf best;      // k uint64 argmax keys + per-round counters
    DevBuf out;       // k seeds (uint32) then k gains (uint64)
    DevBuf big;       // sets above the big-set size (whole pool prefix)
    DevBuf cursor_big; // n uint32: big sets per vertex (inverted index)
    DevBuf flags;     // n uint8 seed marks (coverage)
    DevBuf counters;  // coverage counters
    DevBuf scan_tmp;
    DevBuf topk;      // Equation (8): bin counts and sums, selection state, k + 1 top-k sums
    DevBuf params;    // argument block of the per-round kernels
    alignas(16) unsigned char params_host[256];
    // captured graph of the k greedy rounds and what it was captured for
    hipStream_t capture = nullptr;
    hipGraphExec_t rounds_exec = nullptr;
    uint32_t graph_k = 0, graph_grid[2] = {0, 0}, graph_levels = 0;
    void *graph_params = nullptr;
    size_t bytes() const;
    void release();
};

// Workspace of graph building and stratification: one per device, kept
// between calls (the hash tables take up to 5 GB, and allocating and freeing
// them per call cost more than a small graph's kernels).
struct PrepWorkspace {
    DevBuf k1, vals, k2;                   // (v,u) weight and (v,w) layer hash tables
    DevBuf wmax, pc, tmp;                  // per-vertex maxima, pair prefix sums, scan blocks
    DevBuf counts, base, isum, lmax, hist; // strata counts and statistics
    DevBuf flag, cnt, off64, lists, bm;    // graph build: checks, degrees, offsets, sort lists and marks
    size_t bytes() const;
    void release();
};

// The device's shared workspaces (RR generation, greedy / coverage,
// stratification), locked for the holder's lifetime.
struct DeviceLock {
    RRWorkspace *rr;
    GreedyWorkspace *gr;
    PrepWorkspace *prep;
    void *lock;
    explicit DeviceLock(int device);
    ~DeviceLock();
    DeviceLock(const DeviceLock &) = delete;
    DeviceLock &operator=(const DeviceLock &) = delete;
};

}  // namespace hyperim

struct hyperim_graph_s {
    int device = 0;
    uint32_t n = 0, m = 0;
    uint64_t nnz = 0;
    hyperim_prob prob{};
    bool lt() const { return prob.model == HYPERIM_MODEL_LT_CONST || prob.model == HYPERIM_MODEL_LT_WC; }
    bool layered() const { return prob.model == HYPERIM_MODEL_LAYERED; }   // stratified setting
    // independent cascade drawn by geometric gaps
    bool gaps() const { return prob.model == HYPERIM_MODEL_GAPS_CONST || prob.model == HYPERIM_MODEL_GAPS_WC; }
    // RR-set kernel family: 0 independent cascade by coins, 1 linear
    // threshold, 2 stratified setting, 3 independent cascade by gaps
    int kind() const { return gaps() ? 3 : layered() ? 2 : lt() ? 1 : 0; }
    // weight = d(v) + S(v) incidences read when v is expanded; bytesw = 20 + 12 d(v) + 4 S(v)
    // algorithmic bytes of v as an RR-set member (d = hyperedges of v, S = their total size);
    // phiw = sum over v's hyperedges of ceil(|he| / 4), the Philox blocks of v's expansion
    // v_hbs[e] = (he_off[v_he[e]], size of that hyperedge), uint2 per incidence
    // chan (linear-threshold graphs only): exclusive prefix over v_he of the
    // incidences' channel counts |he| - 1, nnz + 1 entries
    hyperim::DevBuf he_off, he_mem, v_off, v_he, thr, c, weight, bytesw, phiw, v_hbs, chan;
    // stratified setting (built by stratify): A(v) by layers -- members
    // lay_nb[lay_nb_off[v] ..], layer i ending at lay_nb_off[v] +
    // lay_ly_end[lay_ly_off[v] + i - 1] -- and the host-evaluated tables
    // lay_ln[l] = ln(l + 1), lay_expm[l (l - 1) / 2 + i - 1] = e^-P(L_i)
    hyperim::DevBuf lay_nb_off, lay_nb, lay_ly_off, lay_ly_end, lay_ln, lay_expm;
    uint32_t lay_lmax = 0;
    bool stratified = false;
    uint32_t strat_lmax = 0;   // largest l_v (set by stratify)
    // division of the RR sets into R1 / R2 (Section 4.1; hyperim_route):
    // route_on = asked for (kept across stratify), routed = in effect (both
    // sides non-empty); pool 0 roots route_P[0 .. route_n1), pool 1 the rest,
    // each side's strata ending at route_B[side][h]; a pool-0 set of root v
    // starts with force[force_off[v] .. force_off[v + 1])
    bool route_on = false, routed = false;
    uint32_t route_n1 = 0;
    uint32_t route_B[2][HYPERIM_NSTRATA + 1] = {};
    hyperim::DevBuf route_P, force_off, force;
    hyperim::DevBuf l, deg, top, stratum, P;
    hyperim_strata_info info{};
    hyperim_tuning tune{1024, 262144, 256, 512, 0xFFFFFFFFu, 8, 16384, 4, 6, 0xFFFFFFFFu, 1};  // RR execution parameters
    // learned from generated sets (launch-group and stage sizing, admission);
    // -1 = nothing generated yet
    bool rr_used = false;   // RR sets have been generated on this graph
    double rr_members = -1.0, rr_defer = -1.0;
    uint64_t rr_seen_sets = 0, rr_seen_members = 0;
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

constexpr uint64_t kMaxIds = 1ull << 39;   // RR ids use 39 bits of the coin counter
constexpr uint32_t kMaxVertices = 1u << 31; // ids < 2^31: bit 31 of a queue entry marks it expanded
constexpr uint32_t kDefaultQlog = 8;       // pool ladder base Q = 2^8

inline hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

// The graph must live on the current device.
inline int check_device(hyperim_graph g) {
    int d = 0;
    HIM_HIP(hipGetDevice(&d));
    if (d != g->device) {
        set_error_detail("the graph lives on another device than the current one");
        return HYPERIM_EINVAL;
    }
    return HYPERIM_OK;
}

// ---- handles and storage (api.hip) --------------------------------------------
size_t graph_bytes(hyperim_graph g);                       // device bytes of the graph
int pool_init_owned(hyperim_graph g, hyperim_pool p, hipStream_t s);
// Current bytes of the device's shared workspaces: RR slots (lists and
// bitmaps), RR stage and per-set arrays, greedy / coverage.
struct SharedBytes {
    size_t slots, stage, greedy, prep, total;
};
SharedBytes shared_bytes();
void pool_clear(hyperim_pool p);                           // empty, keeps storage
void pool_release(hyperim_pool p);                         // empty, frees owned storage
size_t pool_bytes(const hyperim_pool_s &p);
struct RRStats;
struct RRTask;
// Generate tasks[i] into pools[i] (one generation pass; tasks with empty
// ranges skipped).  With pool_status, a pool that would exceed max_entries
// gets HYPERIM_ECAPACITY there and the others are still filled; without it
// that status is returned.
// time_kernels: time every expansion-kernel launch (RRStats::ms_expand).
// graphs: replay captured superstep batches (HIP graphs) where the device allows.
int generate_into(const std::vector<RRTask> &tasks, const std::vector<hyperim_pool> &pools, uint32_t qlog, int form,
                  uint64_t max_entries, hipStream_t s, RRStats &st, std::vector<int> *pool_status,
                  bool time_kernels = false, bool graphs = true);

// ---- launchers (graph.hip) --------------------------------------------------
int graph_build_device(hyperim_graph g, PrepWorkspace &w, hipStream_t s);
// chan of g (the channel prefix over its incidences); cnt / tmp: scratch
int channel_prefix(hyperim_graph g, DevBuf &cnt, DevBuf &tmp, hipStream_t s);

// ---- launchers (route.hip) ------------------------------------------------------
// Division of g's RR sets into R1 / R2 (Section 4.1) from its strata and
// layer tables (built here when missing); sets route_P, force_off, force,
// route_n1, route_B and routed.  *n1 = the number of R1 vertices.
int route_build(hyperim_graph g, hipStream_t s, uint32_t *n1);

// ---- launchers (stratify.hip) -------------------------------------------------
int stratify_device(hyperim_graph g, PrepWorkspace &w, hipStream_t s);
// Stratified-setting tables of a stratified graph (layers.hip); lmax = largest l_v.
int layers_build_device(hyperim_graph g, uint32_t lmax, hipStream_t s);

// ---- launchers (scan.hip) -----------------------------------------------------
// out[0..count] = exclusive prefix sums of in[0..count) plus init; out[count] = total.
int scan_u32_to_u64(const uint32_t *in, uint64_t *out, uint64_t count, uint64_t init, DevBuf &tmp,
                    hipStream_t s);
int scan_u64(const uint64_t *in, uint64_t *out, uint64_t count, uint64_t init, DevBuf &tmp, hipStream_t s);

// ---- launchers (rr.hip) -------------------------------------------------------
// RR ids [id_begin, id_end) of pool tag `pool` on graph g, Philox key
// (seed mod 2^32, instance).
struct RRTask {
    hyperim_graph g;
    uint64_t seed;
    uint32_t instance, pool;
    uint64_t id_begin, id_end;
};
// Generate tasks[i]'s RR sets and append them to pools[i].  Tasks may name
// different (stratified) graphs on the current device.  form 0 = the tasks
// share launch groups, form 1 = launch groups per (task, ladder block,
// stratum).  Each launch group is compacted into its pools before the next
// one runs; groups are cut so their staged members stay near stage_budget
// bytes.  pool_status[i] = HYPERIM_ECAPACITY when pools[i] would exceed
// max_entries (its remaining sets are dropped; the other pools go on).
// Bytes of slot lists and bitmaps the workspace holds for graphs of up to
// n_max vertices.
size_t rr_slot_bytes(uint32_t n_max);
int rr_generate_into(RRWorkspace &ws, RRStats &st, const std::vector<RRTask> &tasks,
                     const std::vector<hyperim_pool> &pools, uint32_t qlog, int form, uint64_t max_entries,
                     uint64_t stage_budget, hipStream_t s, std::vector<int> &pool_status, bool time_kernels,
                     bool graphs);
// Make room in pool p for `ids` more ids and `entries` more members.
int pool_reserve(hyperim_pool p, uint64_t ids, uint64_t entries, hipStream_t s);
// Work of the pool's first theta sets, summed over their members v:
// incidences d(v) + S(v), algorithmic bytes, coins S(v) - d(v) = c(v) and
// Philox blocks sum over v's hyperedges of ceil(|he| / 4).
struct RRWork {
    uint64_t incidences = 0, alg_bytes = 0, coins = 0, philox = 0;
};
int rr_incidences(hyperim_graph g, hyperim_pool p, uint64_t theta, hipStream_t s, RRWork *out);

// ---- launchers (greedy.hip) ---------------------------------------------------
// Greedy max coverage of the pool's first theta sets; the seeds also stay in
// w.out (device) for coverage_device.
// ub_host (k + 1 entries, may be null): for i = 0..k the sum of the k largest
// marginal coverages given the first i seeds (Equation (8)'s terms).
int greedy_device(GreedyWorkspace &w, hyperim_graph g, hyperim_pool p, uint64_t theta, uint32_t k, hipStream_t s,
                  uint32_t *seeds_host, uint64_t *gains_host, uint64_t *ub_host = nullptr);
int coverage_device(GreedyWorkspace &w, hyperim_graph g, hyperim_pool p, uint64_t theta, const uint32_t *seeds_dev,
                    uint32_t k, hipStream_t s, uint64_t *covered_host);

// ---- host schedule (theta.cpp logic lives in api.hip) ---------------------------
uint32_t query_cu_count();

}  // namespace hyperim
