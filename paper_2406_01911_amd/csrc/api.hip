// C ABI of libhyperim (declared in include/hyperim.h): handles, argument
// validation, pool storage, the per-device RR workspace and the single-call
// entry points.  The HyperIM_BRR loop (Algorithm 4) lives in query.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "dev_common.h"
#include "internal.h"

namespace hyperim {

static thread_local std::string g_detail;

void set_error_detail(const std::string &msg) { g_detail = msg; }
void clear_error_detail() { g_detail.clear(); }

int DevBuf::reserve(size_t need, hipStream_t s, bool keep) {
    if (need <= bytes && ptr) return HYPERIM_OK;
    size_t want = std::max<size_t>(need, bytes + bytes / 2);
    want = (want + 255) & ~(size_t)255;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        want = (need + 255) & ~(size_t)255;
        e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error_detail("hipMalloc of " + std::to_string(want) + " bytes failed");
            return HYPERIM_ENOMEM;
        }
    }
    if (keep && ptr && bytes) {
        HIM_HIP(hipMemcpyAsync(p, ptr, bytes, hipMemcpyDeviceToDevice, s));
        HIM_HIP(hipStreamSynchronize(s));
    }
    if (ptr) {
        HIM_HIP(hipStreamSynchronize(s));
        (void)hipFree(ptr);
    }
    ptr = p;
    bytes = want;
    return HYPERIM_OK;
}

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

// Pool storage: make room for `ids` more ids and `entries` more members
// (owned storage grows and keeps its contents; a caller buffer cannot grow).
int pool_reserve(hyperim_pool p, uint64_t ids, uint64_t entries, hipStream_t s) {
    const uint64_t need_ids = p->count + ids;
    const uint64_t need_mem = p->total + entries;
    if (need_ids <= p->id_cap && need_mem <= p->mem_cap) return HYPERIM_OK;
    if (!p->owned) {
        const uint64_t ic = std::max(need_ids, p->id_cap);
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        p->required = al(8 * (ic + 1)) + al(4 * ic) + 4 * std::max(need_mem, (uint64_t)1);
        set_error_detail("pool buffer too small: " + std::to_string(p->required) + " bytes needed");
        return HYPERIM_ECAPACITY;
    }
    if (need_ids > p->id_cap) {
        const uint64_t ic = std::max<uint64_t>(need_ids, p->id_cap * 2);
        HIM_CHECK(p->off_b.reserve(sizeof(uint64_t) * (ic + 1), s, true));
        HIM_CHECK(p->roots_b.reserve(sizeof(uint32_t) * ic, s, true));
        p->id_cap = ic;
    }
    if (need_mem > p->mem_cap) {
        const uint64_t mc = std::max<uint64_t>(need_mem, p->mem_cap + p->mem_cap / 2);
        HIM_CHECK(p->mem_b.reserve(sizeof(uint32_t) * std::max<uint64_t>(mc, 1), s, true));
        p->mem_cap = mc;
    }
    p->off = p->off_b.as<uint64_t>();
    p->roots = p->roots_b.as<uint32_t>();
    p->mem = p->mem_b.as<uint32_t>();
    return HYPERIM_OK;
}


// Per-device RR workspace (created on first use, kept until the process ends
// or hyperim_workspace_release).
namespace {
struct DevCtx {
    std::mutex mu;
    RRWorkspace rr;
    GreedyWorkspace gr;
    PrepWorkspace prep;
};
constexpr int kMaxDevices = 256;
std::mutex g_ctx_mu;
DevCtx *g_ctx[kMaxDevices];

DevCtx *device_ctx(int device) {
    std::lock_guard<std::mutex> l(g_ctx_mu);
    if (device < 0 || device >= kMaxDevices) return nullptr;
    if (!g_ctx[device]) g_ctx[device] = new DevCtx();
    return g_ctx[device];
}
}  // namespace

DeviceLock::DeviceLock(int device) {
    DevCtx *c = device_ctx(device);
    c->mu.lock();
    rr = &c->rr;
    gr = &c->gr;
    prep = &c->prep;
    lock = c;
}

DeviceLock::~DeviceLock() { static_cast<DevCtx *>(lock)->mu.unlock(); }

void GreedyWorkspace::release() {
    for (DevBuf *x : {&cnt, &inv_off, &cursor, &inv, &covered, &chosen, &best, &out, &big, &cursor_big, &flags,
                      &counters, &scan_tmp, &params, &topk})
        x->release();
    if (rounds_exec) (void)hipGraphExecDestroy(rounds_exec);
    rounds_exec = nullptr;
    graph_k = 0;
    graph_params = nullptr;
}

size_t RRWorkspace::bytes() const {
    size_t b = 0;
    for (const DevBuf *x : {&lists, &bitmaps, &def_idx, &def_u32, &graph_desc, &task_desc, &items, &counters, &stage,
                            &stage_off, &sizes, &roots, &scan_tmp, &big_ids, &ms_seen, &ms_nxt, &ms_cur, &ms_next,
                            &ms_batch, &ms_vcnt, &ms_ctr, &args_dev, &picks})
        b += x->bytes;
    return b;
}

void RRWorkspace::drop_graphs() {
    for (BatchGraph &b : batch_graphs) (void)hipGraphExecDestroy(b.exec);
    batch_graphs.clear();
}

void RRWorkspace::release() {
    drop_graphs();
    if (capture) (void)hipStreamDestroy(capture);
    capture = nullptr;
    for (DevBuf *x : {&lists, &bitmaps, &def_idx, &def_u32, &graph_desc, &task_desc, &items, &counters, &stage,
                      &stage_off, &sizes, &roots, &scan_tmp, &big_ids, &ms_seen, &ms_nxt, &ms_cur, &ms_next,
                      &ms_batch, &ms_vcnt, &ms_ctr, &args_dev, &picks})
        x->release();
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    events.clear();
    if (host) (void)hipHostFree(host);
    host = nullptr;
    host_words = 0;
    grid = waves = slots = grid_b = slot_n = slot_words = 0;
}

size_t PrepWorkspace::bytes() const {
    size_t b = 0;
    for (const DevBuf *x : {&k1, &vals, &k2, &wmax, &pc, &tmp, &counts, &base, &isum, &lmax, &hist, &flag, &cnt, &off64, &lists, &bm}) b += x->bytes;
    return b;
}

void PrepWorkspace::release() {
    for (DevBuf *x : {&k1, &vals, &k2, &wmax, &pc, &tmp, &counts, &base, &isum, &lmax, &hist, &flag, &cnt, &off64, &lists, &bm}) x->release();
}

size_t GreedyWorkspace::bytes() const {
    size_t b = 0;
    for (const DevBuf *x : {&cnt, &inv_off, &cursor, &inv, &covered, &chosen, &best, &out, &big, &cursor_big, &flags,
                            &counters, &scan_tmp, &topk})
        b += x->bytes;
    return b;
}

SharedBytes shared_bytes() {
    SharedBytes b{0, 0, 0, 0, 0};
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return b;
    DeviceLock lk(device);
    b.slots = lk.rr->lists.bytes + lk.rr->bitmaps.bytes;
    b.stage = lk.rr->bytes() - b.slots;
    b.greedy = lk.gr->bytes();
    b.prep = lk.prep->bytes();
    b.total = b.slots + b.stage + b.greedy + b.prep;
    return b;
}

size_t graph_bytes(hyperim_graph g) {
    size_t b = 0;
    for (const DevBuf *x : {&g->he_off, &g->he_mem, &g->v_off, &g->v_he, &g->thr, &g->c, &g->weight, &g->bytesw,
                            &g->phiw, &g->v_hbs, &g->chan, &g->l, &g->deg, &g->top, &g->stratum, &g->P,
                            &g->lay_nb_off, &g->lay_nb, &g->lay_ly_off, &g->lay_ly_end, &g->lay_ln, &g->lay_expm,
                            &g->route_P, &g->force_off, &g->force})
        b += x->bytes;
    return b;
}

void release_graph(hyperim_graph g) {
    for (DevBuf *b : {&g->he_off, &g->he_mem, &g->v_off, &g->v_he, &g->thr, &g->c, &g->weight, &g->bytesw,
                      &g->phiw, &g->v_hbs, &g->chan, &g->l, &g->deg, &g->top, &g->stratum, &g->P,
                            &g->lay_nb_off, &g->lay_nb, &g->lay_ly_off, &g->lay_ly_end, &g->lay_ln, &g->lay_expm,
                            &g->route_P, &g->force_off, &g->force})
        b->release();
}

// Pool storage --------------------------------------------------------------------
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int pool_init_owned(hyperim_graph g, hyperim_pool p, hipStream_t s) {
    p->g = g;
    p->owned = true;
    HIM_CHECK(p->off_b.reserve(sizeof(uint64_t) * 1025, s));
    HIM_CHECK(p->roots_b.reserve(sizeof(uint32_t) * 1024, s));
    HIM_CHECK(p->mem_b.reserve(sizeof(uint32_t) * 4096, s));
    p->id_cap = 1024;
    p->mem_cap = 4096;
    p->off = p->off_b.as<uint64_t>();
    p->roots = p->roots_b.as<uint32_t>();
    p->mem = p->mem_b.as<uint32_t>();
    HIM_HIP(hipMemsetAsync(p->off, 0, sizeof(uint64_t), s));
    return HYPERIM_OK;
}

void pool_clear(hyperim_pool p) {
    p->count = 0;
    p->total = 0;
    p->id_begin = 0;
    p->has_key = false;
}

void pool_release(hyperim_pool p) {
    p->off_b.release();
    p->roots_b.release();
    p->mem_b.release();
    p->off = nullptr;
    p->roots = nullptr;
    p->mem = nullptr;
    p->id_cap = p->mem_cap = 0;
    pool_clear(p);
}

size_t pool_bytes(const hyperim_pool_s &p) { return p.off_b.bytes + p.roots_b.bytes + p.mem_b.bytes; }

// Generate the tasks in one go and append each task's sets to its pool
// (tasks with an empty id range are skipped).
int generate_into(const std::vector<RRTask> &tasks, const std::vector<hyperim_pool> &pools, uint32_t qlog, int form,
                  uint64_t max_entries, hipStream_t s, RRStats &st, std::vector<int> *pool_status,
                  bool time_kernels, bool graphs) {
    std::vector<RRTask> live;
    std::vector<hyperim_pool> dst;
    std::vector<size_t> which;
    std::vector<bool> was_empty;
    for (size_t i = 0; i < tasks.size(); ++i)
        if (tasks[i].id_end > tasks[i].id_begin) {
            tasks[i].g->rr_used = true;
            live.push_back(tasks[i]);
            dst.push_back(pools[i]);
            which.push_back(i);
            was_empty.push_back(pools[i]->count == 0);
        }
    if (pool_status) pool_status->assign(tasks.size(), HYPERIM_OK);
    if (live.empty()) return HYPERIM_OK;
    int device = 0;
    HIM_HIP(hipGetDevice(&device));
    DeviceLock lk(device);
    std::vector<int> status;
    const uint64_t stage_budget = (uint64_t)std::max<uint32_t>(live[0].g->tune.stage_mib, 64) << 20;
    HIM_CHECK(rr_generate_into(*lk.rr, st, live, dst, qlog, form, max_entries, stage_budget, s, status,
                               time_kernels, graphs));
    int first_fail = HYPERIM_OK;
    for (size_t i = 0; i < live.size(); ++i) {
        if (was_empty[i] && dst[i]->count) dst[i]->id_begin = live[i].id_begin;
        if (status[i] != HYPERIM_OK) {
            if (pool_status) (*pool_status)[which[i]] = status[i];
            if (first_fail == HYPERIM_OK) first_fail = status[i];
        }
    }
    return pool_status ? HYPERIM_OK : first_fail;
}

}  // namespace hyperim

using namespace hyperim;

extern "C" {

const char *hyperim_strerror(int status) {
    static thread_local std::string msg;
    const char *base = "unknown status";
    switch (status) {
        case HYPERIM_OK: base = "ok"; break;
        case HYPERIM_EINVAL: base = "invalid argument"; break;
        case HYPERIM_ENOMEM: base = "out of memory"; break;
        case HYPERIM_ECAPACITY: base = "pool capacity exceeded"; break;
        case HYPERIM_ESTATE: base = "call out of order"; break;
        case HYPERIM_EHIP: base = "HIP runtime error"; break;
        default: break;
    }
    msg = base;
    if (status != HYPERIM_OK && !g_detail.empty()) msg += ": " + g_detail;
    return msg.c_str();
}

int hyperim_build_graph(uint32_t n, uint32_t m, const uint32_t *he_off, const uint32_t *he_mem, int ptrs_on_device,
                        hyperim_prob prob, void *stream, hyperim_graph *out) {
    if (!out) return HYPERIM_EINVAL;
    *out = nullptr;
    g_detail.clear();
    // vertex ids stay below 2^31: the grid-wide phase marks expanded queue
    // entries with bit 31
    if (n == 0 || n > kMaxVertices || m == 0xFFFFFFFFu || !he_off || (!he_mem && m)) {
        set_error_detail("n must be in [1, 2^31], m < 2^32-1, arrays non-null");
        return HYPERIM_EINVAL;
    }
    if (prob.model > HYPERIM_MODEL_GAPS_WC ||
        ((prob.model == HYPERIM_MODEL_CONST || prob.model == HYPERIM_MODEL_LT_CONST ||
          prob.model == HYPERIM_MODEL_GAPS_CONST) &&
         (std::isnan(prob.p) || prob.p < 0.0f))) {
        set_error_detail("probability model unknown or p NaN / negative");
        return HYPERIM_EINVAL;
    }
    hipStream_t s = as_stream(stream);
    hyperim_graph g = new (std::nothrow) hyperim_graph_s();
    if (!g) return HYPERIM_ENOMEM;
    int rc = [&]() -> int {
        HIM_HIP(hipGetDevice(&g->device));
        g->n = n;
        g->m = m;
        g->prob = prob;
        const hipMemcpyKind kind = ptrs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        uint32_t nnz = 0, first = 0;
        if (ptrs_on_device) {
            HIM_HIP(hipMemcpyAsync(&nnz, he_off + m, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            HIM_HIP(hipMemcpyAsync(&first, he_off, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            HIM_HIP(hipStreamSynchronize(s));
        } else {
            nnz = he_off[m];
            first = he_off[0];
        }
        if (first != 0) {
            set_error_detail("he_off[0] must be 0");
            return HYPERIM_EINVAL;
        }
        g->nnz = nnz;
        HIM_CHECK(g->he_off.reserve(sizeof(uint32_t) * ((size_t)m + 1), s));
        HIM_CHECK(g->he_mem.reserve(sizeof(uint32_t) * std::max<uint64_t>(nnz, 1), s));
        HIM_HIP(hipMemcpyAsync(g->he_off.ptr, he_off, sizeof(uint32_t) * ((size_t)m + 1), kind, s));
        if (nnz) HIM_HIP(hipMemcpyAsync(g->he_mem.ptr, he_mem, sizeof(uint32_t) * (size_t)nnz, kind, s));
        DeviceLock lk(g->device);
        return graph_build_device(g, *lk.prep, s);
    }();
    if (rc != HYPERIM_OK) {
        release_graph(g);
        delete g;
        return rc;
    }
    *out = g;
    return HYPERIM_OK;
}

int hyperim_stratify(hyperim_graph g, void *stream, hyperim_strata_info *out) {
    if (!g) return HYPERIM_EINVAL;
    g_detail.clear();
    {
        DeviceLock lk(g->device);
        HIM_CHECK(stratify_device(g, *lk.prep, as_stream(stream)));
    }
    if (out) *out = g->info;
    return HYPERIM_OK;
}

int hyperim_route(hyperim_graph g, uint32_t on, void *stream, uint32_t *n_r1) {
    if (!g || on > 1) return HYPERIM_EINVAL;
    g_detail.clear();
    if (n_r1) *n_r1 = 0;
    if (g->lt() || g->layered()) {
        set_error_detail("the division of the RR sets applies to the independent-cascade models only");
        return HYPERIM_EINVAL;
    }
    if (!g->stratified) return HYPERIM_ESTATE;
    if (g->rr_used && (on != 0) != g->route_on) {
        set_error_detail("RR sets were generated on this graph already: divide (or undo) before the first");
        return HYPERIM_ESTATE;
    }
    HIM_CHECK(check_device(g));
    g->routed = false;
    g->route_on = false;   // set once the tables are built (a failed build leaves the graph undivided)
    uint32_t n1 = 0;
    if (on) {
        DeviceLock lk(g->device);
        HIM_CHECK(route_build(g, as_stream(stream), &n1));
        g->route_on = true;
    }
    if (n_r1) *n_r1 = n1;
    return HYPERIM_OK;
}

int hyperim_graph_read(hyperim_graph g, uint32_t *v_off, uint32_t *v_he, uint32_t *thr, uint64_t *c, uint32_t *l,
                       uint32_t *deg, uint32_t *top, uint8_t *stratum, uint32_t *P, int dst_on_device, void *stream) {
    if (!g) return HYPERIM_EINVAL;
    if ((l || deg || top || stratum || P) && !g->stratified) return HYPERIM_ESTATE;
    hipStream_t s = as_stream(stream);
    const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t n = g->n;
    struct Item {
        void *dst;
        const DevBuf *src;
        size_t bytes;
    } items[] = {{v_off, &g->v_off, 4 * (n + 1)}, {v_he, &g->v_he, 4 * (size_t)g->nnz}, {thr, &g->thr, 4 * n},
                 {c, &g->c, 8 * n},           {l, &g->l, 4 * n},                   {deg, &g->deg, 4 * n},
                 {top, &g->top, 4 * n},       {stratum, &g->stratum, n},           {P, &g->P, 4 * n}};
    for (const Item &it : items)
        if (it.dst && it.bytes) HIM_HIP(hipMemcpyAsync(it.dst, it.src->ptr, it.bytes, kind, s));
    HIM_HIP(hipStreamSynchronize(s));
    return HYPERIM_OK;
}

int hyperim_pool_create(hyperim_graph g, void *dev_buf, size_t bytes, uint64_t id_capacity, hyperim_pool *out) {
    if (!g || !out) return HYPERIM_EINVAL;
    *out = nullptr;
    hyperim_pool p = new (std::nothrow) hyperim_pool_s();
    if (!p) return HYPERIM_ENOMEM;
    p->g = g;
    if (dev_buf) {
        const size_t head = align256(8 * (id_capacity + 1)) + align256(4 * id_capacity);
        if (id_capacity == 0 || bytes < head + 4) {
            delete p;
            set_error_detail("pool buffer smaller than its id arrays");
            return HYPERIM_EINVAL;
        }
        p->owned = false;
        p->buf = static_cast<char *>(dev_buf);
        p->bytes = bytes;
        p->off = reinterpret_cast<uint64_t *>(p->buf);
        p->roots = reinterpret_cast<uint32_t *>(p->buf + align256(8 * (id_capacity + 1)));
        p->mem = reinterpret_cast<uint32_t *>(p->buf + head);
        p->id_cap = id_capacity;
        p->mem_cap = (bytes - head) / 4;
        if (hipMemset(p->off, 0, sizeof(uint64_t)) != hipSuccess) {
            delete p;
            return HYPERIM_EHIP;
        }
    } else {
        int rc = pool_init_owned(g, p, nullptr);
        if (rc) {
            delete p;
            return rc;
        }
        if (hipDeviceSynchronize() != hipSuccess) {
            delete p;
            return HYPERIM_EHIP;
        }
    }
    *out = p;
    return HYPERIM_OK;
}

int hyperim_generate_rr(hyperim_graph g, uint64_t seed, uint32_t instance, uint32_t pool_tag, uint64_t id_begin,
                        uint64_t id_end, hyperim_pool pool, void *stream) {
    if (!g || !pool || pool->g != g) return HYPERIM_EINVAL;
    HIM_CHECK(check_device(g));
    g_detail.clear();
    if (!g->stratified) return HYPERIM_ESTATE;
    if (pool_tag > 1 || seed >> 32 || id_end < id_begin || id_end > kMaxIds) {
        set_error_detail("pool_tag must be 0/1, seed < 2^32, id_begin <= id_end <= 2^39");
        return HYPERIM_EINVAL;
    }
    if (pool->count) {
        if (!pool->has_key || pool->seed != seed || pool->instance != instance || pool->tag != pool_tag ||
            id_begin != pool->id_begin + pool->count) {
            set_error_detail("a non-empty pool only grows at its end with its own key");
            return HYPERIM_EINVAL;
        }
    }
    RRStats st;
    HIM_CHECK(generate_into({RRTask{g, seed, instance, pool_tag, id_begin, id_end}}, {pool}, kDefaultQlog, 0, 0,
                            as_stream(stream), st, nullptr));
    pool->has_key = true;
    pool->seed = seed;
    pool->instance = instance;
    pool->tag = pool_tag;
    HIM_HIP(hipStreamSynchronize(as_stream(stream)));
    return HYPERIM_OK;
}

int hyperim_generate_rr_batch(const hyperim_rr_task *tasks, uint32_t count, uint32_t form, void *stream) {
    g_detail.clear();
    if ((!tasks && count) || form > 1) return HYPERIM_EINVAL;
    if (count == 0) return HYPERIM_OK;
    std::vector<RRTask> rt;
    std::vector<hyperim_pool> pools;
    for (uint32_t i = 0; i < count; ++i) {
        const hyperim_rr_task &t = tasks[i];
        if (!t.graph || !t.pool || t.pool->g != t.graph) return HYPERIM_EINVAL;
        HIM_CHECK(check_device(t.graph));
        if (!t.graph->stratified) return HYPERIM_ESTATE;
        if (t.pool_tag > 1 || t.seed >> 32 || t.id_end < t.id_begin || t.id_end > kMaxIds) {
            set_error_detail("pool_tag must be 0/1, seed < 2^32, id_begin <= id_end <= 2^39");
            return HYPERIM_EINVAL;
        }
        const hyperim_pool p = t.pool;
        if (p->count && (!p->has_key || p->seed != t.seed || p->instance != t.instance || p->tag != t.pool_tag ||
                         t.id_begin != p->id_begin + p->count)) {
            set_error_detail("a non-empty pool only grows at its end with its own key");
            return HYPERIM_EINVAL;
        }
        rt.push_back(RRTask{t.graph, t.seed, t.instance, t.pool_tag, t.id_begin, t.id_end});
        pools.push_back(p);
    }
    RRStats st;
    HIM_CHECK(generate_into(rt, pools, kDefaultQlog, (int)form, 0, as_stream(stream), st, nullptr));
    for (uint32_t i = 0; i < count; ++i) {
        if (tasks[i].id_end == tasks[i].id_begin) continue;
        hyperim_pool p = tasks[i].pool;
        p->has_key = true;
        p->seed = tasks[i].seed;
        p->instance = tasks[i].instance;
        p->tag = tasks[i].pool_tag;
    }
    HIM_HIP(hipStreamSynchronize(as_stream(stream)));
    return HYPERIM_OK;
}

int hyperim_pool_view(hyperim_pool pool, const uint64_t **off, const uint32_t **mem, const uint32_t **roots,
                      uint64_t *id_begin, uint64_t *count) {
    if (!pool) return HYPERIM_EINVAL;
    if (off) *off = pool->off;
    if (mem) *mem = pool->mem;
    if (roots) *roots = pool->roots;
    if (id_begin) *id_begin = pool->id_begin;
    if (count) *count = pool->count;
    return HYPERIM_OK;
}

int hyperim_pool_read(hyperim_pool pool, uint64_t *off, uint32_t *mem, uint32_t *roots, int dst_on_device,
                      void *stream) {
    if (!pool) return HYPERIM_EINVAL;
    hipStream_t s = as_stream(stream);
    const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (off) HIM_HIP(hipMemcpyAsync(off, pool->off, sizeof(uint64_t) * (pool->count + 1), kind, s));
    if (mem && pool->total) HIM_HIP(hipMemcpyAsync(mem, pool->mem, sizeof(uint32_t) * pool->total, kind, s));
    if (roots && pool->count) HIM_HIP(hipMemcpyAsync(roots, pool->roots, sizeof(uint32_t) * pool->count, kind, s));
    HIM_HIP(hipStreamSynchronize(s));
    return HYPERIM_OK;
}

int hyperim_pool_required(hyperim_pool pool, size_t *bytes) {
    if (!pool || !bytes) return HYPERIM_EINVAL;
    *bytes = pool->required;
    return HYPERIM_OK;
}

int hyperim_pool_reset(hyperim_pool pool) {
    if (!pool) return HYPERIM_EINVAL;
    pool_clear(pool);
    return HYPERIM_OK;
}

int hyperim_greedy(hyperim_graph g, hyperim_pool pool, uint64_t theta, uint32_t k, void *stream, uint32_t *seeds,
                   uint64_t *gains) {
    if (!g || !pool || pool->g != g || !seeds) return HYPERIM_EINVAL;
    g_detail.clear();
    if (k == 0 || k > g->n || theta > pool->count || theta >= (1ull << 32)) {
        set_error_detail("need 1 <= k <= n and theta <= pool size < 2^32");
        return HYPERIM_EINVAL;
    }
    HIM_CHECK(check_device(g));
    DeviceLock lk(g->device);
    return greedy_device(*lk.gr, g, pool, theta, k, as_stream(stream), seeds, gains);
}

int hyperim_coverage(hyperim_graph g, hyperim_pool pool, uint64_t theta, const uint32_t *seeds, uint32_t k,
                     void *stream, uint64_t *covered) {
    if (!g || !pool || pool->g != g || !covered || (k && !seeds)) return HYPERIM_EINVAL;
    g_detail.clear();
    if (theta > pool->count) return HYPERIM_EINVAL;
    for (uint32_t i = 0; i < k; ++i)
        if (seeds[i] >= g->n) {
            set_error_detail("seed id >= n");
            return HYPERIM_EINVAL;
        }
    hipStream_t s = as_stream(stream);
    DevBuf d;
    HIM_CHECK(d.reserve(sizeof(uint32_t) * std::max<uint32_t>(k, 1), s));
    if (k) HIM_HIP(hipMemcpyAsync(d.ptr, seeds, sizeof(uint32_t) * k, hipMemcpyHostToDevice, s));
    int rc;
    {
        DeviceLock lk(g->device);
        rc = coverage_device(*lk.gr, g, pool, theta, d.as<uint32_t>(), k, s, covered);
    }
    d.release();
    return rc;
}

int hyperim_set_tuning(hyperim_graph g, const hyperim_tuning *t) {
    if (!g || !t) return HYPERIM_EINVAL;
    hyperim_tuning &cur = g->tune;
    if (t->heavy) cur.heavy = t->heavy;
    if (t->budget) cur.budget = t->budget;
    if (t->chunk) cur.chunk = std::max<uint32_t>(t->chunk, 16);
    if (t->seg) cur.seg = t->seg;
    cur.seg = std::max(cur.seg, cur.chunk);
    if (t->prefilter_min) cur.prefilter_min = t->prefilter_min;
    if (t->steps_per_sync) cur.steps_per_sync = std::min<uint32_t>(t->steps_per_sync, 64);
    if (t->stage_mib) cur.stage_mib = std::max<uint32_t>(t->stage_mib, 64);
    if (t->blocks_a) cur.blocks_a = t->blocks_a;
    if (t->blocks_b) cur.blocks_b = t->blocks_b;
    if (t->ms_min) cur.ms_min = t->ms_min;
    if (t->ms_filter) cur.ms_filter = std::min<uint32_t>(t->ms_filter, 65);
    return HYPERIM_OK;
}

int hyperim_get_tuning(hyperim_graph g, hyperim_tuning *t) {
    if (!g || !t) return HYPERIM_EINVAL;
    *t = g->tune;
    return HYPERIM_OK;
}

void hyperim_pool_free(hyperim_pool pool) {
    if (!pool) return;
    pool_release(pool);
    delete pool;
}

int hyperim_workspace_info(size_t *bytes) {
    if (!bytes) return HYPERIM_EINVAL;
    int device = 0;
    HIM_HIP(hipGetDevice(&device));
    DeviceLock lk(device);
    *bytes = lk.rr->bytes() + lk.gr->bytes() + lk.prep->bytes();
    return HYPERIM_OK;
}

int hyperim_workspace_release(void) {
    int device = 0;
    HIM_HIP(hipGetDevice(&device));
    DeviceLock lk(device);
    HIM_HIP(hipDeviceSynchronize());
    lk.rr->release();
    lk.gr->release();
    lk.prep->release();
    return HYPERIM_OK;
}

void hyperim_graph_free(hyperim_graph g) {
    if (!g) return;
    release_graph(g);
    delete g;
}

}  // extern "C"
