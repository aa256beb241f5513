// C ABI of libhyperim (declared in include/hyperim.h): handles, argument
// validation, pool storage, the sample-size schedule and the HyperIM_BRR loop
// (Algorithm 4) that drives the device kernels.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "dev_common.h"
#include "internal.h"

namespace hyperim {

static thread_local std::string g_detail;

void set_error_detail(const std::string &msg) { g_detail = msg; }

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


namespace {

constexpr uint64_t kMaxIds = 1ull << 39;   // RR ids use 39 bits of the coin counter

hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

void release_graph(hyperim_graph g) {
    for (DevBuf *b : {&g->he_off, &g->he_mem, &g->v_off, &g->v_he, &g->thr, &g->c, &g->weight, &g->l, &g->deg,
                      &g->top, &g->stratum, &g->P})
        b->release();
    RRWorkspace &r = g->rr;
    for (DevBuf *b : {&r.lists, &r.bitmaps, &r.counters, &r.stage, &r.stage_off, &r.sizes, &r.roots, &r.scan_tmp,
                      &r.big_ids, &r.def_idx, &r.def_u32, &r.items})
        b->release();
    for (hipEvent_t e : r.events) (void)hipEventDestroy(e);
    r.events.clear();
    g->bytesw.release();
    GreedyWorkspace &w = g->gr;
    for (DevBuf *b : {&w.cnt, &w.inv_off, &w.cursor, &w.inv, &w.covered, &w.chosen, &w.best, &w.out, &w.big,
                      &w.round_big, &w.flags, &w.counters, &w.scan_tmp})
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

// Generate the tasks in one go and append each task's sets to its pool.
int generate_into(hyperim_graph g, const RRKey &key, const std::vector<RRTask> &tasks,
                  const std::vector<hyperim_pool> &pools, int form, uint64_t max_entries, hipStream_t s) {
    std::vector<RRTask> live;
    std::vector<hyperim_pool> dst;
    for (size_t i = 0; i < tasks.size(); ++i)
        if (tasks[i].id_end > tasks[i].id_begin) {
            live.push_back(tasks[i]);
            dst.push_back(pools[i]);
        }
    if (live.empty()) return HYPERIM_OK;
    uint64_t total = 0;
    HIM_CHECK(rr_generate_stage(g, key, live, form, s, &total));
    uint64_t first = 0;
    for (size_t i = 0; i < live.size(); ++i) {
        const uint64_t count = live[i].id_end - live[i].id_begin;
        const bool was_empty = dst[i]->count == 0;
        HIM_CHECK(rr_compact_into(g, dst[i], first, count, max_entries, s));
        if (was_empty) dst[i]->id_begin = live[i].id_begin;
        first += count;
    }
    return HYPERIM_OK;
}

// Sample-size schedule (Section 4): delta = n^-ell; theta_max from Lemma 6 in
// the OPIM-C form it cites, 2n (t sqrt(ln 6/delta) + sqrt(t (ln C(n,k) +
// ln 6/delta)))^2 / (eps^2 k) with t = 1 - 1/e; theta_0 = theta_max eps^2 k / n
// rounded up to a power-of-two ladder size >= Q; i_max = first round whose
// size reaches theta_max; a = ln(3 i_max / delta).
struct Schedule {
    double theta_max, theta0, a, ln_inv_delta;
    uint64_t theta1;
    uint32_t i_max;
};

Schedule make_schedule(uint32_t n, uint32_t k, double eps, double ell, uint32_t qlog) {
    Schedule sc{};
    const double t = 1.0 - std::exp(-1.0);
    sc.ln_inv_delta = ell * std::log((double)n);
    double ln_binom = 0.0;
    for (uint32_t i = 0; i < k; ++i) ln_binom += std::log((double)(n - i) / (double)(i + 1));
    const double l6 = std::log(6.0) + sc.ln_inv_delta;
    const double r = t * std::sqrt(l6) + std::sqrt(t * (ln_binom + l6));
    sc.theta_max = 2.0 * (double)n * r * r / (eps * eps * (double)k);
    sc.theta0 = sc.theta_max * eps * eps * (double)k / (double)n;
    uint64_t th = 1ull << qlog;
    while ((double)th < sc.theta0) th <<= 1;
    sc.theta1 = th;
    uint32_t i = 1;
    while ((double)th < sc.theta_max) {
        th <<= 1;
        ++i;
    }
    sc.i_max = i;
    sc.a = std::log(3.0 * (double)i) + sc.ln_inv_delta;
    return sc;
}

// Equation (12), clamped at zero.
double lower_bound(double lambda2, double a, double n, double theta) {
    const double r = std::sqrt(lambda2 + 2.0 * a / 9.0) - std::sqrt(a / 2.0);
    double v = r * r - a / 18.0;
    if (v < 0.0) v = 0.0;
    return v * n / theta;
}

// Lemma 5 with p_max = 1, lifted by the OPIM-C concentration term.
double upper_bound(double lambda1, uint32_t k, double a, double n, double theta) {
    const double cov = lambda1 / (1.0 - std::pow(1.0 - 1.0 / (double)k, (double)k));
    const double r = std::sqrt(cov + a / 2.0) + std::sqrt(a / 2.0);
    return r * r * n / theta;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace
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
    if (n == 0 || n == 0xFFFFFFFFu || m == 0xFFFFFFFFu || !he_off || (!he_mem && m)) {
        set_error_detail("n must be in [1, 2^32-2], m < 2^32-1, arrays non-null");
        return HYPERIM_EINVAL;
    }
    if (prob.model > HYPERIM_MODEL_WC || (prob.model == HYPERIM_MODEL_CONST && (std::isnan(prob.p) || prob.p < 0.0f))) {
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
        return graph_build_device(g, s);
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
    HIM_CHECK(stratify_device(g, as_stream(stream)));
    if (out) *out = g->info;
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
    RRKey key{seed, instance, 8};
    HIM_CHECK(generate_into(g, key, {RRTask{pool_tag, id_begin, id_end}}, {pool}, 0, 0, as_stream(stream)));
    pool->has_key = true;
    pool->seed = seed;
    pool->instance = instance;
    pool->tag = pool_tag;
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
    return greedy_device(g, pool, theta, k, as_stream(stream), seeds, gains);
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
    int rc = coverage_device(g, pool, theta, d.as<uint32_t>(), k, s, covered);
    d.release();
    return rc;
}

int hyperim_select_seeds(hyperim_graph g, uint32_t k, double eps, double ell, uint64_t seed, uint32_t instance,
                         const hyperim_options *opt, void *stream, uint32_t *seeds, uint64_t *gains,
                         hyperim_result *out) {
    if (!g || !seeds) return HYPERIM_EINVAL;
    g_detail.clear();
    if (!g->stratified) return HYPERIM_ESTATE;
    hyperim_options o{};
    if (opt) o = *opt;
    if (o.qlog == 0) o.qlog = 8;
    if (k == 0 || k > g->n || !(eps > 0.0 && eps < 1.0) || !(ell > 0.0) || seed >> 32 || o.qlog > 24 ||
        o.form > 1) {
        set_error_detail("need 1 <= k <= n, 0 < eps < 1, ell > 0, seed < 2^32, qlog <= 24, form 0/1");
        return HYPERIM_EINVAL;
    }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = as_stream(stream);
    const Schedule sc = make_schedule(g->n, k, eps, ell, o.qlog);
    const double t = 1.0 - std::exp(-1.0);
    hyperim_pool_s r1, r2;
    HIM_CHECK(pool_init_owned(g, &r1, s));
    HIM_CHECK(pool_init_owned(g, &r2, s));
    EventPair ev;
    HIM_HIP(hipEventCreate(&ev.a));
    HIM_HIP(hipEventCreate(&ev.b));
    hyperim_result res{};
    g->rr.ms_bfs = g->rr.ms_light = g->rr.ms_heavy = 0.0;
    g->rr.launches = g->rr.supersteps = g->rr.deferred = 0;
    g->rr.bytes_light = g->rr.bytes_heavy = 0;
    res.i_max = o.theta_fixed ? 1 : sc.i_max;
    res.theta_max = sc.theta_max;
    uint64_t have = 0;
    std::vector<uint64_t> gains_h(k);
    int rc = [&]() -> int {
        for (uint32_t i = 1; i <= res.i_max; ++i) {
            const uint64_t theta = o.theta_fixed ? o.theta_fixed : (sc.theta1 << (i - 1));
            if (theta > kMaxIds || theta >= (1ull << 32)) {
                set_error_detail("theta exceeds the id space");
                return HYPERIM_ECAPACITY;
            }
            float ms = 0.f;
            HIM_HIP(hipEventRecord(ev.a, s));
            // both pools of the round share one launch group
            RRKey key{seed, instance, o.qlog};
            HIM_CHECK(generate_into(g, key, {RRTask{0, have, theta}, RRTask{1, have, theta}}, {&r1, &r2},
                                    (int)o.form, o.max_entries, s));
            HIM_HIP(hipEventRecord(ev.b, s));
            HIM_HIP(hipEventSynchronize(ev.b));
            HIM_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
            res.ms_rr += ms;
            have = theta;
            HIM_HIP(hipEventRecord(ev.a, s));
            HIM_CHECK(greedy_device(g, &r1, theta, k, s, seeds, gains_h.data()));
            uint64_t lambda2 = 0;
            HIM_CHECK(coverage_device(g, &r2, theta, g->gr.out.as<uint32_t>(), k, s, &lambda2));
            HIM_HIP(hipEventRecord(ev.b, s));
            HIM_HIP(hipEventSynchronize(ev.b));
            HIM_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
            res.ms_greedy += ms;
            uint64_t lambda1 = 0;
            for (uint32_t x = 0; x < k; ++x) lambda1 += gains_h[x];
            const double sl = lower_bound((double)lambda2, sc.a, (double)g->n, (double)theta);
            const double su = upper_bound((double)lambda1, k, sc.a, (double)g->n, (double)theta);
            res.rounds = i;
            res.theta = theta;
            res.lambda1 = lambda1;
            res.lambda2 = lambda2;
            res.sigma_l = sl;
            res.sigma_u = su;
            res.spread = (double)g->n * (double)lambda2 / (double)theta;
            res.entries1 = r1.total;   // pools hold exactly [0, theta)
            res.entries2 = r2.total;
            if (o.theta_fixed) break;
            if (su > 0.0 && sl / su >= t - eps) break;
        }
        if (o.flags & HYPERIM_FLAG_INCIDENCES) {
            uint64_t i1 = 0, i2 = 0, b1 = 0, b2 = 0;
            HIM_CHECK(rr_incidences(g, &r1, res.theta, s, &i1, &b1));
            HIM_CHECK(rr_incidences(g, &r2, res.theta, s, &i2, &b2));
            res.incidences = i1 + i2;
            res.alg_bytes = b1 + b2;
        }
        return HYPERIM_OK;
    }();
    for (hyperim_pool_s *p : {&r1, &r2}) {
        p->off_b.release();
        p->roots_b.release();
        p->mem_b.release();
    }
    if (rc != HYPERIM_OK) return rc;
    if (gains)
        for (uint32_t x = 0; x < k; ++x) gains[x] = gains_h[x];
    res.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    res.ms_bfs = g->rr.ms_bfs;
    res.bfs_launches = g->rr.launches;
    res.ms_light = g->rr.ms_light;
    res.ms_heavy = g->rr.ms_heavy;
    res.deferred = g->rr.deferred;
    res.supersteps = g->rr.supersteps;
    res.bytes_light = g->rr.bytes_light;
    res.bytes_heavy = g->rr.bytes_heavy;
    if (out) *out = res;
    return HYPERIM_OK;
}

int hyperim_set_tuning(hyperim_graph g, const hyperim_tuning *t) {
    if (!g || !t) return HYPERIM_EINVAL;
    hyperim_tuning &cur = g->rr.tune;
    if (t->heavy) cur.heavy = t->heavy;
    if (t->budget) cur.budget = t->budget;
    if (t->chunk) cur.chunk = std::max<uint32_t>(t->chunk, 16);
    if (t->seg) cur.seg = t->seg;
    cur.seg = std::max(cur.seg, cur.chunk);
    if (t->prefilter_min) cur.prefilter_min = t->prefilter_min;
    if (t->steps_per_sync) cur.steps_per_sync = std::min<uint32_t>(t->steps_per_sync, 64);
    return HYPERIM_OK;
}

int hyperim_get_tuning(hyperim_graph g, hyperim_tuning *t) {
    if (!g || !t) return HYPERIM_EINVAL;
    *t = g->rr.tune;
    return HYPERIM_OK;
}

void hyperim_pool_free(hyperim_pool pool) {
    if (!pool) return;
    pool->off_b.release();
    pool->roots_b.release();
    pool->mem_b.release();
    delete pool;
}

void hyperim_graph_free(hyperim_graph g) {
    if (!g) return;
    release_graph(g);
    delete g;
}

}  // extern "C"
