// The HyperIM_BRR loop (Algorithm 4) over one or many queries: sample-size
// schedule, rounds of joint RR generation, greedy, the R2 check and the
// bounds; single-query, batched and serving-session entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "internal.h"

namespace hyperim {
namespace {

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
    int create() {
        if (!a) HIM_HIP(hipEventCreate(&a));
        if (!b) HIM_HIP(hipEventCreate(&b));
        return HYPERIM_OK;
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// The two pools of one (graph, seed, instance) key; both hold ids [0, have).
struct PoolPair {
    hyperim_graph g = nullptr;
    uint64_t seed = 0;
    uint32_t instance = 0;
    hyperim_pool_s r[2];
    uint64_t have = 0;
    uint32_t users = 0;        // queries admitted on these pools
    uint64_t last_step = 0;    // for least-recently-used eviction
    bool allocated = false;

    int ensure(hipStream_t s) {
        if (allocated) return HYPERIM_OK;
        for (int x = 0; x < 2; ++x) {
            HIM_CHECK(pool_init_owned(g, &r[x], s));
            r[x].has_key = true;
            r[x].seed = seed;
            r[x].instance = instance;
            r[x].tag = (uint32_t)x;
        }
        allocated = true;
        return HYPERIM_OK;
    }
    void release() {
        for (int x = 0; x < 2; ++x) pool_release(&r[x]);
        have = 0;
        allocated = false;
    }
    size_t bytes() const { return pool_bytes(r[0]) + pool_bytes(r[1]); }
    double members_per_id() const {
        const uint64_t ids = r[0].count + r[1].count;
        return ids ? (double)(r[0].total + r[1].total) / (double)ids : -1.0;
    }
    ~PoolPair() { release(); }
};

struct QueryRun {
    hyperim_query q{};
    Schedule sc{};
    PoolPair *pp = nullptr;
    uint32_t round = 0;   // rounds completed
    bool done = false;
    int status = HYPERIM_OK;
    std::vector<uint32_t> seeds;
    std::vector<uint64_t> gains;
    hyperim_result res{};
    std::chrono::steady_clock::time_point t0;

    uint64_t next_theta(const hyperim_options &o) const {
        if (o.theta_fixed) return o.theta_fixed;
        return round >= 40 ? ~0ull : sc.theta1 << round;
    }
    void fail(int rc) {
        status = rc;
        done = true;
    }
};

hyperim_options normalize(const hyperim_options *opt) {
    hyperim_options o{};
    if (opt) o = *opt;
    if (o.qlog == 0) o.qlog = kDefaultQlog;
    return o;
}

int validate(const hyperim_query &q, const hyperim_options &o) {
    if (!q.graph) {
        set_error_detail("query without a graph");
        return HYPERIM_EINVAL;
    }
    HIM_CHECK(check_device(q.graph));
    if (!q.graph->stratified) {
        set_error_detail("graph not stratified");
        return HYPERIM_ESTATE;
    }
    if (q.k == 0 || q.k > q.graph->n || !(q.eps > 0.0 && q.eps < 1.0) || !(q.ell > 0.0) || q.seed >> 32 ||
        o.qlog > 24 || o.form > 1) {
        set_error_detail("need 1 <= k <= n, 0 < eps < 1, ell > 0, seed < 2^32, qlog <= 24, form 0/1");
        return HYPERIM_EINVAL;
    }
    return HYPERIM_OK;
}

void start(QueryRun &r, const hyperim_options &o) {
    r.sc = make_schedule(r.q.graph->n, r.q.k, r.q.eps, r.q.ell, o.qlog);
    r.seeds.assign(r.q.k, 0u);
    r.gains.assign(r.q.k, 0ull);
    r.res = hyperim_result{};
    r.res.i_max = o.theta_fixed ? 1 : r.sc.i_max;
    r.res.theta_max = r.sc.theta_max;
    r.t0 = std::chrono::steady_clock::now();
}

// One round of every query in qs (none done): RR generation for all their
// pools in one generation pass, then each query's greedy on R1[0, theta),
// coverage of R2[0, theta) and bound test.  Per-query failures (a pool over
// max_entries, theta beyond the id space) end that query only; a HIP error is
// returned and ends them all.
int run_round(const std::vector<QueryRun *> &qs, const hyperim_options &o, hipStream_t s, EventPair &ev,
              uint64_t step) {
    const double tconst = 1.0 - std::exp(-1.0);
    HIM_CHECK(ev.create());
    // targets per pool pair
    std::vector<PoolPair *> pps;
    std::vector<uint64_t> target;
    std::vector<QueryRun *> live;
    for (QueryRun *q : qs) {
        const uint64_t theta = q->next_theta(o);
        if (theta > kMaxIds || theta >= (1ull << 32)) {
            set_error_detail("theta exceeds the id space");
            q->fail(HYPERIM_ECAPACITY);
            continue;
        }
        live.push_back(q);
        size_t i = 0;
        while (i < pps.size() && pps[i] != q->pp) ++i;
        if (i == pps.size()) {
            pps.push_back(q->pp);
            target.push_back(theta);
        } else {
            target[i] = std::max(target[i], theta);
        }
    }
    std::vector<RRTask> tasks;
    std::vector<hyperim_pool> dst;
    std::vector<size_t> task_pp;
    for (size_t i = 0; i < pps.size(); ++i) {
        PoolPair *pp = pps[i];
        pp->last_step = step;
        HIM_CHECK(pp->ensure(s));
        if (target[i] <= pp->have) continue;
        for (uint32_t x = 0; x < 2; ++x) {
            tasks.push_back(RRTask{pp->g, pp->seed, pp->instance, x, pp->have, target[i]});
            dst.push_back(&pp->r[x]);
            task_pp.push_back(i);
        }
    }
    RRStats st;
    float ms_rr = 0.f;
    std::vector<int> pp_status(pps.size(), HYPERIM_OK);
    if (!tasks.empty()) {
        HIM_HIP(hipEventRecord(ev.a, s));
        std::vector<int> pool_status;
        HIM_CHECK(generate_into(tasks, dst, o.qlog, (int)o.form, o.max_entries, s, st, &pool_status));
        HIM_HIP(hipEventRecord(ev.b, s));
        HIM_HIP(hipEventSynchronize(ev.b));
        HIM_HIP(hipEventElapsedTime(&ms_rr, ev.a, ev.b));
        for (size_t t = 0; t < tasks.size(); ++t)
            if (pool_status[t] != HYPERIM_OK) pp_status[task_pp[t]] = pool_status[t];
        for (size_t i = 0; i < pps.size(); ++i) {
            PoolPair *pp = pps[i];
            if (pp_status[i] == HYPERIM_OK) {
                pp->have = std::max(pp->have, target[i]);
            } else {
                // a pool that did not take its new sets: both start over
                pool_clear(&pp->r[0]);
                pool_clear(&pp->r[1]);
                pp->have = 0;
            }
        }
    }
    for (QueryRun *q : live) {
        size_t i = 0;
        while (pps[i] != q->pp) ++i;
        if (pp_status[i] != HYPERIM_OK) {
            set_error_detail("pool would exceed max_entries");
            q->fail(pp_status[i]);
            continue;
        }
        hyperim_result &res = q->res;
        res.ms_rr += ms_rr;
        res.ms_bfs += st.ms_bfs;
        res.ms_light += st.ms_light;
        res.ms_heavy += st.ms_heavy;
        res.bfs_launches += st.launches;
        res.deferred += st.deferred;
        res.supersteps += st.supersteps;
        res.bytes_light += st.bytes_light;
        res.bytes_heavy += st.bytes_heavy;
        res.ms_expand += st.ms_expand;
        res.expand_launches += st.expand_launches;
        hyperim_graph g = q->q.graph;
        const uint64_t theta = q->next_theta(o);
        const uint32_t k = q->q.k;
        float ms = 0.f;
        HIM_HIP(hipEventRecord(ev.a, s));
        HIM_CHECK(greedy_device(g, &q->pp->r[0], theta, k, s, q->seeds.data(), q->gains.data()));
        uint64_t lambda2 = 0;
        HIM_CHECK(coverage_device(g, &q->pp->r[1], theta, g->gr.out.as<uint32_t>(), k, s, &lambda2));
        HIM_HIP(hipEventRecord(ev.b, s));
        HIM_HIP(hipEventSynchronize(ev.b));
        HIM_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        res.ms_greedy += ms;
        uint64_t lambda1 = 0;
        for (uint32_t x = 0; x < k; ++x) lambda1 += q->gains[x];
        const double n = (double)g->n;
        const double sl = lower_bound((double)lambda2, q->sc.a, n, (double)theta);
        const double su = upper_bound((double)lambda1, k, q->sc.a, n, (double)theta);
        q->round += 1;
        res.rounds = q->round;
        res.theta = theta;
        res.lambda1 = lambda1;
        res.lambda2 = lambda2;
        res.sigma_l = sl;
        res.sigma_u = su;
        res.spread = n * (double)lambda2 / (double)theta;
        const bool stop = o.theta_fixed || (su > 0.0 && sl / su >= tconst - q->q.eps) || q->round >= q->sc.i_max;
        if (!stop) continue;
        // members of the two pool prefixes [0, theta)
        uint64_t e[2] = {0, 0};
        for (int x = 0; x < 2; ++x)
            HIM_HIP(hipMemcpyAsync(&e[x], q->pp->r[x].off + theta, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        HIM_HIP(hipStreamSynchronize(s));
        res.entries1 = e[0];
        res.entries2 = e[1];
        if (o.flags & HYPERIM_FLAG_INCIDENCES) {
            uint64_t i1 = 0, i2 = 0, b1 = 0, b2 = 0;
            HIM_CHECK(rr_incidences(g, &q->pp->r[0], theta, s, &i1, &b1));
            HIM_CHECK(rr_incidences(g, &q->pp->r[1], theta, s, &i2, &b2));
            res.incidences = i1 + i2;
            res.alg_bytes = b1 + b2;
        }
        res.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - q->t0).count();
        q->done = true;
    }
    return HYPERIM_OK;
}

// Run queries to completion in lockstep rounds; pools shared by queries with
// the same graph and key live in `pools`.
int run_batch(std::vector<QueryRun> &runs, const hyperim_options &o, hipStream_t s) {
    std::vector<std::unique_ptr<PoolPair>> pools;
    for (QueryRun &r : runs) {
        for (auto &pp : pools)
            if (pp->g == r.q.graph && pp->seed == r.q.seed && pp->instance == r.q.instance) r.pp = pp.get();
        if (!r.pp) {
            pools.emplace_back(new PoolPair());
            PoolPair *pp = pools.back().get();
            pp->g = r.q.graph;
            pp->seed = r.q.seed;
            pp->instance = r.q.instance;
            r.pp = pp;
        }
        start(r, o);
    }
    EventPair ev;
    for (uint64_t step = 0;; ++step) {
        std::vector<QueryRun *> active;
        for (QueryRun &r : runs)
            if (!r.done) active.push_back(&r);
        if (active.empty()) break;
        const int rc = run_round(active, o, s, ev, step);
        if (rc != HYPERIM_OK) {
            for (QueryRun *r : active)
                if (!r->done) r->fail(rc);
            return rc;
        }
    }
    return HYPERIM_OK;
}

}  // namespace
}  // namespace hyperim

using namespace hyperim;

// ---- serving session -------------------------------------------------------
struct hyperim_session_s {
    int device = 0;
    hipStream_t stream = nullptr;
    hyperim_options opt{};
    size_t budget = 0;
    uint64_t next_ticket = 1;
    std::deque<QueryRun *> waiting;
    std::vector<QueryRun *> active;           // admission order
    std::map<uint64_t, QueryRun *> finished;
    std::map<QueryRun *, uint64_t> ticket_of;
    std::vector<std::unique_ptr<PoolPair>> pools;
    std::map<hyperim_graph, double> mpi;      // learned members per RR set, per graph
    EventPair ev;
    hyperim_session_stats stats{};

    ~hyperim_session_s() {
        for (QueryRun *q : waiting) delete q;
        for (QueryRun *q : active) delete q;
        for (auto &kv : finished) delete kv.second;
    }

    PoolPair *pool_for(const hyperim_query &q) {
        for (auto &pp : pools)
            if (pp->g == q.graph && pp->seed == q.seed && pp->instance == q.instance) return pp.get();
        pools.emplace_back(new PoolPair());
        PoolPair *pp = pools.back().get();
        pp->g = q.graph;
        pp->seed = q.seed;
        pp->instance = q.instance;
        return pp;
    }

    double members_per_id(const PoolPair *pp) const {
        const double own = pp->members_per_id();
        if (own >= 0.0) return own;
        auto it = mpi.find(pp->g);
        return it != mpi.end() ? it->second : 16.0;
    }

    // Bytes in use now: graphs with queries or pools, pools, RR workspace.
    size_t resident() {
        std::vector<hyperim_graph> gs;
        auto add = [&](hyperim_graph g) {
            if (std::find(gs.begin(), gs.end(), g) == gs.end()) gs.push_back(g);
        };
        size_t b = 0;
        for (auto &pp : pools) {
            b += pp->bytes();
            if (pp->allocated || pp->users) add(pp->g);
        }
        for (QueryRun *q : active) add(q->q.graph);
        for (hyperim_graph g : gs) b += graph_bytes(g);
        size_t ws = 0;
        if (hyperim_workspace_info(&ws) == HYPERIM_OK) b += ws;
        return b;
    }

    // Estimated extra device bytes for query q's next round: growth of its
    // pools (geometric growth slack 1.5), of its graph's greedy workspace
    // and of the shared stage.
    size_t growth(const QueryRun *q) const {
        const uint64_t theta = q->next_theta(opt);
        const PoolPair *pp = q->pp;
        const double mpi_est = members_per_id(pp);
        double g_b = 0.0;
        if (theta > pp->have) {
            const double pools = 2.0 * 1.5 * (double)theta * (12.0 + 4.0 * mpi_est) + 2.0 * 1.5 * 4.0 * 4096;
            g_b += std::max(0.0, pools - (double)pp->bytes());
            g_b += 2.0 * (double)(theta - pp->have) * (1.3 * 4.0 * mpi_est + 24.0);   // stage and per-id arrays
        }
        const double greedy = 1.5 * (double)theta * (4.0 * mpi_est + 17.0) + 21.0 * (double)q->q.graph->n;
        g_b += std::max(0.0, greedy - (double)q->q.graph->gr.bytes());
        if (!pp->allocated && !pp->users) g_b += (double)graph_bytes(q->q.graph);
        return (size_t)g_b;
    }

    // Free idle pools, least recently used first, until `need` more bytes fit.
    bool make_room(size_t &used, size_t need) {
        while (used + need > budget) {
            PoolPair *victim = nullptr;
            for (auto &pp : pools)
                if (pp->users == 0 && pp->allocated && (!victim || pp->last_step < victim->last_step))
                    victim = pp.get();
            if (!victim) return false;
            const size_t b = victim->bytes();
            victim->release();
            used -= std::min(used, b);
        }
        return true;
    }

    void finish(QueryRun *q) {
        q->pp->users -= 1;
        const double m = q->pp->members_per_id();
        if (m >= 0.0) mpi[q->q.graph] = m;
        if (q->status == HYPERIM_OK)
            stats.finished += 1;
        else
            stats.failed += 1;
        finished[ticket_of[q]] = q;
        ticket_of.erase(q);
    }
};

extern "C" {

int hyperim_select_seeds(hyperim_graph g, uint32_t k, double eps, double ell, uint64_t seed, uint32_t instance,
                         const hyperim_options *opt, void *stream, uint32_t *seeds, uint64_t *gains,
                         hyperim_result *out) {
    if (!g || !seeds) return HYPERIM_EINVAL;
    clear_error_detail();
    const hyperim_options o = normalize(opt);
    hyperim_query q{g, k, instance, eps, ell, seed};
    HIM_CHECK(validate(q, o));
    std::vector<QueryRun> runs(1);
    runs[0].q = q;
    HIM_CHECK(run_batch(runs, o, as_stream(stream)));
    if (runs[0].status != HYPERIM_OK) return runs[0].status;
    std::copy(runs[0].seeds.begin(), runs[0].seeds.end(), seeds);
    if (gains) std::copy(runs[0].gains.begin(), runs[0].gains.end(), gains);
    if (out) *out = runs[0].res;
    return HYPERIM_OK;
}

int hyperim_select_seeds_batch(const hyperim_query *queries, uint32_t count, const hyperim_options *opt,
                               void *stream, uint32_t *seeds, uint64_t *gains, hyperim_result *results,
                               int *status) {
    if ((count && !queries) || !seeds) return HYPERIM_EINVAL;
    clear_error_detail();
    const hyperim_options o = normalize(opt);
    for (uint32_t i = 0; i < count; ++i) {
        const int rc = validate(queries[i], o);
        if (rc != HYPERIM_OK) {
            set_error_detail("query " + std::to_string(i) + ": invalid");
            return rc;
        }
    }
    std::vector<QueryRun> runs(count);
    for (uint32_t i = 0; i < count; ++i) runs[i].q = queries[i];
    const int rc = run_batch(runs, o, as_stream(stream));
    int first_fail = rc;
    uint64_t at = 0;
    for (uint32_t i = 0; i < count; ++i) {
        const QueryRun &r = runs[i];
        if (status) status[i] = r.status;
        if (first_fail == HYPERIM_OK && r.status != HYPERIM_OK) first_fail = r.status;
        if (r.status == HYPERIM_OK) {
            std::copy(r.seeds.begin(), r.seeds.end(), seeds + at);
            if (gains) std::copy(r.gains.begin(), r.gains.end(), gains + at);
            if (results) results[i] = r.res;
        }
        at += r.q.k;
    }
    return first_fail;
}

int hyperim_session_create(size_t hbm_budget, const hyperim_options *opt, void *stream, hyperim_session *out) {
    if (!out) return HYPERIM_EINVAL;
    *out = nullptr;
    clear_error_detail();
    hyperim_options o = normalize(opt);
    if (o.qlog > 24 || o.form > 1) {
        set_error_detail("qlog <= 24, form 0/1");
        return HYPERIM_EINVAL;
    }
    hyperim_session s = new (std::nothrow) hyperim_session_s();
    if (!s) return HYPERIM_ENOMEM;
    s->opt = o;
    s->stream = as_stream(stream);
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return HYPERIM_EHIP;
    }
    if (hbm_budget == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            delete s;
            return HYPERIM_EHIP;
        }
        const size_t reserve = 8ull << 30;
        hbm_budget = total_b > reserve ? total_b - reserve : total_b / 2;
    }
    s->budget = hbm_budget;
    s->stats.hbm_budget = hbm_budget;
    *out = s;
    return HYPERIM_OK;
}

int hyperim_session_submit(hyperim_session s, const hyperim_query *q, uint64_t *ticket) {
    if (!s || !q || !ticket) return HYPERIM_EINVAL;
    clear_error_detail();
    HIM_CHECK(validate(*q, s->opt));
    if (q->graph->device != s->device) {
        set_error_detail("the graph lives on another device than the session");
        return HYPERIM_EINVAL;
    }
    QueryRun *r = new (std::nothrow) QueryRun();
    if (!r) return HYPERIM_ENOMEM;
    r->q = *q;
    start(*r, s->opt);   // latency of the call counts from submission
    const uint64_t t = s->next_ticket++;
    s->ticket_of[r] = t;
    s->waiting.push_back(r);
    s->stats.submitted += 1;
    *ticket = t;
    return HYPERIM_OK;
}

int hyperim_session_step(hyperim_session s, hyperim_session_stats *out) {
    if (!s) return HYPERIM_EINVAL;
    clear_error_detail();
    s->stats.steps += 1;
    const uint64_t step = s->stats.steps;
    size_t used = s->resident();
    std::vector<QueryRun *> run;
    // running queries first, in admission order
    for (QueryRun *q : s->active) {
        const size_t need = q->pp ? s->growth(q) : 0;
        if (used + need <= s->budget || s->make_room(used, need)) {
            run.push_back(q);
            used += need;
        }
    }
    // then new queries, in submission order (no overtaking)
    while (!s->waiting.empty()) {
        QueryRun *q = s->waiting.front();
        PoolPair *pp = s->pool_for(q->q);
        q->pp = pp;
        const size_t need = s->growth(q);
        if (used + need > s->budget && !s->make_room(used, need)) {
            q->pp = nullptr;
            break;
        }
        s->waiting.pop_front();
        pp->users += 1;
        s->active.push_back(q);
        s->stats.admitted += 1;
        run.push_back(q);
        used += need;
    }
    if (run.empty() && (!s->active.empty() || !s->waiting.empty())) {
        // nothing fits: the oldest query cannot run even alone
        QueryRun *q = nullptr;
        if (!s->active.empty()) {
            q = s->active.front();
            s->active.erase(s->active.begin());
        } else {
            q = s->waiting.front();
            s->waiting.pop_front();
            q->pp = s->pool_for(q->q);
            q->pp->users += 1;
        }
        set_error_detail("query does not fit the session's HBM budget");
        q->fail(HYPERIM_ECAPACITY);
        s->finish(q);
    }
    int rc = HYPERIM_OK;
    if (!run.empty()) {
        rc = run_round(run, s->opt, s->stream, s->ev, step);
        if (rc != HYPERIM_OK)
            for (QueryRun *q : run)
                if (!q->done) q->fail(rc);
    }
    s->stats.ran_last = run.size();
    for (size_t i = 0; i < s->active.size();) {
        QueryRun *q = s->active[i];
        if (q->done) {
            s->active.erase(s->active.begin() + (long)i);
            s->finish(q);
        } else {
            ++i;
        }
    }
    s->stats.active = (uint32_t)s->active.size();
    s->stats.waiting = (uint32_t)s->waiting.size();
    s->stats.bytes_resident = s->resident();
    if (out) *out = s->stats;
    return rc;
}

int hyperim_session_poll(hyperim_session s, uint64_t ticket, uint32_t *seeds, uint64_t *gains,
                         hyperim_result *out) {
    if (!s) return HYPERIM_EINVAL;
    auto it = s->finished.find(ticket);
    if (it == s->finished.end()) {
        for (auto &kv : s->ticket_of)
            if (kv.second == ticket) return HYPERIM_PENDING;
        set_error_detail("unknown ticket");
        return HYPERIM_EINVAL;
    }
    QueryRun *q = it->second;
    const int st = q->status;
    if (st == HYPERIM_OK) {
        if (seeds) std::copy(q->seeds.begin(), q->seeds.end(), seeds);
        if (gains) std::copy(q->gains.begin(), q->gains.end(), gains);
        if (out) *out = q->res;
    }
    s->finished.erase(it);
    delete q;
    return st;
}

int hyperim_session_drop(hyperim_session s, hyperim_graph g) {
    if (!s || !g) return HYPERIM_EINVAL;
    for (QueryRun *q : s->active)
        if (q->q.graph == g) return HYPERIM_ESTATE;
    for (QueryRun *q : s->waiting)
        if (q->q.graph == g) return HYPERIM_ESTATE;
    HIM_HIP(hipStreamSynchronize(s->stream));
    for (size_t i = 0; i < s->pools.size();) {
        if (s->pools[i]->g == g) {
            s->pools.erase(s->pools.begin() + (long)i);
        } else {
            ++i;
        }
    }
    s->mpi.erase(g);
    return HYPERIM_OK;
}

int hyperim_session_stats_get(hyperim_session s, hyperim_session_stats *out) {
    if (!s || !out) return HYPERIM_EINVAL;
    s->stats.bytes_resident = s->resident();
    *out = s->stats;
    return HYPERIM_OK;
}

void hyperim_session_free(hyperim_session s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    delete s;
}

}  // extern "C"
