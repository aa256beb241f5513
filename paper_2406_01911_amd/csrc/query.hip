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

// An upper bound on the optimal coverage of R1, lifted to the optimal spread
// by the OPIM-C concentration term.
double upper_bound_cov(double cov, double a, double n, double theta) {
    const double r = std::sqrt(cov + a / 2.0) + std::sqrt(a / 2.0);
    return r * r * n / theta;
}

// Lemma 5 with p_max = 1: Lambda1 / (1 - (1 - 1/k)^k), lifted.
double upper_bound(double lambda1, uint32_t k, double a, double n, double theta) {
    return upper_bound_cov(lambda1 / (1.0 - std::pow(1.0 - 1.0 / (double)k, (double)k)), a, n, theta);
}

// Equation (8) with p_max = 1 from greedy's gains and the top-k sums of the
// marginal coverages before each round and after the last (ub[0..k]).
uint64_t eq8_coverage(const std::vector<uint64_t> &gains, const std::vector<uint64_t> &ub) {
    uint64_t best = ~0ull, cov = 0;
    for (size_t i = 0; i < ub.size(); ++i) {
        best = std::min(best, cov + ub[i]);
        if (i < gains.size()) cov += gains[i];
    }
    return best;
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

// The two pools of one (graph, seed, instance) key; pool x holds ids
// [0, have[x]).
struct PoolPair {
    hyperim_graph g = nullptr;
    uint64_t seed = 0;
    uint32_t instance = 0;
    hyperim_pool_s r[2];
    uint64_t have[2] = {0, 0};
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
    void clear() {
        for (int x = 0; x < 2; ++x) {
            pool_clear(&r[x]);
            have[x] = 0;
        }
    }
    void release() {
        for (int x = 0; x < 2; ++x) {
            pool_release(&r[x]);
            have[x] = 0;
        }
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
        o.qlog > 24 || o.form > 1 || o.bound > 1) {
        set_error_detail("need 1 <= k <= n, 0 < eps < 1, ell > 0, seed < 2^32, qlog <= 24, form 0/1, bound 0/1");
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

// Add one generation pass's device times and counters to a result.
void add_stats(hyperim_result &res, const RRStats &st, float ms_rr) {
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
    res.philox_drawn += st.philox;
    res.philox_bundled += st.philox_bundled;
    res.philox_light += st.philox_light;
    res.bytes_bundled += st.bytes_bundled;
    res.ms_bundled += st.ms_bundled;
    res.bundled_launches += st.bundled_launches;
}

size_t device_shared_bytes() {
    size_t b = 0;
    return hyperim_workspace_info(&b) == HYPERIM_OK ? b : 0;
}

// Queries in flight over resident pools, advanced one doubling round at a
// time.  With a finite budget, queries are admitted in submission order while
// the estimated device bytes fit (see hyperim_session_create).
struct Engine {
    hipStream_t stream = nullptr;
    hyperim_options opt{};
    size_t budget = ~(size_t)0;
    uint64_t steps = 0;
    std::deque<QueryRun *> waiting;
    std::vector<QueryRun *> active;   // admission order
    std::vector<std::unique_ptr<PoolPair>> pools;
    EventPair ev;
    // whole-engine totals: device times and counters of every shared launch
    // (pilot samples included), steps in `rounds`
    hyperim_result total{};

    bool bounded() const { return budget != ~(size_t)0; }

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
        return own >= 0.0 ? own : pp->g->rr_members;
    }

    // Device bytes in use: graphs with queries or pools here, pools, shared workspaces.
    size_t resident() const {
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
        return b + device_shared_bytes();
    }

    // Estimated extra device bytes for query q's next round that q alone
    // needs: its pools (plus the old storage while a pool grows and keeps its
    // contents) and its graph if nothing here uses it yet.  Its share of the
    // shared workspaces goes to `need`.  A graph without a members-per-set
    // estimate is priced at the worst case, n members per set.
    struct Shared {
        uint32_t n_max = 0;      // largest graph of the step (RR slots)
        double stage = 0.0;      // staged bytes of the step
        double greedy = 0.0;     // largest greedy index of the step
    };
    size_t own_growth(const QueryRun *q, Shared &need) const {
        const uint64_t theta = q->next_theta(opt);
        const PoolPair *pp = q->pp;
        const double n = (double)q->q.graph->n;
        double m = members_per_id(pp);
        if (m < 0.0) m = n;
        double b = 0.0;
        for (int x = 0; x < 2; ++x) {
            if (theta <= pp->have[x]) continue;
            const double add = (double)(theta - pp->have[x]) * m;
            const double bytes = ((double)theta + 1.0) * 12.0 + 4.0 * ((double)pp->r[x].total + add);
            const double cur = (double)pool_bytes(pp->r[x]);
            if (bytes > cur) b += bytes - cur + 4.0 * (double)pp->r[x].total;
            need.stage += 4.0 * 1.3 * add + 24.0 * (double)(theta - pp->have[x]);
        }
        need.greedy = std::max(need.greedy, 4.0 * 1.1 * (double)theta * m + 17.0 * (double)theta + 21.0 * n);
        need.n_max = std::max(need.n_max, q->q.graph->n);
        if (!pp->allocated && !pp->users) b += (double)graph_bytes(q->q.graph);
        return (size_t)b;
    }

    // Growth of the shared workspaces beyond what they hold now.
    size_t shared_growth(const Shared &need, const SharedBytes &have, hyperim_graph g) const {
        const double stage_cap = (double)((uint64_t)std::max<uint32_t>(g->tune.stage_mib, 64) << 20);
        const double slots = (double)rr_slot_bytes(need.n_max);
        double b = std::max(0.0, slots - (double)have.slots);
        b += std::max(0.0, std::min(need.stage, stage_cap) - (double)have.stage);
        b += std::max(0.0, need.greedy - (double)have.greedy);
        return (size_t)b;
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

    // A first sample of R1 (ids [0, Q)) for waiting queries on graphs without
    // a members-per-set estimate; those sets are the start of R1 anyway.
    int pilot(size_t used) {
        const uint64_t Q = 1ull << opt.qlog;
        std::vector<PoolPair *> pps;
        for (QueryRun *q : waiting) {
            PoolPair *pp = pool_for(q->q);
            if (members_per_id(pp) >= 0.0 || std::find(pps.begin(), pps.end(), pp) != pps.end()) continue;
            const uint64_t ids = std::min<uint64_t>(Q, q->next_theta(opt));
            const size_t worst = (size_t)(2.0 * 4.0 * 1.3 * (double)ids * (double)pp->g->n) + graph_bytes(pp->g);
            if (used + worst > budget) break;
            used += worst;
            pps.push_back(pp);
        }
        if (pps.empty()) return HYPERIM_OK;
        std::vector<RRTask> tasks;
        std::vector<hyperim_pool> dst;
        for (PoolPair *pp : pps) {
            HIM_CHECK(pp->ensure(stream));
            tasks.push_back(RRTask{pp->g, pp->seed, pp->instance, 0, 0, Q});
            dst.push_back(&pp->r[0]);
        }
        RRStats st;
        std::vector<int> status;
        HIM_CHECK(ev.create());
        float ms = 0.f;
        HIM_HIP(hipEventRecord(ev.a, stream));
        HIM_CHECK(generate_into(tasks, dst, opt.qlog, (int)opt.form, opt.max_entries, stream, st, &status,
                                (opt.flags & HYPERIM_FLAG_KERNEL_TIMES) != 0, (opt.flags & HYPERIM_FLAG_NO_GRAPHS) == 0));
        HIM_HIP(hipEventRecord(ev.b, stream));
        HIM_HIP(hipEventSynchronize(ev.b));
        HIM_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
        for (size_t i = 0; i < pps.size(); ++i) {
            if (status[i] == HYPERIM_OK)
                pps[i]->have[0] = Q;
            else
                pps[i]->clear();
        }
        add_stats(total, st, ms);
        // the sample is part of the piloted queries' generation
        for (QueryRun *q : waiting)
            if (std::find(pps.begin(), pps.end(), pool_for(q->q)) != pps.end()) add_stats(q->res, st, ms);
        return HYPERIM_OK;
    }

    // Generate ahead.  A generation call pays the traversal depth of its
    // deepest sets in supersteps however few sets it holds, and a call with
    // fewer sets than the device has phase-A wavefronts leaves some idle.  A
    // round whose call would add fewer than `ahead` sets (both pools, every
    // pool pair) therefore also takes the ids of the following rounds, a
    // doubling at a time, up to each pool pair's last admissible round; a
    // later round then finds its prefix in the pools.  The ids and their sets
    // are the same, so no result changes; sets a query never reaches are
    // spent work, at most about one call's worth.  With a finite budget, a
    // doubling is taken only while its estimated pool and stage bytes fit.
    int generate_ahead(const std::vector<QueryRun *> &live, const std::vector<PoolPair *> &pps,
                       std::vector<uint64_t> &target) {
        if (pps.empty() || opt.ahead == 1) return HYPERIM_OK;
        uint64_t want = opt.ahead;
        if (want == 0) {
            // two sets per phase-A wavefront of the device
            int device = 0, cus = 0;
            HIM_HIP(hipGetDevice(&device));
            HIM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
            const uint32_t per_cu = pps[0]->g->tune.blocks_a ? pps[0]->g->tune.blocks_a : 4u;
            want = 2ull * (uint64_t)cus * per_cu * 4u;
        }
        std::vector<uint64_t> cap(pps.size(), 0);
        for (QueryRun *q : live) {
            const size_t i = (size_t)(std::find(pps.begin(), pps.end(), q->pp) - pps.begin());
            cap[i] = std::max(cap[i], q->sc.theta1 << (q->sc.i_max ? q->sc.i_max - 1u : 0u));
        }
        auto added = [&](const std::vector<uint64_t> &t) {
            uint64_t a = 0;
            for (size_t i = 0; i < pps.size(); ++i)
                for (int x = 0; x < 2; ++x)
                    if (t[i] > pps[i]->have[x]) a += t[i] - pps[i]->have[x];
            return a;
        };
        size_t used = bounded() ? resident() : 0;
        for (;;) {
            const uint64_t now = added(target);
            if (now == 0 || now >= want) break;
            std::vector<uint64_t> next(target);
            double extra = 0.0;
            for (size_t i = 0; i < pps.size(); ++i) {
                if (2 * target[i] > cap[i] || 2 * target[i] > kMaxIds) continue;
                next[i] = 2 * target[i];
                double m = members_per_id(pps[i]);
                if (m < 0.0) m = (double)pps[i]->g->n;
                // both pools' members and offsets, old storage kept while growing, stage
                extra += 2.0 * (double)(next[i] - target[i]) * (4.0 * m * (2.0 + 1.3) + 36.0);
            }
            if (next == target) break;
            if (bounded() && (double)used + extra > (double)budget) break;
            used += (size_t)extra;
            target.swap(next);
        }
        return HYPERIM_OK;
    }

    // One round of every query in qs (none done): RR generation for all their
    // pools in one generation pass, then each query's greedy on R1[0, theta),
    // coverage of R2[0, theta) and bound test.  Per-query failures (a pool
    // over max_entries, theta beyond the id space) end that query only; a HIP
    // error is returned and ends them all.
    int run_round(const std::vector<QueryRun *> &qs) {
        const double tconst = 1.0 - std::exp(-1.0);
        const hipStream_t s = stream;
        const hyperim_options &o = opt;
        HIM_CHECK(ev.create());
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
        if (!o.theta_fixed && o.form == 0) HIM_CHECK(generate_ahead(live, pps, target));
        std::vector<RRTask> tasks;
        std::vector<hyperim_pool> dst;
        std::vector<size_t> task_pp;
        for (size_t i = 0; i < pps.size(); ++i) {
            PoolPair *pp = pps[i];
            pp->last_step = steps;
            HIM_CHECK(pp->ensure(s));
            for (uint32_t x = 0; x < 2; ++x) {
                if (target[i] <= pp->have[x]) continue;
                tasks.push_back(RRTask{pp->g, pp->seed, pp->instance, x, pp->have[x], target[i]});
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
            HIM_CHECK(generate_into(tasks, dst, o.qlog, (int)o.form, o.max_entries, s, st, &pool_status,
                                    (o.flags & HYPERIM_FLAG_KERNEL_TIMES) != 0, (o.flags & HYPERIM_FLAG_NO_GRAPHS) == 0));
            HIM_HIP(hipEventRecord(ev.b, s));
            HIM_HIP(hipEventSynchronize(ev.b));
            HIM_HIP(hipEventElapsedTime(&ms_rr, ev.a, ev.b));
            add_stats(total, st, ms_rr);
            for (size_t t = 0; t < tasks.size(); ++t)
                if (pool_status[t] != HYPERIM_OK) pp_status[task_pp[t]] = pool_status[t];
            for (size_t i = 0; i < pps.size(); ++i) {
                PoolPair *pp = pps[i];
                if (pp_status[i] == HYPERIM_OK) {
                    for (int x = 0; x < 2; ++x) pp->have[x] = std::max(pp->have[x], target[i]);
                } else {
                    pp->clear();   // a pool that did not take its new sets: both start over
                }
            }
        }
        int device = 0;
        HIM_HIP(hipGetDevice(&device));
        for (QueryRun *q : live) {
            size_t i = 0;
            while (pps[i] != q->pp) ++i;
            if (pp_status[i] != HYPERIM_OK) {
                set_error_detail("pool would exceed max_entries");
                q->fail(pp_status[i]);
                continue;
            }
            hyperim_result &res = q->res;
            add_stats(res, st, ms_rr);
            hyperim_graph g = q->q.graph;
            const uint64_t theta = q->next_theta(o);
            const uint32_t k = q->q.k;
            float ms = 0.f;
            uint64_t lambda2 = 0;
            std::vector<uint64_t> ub(o.bound == 0 ? (size_t)k + 1 : 0, 0ull);
            {
                DeviceLock lk(device);
                HIM_HIP(hipEventRecord(ev.a, s));
                HIM_CHECK(greedy_device(*lk.gr, g, &q->pp->r[0], theta, k, s, q->seeds.data(), q->gains.data(),
                                        o.bound == 0 ? ub.data() : nullptr));
                HIM_CHECK(coverage_device(*lk.gr, g, &q->pp->r[1], theta, lk.gr->out.as<uint32_t>(), k, s,
                                          &lambda2));
                HIM_HIP(hipEventRecord(ev.b, s));
                HIM_HIP(hipEventSynchronize(ev.b));
            }
            HIM_HIP(hipEventElapsedTime(&ms, ev.a, ev.b));
            res.ms_greedy += ms;
            total.ms_greedy += ms;
            uint64_t lambda1 = 0;
            for (uint32_t x = 0; x < k; ++x) lambda1 += q->gains[x];
            const double n = (double)g->n;
            const double sl = lower_bound((double)lambda2, q->sc.a, n, (double)theta);
            // the stop test's upper bound: Equation (8), or Lemma 5's closed form
            const uint64_t lam_u = o.bound == 0 ? eq8_coverage(q->gains, ub) : 0ull;
            const double su = o.bound == 0 ? upper_bound_cov((double)lam_u, q->sc.a, n, (double)theta)
                                           : upper_bound((double)lambda1, k, q->sc.a, n, (double)theta);
            q->round += 1;
            res.rounds = q->round;
            res.theta = theta;
            res.lambda1 = lambda1;
            res.lambda2 = lambda2;
            res.sigma_l = sl;
            res.sigma_u = su;
            res.lambda_u = lam_u;
            res.spread = n * (double)lambda2 / (double)theta;
            const bool stop =
                o.theta_fixed || (su > 0.0 && sl / su >= tconst - q->q.eps) || q->round >= q->sc.i_max;
            if (!stop) continue;
            // members of the two pool prefixes [0, theta)
            uint64_t e[2] = {0, 0};
            for (int x = 0; x < 2; ++x)
                HIM_HIP(hipMemcpyAsync(&e[x], q->pp->r[x].off + theta, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
            HIM_HIP(hipStreamSynchronize(s));
            res.entries1 = e[0];
            res.entries2 = e[1];
            if (o.flags & HYPERIM_FLAG_INCIDENCES) {
                RRWork w1, w2;
                HIM_CHECK(rr_incidences(g, &q->pp->r[0], theta, s, &w1));
                HIM_CHECK(rr_incidences(g, &q->pp->r[1], theta, s, &w2));
                res.incidences = w1.incidences + w2.incidences;
                res.alg_bytes = w1.alg_bytes + w2.alg_bytes;
                res.coins = w1.coins + w2.coins;
                res.philox_alg = w1.philox + w2.philox;
            }
            total.entries1 += res.entries1;
            total.entries2 += res.entries2;
            total.theta += theta;
            total.incidences += res.incidences;
            total.alg_bytes += res.alg_bytes;
            total.coins += res.coins;
            total.philox_alg += res.philox_alg;
            res.ms_total =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - q->t0).count();
            q->done = true;
        }
        return HYPERIM_OK;
    }

    // Admit what fits and run one round; `finished` receives the queries that
    // ended in this step (done or failed).
    int step(std::vector<QueryRun *> &finished, size_t *ran) {
        steps += 1;
        total.rounds = (uint32_t)steps;
        size_t used = bounded() ? resident() : 0;
        if (bounded()) HIM_CHECK(pilot(used));
        if (bounded()) used = resident();
        std::vector<QueryRun *> run;
        Shared need;
        const SharedBytes have = bounded() ? shared_bytes() : SharedBytes{0, 0, 0, 0, 0};
        size_t shared_so_far = 0;
        auto fits = [&](QueryRun *q) {
            if (!bounded()) return true;
            Shared trial = need;
            const size_t own = own_growth(q, trial);
            const size_t shared = shared_growth(trial, have, q->q.graph);
            const size_t delta = own + (shared > shared_so_far ? shared - shared_so_far : 0);
            if (used + delta > budget && !make_room(used, delta)) return false;
            need = trial;
            used += delta;
            shared_so_far = std::max(shared, shared_so_far);
            return true;
        };
        // running queries first, in admission order
        for (QueryRun *q : active)
            if (fits(q)) run.push_back(q);
        // then new queries, in submission order (no overtaking)
        while (!waiting.empty()) {
            QueryRun *q = waiting.front();
            q->pp = pool_for(q->q);
            if (!fits(q)) break;
            waiting.pop_front();
            q->pp->users += 1;
            active.push_back(q);
            run.push_back(q);
        }
        if (run.empty() && (!active.empty() || !waiting.empty())) {
            // nothing fits: the oldest query cannot run even alone
            QueryRun *q = nullptr;
            if (!active.empty()) {
                q = active.front();
                active.erase(active.begin());
            } else {
                q = waiting.front();
                waiting.pop_front();
                q->pp = pool_for(q->q);
                q->pp->users += 1;
            }
            set_error_detail("query does not fit the HBM budget");
            q->fail(HYPERIM_ECAPACITY);
            q->pp->users -= 1;
            finished.push_back(q);
        }
        int rc = HYPERIM_OK;
        if (!run.empty()) {
            rc = run_round(run);
            if (rc != HYPERIM_OK)
                for (QueryRun *q : run)
                    if (!q->done) q->fail(rc);
        }
        if (ran) *ran = run.size();
        for (size_t i = 0; i < active.size();) {
            QueryRun *q = active[i];
            if (q->done) {
                active.erase(active.begin() + (long)i);
                q->pp->users -= 1;
                finished.push_back(q);
            } else {
                ++i;
            }
        }
        return rc;
    }
};

}  // namespace
}  // namespace hyperim

using namespace hyperim;

// ---- serving session -------------------------------------------------------
struct hyperim_session_s {
    int device = 0;
    Engine eng;
    uint64_t next_ticket = 1;
    std::map<uint64_t, QueryRun *> finished;
    std::map<QueryRun *, uint64_t> ticket_of;
    hyperim_session_stats stats{};

    ~hyperim_session_s() {
        for (QueryRun *q : eng.waiting) delete q;
        for (QueryRun *q : eng.active) delete q;
        for (auto &kv : finished) delete kv.second;
    }
};

namespace {

// Lockstep rounds for queries[0, count) (none waits once admitted); with a
// finite budget, admission as in a session.
int run_queries(const hyperim_query *queries, uint32_t count, const hyperim_options &o, hipStream_t s, size_t budget,
                std::vector<std::unique_ptr<QueryRun>> &runs, hyperim_result *total) {
    const auto t0 = std::chrono::steady_clock::now();
    Engine eng;
    eng.stream = s;
    eng.opt = o;
    eng.budget = budget;
    for (uint32_t i = 0; i < count; ++i) {
        runs.emplace_back(new QueryRun());
        QueryRun *r = runs.back().get();
        r->q = queries[i];
        start(*r, o);
        eng.waiting.push_back(r);
    }
    std::vector<QueryRun *> finished;
    int rc = HYPERIM_OK;
    while (!eng.waiting.empty() || !eng.active.empty()) {
        rc = eng.step(finished, nullptr);
        if (rc != HYPERIM_OK) {
            for (QueryRun *q : eng.active)
                if (!q->done) q->fail(rc);
            for (QueryRun *q : eng.waiting) q->fail(rc);
            break;
        }
    }
    if (total) {
        *total = eng.total;
        total->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return rc;
}

}  // namespace

extern "C" {

int hyperim_select_seeds(hyperim_graph g, uint32_t k, double eps, double ell, uint64_t seed, uint32_t instance,
                         const hyperim_options *opt, void *stream, uint32_t *seeds, uint64_t *gains,
                         hyperim_result *out) {
    if (!g || !seeds) return HYPERIM_EINVAL;
    clear_error_detail();
    const hyperim_options o = normalize(opt);
    hyperim_query q{g, k, instance, eps, ell, seed};
    HIM_CHECK(validate(q, o));
    std::vector<std::unique_ptr<QueryRun>> runs;
    HIM_CHECK(run_queries(&q, 1, o, as_stream(stream), ~(size_t)0, runs, nullptr));
    const QueryRun &r = *runs[0];
    if (r.status != HYPERIM_OK) return r.status;
    std::copy(r.seeds.begin(), r.seeds.end(), seeds);
    if (gains) std::copy(r.gains.begin(), r.gains.end(), gains);
    if (out) *out = r.res;
    return HYPERIM_OK;
}

int hyperim_select_seeds_batch(const hyperim_query *queries, uint32_t count, const hyperim_options *opt,
                               void *stream, uint32_t *seeds, uint64_t *gains, hyperim_result *results,
                               int *status, hyperim_result *total) {
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
    // budget: the device memory free now plus what the batch already holds
    // (its graphs, the shared workspaces), less a reserve
    size_t free_b = 0, total_b = 0;
    HIM_HIP(hipMemGetInfo(&free_b, &total_b));
    std::vector<hyperim_graph> gs;
    size_t held = device_shared_bytes();
    for (uint32_t i = 0; i < count; ++i)
        if (std::find(gs.begin(), gs.end(), queries[i].graph) == gs.end()) {
            gs.push_back(queries[i].graph);
            held += graph_bytes(queries[i].graph);
        }
    const size_t reserve = 4ull << 30;
    const size_t budget = free_b + held > reserve ? free_b + held - reserve : 0;
    std::vector<std::unique_ptr<QueryRun>> runs;
    const int rc = run_queries(queries, count, o, as_stream(stream), budget, runs, total);
    int first_fail = rc;
    uint64_t at = 0;
    for (uint32_t i = 0; i < count; ++i) {
        const QueryRun &r = *runs[i];
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
    s->eng.opt = o;
    s->eng.stream = as_stream(stream);
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
    s->eng.budget = hbm_budget;
    s->stats.hbm_budget = hbm_budget;
    *out = s;
    return HYPERIM_OK;
}

int hyperim_session_submit(hyperim_session s, const hyperim_query *q, uint64_t *ticket) {
    if (!s || !q || !ticket) return HYPERIM_EINVAL;
    clear_error_detail();
    HIM_CHECK(validate(*q, s->eng.opt));
    if (q->graph->device != s->device) {
        set_error_detail("the graph lives on another device than the session");
        return HYPERIM_EINVAL;
    }
    QueryRun *r = new (std::nothrow) QueryRun();
    if (!r) return HYPERIM_ENOMEM;
    r->q = *q;
    start(*r, s->eng.opt);   // latency of the query counts from submission
    const uint64_t t = s->next_ticket++;
    s->ticket_of[r] = t;
    s->eng.waiting.push_back(r);
    s->stats.submitted += 1;
    *ticket = t;
    return HYPERIM_OK;
}

int hyperim_session_step(hyperim_session s, hyperim_session_stats *out) {
    if (!s) return HYPERIM_EINVAL;
    clear_error_detail();
    const size_t waiting_before = s->eng.waiting.size();
    std::vector<QueryRun *> done;
    size_t ran = 0;
    const int rc = s->eng.step(done, &ran);
    s->stats.steps = s->eng.steps;
    s->stats.admitted += waiting_before - s->eng.waiting.size();
    s->stats.ran_last = ran;
    for (QueryRun *q : done) {
        if (q->status == HYPERIM_OK)
            s->stats.finished += 1;
        else
            s->stats.failed += 1;
        s->finished[s->ticket_of[q]] = q;
        s->ticket_of.erase(q);
    }
    s->stats.active = (uint32_t)s->eng.active.size();
    s->stats.waiting = (uint32_t)s->eng.waiting.size();
    s->stats.bytes_resident = s->eng.resident();
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
    for (QueryRun *q : s->eng.active)
        if (q->q.graph == g) return HYPERIM_ESTATE;
    for (QueryRun *q : s->eng.waiting)
        if (q->q.graph == g) return HYPERIM_ESTATE;
    HIM_HIP(hipStreamSynchronize(s->eng.stream));
    auto &pools = s->eng.pools;
    for (size_t i = 0; i < pools.size();) {
        if (pools[i]->g == g)
            pools.erase(pools.begin() + (long)i);
        else
            ++i;
    }
    return HYPERIM_OK;
}

int hyperim_session_stats_get(hyperim_session s, hyperim_session_stats *out) {
    if (!s || !out) return HYPERIM_EINVAL;
    s->stats.bytes_resident = s->eng.resident();
    *out = s->stats;
    return HYPERIM_OK;
}

void hyperim_session_free(hyperim_session s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->eng.stream);
    delete s;
}

}  // extern "C"
