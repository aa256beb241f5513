/*
 * hyperim.h -- C ABI of libhyperim.so, an MI355X (gfx950) implementation of
 * the hot path of HyperIM: influence maximization in hypergraphs by
 * stratified reverse-reachable (RR) set sampling and greedy max coverage.
 *
 * Problem (Section 2.1, Definition 1): given a hypergraph G = (V, HE), an
 * integer k and a cascade model, find k vertices of largest expected
 * influence in the weighted clique graph G_w.  Influence is estimated from
 * RR sets (Equation (1)): I(S) = |V| Pr[S meets R], estimated as
 * |V| Lambda_R(S) / |R|.
 *
 * Conventions for every call:
 *   - return value: HYPERIM_OK (0) or a negative status below; on error no
 *     output is partially valid and hyperim_strerror() names the cause;
 *   - `stream` is a hipStream_t (NULL = the default stream); device work is
 *     ordered on it; calls that return host values synchronise it first;
 *   - input arrays are borrowed for the duration of the call and never
 *     retained; handles own their device memory until *_free;
 *   - vertex ids are uint32 in [0, n); hyperedge ids uint32 in [0, m);
 *     1 <= n <= 2^31, m < 2^32 - 1 and the number of incidences
 *     nnz = he_off[m] < 2^32 (else HYPERIM_EINVAL);
 *   - distinct handles may be used from different threads; one handle must
 *     not be used by two threads at once (RR generation on one device is
 *     serialised internally: it shares that device's workspace).
 */
#ifndef HYPERIM_H
#define HYPERIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HYPERIM_OK 0
#define HYPERIM_EINVAL (-1)     /* bad argument or malformed hypergraph        */
#define HYPERIM_ENOMEM (-2)     /* device or host allocation failed             */
#define HYPERIM_ECAPACITY (-3)  /* caller-provided pool buffer too small        */
#define HYPERIM_ESTATE (-4)     /* call out of order (e.g. before stratify)     */
#define HYPERIM_EHIP (-5)       /* HIP runtime error (see hyperim_strerror)     */
#define HYPERIM_PENDING 1       /* hyperim_session_poll: query not finished yet */

#define HYPERIM_MODEL_CONST 0u  /* every channel into v live with probability p */
#define HYPERIM_MODEL_WC 1u     /* weighted cascade: p_v = 1 / c(v)             */
#define HYPERIM_MODEL_LT_CONST 2u /* linear threshold, channel weight p         */
#define HYPERIM_MODEL_LT_WC 3u  /* linear threshold, channel weight 1 / c(v)    */
#define HYPERIM_MODEL_LAYERED 4u /* stratified setting of Section 3.1.1         */
#define HYPERIM_MODEL_GAPS_CONST 5u /* IC with constant p, by geometric gaps    */
#define HYPERIM_MODEL_GAPS_WC 6u /* weighted-cascade IC, by geometric gaps      */
#define HYPERIM_NSTRATA 8u

typedef struct hyperim_graph_s *hyperim_graph;
typedef struct hyperim_pool_s *hyperim_pool;
typedef struct hyperim_session_s *hyperim_session;

/* Independent-cascade channel probabilities (Section 2.1, "Cascade models",
 * IC).  Every hyperedge he and every ordered pair u != v of its members is
 * one channel u -> v, live with probability p_v of the target:
 *   HYPERIM_MODEL_CONST: p_v = p (p >= 1 means always live; p must not be
 *                        NaN or negative);
 *   HYPERIM_MODEL_WC:    p_v = (float)(1.0 / c(v)), c(v) = sum over
 *                        hyperedges he containing v of (|he| - 1), the
 *                        weighted in-degree of v in G_w; p is ignored.
 * A channel is live when its coin is below floor(p_v * 2^32).
 *
 * Linear-threshold model (Section 2.1, "Cascade models", LT), in its
 * live-edge form: HYPERIM_MODEL_LT_CONST and HYPERIM_MODEL_LT_WC take p_v as
 * the two IC models do; every vertex v keeps at most one of its c(v) channels
 * (hyperedges of v in ascending order, members in the caller's order, v
 * skipped), each with weight W_v / 2^32, W_v = min(floor(p_v * 2^32),
 * floor(2^32 / c(v))) (p_v >= 1 counting as 2^32), so that the weights into v
 * sum to at most 1.  The Philox word of (RR id, v) at hyperedge slot
 * 0xFFFFFFFE, position 0, picks channel floor(x / W_v) when x < W_v c(v),
 * none otherwise; an RR set is the reverse walk from its root along kept
 * channels until none is kept or the walk meets a vertex already in it.
 *
 * Stratified setting (Section 3.1.1, "Activation probability" and
 * "Sampling strategy"; Algorithm 3's per-layer draws), HYPERIM_MODEL_LAYERED,
 * p ignored: A(v), the co-members of v, in layers by w(v,u) (layer 1 the
 * largest, ascending ids within a layer); a member of layer i (n members, l
 * layers) activates v with p = min(1, P / n), P = 1 / (i ln(l + 1)).  RR
 * sets: per popped vertex v and layer i, the Philox blocks at counter
 * (j_lo, i, v, pool << 31 | j_hi << 24 | r), r = 0, 1, ...; block 0's words 0
 * and 1 give U = (w0 >> 11 | w1 << 21) / 2^53 and the count h inverts U --
 * Binomial(n, p) for n <= 20 (p = 1: h = n), else Poisson(P) truncated at
 * min(n, 64) -- with the recursions prob_{h+1} = ((prob_h (n - h)) / (h + 1))
 * (p / q) from q^n, and prob_{h+1} = (prob_h P) / (h + 1) from e^-P; the
 * following words x pick, h times, index floor(x (n - r) / 2^32) among the
 * layer's members not picked yet (ascending).  Picked members outside the
 * set join it.  ln and exp come from the host's C library.
 *
 * Independent cascade drawn by geometric gaps (the subset sampling of Section
 * 2.2.1, Algorithm 2), HYPERIM_MODEL_GAPS_CONST and HYPERIM_MODEL_GAPS_WC (p_v
 * as for the two IC models): the same cascade, with
 * the live positions of each stream (RR id j, hyperedge he, target v) -- he's
 * member positions in the caller's order, each live with p_v, a live
 * position holding v itself ignored -- found by skipping over the dead ones.
 * Gap r of the stream (the dead positions before the next live one, G
 * positions left) comes from word r mod 4 of the Philox block at counter
 * (j_lo, he, v, pool << 31 | j_hi << 24 | r / 4): with t = (2^32 - x) / 2^32
 * for word x, q = 1 - p_v and S_0 = q, S_{i+1} = S_i * S_i, the gap is built
 * bit by bit from the top bit of G, taking bit i when the gap stays <= G and
 * acc * S_i >= t (then acc *= S_i; acc starts at 1), in IEEE double; a gap of
 * G ends the stream.  Sets are not equal to the coin models' sets for the
 * same seed (different random numbers), but have the same distribution. */
typedef struct {
    uint32_t model;
    float p;
} hyperim_prob;

/* Statistics of the sample-set layers (Section 3.1.1; Section 4.1's F_cnt,
 * T_cnt, L_cnt; Theorem 2's theta(l*)) and the strata boundaries. */
typedef struct {
    uint32_t B[HYPERIM_NSTRATA + 1]; /* stratum h holds P[B[h] .. B[h+1])      */
    uint64_t sum_top;                /* F_cnt = sum_v n(L_1(v))                 */
    uint64_t sum_deg;                /* T_cnt = sum_v deg(v) in G_w             */
    uint64_t sum_l;                  /* L_cnt = sum_v l_v                       */
    double alpha;                    /* F_cnt / T_cnt                           */
    double beta;                     /* L_cnt / |V|                             */
    double theta_l;                  /* (1/|V|) sum_v l_v / ln(l_v + 1)         */
} hyperim_strata_info;

/* Options of hyperim_select_seeds (zero-initialised = defaults). */
typedef struct {
    uint32_t qlog;          /* pool ladder base Q = 2^qlog; 0 -> 8; max 24    */
    uint32_t form;          /* 0: one persistent launch per pool block;
                               1: plain form, one launch per stratum          */
    uint64_t theta_fixed;   /* > 0: one round of exactly this many RR sets per
                               pool and no bound test                         */
    uint64_t max_entries;   /* > 0: fail with HYPERIM_ECAPACITY rather than let
                               a pool exceed this many members                */
    uint32_t flags;         /* HYPERIM_FLAG_* bits                            */
    uint32_t ahead;         /* a round whose RR generation would add fewer
                               sets than this (both pools, all queries) also
                               generates the ids of the following rounds, a
                               doubling at a time (same sets, same results;
                               unreached sets are spent work); 0 -> two per
                               phase-A wavefront of the device, 1 -> off.
                               Not with theta_fixed or form 1.              */
    uint32_t bound;         /* upper bound of the stop test: 0 = Equation (8),
                               the smallest over the greedy prefixes S_i*
                               (i = 0..k) of Lambda_R1(S_i*) plus the k
                               largest marginal coverages given S_i*
                               (Lemma 4, p_max = 1); 1 = Lemma 5's closed
                               form Lambda_R1(S_k*) / (1 - (1 - 1/k)^k)      */
} hyperim_options;

#define HYPERIM_FLAG_KERNEL_TIMES 2u /* time every expansion-kernel launch
                                         with events its launch stamps
                                         (fills ms_expand; costs a few
                                         percent of a small query)       */
#define HYPERIM_FLAG_INCIDENCES 1u  /* fill hyperim_result.incidences (one extra
                                       pass over the final pools)            */
#define HYPERIM_FLAG_NO_GRAPHS 4u   /* launch every superstep kernel directly
                                       instead of replaying captured batches
                                       (HIP graphs); same results           */

/* Outcome of hyperim_select_seeds. */
typedef struct {
    uint32_t rounds;        /* doubling rounds executed                       */
    uint32_t i_max;         /* last admissible round                          */
    uint64_t theta;         /* RR sets per pool in the final round            */
    uint64_t lambda1;       /* coverage of S* in R1 (sum of the gains)        */
    uint64_t lambda2;       /* coverage of S* in R2                           */
    double sigma_l;         /* Equation (12) lower bound on I(S*)             */
    double sigma_u;         /* Lemma 5 upper bound on the optimum             */
    double spread;          /* |V| lambda2 / theta, unbiased estimate of I(S*)*/
    double theta_max;       /* Lemma 6 / Equation (13) cap                    */
    uint64_t entries1;      /* members stored in R1[0, theta)                 */
    uint64_t entries2;      /* members stored in R2[0, theta)                 */
    uint64_t incidences;    /* incidences read by RR generation (both pools)  */
    double ms_rr;           /* device time in RR generation + compaction      */
    double ms_greedy;       /* device time in coverage, greedy and R2 check   */
    double ms_total;        /* wall time of the call                          */
    uint64_t alg_bytes;     /* algorithmic bytes of RR generation (both pools):
                               sum over members v of 20 + 12 d(v) + 4 S(v),
                               d(v) = hyperedges of v, S(v) = their total size;
                               filled with HYPERIM_FLAG_INCIDENCES            */
    double ms_bfs;          /* device time of the RR-generation kernels alone  */
    uint64_t bfs_launches;  /* number of RR-generation kernel launches         */
    double ms_light;        /* part of ms_bfs spent in the per-set phase       */
    double ms_heavy;        /* part of ms_bfs spent in the grid-wide phase     */
    uint64_t deferred;      /* RR sets handed to the grid-wide phase           */
    uint64_t supersteps;    /* grid-wide supersteps launched                   */
    uint64_t bytes_light;   /* algorithmic bytes expanded by the per-set phase */
    uint64_t bytes_heavy;   /* ... by the grid-wide phase's per-set expansion  */
    double ms_expand;       /* with HYPERIM_FLAG_KERNEL_TIMES: part of ms_heavy
                               spent in the per-set expansion kernel of the
                               grid-wide phase (events each launch stamps)  */
    uint64_t expand_launches; /* its launches (one per superstep)              */
    uint64_t philox_drawn;  /* Philox4x32-10 blocks the RR-generation kernels
                               drew (a block gives the coins of up to four
                               channels; channels from members a set already
                               holds need none)                               */
    uint64_t coins;         /* with HYPERIM_FLAG_INCIDENCES: channels of the
                               final pools' members, sum of c(v) = S(v) - d(v)
                               over the members of R1[0, theta) and
                               R2[0, theta)                                   */
    uint64_t philox_alg;    /* with HYPERIM_FLAG_INCIDENCES: Philox blocks a
                               per-set traversal of the same sets draws, sum
                               over their members of sum over v's hyperedges
                               of ceil(|he| / 4)                              */
    uint64_t philox_bundled; /* part of philox_drawn drawn in bundled mode     */
    uint64_t bytes_bundled; /* algorithmic bytes expanded in bundled mode      */
    double ms_bundled;      /* with HYPERIM_FLAG_KERNEL_TIMES: device time of
                               the bundled expansion kernel's launches        */
    uint64_t bundled_launches; /* its launches                                */
    uint64_t philox_light;  /* part of philox_drawn drawn by the per-set phase */
    uint64_t lambda_u;      /* upper bound on the optimal coverage of R1 that
                               sigma_u lifts (Equation (8) or Lemma 5)       */
} hyperim_result;

/* Build the device-resident hypergraph (Section 2.1: G = (V, HE), V(he)).
 * he_off[m+1] (nondecreasing, he_off[0] = 0) and he_mem[he_off[m]] give the
 * members of every hyperedge in the caller's order; ptrs_on_device != 0 means
 * both are device pointers, else host pointers.  Hyperedges of size 0 or 1
 * are legal (no channels); a vertex repeated inside one hyperedge, an id >= n
 * or decreasing offsets give HYPERIM_EINVAL.  Builds the vertex -> hyperedge
 * incidence lists (ascending hyperedge ids) and per-target coin thresholds;
 * the clique graph G_w is never materialised.  *out receives a new handle. */
int hyperim_build_graph(uint32_t n, uint32_t m, const uint32_t *he_off, const uint32_t *he_mem,
                        int ptrs_on_device, hyperim_prob prob, void *stream, hyperim_graph *out);

/* Sample-set division (Section 3.1.1): for each vertex v, the co-membership
 * weight w(v,u) = number of hyperedges shared with u; the layers of A(v) are
 * its groups of equal w (layer 1 = largest w); l_v = number of layers,
 * deg(v) = |A(v)|, top(v) = n(L_1).  Stratum s(v) = 0 if l_v = 0, else
 * min(7, 1 + floor(log2 l_v)); P = vertices sorted by (s(v), v).  Required
 * before hyperim_generate_rr / hyperim_select_seeds.  `out` may be NULL. */
int hyperim_stratify(hyperim_graph g, void *stream, hyperim_strata_info *out);

/* Division of the RR sets into R1 and R2 (Section 4.1, "Division of the RR
 * sets"), opt-in and biased.  With alpha = F_cnt / T_cnt and beta =
 * L_cnt / |V| of the graph's strata, layer i (1 <= i <= floor(beta)) of A(v)
 * is small when n(L_i) < alpha |A(v)| (compared exactly as
 * n(L_i) T_cnt < F_cnt |A(v)|).  on = 1: pool 0 (R1) draws its roots, with the
 * usual stratified sampling, only from the vertices that have a small layer
 * (in the order of P), and each of its RR sets starts from the root and all
 * members of the root's small layers together (their channels into the root
 * count as live); pool 1 (R2) draws its roots from the other vertices.  The
 * estimators keep their factor n / theta, so R2's lower bound estimates n
 * times the mean over the R2 vertices only, not the spread.  on = 0 undoes it.
 * When every vertex or none has a small layer the division is inert.
 * Independent-cascade models only (HYPERIM_EINVAL otherwise); needs
 * hyperim_stratify first (HYPERIM_ESTATE); switching the division on or off
 * after the graph's first RR set gives HYPERIM_ESTATE (pools would mix both
 * kinds of sets); a later hyperim_stratify keeps it; a failed call leaves
 * the graph undivided.  Builds the layer tables of A(v) on the device
 * when the graph has none (HYPERIM_EINVAL beyond 2^32 co-member occurrences
 * or 16384 layers).  *n_r1 (may be NULL) receives the number of R1 vertices. */
int hyperim_route(hyperim_graph g, uint32_t on, void *stream, uint32_t *n_r1);

/* Copy the graph's derived arrays to caller buffers (host pointers unless
 * dst_on_device != 0); any pointer may be NULL.  Sizes: v_off n+1, v_he nnz,
 * thr n, c n (uint64), l/deg/top/P n, stratum n (uint8).  The strata arrays
 * need a prior hyperim_stratify (else HYPERIM_ESTATE). */
int hyperim_graph_read(hyperim_graph g, uint32_t *v_off, uint32_t *v_he, uint32_t *thr, uint64_t *c,
                       uint32_t *l, uint32_t *deg, uint32_t *top, uint8_t *stratum, uint32_t *P,
                       int dst_on_device, void *stream);

/* A pool of RR sets stored as a CSR over consecutive ids.  dev_buf == NULL:
 * the library allocates and grows the storage.  Otherwise the caller's
 * device buffer of `bytes` bytes holds everything (it is never freed by the
 * library) and `id_capacity` bounds the number of ids; a generate call that
 * does not fit returns HYPERIM_ECAPACITY and hyperim_pool_required() then
 * reports the bytes needed. */
int hyperim_pool_create(hyperim_graph g, void *dev_buf, size_t bytes, uint64_t id_capacity,
                        hyperim_pool *out);

/* RR sets [id_begin, id_end) of pool `pool_tag` (0 = R1, 1 = R2) for key
 * (seed, instance), appended to `pool`.  An empty pool accepts any id_begin;
 * a non-empty pool only its current end and the same (seed, instance,
 * pool_tag) (else HYPERIM_EINVAL).  seed must be < 2^32.
 * RR set j (Algorithm 3's skeleton): root r(j) from the stratified ladder
 * (block b of the pool's ladder, t-th id of the block: P[floor((t n + o_b) /
 * T_b)]), then every vertex with a live path of channels to the root.
 * Channel (he, u -> v) of RR set j is live when word (pos & 3) of
 * Philox4x32-10 with key (seed, instance) and counter
 * (j mod 2^32, he, v, pool_tag << 31 | (j >> 32) << 24 | pos >> 2), pos being
 * u's index in he, is below v's threshold.  Members are stored ascending. */
int hyperim_generate_rr(hyperim_graph g, uint64_t seed, uint32_t instance, uint32_t pool_tag,
                        uint64_t id_begin, uint64_t id_end, hyperim_pool pool, void *stream);

/* One RR-generation task of a batched call: ids [id_begin, id_end) of pool
 * `pool_tag` on `graph` for key (seed, instance), appended to `pool` (whose
 * graph it must be), with the rules of hyperim_generate_rr. */
typedef struct {
    hyperim_graph graph;
    hyperim_pool pool;
    uint64_t seed;
    uint32_t instance, pool_tag;
    uint64_t id_begin, id_end;
} hyperim_rr_task;

/* hyperim_generate_rr for `count` tasks at once (Algorithm 3 for every id of
 * every task): form 0 lays the tasks back to back into shared launch groups
 * -- all strata, both pools and many IM instances in the same persistent
 * launches -- and form 1 launches each (task, ladder block, stratum) range
 * on its own.  The pools receive exactly the sets that one
 * hyperim_generate_rr call per task would give them.  Two tasks must not name
 * the same pool.  Stream-ordered; returns after the stream has drained.
 * Errors as for hyperim_generate_rr, checked for every task before any work. */
int hyperim_generate_rr_batch(const hyperim_rr_task *tasks, uint32_t count, uint32_t form, void *stream);

/* Device pointers of the pool's CSR (rr_off[count+1] uint64 relative to the
 * pool, rr_mem, rr_root[count]) and its id range; valid until the next call
 * on the pool. */
int hyperim_pool_view(hyperim_pool pool, const uint64_t **off, const uint32_t **mem,
                      const uint32_t **roots, uint64_t *id_begin, uint64_t *count);

/* Copy the pool's CSR to caller buffers (host unless dst_on_device != 0). */
int hyperim_pool_read(hyperim_pool pool, uint64_t *off, uint32_t *mem, uint32_t *roots,
                      int dst_on_device, void *stream);

/* Bytes a caller buffer needs for the last failed generate call. */
int hyperim_pool_required(hyperim_pool pool, size_t *bytes);

/* Empty the pool (keeps its storage). */
int hyperim_pool_reset(hyperim_pool pool);

/* Greedy max coverage over the first theta sets of a pool (Algorithm 1 with
 * Equation (2)): k rounds, each taking the unchosen vertex of largest
 * marginal coverage (ties to the smallest id) and removing the sets it
 * covers.  seeds[k] and gains[k] are host arrays. */
int hyperim_greedy(hyperim_graph g, hyperim_pool pool, uint64_t theta, uint32_t k, void *stream,
                   uint32_t *seeds, uint64_t *gains);

/* Lambda_R(S): how many of the first theta sets of the pool meet the k seeds
 * (host array). */
int hyperim_coverage(hyperim_graph g, hyperim_pool pool, uint64_t theta, const uint32_t *seeds,
                     uint32_t k, void *stream, uint64_t *covered);

/* hyperim_coverage for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the seeds (seeds_dev[k]) and the result (*covered_dev) are in
 * device memory, the work is queued on `stream` and the call returns without
 * waiting.  It allocates nothing: its scratch (hit counters, n bytes of seed
 * flags, 8 bytes per set for the sets above 4096 members) lives in a 32 MiB
 * static device array of the library, held by every device the library runs
 * on until the process ends; n + 8 theta above about 32 MiB gives
 * HYPERIM_ECAPACITY.  Seed ids >= n are ignored.  Calls on one device share
 * that array, so calls that overlap on one device race (order them on one
 * stream); each call clears what it uses with a fill kernel, no memset. */
int hyperim_coverage_noalloc(hyperim_graph g, hyperim_pool pool, uint64_t theta, const uint32_t *seeds_dev,
                             uint32_t k, void *stream, uint64_t *covered_dev);

/* HyperIM_BRR (Algorithm 4) with delta = n^-ell: pools R1 and R2 grow over
 * the ladder theta_i = theta_1 2^(i-1) (theta_1 = theta_0 of Section 4.3
 * rounded up to the ladder); S* = greedy on R1[0, theta_i); Lambda2 =
 * coverage of S* in R2[0, theta_i); stop when sigma_l / sigma_u >=
 * 1 - 1/e - eps (Equation (12), Lemma 5 with p_max = 1) or at round i_max,
 * where theta_i reaches theta_max (Lemma 6 in its OPIM-C form).
 * seeds[k] and gains[k] are host arrays; `opt` may be NULL. */
int hyperim_select_seeds(hyperim_graph g, uint32_t k, double eps, double ell, uint64_t seed,
                         uint32_t instance, const hyperim_options *opt, void *stream,
                         uint32_t *seeds, uint64_t *gains, hyperim_result *out);

/* One influence-maximization query (Definition 1's input plus the sampling
 * key): a stratified graph on the current device, k, eps, ell, and the
 * Philox key (seed < 2^32, instance). */
typedef struct {
    hyperim_graph graph;
    uint32_t k;
    uint32_t instance;
    double eps, ell;
    uint64_t seed;
} hyperim_query;

/* hyperim_select_seeds for `count` queries at once, on one or several graphs.
 * Round i of every unfinished query runs together: the RR sets that all of
 * them need for the round are generated in shared launches (all strata, both
 * pools, all instances), then each query takes its greedy step and bound test.
 * Queries with the same graph and key share their pools.  Every query's
 * seeds, gains and result fields other than the timings equal those of
 * hyperim_select_seeds on that query alone; timings cover the shared launches
 * the query took part in.  seeds and gains (may be NULL) are host arrays
 * holding query 0's k_0 entries, then query 1's, and so on; results[count]
 * and status[count] may be NULL.  *total (may be NULL) receives the whole
 * batch: rounds = rounds run, theta / entries / incidences / alg_bytes summed
 * over the queries, device times and kernel counters of every launch once,
 * ms_total the wall time.  Queries are admitted as the device memory allows
 * (as in a session whose budget is the memory free at the call plus what the
 * batch already holds, less 4 GiB); the first sample of R1 on a graph not
 * seen before also sizes its admission.  Returns HYPERIM_OK when every query
 * succeeded, else the first failing query's status (status[] tells which);
 * a malformed query (as for hyperim_select_seeds) fails the whole call with
 * HYPERIM_EINVAL before any work. */
int hyperim_select_seeds_batch(const hyperim_query *queries, uint32_t count, const hyperim_options *opt,
                               void *stream, uint32_t *seeds, uint64_t *gains, hyperim_result *results,
                               int *status, hyperim_result *total);

/* Serving session: queries are submitted at any time and advanced together,
 * one doubling round of every admitted query per hyperim_session_step
 * (continuous batching: a query submitted while others run joins at the next
 * step).  RR pools stay resident, keyed by (graph, seed, instance), so a
 * later query with the same key reuses the prefix already generated.
 * Admission (at each step, in submission order) keeps the device bytes of
 * the graphs in use, the resident pools, the greedy workspaces and the RR
 * workspace within hbm_budget (0 = the device's memory less 8 GiB), using a
 * learned members-per-RR-set estimate; idle pools are evicted least recently
 * used first; a running query whose next round does not fit waits; a query
 * that cannot fit even alone fails with HYPERIM_ECAPACITY.  Results are those
 * of hyperim_select_seeds on the query alone.  `opt` applies to every query
 * (theta_fixed, form, qlog, max_entries, flags).  A session handle must not
 * be used by two threads at once; graphs must outlive their use by the
 * session (hyperim_session_drop releases a graph's pools). */
typedef struct {
    uint64_t submitted, admitted, finished, failed;  /* totals since creation       */
    uint32_t active, waiting;   /* queries admitted and running / not yet admitted */
    uint64_t steps;             /* hyperim_session_step calls                      */
    uint64_t ran_last;          /* queries advanced by the last step               */
    size_t bytes_resident;      /* graphs in use + pools + greedy + RR workspace  */
    size_t hbm_budget;
} hyperim_session_stats;

int hyperim_session_create(size_t hbm_budget, const hyperim_options *opt, void *stream, hyperim_session *out);
/* Queue a query (validated as for hyperim_select_seeds); *ticket names it. */
int hyperim_session_submit(hyperim_session s, const hyperim_query *q, uint64_t *ticket);
/* Admit what fits and advance every admitted query by one round; `out` may
 * be NULL.  Returns a HIP error if the device work failed (then the session's
 * queries of that step fail). */
int hyperim_session_step(hyperim_session s, hyperim_session_stats *out);
/* HYPERIM_PENDING while the query runs or waits; else its status, with
 * seeds[k], gains[k] (may be NULL) and *out (may be NULL) filled on
 * HYPERIM_OK.  A finished ticket is forgotten once polled. */
int hyperim_session_poll(hyperim_session s, uint64_t ticket, uint32_t *seeds, uint64_t *gains,
                         hyperim_result *out);
/* Release the resident pools of graph g (HYPERIM_ESTATE while a query on g
 * is running or waiting). */
int hyperim_session_drop(hyperim_session s, hyperim_graph g);
int hyperim_session_stats_get(hyperim_session s, hyperim_session_stats *out);
void hyperim_session_free(hyperim_session s);

/* The RR-generation workspace is shared by every graph of a device and kept
 * between calls: its current size on the current device, and its release. */
int hyperim_workspace_info(size_t *bytes);
int hyperim_workspace_release(void);

/* Execution parameters of RR generation (a schedule, not the method: every
 * setting produces the same bytes).  Zero fields keep their defaults.
 *   heavy:         a set whose next frontier batch holds a vertex with more
 *                  hyperedges than this moves to the grid-wide phase (1024);
 *   budget:        ... or once it has read this many incidences (262144);
 *   chunk:         incidences per heavy-vertex work item (256);
 *   seg:           light incidences per frontier-segment work item (512,
 *                  raised to chunk if smaller);
 *   prefilter_min: the grid-wide phase tests visited marks before coins in
 *                  sets of at least this many members (0xFFFFFFFF: never;
 *                  the scattered mark loads cost more than the coins they
 *                  save on the workloads measured);
 *   steps_per_sync: grid-wide supersteps launched between host checks (8);
 *   stage_mib:     staging memory a generation pass aims at: launch groups
 *                  are cut so that their members fit (16384 MiB, min 64);
 *   blocks_a:      per-set phase workgroups per compute unit, at most the
 *                  occupancy limit (4; 0 = the occupancy limit);
 *   blocks_b:      grid-wide expansion workgroups per compute unit (6; 0 =
 *                  the occupancy limit);
 *   ms_filter:     bundled mode reads the members' seen masks before drawing
 *                  coins only for frontier entries that carry at least this
 *                  many sets (1 = always; 65 = never: every set of an entry
 *                  draws its coins and the level's advance drops members a
 *                  set already holds);
 *   ms_min:        graphs whose RR sets hold at least this many members on
 *                  average (learned from earlier launches) grow their sets
 *                  in bundles of 64, bit-parallel over the sets: each vertex
 *                  expansion serves every set that reached it in the same
 *                  level (0xFFFFFFFF = never, the default: it helps on some
 *                  supercritical graphs and hurts on others, so the
 *                  autotuner decides). */
typedef struct {
    uint32_t heavy, budget, chunk, seg, prefilter_min, steps_per_sync;
    uint32_t stage_mib, blocks_a, blocks_b, ms_min, ms_filter;
} hyperim_tuning;

/* Set / read the execution parameters of graph g (host-side values).  A
 * launch that covers several graphs uses those of its first task's graph. */
int hyperim_set_tuning(hyperim_graph g, const hyperim_tuning *t);
int hyperim_get_tuning(hyperim_graph g, hyperim_tuning *t);

void hyperim_pool_free(hyperim_pool pool);
void hyperim_graph_free(hyperim_graph g);

/* Text for a status code (thread-local detail of the last HIP error). */
const char *hyperim_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* HYPERIM_H */
