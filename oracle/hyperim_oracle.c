/*
 * hyperim_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU implementation of HyperIM's hot path
 * (influence maximization in hypergraphs by RR-set sampling plus greedy max
 * coverage).  It exists to check the GPU library: only the test suite, the
 * smoke entry point and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or constant generator with the GPU library.
 *
 * What it computes, and where in the paper each step comes from:
 *   - the hypergraph G=(V,HE) and its implicit weighted clique graph G_w
 *     (Section 2.1, problem definition); G_w is never built, only walked;
 *   - independent-cascade channels (Section 2.1, "Cascade models", IC):
 *     every hyperedge he and every ordered pair of distinct members u->v of he
 *     is one channel, live with probability p_v;
 *   - the stratified setting (Section 3.1.1, "Activation probability" and
 *     "Sampling strategy"; Algorithm 3's per-layer draws): a member of layer
 *     i of A(v) activates v with probability P(L_i) / n(L_i),
 *     P(L_i) = 1 / (i ln(l_v + 1)); an RR set draws per popped vertex and
 *     layer a count (Binomial for layers of at most 20 members, Poisson
 *     above) and selects that many members without replacement;
 *   - independent cascade drawn by geometric gaps (models 5 and 6; the
 *     subset sampling of Section 2.2.1, Algorithm 2, on IC channels): the same
 *     channels and probabilities as models 0 and 1, but the live positions
 *     of each stream (RR id, hyperedge, target) are drawn as gaps of dead
 *     positions instead of one coin per position;
 *   - the linear-threshold model (Section 2.1, "Cascade models", LT) in its
 *     live-edge form: every vertex v keeps at most one of its channels, each
 *     with weight W_v (the per-channel probability, capped so that the
 *     weights into v sum to at most 1), and an RR set is the reverse walk
 *     along kept channels until it meets a vertex already in the set;
 *   - the sample-set layers of each vertex by co-membership weight w(v,u)
 *     (Section 3.1.1, "Sample set division"), the layer count l_v, and the
 *     statistics alpha, beta of Section 4.1 and theta(l*) of Theorem 2;
 *   - RR sets: a root, then the reverse breadth-first closure over live
 *     channels (Algorithm 3's skeleton: root, queue, activated marks);
 *   - optionally, the division of the RR sets into R1 and R2 of Section 4.1
 *     (roots with a small layer among the first beta go to R1, whose sets
 *     contain those layers' members; the others to R2), which biases the
 *     estimates and is off unless switched on;
 *   - greedy max coverage (Algorithm 1, Equations (1)-(2));
 *   - the sample-size loop of HyperIM_BRR (Algorithm 4): theta_max
 *     (Lemma 6 / Equation (13)), theta_0, the lower bound of Equation (12)
 *     and the upper bound of Lemma 5, doubling until the ratio test passes.
 *
 * Readings where the paper is silent or garbled (each restated in the design
 * notes): one independent channel per (hyperedge, ordered pair); coins are
 * Philox4x32-10 words keyed by (seed, instance) with counter
 * (j_lo, he, v, pool<<31 | j_hi<<24 | pos>>2); thresholds floor(p * 2^32)
 * from float32 p; layers by descending w; stratum = min(7, 1+floor(log2 l_v))
 * (0 for l_v = 0); roots by systematic sampling over the stratum-sorted vertex
 * list with one 64-bit random offset per ladder block; theta_max in the
 * OPIM-C form; the stop test sigma_l/sigma_u >= 1-1/e-eps.  Under LT each
 * channel into v weighs min(thr[v], floor(2^32 / c(v))) / 2^32 and one Philox
 * word per (RR id, v), the coin at hyperedge slot 0xFFFFFFFE and position 0,
 * picks the kept channel.
 *
 * Build: gcc -O2 -shared -fPIC -pthread -o liboracle.so hyperim_oracle.c -lm
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_NSTRATA 8u
#define ORC_ALWAYS 0xFFFFFFFFu

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Ten rounds of the 4x32 Philox S-P network; the */
/* two-word key is bumped by the Weyl constants between rounds.              */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Philox over a batch of (counter, key) records, for cross-checks. */
void orc_philox_batch(uint64_t count, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (uint64_t i = 0; i < count; ++i) orc_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

/* The coin of channel (he, u -> v) in RR set j of pool `pool`, where pos is
 * u's index inside he's member list.  IC, Section 2.1: one independent
 * Bernoulli trial per channel. */
uint32_t orc_coin(uint64_t seed, uint32_t instance, uint32_t pool, uint64_t j,
                  uint32_t he, uint32_t v, uint32_t pos)
{
    uint32_t ctr[4], key[2], out[4];
    ctr[0] = (uint32_t)j;
    ctr[1] = he;
    ctr[2] = v;
    ctr[3] = (pool << 31) | ((uint32_t)(j >> 32) << 24) | (pos >> 2);
    key[0] = (uint32_t)seed;
    key[1] = instance;
    orc_philox4x32_10(ctr, key, out);
    return out[pos & 3u];
}

static int orc_live(uint32_t coin, uint32_t thr)
{
    return thr == ORC_ALWAYS || coin < thr;
}

/* ------------------------------------------------------------------------ */
/* Graph                                                                     */
/* ------------------------------------------------------------------------ */
typedef struct orc_graph {
    uint32_t n, m;
    uint64_t nnz;
    uint32_t *he_off, *he_mem;     /* hyperedge -> members (caller's order) */
    uint32_t *v_off, *v_he;        /* vertex -> hyperedges (ascending ids)  */
    uint32_t *thr;                 /* coin threshold of channels into v     */
    uint64_t *c;                   /* sum over he containing v of |he|-1    */
    int lt;                        /* linear-threshold model (else IC)      */
    int layered;                   /* stratified-setting model (model 4)    */
    int gaps;                      /* IC drawn by geometric gaps (5, 6)     */
    /* stratified setting: per vertex v the members of A(v), layer by layer
     * (layer 1 = largest w(v,u)), ascending ids within a layer:
     * nb[nb_off[v] .. nb_off[v+1]); layer i (1-based) of v ends at
     * nb_off[v] + ly_end[ly_off[v] + i - 1] */
    uint64_t *nb_off, *ly_off;
    uint32_t *nb, *ly_end;
    int stratified;
    uint32_t *l, *deg, *top, *P;   /* layers, G_w degree, |L_1|, ordering   */
    uint8_t *stratum;
    uint32_t B[ORC_NSTRATA + 1];
    double alpha, beta, theta_l;
    /* division of the RR sets (Section 4.1), when switched on: R1 (pool 0)
     * draws its roots from rP[0 .. n1), the vertices with a small layer,
     * R2 (pool 1) from rP[n1 .. n); an R1 set of root v starts from v and
     * f_mem[f_off[v] .. f_off[v+1]) */
    int route_on, routed;          /* asked for; in effect (both sides)     */
    uint32_t n1;
    uint32_t *rP, *f_mem;
    uint64_t *f_off;
} orc_graph;

void orc_graph_free(orc_graph *g)
{
    if (!g) return;
    free(g->he_off); free(g->he_mem); free(g->v_off); free(g->v_he);
    free(g->thr); free(g->c); free(g->l); free(g->deg); free(g->top);
    free(g->P); free(g->stratum);
    free(g->nb_off); free(g->ly_off); free(g->nb); free(g->ly_end);
    free(g->rP); free(g->f_off); free(g->f_mem);
    free(g);
}

/* Probability threshold: a channel into v is live when its coin is below
 * thr[v]; thr = ALWAYS when p_v >= 1.  p_v is float32; floor(p_v * 2^32) is
 * exact in double because a float32 has a 24-bit significand. */
static uint32_t orc_threshold(float pv)
{
    if (pv >= 1.0f) return ORC_ALWAYS;
    if (!(pv > 0.0f)) return 0u;
    return (uint32_t)floor(ldexp((double)pv, 32));
}

/* Section 2.1: G = (V, HE) with V(he) given as member lists.  Validates the
 * input, builds the vertex -> hyperedge incidence lists and the per-target
 * thresholds (model 0: IC, constant p; model 1: IC, weighted cascade,
 * p_v = 1/c(v) with c(v) the weighted in-degree of v in G_w; models 2 and 3:
 * the linear-threshold model with the thresholds of models 0 and 1). */
int orc_graph_new(uint32_t n, uint32_t m, const uint32_t *he_off, const uint32_t *he_mem,
                  uint32_t model, float p, orc_graph **out)
{
    *out = NULL;
    if (model > 6u) return ORC_EINVAL;
    if ((model == 0u || model == 2u || model == 5u) && (isnan(p) || p < 0.0f)) return ORC_EINVAL;
    if (he_off[0] != 0u) return ORC_EINVAL;
    for (uint32_t e = 0; e < m; ++e)
        if (he_off[e + 1] < he_off[e]) return ORC_EINVAL;
    uint64_t nnz = he_off[m];
    for (uint64_t i = 0; i < nnz; ++i)
        if (he_mem[i] >= n) return ORC_EINVAL;
    /* duplicate member inside one hyperedge */
    uint32_t *stamp = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!stamp) return ORC_ENOMEM;
    for (uint32_t v = 0; v < n; ++v) stamp[v] = 0xFFFFFFFFu;
    for (uint32_t e = 0; e < m; ++e)
        for (uint32_t i = he_off[e]; i < he_off[e + 1]; ++i) {
            if (stamp[he_mem[i]] == e) { free(stamp); return ORC_EINVAL; }
            stamp[he_mem[i]] = e;
        }
    free(stamp);

    orc_graph *g = (orc_graph *)calloc(1, sizeof(orc_graph));
    if (!g) return ORC_ENOMEM;
    g->n = n; g->m = m; g->nnz = nnz;
    g->lt = model == 2u || model == 3u;
    g->layered = model == 4u;
    g->gaps = model == 5u || model == 6u;
    g->he_off = (uint32_t *)malloc(sizeof(uint32_t) * (m + 1));
    g->he_mem = (uint32_t *)malloc(sizeof(uint32_t) * (nnz ? nnz : 1));
    g->v_off = (uint32_t *)calloc(n + 1, sizeof(uint32_t));
    g->v_he = (uint32_t *)malloc(sizeof(uint32_t) * (nnz ? nnz : 1));
    g->thr = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    g->c = (uint64_t *)calloc(n ? n : 1, sizeof(uint64_t));
    if (!g->he_off || !g->he_mem || !g->v_off || !g->v_he || !g->thr || !g->c) {
        orc_graph_free(g);
        return ORC_ENOMEM;
    }
    memcpy(g->he_off, he_off, sizeof(uint32_t) * (m + 1));
    if (nnz) memcpy(g->he_mem, he_mem, sizeof(uint32_t) * nnz);

    /* incidence lists: count, prefix sum, fill in ascending hyperedge order */
    for (uint64_t i = 0; i < nnz; ++i) g->v_off[he_mem[i] + 1]++;
    for (uint32_t v = 0; v < n; ++v) g->v_off[v + 1] += g->v_off[v];
    uint32_t *fill = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    if (!fill) { orc_graph_free(g); return ORC_ENOMEM; }
    for (uint32_t e = 0; e < m; ++e)
        for (uint32_t i = he_off[e]; i < he_off[e + 1]; ++i) {
            uint32_t v = he_mem[i];
            g->v_he[g->v_off[v] + fill[v]++] = e;
            g->c[v] += (uint64_t)(he_off[e + 1] - he_off[e] - 1u);
        }
    free(fill);

    for (uint32_t v = 0; v < n; ++v) {
        float pv;
        if (model == 0u || model == 2u || model == 5u) pv = p;
        else pv = g->c[v] ? (float)(1.0 / (double)g->c[v]) : 0.0f;   /* model 4 keeps these unused */
        g->thr[v] = orc_threshold(pv);
    }
    *out = g;
    return ORC_OK;
}

int orc_graph_export(const orc_graph *g, uint32_t *v_off, uint32_t *v_he, uint32_t *thr, uint64_t *c)
{
    memcpy(v_off, g->v_off, sizeof(uint32_t) * (g->n + 1));
    if (g->nnz) memcpy(v_he, g->v_he, sizeof(uint32_t) * g->nnz);
    memcpy(thr, g->thr, sizeof(uint32_t) * g->n);
    memcpy(c, g->c, sizeof(uint64_t) * g->n);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Sample-set layers (Section 3.1.1) and strata                              */
/* ------------------------------------------------------------------------ */
static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

static uint32_t orc_stratum_of(uint32_t l)
{
    if (l == 0u) return 0u;
    uint32_t lg = 0;                 /* floor(log2 l) */
    while ((l >> (lg + 1)) != 0u) ++lg;
    uint32_t s = 1u + lg;
    return s < ORC_NSTRATA - 1u ? s : ORC_NSTRATA - 1u;
}

/* For each vertex v: w(v,u) = number of hyperedges shared with co-member u;
 * deg(v) = number of distinct u (degree in G_w); the sample set A(v) is
 * divided into layers of equal w, layer 1 holding the largest w; l_v is the
 * number of layers and top(v) = n(L_1).  Strata group vertices by l_v; P is
 * the vertex list sorted by (stratum, id) and B[h] the first index of
 * stratum h.  Section 4.1 statistics: alpha = F_cnt / T_cnt (first-layer
 * vertices over all layered vertices), beta = L_cnt / |V|, and Theorem 2's
 * theta(l*) = (1/|V|) sum_v l_v / ln(l_v + 1). */
/* (w, u) pairs: w descending, then u ascending */
static int cmp_wu_desc(const void *a, const void *b)
{
    const uint32_t *x = (const uint32_t *)a, *y = (const uint32_t *)b;
    if (x[0] != y[0]) return x[0] > y[0] ? -1 : 1;
    return (x[1] > y[1]) - (x[1] < y[1]);
}

/* Sample-set division (Section 3.1.1) written out for the stratified
 * setting: A(v) = the co-members of v, in layers by w(v,u) (layer 1 the
 * largest), ascending ids within a layer.  Uses l and deg from orc_stratify. */
static int orc_build_layers(orc_graph *g)
{
    uint32_t n = g->n;
    free(g->nb_off); free(g->ly_off); free(g->nb); free(g->ly_end);
    g->nb_off = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    g->ly_off = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    if (!g->nb_off || !g->ly_off) return ORC_ENOMEM;
    for (uint32_t v = 0; v < n; ++v) {
        g->nb_off[v + 1] = g->nb_off[v] + g->deg[v];
        g->ly_off[v + 1] = g->ly_off[v] + g->l[v];
    }
    g->nb = (uint32_t *)malloc(sizeof(uint32_t) * (g->nb_off[n] ? g->nb_off[n] : 1));
    g->ly_end = (uint32_t *)malloc(sizeof(uint32_t) * (g->ly_off[n] ? g->ly_off[n] : 1));
    if (!g->nb || !g->ly_end) return ORC_ENOMEM;
    uint64_t cap = 16;
    uint32_t *buf = (uint32_t *)malloc(sizeof(uint32_t) * cap);
    uint32_t *wu = (uint32_t *)malloc(sizeof(uint32_t) * 2 * cap);
    if (!buf || !wu) { free(buf); free(wu); return ORC_ENOMEM; }
    for (uint32_t v = 0; v < n; ++v) {
        uint64_t cnt = 0;
        for (uint32_t e = g->v_off[v]; e < g->v_off[v + 1]; ++e) {
            uint32_t he = g->v_he[e];
            for (uint32_t i = g->he_off[he]; i < g->he_off[he + 1]; ++i) {
                uint32_t u = g->he_mem[i];
                if (u == v) continue;
                if (cnt == cap) {
                    cap *= 2;
                    uint32_t *nb = (uint32_t *)realloc(buf, sizeof(uint32_t) * cap);
                    uint32_t *nw = (uint32_t *)realloc(wu, sizeof(uint32_t) * 2 * cap);
                    if (!nb || !nw) { free(nb ? nb : buf); free(nw ? nw : wu); return ORC_ENOMEM; }
                    buf = nb; wu = nw;
                }
                buf[cnt++] = u;
            }
        }
        qsort(buf, cnt, sizeof(uint32_t), cmp_u32);
        uint64_t d = 0;
        for (uint64_t i = 0; i < cnt;) {
            uint64_t r = i;
            while (r < cnt && buf[r] == buf[i]) ++r;
            wu[2 * d] = (uint32_t)(r - i);
            wu[2 * d + 1] = buf[i];
            ++d;
            i = r;
        }
        qsort(wu, d, 2 * sizeof(uint32_t), cmp_wu_desc);
        uint64_t base = g->nb_off[v], lb = g->ly_off[v];
        uint32_t layer = 0;
        for (uint64_t i = 0; i < d; ++i) {
            g->nb[base + i] = wu[2 * i + 1];
            if (i + 1 == d || wu[2 * (i + 1)] != wu[2 * i]) g->ly_end[lb + layer++] = (uint32_t)(i + 1);
        }
    }
    free(buf);
    free(wu);
    return ORC_OK;
}

int orc_layers_export(const orc_graph *g, uint64_t *nb_off, uint32_t *nb, uint64_t *ly_off, uint32_t *ly_end)
{
    if (!g->stratified || !g->nb_off) return ORC_EINVAL;
    uint32_t n = g->n;
    memcpy(nb_off, g->nb_off, sizeof(uint64_t) * ((size_t)n + 1));
    memcpy(ly_off, g->ly_off, sizeof(uint64_t) * ((size_t)n + 1));
    if (g->nb_off[n]) memcpy(nb, g->nb, sizeof(uint32_t) * g->nb_off[n]);
    if (g->ly_off[n]) memcpy(ly_end, g->ly_end, sizeof(uint32_t) * g->ly_off[n]);
    return ORC_OK;
}

int orc_route(orc_graph *g, int on, uint32_t *n1);

int orc_stratify(orc_graph *g)
{
    uint32_t n = g->n;
    /* new strata: the division of the RR sets is rebuilt at the end */
    free(g->rP); free(g->f_off); free(g->f_mem);
    g->rP = NULL; g->f_off = NULL; g->f_mem = NULL;
    g->routed = 0; g->n1 = 0;
    free(g->nb_off); free(g->ly_off); free(g->nb); free(g->ly_end);
    g->nb_off = NULL; g->ly_off = NULL; g->nb = NULL; g->ly_end = NULL;
    free(g->l); free(g->deg); free(g->top); free(g->P); free(g->stratum);
    g->l = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    g->deg = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    g->top = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
    g->P = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    g->stratum = (uint8_t *)calloc(n ? n : 1, 1);
    if (!g->l || !g->deg || !g->top || !g->P || !g->stratum) return ORC_ENOMEM;

    uint64_t cap = 16;
    uint32_t *buf = (uint32_t *)malloc(sizeof(uint32_t) * cap);
    uint32_t *wv = (uint32_t *)malloc(sizeof(uint32_t) * cap);
    if (!buf || !wv) { free(buf); free(wv); return ORC_ENOMEM; }
    uint64_t sum_top = 0, sum_deg = 0, sum_l = 0;
    double theta_l = 0.0;
    for (uint32_t v = 0; v < n; ++v) {
        /* gather every co-member occurrence of v */
        uint64_t cnt = 0;
        for (uint32_t e = g->v_off[v]; e < g->v_off[v + 1]; ++e) {
            uint32_t he = g->v_he[e];
            for (uint32_t i = g->he_off[he]; i < g->he_off[he + 1]; ++i) {
                uint32_t u = g->he_mem[i];
                if (u == v) continue;
                if (cnt == cap) {
                    cap *= 2;
                    uint32_t *nb = (uint32_t *)realloc(buf, sizeof(uint32_t) * cap);
                    uint32_t *nw = (uint32_t *)realloc(wv, sizeof(uint32_t) * cap);
                    if (!nb || !nw) { free(nb ? nb : buf); free(nw ? nw : wv); return ORC_ENOMEM; }
                    buf = nb; wv = nw;
                }
                buf[cnt++] = u;
            }
        }
        qsort(buf, cnt, sizeof(uint32_t), cmp_u32);
        /* run lengths = w(v,u) */
        uint64_t d = 0;
        for (uint64_t i = 0; i < cnt;) {
            uint64_t r = i;
            while (r < cnt && buf[r] == buf[i]) ++r;
            wv[d++] = (uint32_t)(r - i);
            i = r;
        }
        qsort(wv, d, sizeof(uint32_t), cmp_u32);
        uint32_t layers = 0, top = 0;
        for (uint64_t i = 0; i < d; ++i)
            if (i == 0 || wv[i] != wv[i - 1]) ++layers;
        if (d) {
            uint32_t wmax = wv[d - 1];
            for (uint64_t i = 0; i < d; ++i)
                if (wv[i] == wmax) ++top;
        }
        g->l[v] = layers;
        g->deg[v] = (uint32_t)d;
        g->top[v] = top;
        g->stratum[v] = (uint8_t)orc_stratum_of(layers);
        sum_top += top;
        sum_deg += d;
        sum_l += layers;
        if (layers) theta_l += (double)layers / log((double)layers + 1.0);
    }
    free(buf);
    free(wv);

    uint32_t idx = 0;
    for (uint32_t h = 0; h < ORC_NSTRATA; ++h) {
        g->B[h] = idx;
        for (uint32_t v = 0; v < n; ++v)
            if (g->stratum[v] == h) g->P[idx++] = v;
    }
    g->B[ORC_NSTRATA] = idx;
    g->alpha = sum_deg ? (double)sum_top / (double)sum_deg : 0.0;
    g->beta = n ? (double)sum_l / (double)n : 0.0;
    g->theta_l = n ? theta_l / (double)n : 0.0;
    g->stratified = 1;
    if (g->layered) {
        int rc = orc_build_layers(g);
        if (rc) return rc;
    }
    if (g->route_on) {
        uint32_t n1;
        return orc_route(g, 1, &n1);
    }
    return ORC_OK;
}

int orc_strata_export(const orc_graph *g, uint32_t *l, uint32_t *deg, uint32_t *top,
                      uint8_t *stratum, uint32_t *P, uint32_t *B, double *stats)
{
    if (!g->stratified) return ORC_EINVAL;
    memcpy(l, g->l, sizeof(uint32_t) * g->n);
    memcpy(deg, g->deg, sizeof(uint32_t) * g->n);
    memcpy(top, g->top, sizeof(uint32_t) * g->n);
    memcpy(stratum, g->stratum, g->n);
    memcpy(P, g->P, sizeof(uint32_t) * g->n);
    memcpy(B, g->B, sizeof(uint32_t) * (ORC_NSTRATA + 1));
    stats[0] = g->alpha;
    stats[1] = g->beta;
    stats[2] = g->theta_l;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Division of the RR sets into R1 and R2 (Section 4.1), opt-in              */
/* ------------------------------------------------------------------------ */
/* alpha = F_cnt / T_cnt (the share of first-layer vertices among all layer
 * vertices) and beta = L_cnt / |V| (the mean number of layers).  For a
 * vertex v and each layer i of A(v) with 1 <= i <= beta (i <= floor(beta)),
 * the layer is small when |L_i| < alpha |A(v)|, compared exactly as
 * |L_i| T_cnt < F_cnt |A(v)| in 128-bit integers.  v's RR sets go to R1 when
 * some layer is small, and then contain every member of the small layers;
 * otherwise to R2.  Here R1 (pool 0) draws its roots, stratified as usual,
 * from the R1 vertices only (the stratum order of P kept), R2 (pool 1) from
 * the others; an R1 set starts its reverse traversal from the root and the
 * members of its small layers together (their channels into the root count
 * as live).  When either side is empty the division is inert (both pools
 * over V, no forced members).  Not for the linear-threshold or stratified-
 * setting models.  *n1 = the number of R1 vertices. */
int orc_route(orc_graph *g, int on, uint32_t *n1)
{
    uint32_t n = g->n;
    *n1 = 0;
    if (!g->stratified || g->lt || g->layered) return ORC_EINVAL;
    free(g->rP); free(g->f_off); free(g->f_mem);
    g->rP = NULL; g->f_off = NULL; g->f_mem = NULL;
    g->routed = 0; g->n1 = 0;
    g->route_on = on != 0;
    if (!on) return ORC_OK;
    if (!g->nb_off) {
        int rc = orc_build_layers(g);
        if (rc) return rc;
    }
    uint64_t Fc = 0, Tc = 0, Lc = 0;
    for (uint32_t v = 0; v < n; ++v) {
        Fc += g->top[v];
        Tc += g->deg[v];
        Lc += g->l[v];
    }
    uint64_t ilim = n ? Lc / n : 0;   /* layers 1 .. floor(beta) */
    g->f_off = (uint64_t *)calloc((size_t)n + 1, sizeof(uint64_t));
    if (!g->f_off) return ORC_ENOMEM;
    for (int pass = 0; pass < 2; ++pass) {
        for (uint32_t v = 0; v < n; ++v) {
            uint64_t at = pass ? g->f_off[v] : 0;   /* pass 0 counts, pass 1 writes */
            uint32_t prev = 0;
            for (uint64_t i = 0; i < g->l[v] && i < ilim; ++i) {
                uint32_t end = g->ly_end[g->ly_off[v] + i];
                uint32_t size = end - prev;
                if ((unsigned __int128)size * Tc < (unsigned __int128)Fc * g->deg[v]) {
                    if (pass == 0) {
                        at += size;
                    } else {
                        for (uint32_t k = prev; k < end; ++k) g->f_mem[at++] = g->nb[g->nb_off[v] + k];
                    }
                }
                prev = end;
            }
            if (pass == 0) g->f_off[v + 1] = at;   /* count, summed below */
        }
        if (pass == 0) {
            for (uint32_t v = 0; v < n; ++v) g->f_off[v + 1] += g->f_off[v];
            g->f_mem = (uint32_t *)malloc(sizeof(uint32_t) * (g->f_off[n] ? g->f_off[n] : 1));
            if (!g->f_mem) return ORC_ENOMEM;
        }
    }
    uint32_t c1 = 0;
    for (uint32_t v = 0; v < n; ++v) c1 += g->f_off[v + 1] > g->f_off[v];
    *n1 = c1;
    if (c1 == 0 || c1 == n) {
        free(g->f_off); free(g->f_mem);
        g->f_off = NULL; g->f_mem = NULL;
        return ORC_OK;
    }
    g->rP = (uint32_t *)malloc(sizeof(uint32_t) * n);
    if (!g->rP) return ORC_ENOMEM;
    uint32_t a = 0, b = c1;
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t v = g->P[i];
        if (g->f_off[v + 1] > g->f_off[v]) g->rP[a++] = v;
        else g->rP[b++] = v;
    }
    g->n1 = c1;
    g->routed = 1;
    return ORC_OK;
}

/* The division's tables: rP (n), f_off (n + 1), f_mem (f_off[n]). */
int orc_route_export(const orc_graph *g, uint32_t *rP, uint64_t *f_off, uint32_t *f_mem)
{
    if (!g->routed) return ORC_EINVAL;
    memcpy(rP, g->rP, sizeof(uint32_t) * g->n);
    memcpy(f_off, g->f_off, sizeof(uint64_t) * ((size_t)g->n + 1));
    if (g->f_off[g->n]) memcpy(f_mem, g->f_mem, sizeof(uint32_t) * g->f_off[g->n]);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Roots: stratified (systematic, proportional) root sampling                */
/* ------------------------------------------------------------------------ */
/* The pool's ids are cut into a ladder of blocks: block 0 = [0, Q), block
 * b >= 1 = [Q 2^(b-1), Q 2^b), with Q = 2^qlog.  */
void orc_block_of(uint64_t j, uint32_t qlog, uint32_t *b, uint64_t *J, uint64_t *T)
{
    uint64_t Q = (uint64_t)1 << qlog;
    if (j < Q) { *b = 0; *J = 0; *T = Q; return; }
    uint32_t bb = 1;
    while (((Q << bb)) <= j) ++bb;
    *b = bb;
    *J = Q << (bb - 1);
    *T = Q << (bb - 1);
}

/* The one random offset of block b in pool `pool`: o_b = floor(x * n / 2^64)
 * with x the first two words of Philox at counter (b, ~0, ~0, pool). */
uint64_t orc_block_offset(uint32_t n, uint64_t seed, uint32_t instance, uint32_t pool, uint32_t b)
{
    uint32_t ctr[4] = {b, 0xFFFFFFFFu, 0xFFFFFFFFu, pool};
    uint32_t key[2] = {(uint32_t)seed, instance};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    uint64_t x = (uint64_t)out[0] | ((uint64_t)out[1] << 32);
    return (uint64_t)(((unsigned __int128)x * n) >> 64);
}

/* Algorithm 3 starts from "a randomly sampled node".  Here the sample is
 * stratified: inside block b (size T) the t-th id takes the vertex at
 * position floor((t n + o_b) / T) of the stratum-sorted list P, so every
 * vertex is a root exactly T/n times in expectation and each stratum gets a
 * quota within one of T N_h / n. */
uint32_t orc_root(const orc_graph *g, uint64_t seed, uint32_t instance, uint32_t pool,
                  uint64_t j, uint32_t qlog)
{
    uint32_t b;
    uint64_t J, T;
    orc_block_of(j, qlog, &b, &J, &T);
    /* with the RR sets divided (Section 4.1), each pool samples its own
     * vertices, in the same way */
    const uint32_t *P = g->P;
    uint32_t n = g->n;
    if (g->routed) {
        P = pool == 0u ? g->rP : g->rP + g->n1;
        n = pool == 0u ? g->n1 : g->n - g->n1;
    }
    uint64_t o = orc_block_offset(n, seed, instance, pool, b);
    unsigned __int128 pos = ((unsigned __int128)(j - J) * n + o) / T;
    return P[(uint64_t)pos];
}

/* ------------------------------------------------------------------------ */
/* One RR set (Algorithm 3's skeleton with per-channel coins)                */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint8_t *inR;
    uint32_t *queue;
} orc_scratch;

/* An R1 set of a divided graph (Section 4.1) starts with the members of its
 * root's small layers beside the root. */
static void orc_seed_forced(const orc_graph *g, uint32_t pool, uint32_t root, orc_scratch *s, uint32_t *tail)
{
    if (!g->routed || pool != 0u) return;
    for (uint64_t f = g->f_off[root]; f < g->f_off[root + 1]; ++f) {
        uint32_t u = g->f_mem[f];
        if (s->inR[u]) continue;
        s->inR[u] = 1;
        s->queue[(*tail)++] = u;
    }
}

/* R = {root}; pop v; for every hyperedge he containing v and every member u
 * of he other than v, the channel u -> v is tested with its own coin; a live
 * channel from a vertex outside R adds it to R and to the queue.  The result
 * is the set of vertices with a live path to the root, written ascending. */
static uint32_t orc_rr_into(const orc_graph *g, uint64_t seed, uint32_t instance, uint32_t pool,
                            uint64_t j, uint32_t root, orc_scratch *s, uint32_t *out)
{
    uint32_t head = 0, tail = 0;
    s->queue[tail++] = root;
    s->inR[root] = 1;
    orc_seed_forced(g, pool, root, s, &tail);
    while (head < tail) {
        uint32_t v = s->queue[head++];
        uint32_t thr = g->thr[v];
        for (uint32_t e = g->v_off[v]; e < g->v_off[v + 1]; ++e) {
            uint32_t he = g->v_he[e];
            uint32_t base = g->he_off[he];
            uint32_t size = g->he_off[he + 1] - base;
            for (uint32_t pos = 0; pos < size; ++pos) {
                uint32_t u = g->he_mem[base + pos];
                if (u == v) continue;
                if (!orc_live(orc_coin(seed, instance, pool, j, he, v, pos), thr)) continue;
                if (s->inR[u]) continue;
                s->inR[u] = 1;
                s->queue[tail++] = u;
            }
        }
    }
    for (uint32_t i = 0; i < tail; ++i) {
        out[i] = s->queue[i];
        s->inR[s->queue[i]] = 0;
    }
    qsort(out, tail, sizeof(uint32_t), cmp_u32);
    return tail;
}

/* Linear-threshold model, live-edge form (Section 2.1, LT bullet; the
 * threshold process and this form give every vertex the same activation
 * probability).  The channels into v are its (hyperedge, member) pairs in
 * ascending hyperedge order and the hyperedge's stored member order, v
 * itself skipped: c(v) of them.  Each has weight W / 2^32 with
 * W = min(thr[v], floor(2^32 / c(v))) (thr = ALWAYS counting as 2^32), so
 * the weights into v sum to at most 1.  One Philox word per (RR id, v) -- the
 * coin at hyperedge slot 0xFFFFFFFE, position 0 -- picks channel
 * floor(x / W) when x < W c(v), and none otherwise.  Returns 1 and the
 * picked member in *u, or 0. */
static int orc_lt_pick(const orc_graph *g, uint64_t seed, uint32_t instance, uint32_t pool, uint64_t j,
                       uint32_t v, uint32_t *u)
{
    uint64_t C = g->c[v];
    if (C == 0) return 0;
    uint64_t W = g->thr[v] == ORC_ALWAYS ? (1ull << 32) : (uint64_t)g->thr[v];
    uint64_t cap = (1ull << 32) / C;
    if (W > cap) W = cap;
    uint64_t x = orc_coin(seed, instance, pool, j, 0xFFFFFFFEu, v, 0u);
    if (x >= W * C) return 0;
    uint64_t k = x / W;
    for (uint32_t e = g->v_off[v]; e < g->v_off[v + 1]; ++e) {
        uint32_t he = g->v_he[e];
        uint32_t base = g->he_off[he];
        uint32_t size = g->he_off[he + 1] - base;
        if (k >= (uint64_t)(size - 1u)) {
            k -= size - 1u;
            continue;
        }
        for (uint32_t pos = 0; pos < size; ++pos) {
            uint32_t w = g->he_mem[base + pos];
            if (w == v) continue;
            if (k == 0) { *u = w; return 1; }
            --k;
        }
    }
    return 0;   /* not reached: k < c(v) */
}

/* The LT RR set of root r: r, the member r's kept channel comes from, that
 * member's, and so on, until no channel is kept or the walk meets a vertex
 * already in the set; written ascending. */
static uint32_t orc_lt_into(const orc_graph *g, uint64_t seed, uint32_t instance, uint32_t pool,
                            uint64_t j, uint32_t root, orc_scratch *s, uint32_t *out)
{
    uint32_t len = 0, cur = root, u = 0;
    s->queue[len++] = root;
    s->inR[root] = 1;
    while (orc_lt_pick(g, seed, instance, pool, j, cur, &u) && !s->inR[u]) {
        s->inR[u] = 1;
        s->queue[len++] = u;
        cur = u;
    }
    for (uint32_t i = 0; i < len; ++i) {
        out[i] = s->queue[i];
        s->inR[s->queue[i]] = 0;
    }
    qsort(out, len, sizeof(uint32_t), cmp_u32);
    return len;
}

/* Stratified setting.  Random numbers of (RR id j, vertex v, layer i): the
 * Philox blocks at counter (j_lo, i, v, pool<<31 | j_hi<<24 | r), r = 0, 1, ...
 * Block 0's words 0 and 1 give U = (w0 >> 11 | w1 << 21) / 2^53 in [0, 1);
 * block 0's words 2, 3 and every word of the blocks r >= 1, in order, are the
 * selection draws. */
static void orc_layer_block(uint64_t seed, uint32_t instance, uint32_t pool, uint64_t j, uint32_t i, uint32_t v,
                            uint32_t r, uint32_t out[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = (uint32_t)j;
    ctr[1] = i;
    ctr[2] = v;
    ctr[3] = (pool << 31) | ((uint32_t)(j >> 32) << 24) | r;
    key[0] = (uint32_t)seed;
    key[1] = instance;
    orc_philox4x32_10(ctr, key, out);
}

/* Count h of layer i of v (n members, l layers): the layer's probability is
 * P = 1 / (i ln(l + 1)) (Section 3.1.1), each member's p = P / n, at most 1
 * (the P of the top layers exceed 1 / n when l is small).  n <= 20: Binomial
 * (n, p) by inversion of U, probabilities q^n, then
 * prob_{h+1} = ((prob_h (n - h)) / (h + 1)) (p / q); n > 20: Poisson with
 * lambda = n p = P, prob_0 = e^-lambda, prob_{h+1} = (prob_h lambda) / (h + 1),
 * truncated at min(n, 64) (lambda < 1.5, so a count above 64 has probability
 * below 1e-70).  h is the first count whose cumulative probability exceeds
 * U. */
#define ORC_MAX_PICK 64u
static uint32_t orc_layer_count(uint32_t n, uint32_t i, uint32_t l, double U)
{
    double P = 1.0 / ((double)i * log((double)l + 1.0));
    double p = P / (double)n;
    if (n <= 20u) {
        if (p >= 1.0) return n;
        double q = 1.0 - p;
        double prob = 1.0;
        for (uint32_t t = 0; t < n; ++t) prob = prob * q;
        double ratio = p / q, cdf = prob;
        uint32_t h = 0;
        while (U >= cdf && h < n) {
            prob = ((prob * (double)(n - h)) / (double)(h + 1)) * ratio;
            ++h;
            cdf = cdf + prob;
        }
        return h;
    }
    double lambda = P;
    double prob = exp(-lambda), cdf = prob;
    uint32_t h = 0, hmax = n < ORC_MAX_PICK ? n : ORC_MAX_PICK;
    while (U >= cdf && h < hmax) {
        prob = (prob * lambda) / (double)(h + 1);
        ++h;
        cdf = cdf + prob;
    }
    return h;
}

/* R = {root}; pop v; for each layer i of A(v): draw the count h, then h
 * members without replacement -- draw r picks index floor(x (n - r) / 2^32)
 * among the layer's members not picked yet, in ascending order -- and every
 * picked member outside R joins R and the queue (Algorithm 3's loop). */
static uint32_t orc_layered_into(const orc_graph *g, uint64_t seed, uint32_t instance, uint32_t pool,
                                 uint64_t j, uint32_t root, orc_scratch *s, uint32_t *out)
{
    uint32_t head = 0, tail = 0;
    uint32_t picked[ORC_MAX_PICK];
    s->queue[tail++] = root;
    s->inR[root] = 1;
    while (head < tail) {
        uint32_t v = s->queue[head++];
        uint32_t l = g->l[v];
        uint64_t base = g->nb_off[v];
        for (uint32_t i = 1; i <= l; ++i) {
            uint32_t lo = i == 1 ? 0u : g->ly_end[g->ly_off[v] + i - 2];
            uint32_t hi = g->ly_end[g->ly_off[v] + i - 1];
            uint32_t n = hi - lo;
            uint32_t w[4];
            orc_layer_block(seed, instance, pool, j, i, v, 0u, w);
            double U = (double)(((uint64_t)(w[0] >> 11)) | ((uint64_t)w[1] << 21)) * 0x1.0p-53;
            uint32_t h = orc_layer_count(n, i, l, U);
            uint32_t r_blk = 0, word = 2, np = 0;
            for (uint32_t r = 0; r < h; ++r) {
                if (word == 4) {
                    orc_layer_block(seed, instance, pool, j, i, v, ++r_blk, w);
                    word = 0;
                }
                uint32_t x = w[word++];
                uint32_t a = (uint32_t)(((uint64_t)x * (uint64_t)(n - r)) >> 32);
                /* the a-th index not picked yet: walk the picked ones ascending */
                uint32_t idx = a;
                for (uint32_t t = 0; t < np; ++t) {     /* picked[] kept ascending */
                    if (picked[t] <= idx) ++idx;
                    else break;
                }
                uint32_t t = np;
                while (t > 0 && picked[t - 1] > idx) { picked[t] = picked[t - 1]; --t; }
                picked[t] = idx;
                ++np;
                uint32_t u = g->nb[base + lo + idx];
                if (!s->inR[u]) {
                    s->inR[u] = 1;
                    s->queue[tail++] = u;
                }
            }
        }
    }
    for (uint32_t i = 0; i < tail; ++i) {
        out[i] = s->queue[i];
        s->inR[s->queue[i]] = 0;
    }
    qsort(out, tail, sizeof(uint32_t), cmp_u32);
    return tail;
}

/* Independent cascade by geometric gaps.  The stream of (RR id j, hyperedge
 * he, target v) is he's positions 0 .. |he|-1 in stored order, each live with
 * p_v = thr[v] / 2^32 (2^32 for thr = ALWAYS); a live position holding v
 * itself is no channel and is dropped, so every channel u -> v is live with
 * p_v independently, as under coins.  The gaps -- dead positions before the
 * next live one, Geometric(p_v) -- come from the words of the Philox blocks
 * at counter (j_lo, he, v, pool<<31 | j_hi<<24 | r/4), word r mod 4 for gap r.
 *
 * Gap from word x with G positions left: t = (2^32 - x) / 2^32 in (0, 1]; the
 * gap is the largest g <= G with Q(g) >= t, found by descending over the bits
 * i = b-1 .. 0 of G (b bits): take bit i when g + 2^i <= G and
 * acc * S_i >= t, then acc = acc * S_i, where S_0 = q = 1 - p_v and
 * S_{i+1} = S_i * S_i (Q(g) is q^g up to rounding).  g = G means no live
 * position is left. */
static uint32_t orc_gap(double q, uint32_t x, uint32_t G)
{
    double t = (double)((1ull << 32) - (uint64_t)x) * 0x1.0p-32;
    uint32_t b = 0;
    while (b < 32u && (G >> b) != 0u) ++b;
    uint32_t g = 0;
    double acc = 1.0;
    for (int i = (int)b - 1; i >= 0; --i) {
        double S = q;
        for (int k = 0; k < i; ++k) S = S * S;
        if ((uint64_t)g + (1ull << i) <= (uint64_t)G && acc * S >= t) {
            acc = acc * S;
            g += 1u << i;
        }
    }
    return g;
}

uint32_t orc_gap_draw(double q, uint32_t x, uint32_t G) { return orc_gap(q, x, G); }

static uint32_t orc_gaps_into(const orc_graph *g, uint64_t seed, uint32_t instance, uint32_t pool,
                              uint64_t j, uint32_t root, orc_scratch *s, uint32_t *out)
{
    uint32_t head = 0, tail = 0;
    s->queue[tail++] = root;
    s->inR[root] = 1;
    orc_seed_forced(g, pool, root, s, &tail);
    while (head < tail) {
        uint32_t v = s->queue[head++];
        uint32_t thr = g->thr[v];
        if (thr == 0u) continue;
        double p = thr == ORC_ALWAYS ? 1.0 : (double)thr * 0x1.0p-32;
        double q = 1.0 - p;
        for (uint32_t e = g->v_off[v]; e < g->v_off[v + 1]; ++e) {
            uint32_t he = g->v_he[e];
            uint32_t base = g->he_off[he];
            uint32_t size = g->he_off[he + 1] - base;
            uint32_t cur = 0, r = 0, w[4] = {0, 0, 0, 0};
            while (cur < size) {
                if ((r & 3u) == 0u) {
                    uint32_t ctr[4], key[2];
                    ctr[0] = (uint32_t)j;
                    ctr[1] = he;
                    ctr[2] = v;
                    ctr[3] = (pool << 31) | ((uint32_t)(j >> 32) << 24) | (r >> 2);
                    key[0] = (uint32_t)seed;
                    key[1] = instance;
                    orc_philox4x32_10(ctr, key, w);
                }
                uint32_t x = w[r & 3u];
                ++r;
                uint32_t G = size - cur;
                uint32_t gap = orc_gap(q, x, G);
                if (gap == G) break;
                uint32_t pos = cur + gap;
                uint32_t u = g->he_mem[base + pos];
                if (u != v && !s->inR[u]) {
                    s->inR[u] = 1;
                    s->queue[tail++] = u;
                }
                cur = pos + 1;
            }
        }
    }
    for (uint32_t i = 0; i < tail; ++i) {
        out[i] = s->queue[i];
        s->inR[s->queue[i]] = 0;
    }
    qsort(out, tail, sizeof(uint32_t), cmp_u32);
    return tail;
}

static uint32_t orc_set_into(const orc_graph *g, uint64_t seed, uint32_t instance, uint32_t pool,
                             uint64_t j, uint32_t root, orc_scratch *s, uint32_t *out)
{
    if (g->gaps) return orc_gaps_into(g, seed, instance, pool, j, root, s, out);
    if (g->layered) return orc_layered_into(g, seed, instance, pool, j, root, s, out);
    return g->lt ? orc_lt_into(g, seed, instance, pool, j, root, s, out)
                 : orc_rr_into(g, seed, instance, pool, j, root, s, out);
}

/* RR set j of pool `pool` into out[] (room for n ids); returns its size. */
uint32_t orc_rr_set(const orc_graph *g, uint64_t seed, uint32_t instance, uint32_t pool,
                    uint64_t j, uint32_t qlog, uint32_t *out)
{
    orc_scratch s;
    s.inR = (uint8_t *)calloc(g->n, 1);
    s.queue = (uint32_t *)malloc(sizeof(uint32_t) * g->n);
    uint32_t root = orc_root(g, seed, instance, pool, j, qlog);
    uint32_t size = orc_set_into(g, seed, instance, pool, j, root, &s, out);
    free(s.inR);
    free(s.queue);
    return size;
}

/* Same, with a caller-chosen root (used by the statistical tests). */
uint32_t orc_rr_set_rooted(const orc_graph *g, uint64_t seed, uint32_t instance, uint32_t pool,
                           uint64_t j, uint32_t root, uint32_t *out)
{
    orc_scratch s;
    s.inR = (uint8_t *)calloc(g->n, 1);
    s.queue = (uint32_t *)malloc(sizeof(uint32_t) * g->n);
    uint32_t size = orc_set_into(g, seed, instance, pool, j, root, &s, out);
    free(s.inR);
    free(s.queue);
    return size;
}

/* ---- many RR sets, one worker thread per host core ---------------------- */
typedef struct {
    const orc_graph *g;
    uint64_t seed;
    uint32_t instance, pool, qlog, tid, nthreads;
    uint64_t id_begin, id_end;
    const uint32_t *roots;    /* optional caller roots (iid baseline), else NULL */
    uint32_t **buf;           /* per-id member arrays */
    uint32_t *size;           /* per-id sizes */
    uint32_t *root_out;
    int err;
} orc_gen_job;

static void *orc_gen_worker(void *arg)
{
    orc_gen_job *job = (orc_gen_job *)arg;
    const orc_graph *g = job->g;
    orc_scratch s;
    s.inR = (uint8_t *)calloc(g->n, 1);
    s.queue = (uint32_t *)malloc(sizeof(uint32_t) * g->n);
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * g->n);
    if (!s.inR || !s.queue || !tmp) { job->err = ORC_ENOMEM; goto done; }
    for (uint64_t j = job->id_begin + job->tid; j < job->id_end; j += job->nthreads) {
        uint64_t k = j - job->id_begin;
        uint32_t root = job->roots ? job->roots[k]
                                   : orc_root(g, job->seed, job->instance, job->pool, j, job->qlog);
        uint32_t sz = orc_set_into(g, job->seed, job->instance, job->pool, j, root, &s, tmp);
        job->buf[k] = (uint32_t *)malloc(sizeof(uint32_t) * (sz ? sz : 1));
        if (!job->buf[k]) { job->err = ORC_ENOMEM; goto done; }
        memcpy(job->buf[k], tmp, sizeof(uint32_t) * sz);
        job->size[k] = sz;
        job->root_out[k] = root;
    }
done:
    free(s.inR);
    free(s.queue);
    free(tmp);
    return NULL;
}

/* RR sets [id_begin, id_end) of one pool as a CSR: *off_out (count+1, u64),
 * *mem_out (members, ascending inside each set), *roots_out.  The arrays are
 * malloc'ed here and released with orc_free. */
int orc_generate(const orc_graph *g, uint64_t seed, uint32_t instance, uint32_t pool,
                 uint64_t id_begin, uint64_t id_end, uint32_t qlog, uint32_t nthreads,
                 const uint32_t *roots_in,
                 uint64_t **off_out, uint32_t **mem_out, uint32_t **roots_out)
{
    if (!g->stratified && !roots_in) return ORC_EINVAL;
    if (id_end < id_begin) return ORC_EINVAL;
    uint64_t count = id_end - id_begin;
    if (nthreads == 0) nthreads = 1;
    uint32_t **buf = (uint32_t **)calloc(count ? count : 1, sizeof(uint32_t *));
    uint32_t *size = (uint32_t *)calloc(count ? count : 1, sizeof(uint32_t));
    uint32_t *roots = (uint32_t *)malloc(sizeof(uint32_t) * (count ? count : 1));
    uint64_t *off = (uint64_t *)malloc(sizeof(uint64_t) * (count + 1));
    if (!buf || !size || !roots || !off) {
        free(buf); free(size); free(roots); free(off);
        return ORC_ENOMEM;
    }
    orc_gen_job *jobs = (orc_gen_job *)calloc(nthreads, sizeof(orc_gen_job));
    pthread_t *th = (pthread_t *)calloc(nthreads, sizeof(pthread_t));
    int err = ORC_OK;
    for (uint32_t t = 0; t < nthreads; ++t) {
        orc_gen_job jb = {g, seed, instance, pool, qlog, t, nthreads, id_begin, id_end,
                          roots_in, buf, size, roots, ORC_OK};
        jobs[t] = jb;
        if (nthreads == 1) orc_gen_worker(&jobs[t]);
        else pthread_create(&th[t], NULL, orc_gen_worker, &jobs[t]);
    }
    if (nthreads > 1)
        for (uint32_t t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    for (uint32_t t = 0; t < nthreads; ++t)
        if (jobs[t].err) err = jobs[t].err;
    free(jobs);
    free(th);
    uint32_t *mem = NULL;
    if (err == ORC_OK) {
        off[0] = 0;
        for (uint64_t k = 0; k < count; ++k) off[k + 1] = off[k] + size[k];
        mem = (uint32_t *)malloc(sizeof(uint32_t) * (off[count] ? off[count] : 1));
        if (!mem) err = ORC_ENOMEM;
        else
            for (uint64_t k = 0; k < count; ++k)
                memcpy(mem + off[k], buf[k], sizeof(uint32_t) * size[k]);
    }
    for (uint64_t k = 0; k < count; ++k) free(buf[k]);
    free(buf);
    free(size);
    if (err != ORC_OK) { free(off); free(roots); free(mem); return err; }
    *off_out = off;
    *mem_out = mem;
    *roots_out = roots;
    return ORC_OK;
}

void orc_free(void *p) { free(p); }

/* ------------------------------------------------------------------------ */
/* Greedy max coverage (Algorithm 1, Equations (1)-(2))                      */
/* ------------------------------------------------------------------------ */
/* k rounds over the first theta sets of a pool: take the vertex of largest
 * marginal coverage (ties -> smallest id; a chosen vertex is never chosen
 * again, even when every count has dropped to zero), add it to S and remove
 * every set it covers.  gains[i] is the marginal coverage of the i-th seed;
 * their sum is the coverage Lambda_R(S_k). */
int orc_greedy(uint32_t n, uint64_t theta, const uint64_t *off, const uint32_t *mem, uint32_t k,
               uint32_t *seeds, uint64_t *gains)
{
    if (k == 0 || k > n) return ORC_EINVAL;
    uint64_t total = off[theta];
    uint64_t *cnt = (uint64_t *)calloc(n, sizeof(uint64_t));
    uint64_t *inv_off = (uint64_t *)calloc((uint64_t)n + 1, sizeof(uint64_t));
    uint64_t *fill = (uint64_t *)calloc(n, sizeof(uint64_t));
    uint64_t *inv = (uint64_t *)malloc(sizeof(uint64_t) * (total ? total : 1));
    uint8_t *covered = (uint8_t *)calloc(theta ? theta : 1, 1);
    uint8_t *chosen = (uint8_t *)calloc(n, 1);
    if (!cnt || !inv_off || !fill || !inv || !covered || !chosen) {
        free(cnt); free(inv_off); free(fill); free(inv); free(covered); free(chosen);
        return ORC_ENOMEM;
    }
    for (uint64_t e = 0; e < total; ++e) cnt[mem[e]]++;
    for (uint32_t v = 0; v < n; ++v) inv_off[v + 1] = inv_off[v] + cnt[v];
    for (uint64_t j = 0; j < theta; ++j)
        for (uint64_t e = off[j]; e < off[j + 1]; ++e) {
            uint32_t u = mem[e];
            inv[inv_off[u] + fill[u]++] = j;
        }
    for (uint32_t i = 0; i < k; ++i) {
        uint32_t best = 0xFFFFFFFFu;
        for (uint32_t v = 0; v < n; ++v) {
            if (chosen[v]) continue;
            if (best == 0xFFFFFFFFu || cnt[v] > cnt[best]) best = v;
        }
        seeds[i] = best;
        gains[i] = cnt[best];
        chosen[best] = 1;
        for (uint64_t x = inv_off[best]; x < inv_off[best + 1]; ++x) {
            uint64_t j = inv[x];
            if (covered[j]) continue;
            covered[j] = 1;
            for (uint64_t e = off[j]; e < off[j + 1]; ++e) cnt[mem[e]]--;
        }
    }
    free(cnt); free(inv_off); free(fill); free(inv); free(covered); free(chosen);
    return ORC_OK;
}

/* Lambda_R(S): the number of sets among the first theta that meet S. */
uint64_t orc_coverage(uint32_t n, uint64_t theta, const uint64_t *off, const uint32_t *mem,
                      uint32_t k, const uint32_t *seeds)
{
    uint8_t *inS = (uint8_t *)calloc(n ? n : 1, 1);
    for (uint32_t i = 0; i < k; ++i) inS[seeds[i]] = 1;
    uint64_t hit = 0;
    for (uint64_t j = 0; j < theta; ++j) {
        int h = 0;
        for (uint64_t e = off[j]; e < off[j + 1] && !h; ++e) h = inS[mem[e]];
        hit += (uint64_t)h;
    }
    free(inS);
    return hit;
}

/* Equation (8) with p_max = 1: the smallest, over the greedy prefixes
 * S_0* = {}, S_1*, ..., S_k* (seeds[] in selection order), of
 * Lambda_R1(S_i*) plus the sum of the k largest marginal coverages
 * Lambda_R1(u | S_i*) over all vertices u -- Lemma 4's bound on the coverage
 * of an optimal k-set, from each prefix.  Marginal coverages are recounted
 * from the sets S_i* leaves uncovered, one prefix at a time. */
static int cmp_u64_desc(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x < y) - (x > y);
}

uint64_t orc_upper_eq8(uint32_t n, uint64_t theta, const uint64_t *off, const uint32_t *mem,
                       uint32_t k, const uint32_t *seeds)
{
    uint8_t *covered = (uint8_t *)calloc(theta ? theta : 1, 1);
    uint64_t *marg = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t best = UINT64_MAX, cov = 0;
    for (uint32_t i = 0; i <= k; ++i) {
        memset(marg, 0, sizeof(uint64_t) * (n ? n : 1));
        for (uint64_t j = 0; j < theta; ++j)
            if (!covered[j])
                for (uint64_t e = off[j]; e < off[j + 1]; ++e) marg[mem[e]] += 1;
        qsort(marg, n, sizeof(uint64_t), cmp_u64_desc);
        uint64_t top = 0;
        for (uint32_t x = 0; x < k && x < n; ++x) top += marg[x];
        if (cov + top < best) best = cov + top;
        if (i == k) break;
        for (uint64_t j = 0; j < theta; ++j) {
            if (covered[j]) continue;
            for (uint64_t e = off[j]; e < off[j + 1]; ++e)
                if (mem[e] == seeds[i]) { covered[j] = 1; cov += 1; break; }
        }
    }
    free(covered);
    free(marg);
    return best;
}

/* ------------------------------------------------------------------------ */
/* Sample-size control (Section 4, Algorithm 4)                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    double delta, lnC, theta_max, theta0, a;
    uint64_t theta1;
    uint32_t i_max;
} orc_schedule;

/* delta = |V|^-ell.  ln C(n,k) summed term by term in ascending i.
 * theta_max follows Lemma 6 in the OPIM-C form the lemma cites:
 *   2n (t sqrt(ln(6/delta)) + sqrt(t (ln C(n,k) + ln(6/delta))))^2 / (eps^2 k),
 * t = 1 - 1/e.  theta_0 = theta_max eps^2 k / n, rounded up to a ladder
 * boundary Q 2^b (and at least Q).  i_max is the first round whose size
 * reaches theta_max; a = ln(3 i_max / delta) spreads delta over the rounds
 * and the two bounds. */
int orc_make_schedule(uint32_t n, uint32_t k, double eps, double ell, uint32_t qlog, orc_schedule *s)
{
    if (n == 0 || k == 0 || k > n || !(eps > 0.0 && eps < 1.0) || !(ell > 0.0)) return ORC_EINVAL;
    double t = 1.0 - exp(-1.0);
    double lndelta_inv = ell * log((double)n);          /* ln(1/delta) */
    s->delta = exp(-lndelta_inv);
    double lnC = 0.0;
    for (uint32_t i = 0; i < k; ++i) lnC += log((double)(n - i) / (double)(i + 1));
    s->lnC = lnC;
    double l6 = log(6.0) + lndelta_inv;
    double root = t * sqrt(l6) + sqrt(t * (lnC + l6));
    s->theta_max = 2.0 * (double)n * root * root / (eps * eps * (double)k);
    s->theta0 = s->theta_max * eps * eps * (double)k / (double)n;
    uint64_t Q = (uint64_t)1 << qlog;
    uint64_t th = Q;
    while ((double)th < s->theta0) th <<= 1;
    s->theta1 = th;
    uint32_t i = 1;
    while ((double)th < s->theta_max) { th <<= 1; ++i; }
    s->i_max = i;
    s->a = log(3.0 * (double)i) + lndelta_inv;
    return ORC_OK;
}

/* Equation (12): lower bound on the spread of S* from its coverage Lambda2
 * in the independent pool R2 of size theta (clamped at zero). */
double orc_sigma_lower(double lambda2, double a, double n, double theta)
{
    double r = sqrt(lambda2 + 2.0 * a / 9.0) - sqrt(a / 2.0);
    double v = r * r - a / 18.0;
    if (v < 0.0) v = 0.0;
    return v * n / theta;
}

/* Lemma 5 with p_max = 1: the optimum's coverage in R1 is at most
 * Lambda1 / (1 - (1 - 1/k)^k); lifted to spread by the same concentration
 * term as the lower bound. */
/* The concentration lift of a coverage upper bound on R1 to an upper bound
 * on the optimal spread, as in orc_sigma_upper. */
double orc_sigma_upper_cov(double cov_upper, double a, double n, double theta)
{
    double r = sqrt(cov_upper + a / 2.0) + sqrt(a / 2.0);
    return r * r * n / theta;
}

double orc_sigma_upper(double lambda1, uint32_t k, double a, double n, double theta)
{
    double up = lambda1 / (1.0 - pow(1.0 - 1.0 / (double)k, (double)k));
    double r = sqrt(up + a / 2.0) + sqrt(a / 2.0);
    return r * r * n / theta;
}

typedef struct {
    uint32_t rounds;
    uint32_t i_max;
    uint64_t theta;
    uint64_t lambda1, lambda2;
    double sigma_l, sigma_u, spread, theta_max;
    uint64_t entries1, entries2;
    uint64_t lambda_u;   /* Equation (8) coverage bound of the last round (bound 0) */
} orc_result;

/* HyperIM_BRR (Algorithm 4): two independent pools R1 (tag 0) and R2 (tag 1)
 * grow together over ladder prefixes theta_i = theta_1 2^(i-1); S* = greedy
 * on R1; Lambda2 = coverage of S* in R2; stop once sigma_l / sigma_u >=
 * 1 - 1/e - eps or at round i_max.  theta_fixed > 0 runs one round of that
 * size with no bound test. */
int orc_select_seeds(const orc_graph *g, uint32_t k, double eps, double ell, uint64_t seed,
                     uint32_t instance, uint32_t qlog, uint64_t theta_fixed, uint32_t nthreads,
                     uint32_t bound, uint32_t *seeds, uint64_t *gains, orc_result *res)
{
    if (!g->stratified) return ORC_EINVAL;
    orc_schedule s;
    int rc = orc_make_schedule(g->n, k, eps, ell, qlog, &s);
    if (rc) return rc;
    memset(res, 0, sizeof(*res));
    res->i_max = s.i_max;
    res->theta_max = s.theta_max;
    double t = 1.0 - exp(-1.0);
    uint64_t have = 0;
    uint64_t *off1 = (uint64_t *)calloc(1, sizeof(uint64_t)), *off2 = (uint64_t *)calloc(1, sizeof(uint64_t));
    uint32_t *mem1 = NULL, *mem2 = NULL;
    uint32_t i_max = theta_fixed ? 1u : s.i_max;
    for (uint32_t i = 1; i <= i_max; ++i) {
        uint64_t theta = theta_fixed ? theta_fixed : (s.theta1 << (i - 1));
        for (uint32_t pool = 0; pool < 2; ++pool) {
            uint64_t *o, *noff; uint32_t *mm, *r;
            rc = orc_generate(g, seed, instance, pool, have, theta, qlog, nthreads, NULL, &o, &mm, &r);
            if (rc) goto out;
            uint64_t **poff = pool ? &off2 : &off1;
            uint32_t **pmem = pool ? &mem2 : &mem1;
            uint64_t old_total = (*poff)[have];
            uint64_t add = o[theta - have];
            noff = (uint64_t *)realloc(*poff, sizeof(uint64_t) * (theta + 1));
            uint32_t *nmem = (uint32_t *)realloc(*pmem, sizeof(uint32_t) * (old_total + add + 1));
            if (!noff || !nmem) { rc = ORC_ENOMEM; free(o); free(mm); free(r); goto out; }
            for (uint64_t x = 1; x <= theta - have; ++x) noff[have + x] = old_total + o[x];
            memcpy(nmem + old_total, mm, sizeof(uint32_t) * add);
            *poff = noff;
            *pmem = nmem;
            free(o); free(mm); free(r);
        }
        have = theta;
        rc = orc_greedy(g->n, theta, off1, mem1, k, seeds, gains);
        if (rc) goto out;
        uint64_t lambda1 = 0;
        for (uint32_t x = 0; x < k; ++x) lambda1 += gains[x];
        uint64_t lambda2 = orc_coverage(g->n, theta, off2, mem2, k, seeds);
        double sl = orc_sigma_lower((double)lambda2, s.a, (double)g->n, (double)theta);
        /* upper bound: Equation (8) (bound 0) or Lemma 5's closed form (1) */
        double su;
        if (bound == 0) {
            res->lambda_u = orc_upper_eq8(g->n, theta, off1, mem1, k, seeds);
            su = orc_sigma_upper_cov((double)res->lambda_u, s.a, (double)g->n, (double)theta);
        } else {
            su = orc_sigma_upper((double)lambda1, k, s.a, (double)g->n, (double)theta);
        }
        res->rounds = i;
        res->theta = theta;
        res->lambda1 = lambda1;
        res->lambda2 = lambda2;
        res->sigma_l = sl;
        res->sigma_u = su;
        res->spread = (double)g->n * (double)lambda2 / (double)theta;
        res->entries1 = off1[theta];
        res->entries2 = off2[theta];
        if (theta_fixed) break;
        if (su > 0.0 && sl / su >= t - eps) break;
    }
out:
    free(off1); free(off2); free(mem1); free(mem2);
    return rc;
}
