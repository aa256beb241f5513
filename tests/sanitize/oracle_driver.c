/* Drives the CPU oracle through its whole API on one hypergraph read from a
 * file, for an AddressSanitizer / UndefinedBehaviorSanitizer build: graph
 * construction (and its rejection of malformed input), stratification,
 * roots, RR sets one by one and in threads, greedy, coverage, the schedule
 * and the HyperIM_BRR loop.  Prints a checksum line; any sanitizer report
 * makes the process fail.
 *
 * Input file: uint32 n, m, model; float p; uint32 k; double eps;
 * then he_off[m+1] and he_mem[he_off[m]] (uint32). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_graph orc_graph;
typedef struct {
    uint32_t rounds, i_max;
    uint64_t theta, lambda1, lambda2;
    double sigma_l, sigma_u, spread, theta_max;
    uint64_t entries1, entries2;
    uint64_t lambda_u;
} orc_result;

int orc_graph_new(uint32_t n, uint32_t m, const uint32_t *he_off, const uint32_t *he_mem, uint32_t model, float p,
                  orc_graph **out);
void orc_graph_free(orc_graph *g);
int orc_stratify(orc_graph *g);
uint32_t orc_root(const orc_graph *g, uint64_t seed, uint32_t instance, uint32_t pool, uint64_t j, uint32_t qlog);
uint32_t orc_rr_set(const orc_graph *g, uint64_t seed, uint32_t instance, uint32_t pool, uint64_t j, uint32_t qlog,
                    uint32_t *out);
int orc_generate(const orc_graph *g, uint64_t seed, uint32_t instance, uint32_t pool, uint64_t id_begin,
                 uint64_t id_end, uint32_t qlog, uint32_t nthreads, const uint32_t *roots_in, uint64_t **off_out,
                 uint32_t **mem_out, uint32_t **roots_out);
void orc_free(void *p);
int orc_greedy(uint32_t n, uint64_t theta, const uint64_t *off, const uint32_t *mem, uint32_t k, uint32_t *seeds,
               uint64_t *gains);
uint64_t orc_coverage(uint32_t n, uint64_t theta, const uint64_t *off, const uint32_t *mem, uint32_t k,
                      const uint32_t *seeds);
int orc_select_seeds(const orc_graph *g, uint32_t k, double eps, double ell, uint64_t seed, uint32_t instance,
                     uint32_t qlog, uint64_t theta_fixed, uint32_t nthreads, uint32_t bound, uint32_t *seeds,
                     uint64_t *gains, orc_result *res);
uint64_t orc_upper_eq8(uint32_t n, uint64_t theta, const uint64_t *off, const uint32_t *mem, uint32_t k,
                       const uint32_t *seeds);

static void *read_all(FILE *f, size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv)
{
    if (argc != 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    uint32_t n, m, model, k;
    float p;
    double eps;
    if (fread(&n, 4, 1, f) != 1 || fread(&m, 4, 1, f) != 1 || fread(&model, 4, 1, f) != 1 ||
        fread(&p, 4, 1, f) != 1 || fread(&k, 4, 1, f) != 1 || fread(&eps, 8, 1, f) != 1)
        return 2;
    uint32_t *he_off = (uint32_t *)read_all(f, 4 * ((size_t)m + 1));
    uint32_t *he_mem = (uint32_t *)read_all(f, 4 * (size_t)he_off[m]);
    fclose(f);

    /* malformed inputs are rejected without touching memory they do not own */
    orc_graph *bad = NULL;
    uint32_t off_bad[3] = {0, 3, 2}, mem_bad[3] = {0, 1, 0};
    if (orc_graph_new(4, 2, off_bad, mem_bad, 0, 0.5f, &bad) == 0) return 3;
    uint32_t off_dup[2] = {0, 3};
    if (orc_graph_new(4, 1, off_dup, mem_bad, 0, 0.5f, &bad) == 0) return 3;
    uint32_t mem_big[3] = {0, 1, 9};
    if (orc_graph_new(4, 1, off_dup, mem_big, 0, 0.5f, &bad) == 0) return 3;

    orc_graph *g = NULL;
    if (orc_graph_new(n, m, he_off, he_mem, model, p, &g) != 0) return 4;
    if (orc_stratify(g) != 0) return 5;
    uint64_t sum = 0;
    uint32_t *set = (uint32_t *)malloc(sizeof(uint32_t) * n);
    for (uint64_t j = 0; j < 300; ++j) {
        sum += orc_root(g, 1, 2, (uint32_t)(j & 1), j * 37, 8);
        uint32_t sz = orc_rr_set(g, 1, 2, (uint32_t)(j & 1), j * 37, 8, set);
        for (uint32_t i = 0; i < sz; ++i) sum += set[i] * (i + 1);
    }
    uint64_t *off = NULL;
    uint32_t *mem = NULL, *roots = NULL;
    if (orc_generate(g, 0, 0, 0, 0, 2048, 8, 4, NULL, &off, &mem, &roots) != 0) return 6;
    uint32_t *seeds = (uint32_t *)malloc(sizeof(uint32_t) * k);
    uint64_t *gains = (uint64_t *)malloc(sizeof(uint64_t) * k);
    if (orc_greedy(n, 2048, off, mem, k, seeds, gains) != 0) return 7;
    sum += orc_coverage(n, 2048, off, mem, k, seeds);
    if (orc_greedy(n, 2048, off, mem, 0, seeds, gains) == 0) return 7;
    sum += orc_upper_eq8(n, 2048, off, mem, k, seeds);
    orc_free(off);
    orc_free(mem);
    orc_free(roots);
    orc_result r;
    for (uint32_t bound = 0; bound < 2; ++bound) {
        if (orc_select_seeds(g, k, eps, 1.0, 0, 0, 8, 0, 4, bound, seeds, gains, &r) != 0) return 8;
        for (uint32_t i = 0; i < k; ++i) sum += seeds[i] + gains[i];
    }
    if (orc_select_seeds(g, k, eps, 1.0, 0, 0, 8, 4096, 2, 0, seeds, gains, &r) != 0) return 8;
    printf("ok %llu theta %llu\n", (unsigned long long)sum, (unsigned long long)r.theta);
    free(set);
    free(seeds);
    free(gains);
    orc_graph_free(g);
    free(he_off);
    free(he_mem);
    return 0;
}
