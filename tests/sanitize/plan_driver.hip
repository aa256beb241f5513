// Drives the host model of the grid-wide planners (plan_model.hip) and the
// loop checks on random and extreme batches, for a build whose host code
// carries AddressSanitizer / UndefinedBehaviorSanitizer; prints a checksum.
#include <stdint.h>
#include <stdio.h>

#include <random>
#include <vector>

extern "C" int hyperim_model_plan_batch(uint32_t mode, uint32_t nb, const uint32_t *deg, const uint32_t *e0,
                                        const uint32_t *sets, const uint8_t *expanded, uint32_t chunk, uint32_t seg,
                                        uint32_t item_cap, uint32_t *items, uint32_t cap_out, uint32_t *n_items,
                                        uint32_t *taken);
extern "C" int hyperim_model_loop_check(uint32_t which, uint64_t a, uint64_t b, uint64_t c, uint64_t d, uint64_t e,
                                        uint64_t f);

int main() {
    std::mt19937_64 rng(7);
    const uint32_t cap_out = (1u << 20) + 128;
    std::vector<uint32_t> items(4 * (size_t)cap_out);
    uint64_t sum = 0;
    const uint32_t chunks[] = {1, 16, 256, 4096};
    for (int trial = 0; trial < 2000; ++trial) {
        const uint32_t mode = trial & 1, nb = 1 + (uint32_t)(rng() % 64);
        const uint32_t chunk = chunks[rng() % 4], seg = chunks[rng() % 4];
        uint32_t deg[64], e0[64], sets[64];
        uint8_t exp[64];
        for (uint32_t l = 0; l < nb; ++l) {
            const uint32_t kind = (uint32_t)(rng() % 5);
            deg[l] = kind == 0 ? 0u : kind == 1 ? (uint32_t)(rng() % (chunk + 1))
                   : kind == 2 ? chunk + 1 + (uint32_t)(rng() % (8 * chunk + 1))
                   : kind == 3 ? (uint32_t)(rng() % 60000) : 0xFFFFFFF0u - (uint32_t)(rng() % 1000);
            if (mode == 1 && kind == 4) deg[l] = (uint32_t)(rng() % 4000);
            e0[l] = kind == 4 && mode == 0 ? 5u : (uint32_t)(rng() % (1u << 30));
            sets[l] = 1 + (uint32_t)(rng() % 64);
            exp[l] = (uint8_t)(rng() % 4 == 0);
        }
        uint32_t n = 0, taken = 0;
        const uint32_t cap = (trial % 7 == 0) ? 8u : (1u << 22);
        const int rc = hyperim_model_plan_batch(mode, nb, deg, e0, sets, exp, chunk, seg, cap, items.data(), cap_out,
                                                &n, &taken);
        if (rc == 0)
            for (uint32_t i = 0; i < 4 * n; ++i) sum += items[i];
        sum += (uint64_t)rc + taken;
    }
    // argument errors are reported, not dereferenced
    uint32_t n = 0, taken = 0;
    if (hyperim_model_plan_batch(2, 1, nullptr, nullptr, nullptr, nullptr, 1, 1, 1, items.data(), 1, &n, &taken) != -1)
        return 3;
    if (hyperim_model_plan_batch(0, 65, nullptr, nullptr, nullptr, nullptr, 1, 1, 1, items.data(), 1, &n, &taken) != -1)
        return 3;
    for (uint64_t a = 0; a < 4; ++a)
        for (uint64_t b = 0; b < 4; ++b) {
            sum += (uint64_t)hyperim_model_loop_check(0, a, b, a ^ b, 3, 0, 0);
            sum += (uint64_t)hyperim_model_loop_check(1, a, b, b, a, a & 1, 2);
        }
    printf("ok %llu\n", (unsigned long long)sum);
    return 0;
}
