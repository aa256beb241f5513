// Host model of one planning wave of the grid-wide RR-generation phase and of
// the progress rules of the host loops, for the CPU tests.  It runs the same
// layout arithmetic the device planners k_plan and k_ms_plan use
// (plan_layout.h) over plain arrays instead of wave registers: per-lane
// heavy splits, light segments, the reservation fallback of the per-set
// planner, and the owner search that spreads a batch's heavy chunks over the
// wave.  Nothing here runs on the device or in the generation path.
#include <stdint.h>

#include "internal.h"
#include "plan_layout.h"

using namespace hyperim;

// mode 0: per-set planner (entries may be marked expanded; a batch whose
// items exceed item_cap plans its first entry alone); mode 1: bundled
// planner (entry weights are incidences times sets).
// Lanes [0, nb) carry deg[l], e0[l], sets[l] (mode 1) and expanded[l]
// (mode 0).  Items go to items[4 * i ..] as (lane, count, 0, 0) for a light
// segment starting at `lane` and (lane | 1 << 31, lo, hi, 0) for a heavy
// chunk of lane's incidences [lo, hi); *n_items receives the batch's
// reservation, *taken the entries the batch consumes.  Returns 0, or -1 when
// an argument is out of range or `items` holds fewer than cap_out items.
extern "C" int hyperim_model_plan_batch(uint32_t mode, uint32_t nb, const uint32_t *deg, const uint32_t *e0,
                                        const uint32_t *sets, const uint8_t *expanded, uint32_t chunk, uint32_t seg,
                                        uint32_t item_cap, uint32_t *items, uint32_t cap_out, uint32_t *n_items,
                                        uint32_t *taken) {
    constexpr uint32_t W = 64;
    if (mode > 1 || nb == 0 || nb > W || !deg || !e0 || !items || !n_items || !taken || chunk == 0 || seg == 0 ||
        (mode == 1 && !sets))
        return -1;
    seg = seg > chunk ? seg : chunk;   // as the library sets it
    uint32_t hv[W] = {0}, len[W] = {0}, light[W] = {0};
    bool live[W] = {false};
    bool any = false;
    for (uint32_t l = 0; l < nb; ++l) {
        live[l] = mode == 1 || !expanded || !expanded[l];
        if (!live[l]) continue;
        any = true;
        const HeavySplit h = mode == 0 ? heavy_split(deg[l], chunk) : ms_heavy_split(deg[l], sets[l], chunk);
        hv[l] = h.count;
        len[l] = h.len;
        light[l] = hv[l] ? 0u : (mode == 0 ? deg[l] : deg[l] * sets[l]);
    }
    *n_items = 0;
    *taken = nb;
    if (!any) return 0;   // every entry already expanded
    // segments of light entries: a lane starts one when its segment index
    // differs from the previous lane's
    uint32_t segidx[W] = {0};
    bool first[W] = {false};
    uint32_t acc = 0, nseg = 0;
    for (uint32_t l = 0; l < nb; ++l) {
        acc += light[l];
        segidx[l] = segment_of(acc, light[l], seg);
        first[l] = l == 0 || segidx[l] != segidx[l - 1];
        nseg += first[l] ? 1u : 0u;
    }
    uint32_t hscan[W] = {0};
    auto rescan = [&]() {
        uint32_t s = 0;
        for (uint32_t l = 0; l < W; ++l) {
            s += hv[l];
            hscan[l] = s;
        }
    };
    rescan();
    uint64_t need = (uint64_t)nseg + hscan[W - 1];
    if (mode == 0 && need > item_cap) {   // plan the first entry alone
        nb = 1;
        for (uint32_t l = 1; l < W; ++l) hv[l] = 0;
        for (uint32_t l = 1; l < W; ++l) first[l] = false;
        nseg = 1;
        rescan();
        need = 1u + (uint64_t)hscan[W - 1];
        *taken = 1;
    }
    if (need > cap_out) return -1;
    uint32_t out = 0;
    for (uint32_t l = 0; l < nb; ++l) {
        if (!first[l]) continue;
        uint32_t next = l + 1;
        while (next < nb && !first[next]) ++next;
        uint32_t *it = items + 4 * (size_t)out++;
        it[0] = l;
        it[1] = next - l;
        it[2] = it[3] = 0;
    }
    const uint32_t H = hscan[W - 1];
    for (uint32_t q = 0; q < H; ++q) {
        const uint32_t k = scan_owner([&](uint32_t i) { return hscan[i]; }, q);
        const uint32_t excl = hscan[k] - hv[k];
        const ChunkRange c = chunk_range(e0[k], deg[k], len[k], q - excl);
        uint32_t *it = items + 4 * (size_t)(nseg + q);
        it[0] = k | 0x80000000u;
        it[1] = c.lo;
        it[2] = c.hi;
        it[3] = 0;
    }
    *n_items = (uint32_t)need;
    return 0;
}

// which 0: phase_b_check(a, b, c, d); which 1: bundled_check(a, b, c, d, e, f).
extern "C" int hyperim_model_loop_check(uint32_t which, uint64_t a, uint64_t b, uint64_t c, uint64_t d, uint64_t e,
                                        uint64_t f) {
    if (which == 0) return phase_b_check(a, b, c, d);
    if (which == 1) return bundled_check(a, b, c, d, e, f);
    return -1;
}
