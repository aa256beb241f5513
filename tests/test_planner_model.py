"""Work-item layout of the grid-wide RR-generation planners and the progress
rules of the host loops that drive them, checked on the CPU.

The library exports a host model of one planning wave that runs the same
layout arithmetic as the device planners (per-lane heavy splits, light
segments, the reservation fallback, and the owner search that spreads a
batch's heavy chunks over the wave).  Its items are compared with a plain
sequential loop: every incidence of every entry that is not yet expanded is
covered exactly once, chunks keep their length bound, segments their weight
bound, and items come in the planner's order.  The loop checks must stop a
loop that has no work left, keep one that progresses, and flag one that
stalls or overruns."""
import ctypes as C
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2406_01911_amd", "libhyperim.so")

ITEM_CAP = 1 << 22
MAX_ITEMS_PER_VERTEX = 1 << 20
CONTINUE, DONE, STALLED, OVER = 0, 1, 2, 3


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2406_01911_amd import build
        build.build()
    import torch  # noqa: F401  (binds the HIP runtime first, as the binding does)
    L = C.CDLL(LIB)
    vp = C.c_void_p
    L.hyperim_model_plan_batch.argtypes = [C.c_uint32, C.c_uint32, vp, vp, vp, vp, C.c_uint32, C.c_uint32,
                                           C.c_uint32, vp, C.c_uint32, C.POINTER(C.c_uint32),
                                           C.POINTER(C.c_uint32)]
    L.hyperim_model_loop_check.argtypes = [C.c_uint32] + [C.c_uint64] * 6
    return L


def model(lib, mode, deg, e0, sets=None, expanded=None, chunk=256, seg=512, item_cap=ITEM_CAP):
    nb = len(deg)
    deg = np.ascontiguousarray(deg, np.uint32)
    e0 = np.ascontiguousarray(e0, np.uint32)
    sets_a = np.ascontiguousarray(sets if sets is not None else np.ones(nb), np.uint32)
    exp_a = np.ascontiguousarray(expanded if expanded is not None else np.zeros(nb), np.uint8)
    # items a batch can need: one segment per entry plus every heavy chunk
    # (chunk lengths never go below 1 incidence)
    cap_out = int(min(nb + int(np.sum(deg.astype(np.int64))), (1 << 20) + 64))
    items = np.zeros((cap_out, 4), np.uint32)
    n, taken = C.c_uint32(0), C.c_uint32(0)
    rc = lib.hyperim_model_plan_batch(mode, nb, deg.ctypes.data, e0.ctypes.data, sets_a.ctypes.data,
                                      exp_a.ctypes.data, chunk, seg, item_cap, items.ctypes.data, cap_out,
                                      C.byref(n), C.byref(taken))
    assert rc == 0
    return items[:n.value].copy(), taken.value


def div_up(a, b):
    return (a + b - 1) // b


def reference(mode, deg, e0, sets, expanded, chunk, seg, item_cap=ITEM_CAP):
    """The planner's layout written as a plain loop over the batch's entries."""
    seg = max(seg, chunk)
    nb = len(deg)
    live = [mode == 1 or not expanded[l] for l in range(nb)]
    if not any(live):
        return [], nb
    split = []
    for l in range(nb):
        d = int(deg[l])
        if not live[l]:
            split.append((0, 0))
        elif mode == 0:
            ln = max(chunk, div_up(d, MAX_ITEMS_PER_VERTEX))
            split.append((ln, div_up(d, ln) if d > chunk else 0))
        else:
            ln = max(max(1, chunk // max(int(sets[l]), 1)), div_up(d, ITEM_CAP // 128))
            split.append((ln, div_up(d, ln) if d > ln else 0))
    weight = [0 if (not live[l] or split[l][1]) else (int(deg[l]) if mode == 0 else int(deg[l]) * int(sets[l]))
              for l in range(nb)]
    starts, before, prev = [], 0, None
    for l in range(nb):
        s = before // seg
        if l == 0 or s != prev:
            starts.append(l)
        prev = s
        before += weight[l]
    heavy_lanes = list(range(nb))
    if mode == 0 and len(starts) + sum(c for _, c in split) > item_cap:
        starts, heavy_lanes, nb = [0], [0], 1
    items = []
    for i, l in enumerate(starts):
        nxt = starts[i + 1] if i + 1 < len(starts) else nb
        items.append((l, nxt - l, 0, 0))
    for l in heavy_lanes:
        ln, cnt = split[l]
        for r in range(cnt):
            lo = int(e0[l]) + r * ln
            items.append((l | 0x80000000, lo, min(lo + ln, int(e0[l]) + int(deg[l])), 0))
    return items, nb


def coverage_ok(mode, items, deg, e0, sets, expanded, chunk, seg, taken):
    """Every live entry's incidences covered once; bounds hold."""
    seg = max(seg, chunk)
    covered_light = np.zeros(taken, bool)
    ranges = {}
    for x, a, b, _ in items:
        if x & 0x80000000:
            l = x & 0x7FFFFFFF
            ranges.setdefault(l, []).append((a, b))
        else:
            assert not covered_light[x:x + a].any()
            covered_light[x:x + a] = True
            w = sum(0 if l in ranges else int(deg[l]) * (int(sets[l]) if mode == 1 else 1)
                    for l in range(x, x + a))
            assert a >= 1
    assert covered_light.all()   # every consumed entry is in one segment
    for l in range(taken):
        live = mode == 1 or not expanded[l]
        if l in ranges:
            rs = sorted(ranges[l])
            assert rs[0][0] == e0[l] and rs[-1][1] == int(e0[l]) + int(deg[l])
            for (a0, b0), (a1, b1) in zip(rs, rs[1:]):
                assert b0 == a1 and b0 > a0
            assert live


def random_batch(rng, mode, nb, chunk):
    kind = rng.integers(0, 4, nb)   # 0 expanded, 1 light, 2 heavy, 3 hub
    hub = 400 if mode == 0 else 60
    deg = np.where(kind == 1, rng.integers(0, chunk + 1, nb),
                   np.where(kind == 2, rng.integers(chunk + 1, 20 * chunk, nb),
                            np.where(kind == 3, rng.integers(50 * chunk, hub * chunk, nb), rng.integers(0, 9, nb))))
    e0 = rng.integers(0, 1 << 28, nb)
    sets = rng.integers(1, 65, nb)
    expanded = (kind == 0) if mode == 0 else np.zeros(nb, bool)
    return deg.astype(np.uint32), e0.astype(np.uint32), sets.astype(np.uint32), expanded


@pytest.mark.parametrize("mode", [0, 1])
def test_layout_matches_plain_loop(lib, mode):
    rng = np.random.default_rng(11 + mode)
    for trial in range(300):
        nb = int(rng.integers(1, 65))
        chunk = int(rng.choice([16, 64, 256, 1024]))
        seg = int(rng.choice([16, 128, 512, 2048]))
        deg, e0, sets, expanded = random_batch(rng, mode, nb, chunk)
        got, taken = model(lib, mode, deg, e0, sets, expanded, chunk, seg)
        want, want_taken = reference(mode, deg, e0, sets, expanded, chunk, seg)
        assert taken == want_taken, trial
        assert [tuple(map(int, r)) for r in got] == [tuple(x) for x in want], trial
        if want:
            coverage_ok(mode, got, deg, e0, sets, expanded, chunk, seg, taken)


def test_all_expanded_batch_takes_its_entries_without_items(lib):
    items, taken = model(lib, 0, [5, 9000, 1], [0, 10, 20], expanded=[1, 1, 1])
    assert len(items) == 0 and taken == 3


def test_reservation_fallback_plans_the_first_entry_alone(lib):
    # 64 hubs of 2^28 incidences: 2^20 chunks each, far above the item cap
    deg = np.full(64, 1 << 28, np.uint32)
    e0 = np.arange(64, dtype=np.uint32) * 7
    items, taken = model(lib, 0, deg, e0, chunk=256, item_cap=ITEM_CAP)
    assert taken == 1
    assert len(items) == 1 + MAX_ITEMS_PER_VERTEX <= ITEM_CAP
    assert tuple(items[0]) == (0, 1, 0, 0)
    heavy = items[1:]
    assert np.all(heavy[:, 0] == 0x80000000)
    assert heavy[0, 1] == 0 and heavy[-1, 2] == 1 << 28
    assert np.all(heavy[1:, 1] == heavy[:-1, 2])
    # a smaller cap forces the same fallback on an ordinary batch
    deg = np.array([3000, 40, 5000, 7], np.uint32)
    items, taken = model(lib, 0, deg, np.zeros(4, np.uint32), chunk=256, seg=512, item_cap=8)
    want, want_taken = reference(0, deg, np.zeros(4), None, np.zeros(4, bool), 256, 512, item_cap=8)
    assert taken == want_taken == 1 and [tuple(map(int, r)) for r in items] == want


def test_chunk_growth_bounds_items_per_vertex(lib):
    # per-set mode: one vertex never needs more than 2^20 items; bundled mode:
    # a batch of 64 entries always fits half the item buffer plus its segments
    for d in (1 << 20, (1 << 28) + 5, 0xFFFF0000):
        items, _ = model(lib, 0, [d], [0], chunk=16)
        assert len(items) - 1 <= MAX_ITEMS_PER_VERTEX
    deg = np.full(1, 0xFFFF0000, np.uint32)
    items, _ = model(lib, 1, deg, np.zeros(1, np.uint32), sets=np.full(1, 64, np.uint32), chunk=16)
    assert len(items) - 1 <= ITEM_CAP // 128


def test_phase_b_progress_rule(lib):
    chk = lambda a, b, c, d: lib.hyperim_model_loop_check(0, a, b, c, d, 0, 0)
    assert chk(0, 0, 0, 100) == DONE          # no items in the last superstep: nothing left
    assert chk(10, 10, 0, 100) == DONE
    assert chk(0, 5, 3, 100) == CONTINUE      # work planned and entries taken
    assert chk(5, 5, 3, 100) == STALLED       # work pending but no entry taken in a whole batch
    assert chk(5, 4, 3, 100) == STALLED
    assert chk(5, 101, 3, 100) == OVER        # more entries than the sets can hold


def test_bundled_progress_rule(lib):
    chk = lambda *a: lib.hyperim_model_loop_check(1, *a)
    big = 1 << 40
    assert chk(0, 2 ** 64 - 1, 0, 7, 0, big) == CONTINUE   # first batch
    assert chk(3, 7, 3, 2, 0, big) == CONTINUE             # pending batches planned
    assert chk(3, 7, 4, 9, 0, big) == CONTINUE             # next level
    assert chk(3, 7, 3, 7, 0, big) == STALLED
    assert chk(3, 7, 3, 8, 0, big) == STALLED
    assert chk(3, 7, 3, 7, 1, big) == DONE
    assert chk(3, 7, big + 1, 0, 0, big) == OVER


def test_chunks_near_the_end_of_the_incidence_space(lib):
    # a vertex whose incidences end just below 2^32: chunk ends must not wrap
    e0 = np.array([(1 << 32) - 1000], np.uint32)
    deg = np.array([999], np.uint32)
    items, _ = model(lib, 0, deg, e0, chunk=16)
    heavy = items[1:].astype(np.int64)
    assert heavy[0, 1] == int(e0[0]) and heavy[-1, 2] == int(e0[0]) + 999
    assert np.all(heavy[:, 2] > heavy[:, 1]) and np.all(heavy[1:, 1] == heavy[:-1, 2])
