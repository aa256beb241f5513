"""The allocation-free coverage entry point against hyperim_coverage.

hyperim_coverage_noalloc keeps its scratch in a static device array of the
library and takes seeds and result in device memory.  Two calls in a row --
the second on a smaller input, so that it runs over what the first left in
the shared scratch -- must each return exactly what hyperim_coverage returns
for the same pool prefix and seeds; ids >= n are ignored; inputs beyond the
scratch fail with HYPERIM_ECAPACITY before any work."""
import numpy as np
import pytest

import hypergen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hy():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_01911_amd as hy
    hy.load_library()
    return hy


def _noalloc(hy, g, pool, theta, seeds):
    import torch
    sd = torch.from_numpy(np.asarray(seeds, np.uint32).view(np.int32)).cuda()
    out = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    hy.coverage_noalloc(g, pool, theta, sd, out)
    torch.cuda.synchronize()
    return int(out.item())


def test_noalloc_coverage_matches_coverage_twice(hy):
    print("[gpu] coverage without allocation: two calls", flush=True)
    w = hypergen.workload("mid")
    hg = w.build()
    g = hy.build_graph(hg.n, hg.he_off, hg.he_mem, w.model, w.p)
    g.stratify()
    pool = hy.Pool(g)
    hy.generate_rr(g, 3, 1, 0, 0, 6000, pool)
    seeds, _ = hy.greedy(g, pool, 6000, 40)
    first = (6000, seeds)                          # large sets included
    second = (700, seeds[:5][::-1].copy())         # smaller input
    for theta, sd in (first, second):
        want = hy.coverage(g, pool, theta, sd)
        got = _noalloc(hy, g, pool, theta, sd)
        assert got == want, (theta, len(sd), got, want)
        assert want > 0
    # ids >= n are ignored; no seeds covers nothing
    assert _noalloc(hy, g, pool, 700, np.array([hg.n + 5, 0xFFFFFFFF], np.uint32)) == 0
    assert _noalloc(hy, g, pool, 700, np.zeros(0, np.uint32)) == 0
    assert _noalloc(hy, g, pool, 700, seeds[:5]) == hy.coverage(g, pool, 700, seeds[:5])


def test_noalloc_coverage_rejects_inputs_beyond_its_scratch(hy):
    import torch
    n = 34_000_000   # n bytes of seed flags exceed the 32 MiB scratch
    hg = hypergen.from_lists(n, [[0, 1], [2, 3, n - 1]])
    g = hy.build_graph(n, hg.he_off, hg.he_mem, 0, 0.5)
    g.stratify()
    pool = hy.Pool(g)
    hy.generate_rr(g, 0, 0, 0, 0, 16, pool)
    sd = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    with pytest.raises(hy.HyperIMError) as e:
        hy.coverage_noalloc(g, pool, 16, sd, out)
    assert e.value.status == hy.ECAPACITY
    torch.cuda.synchronize()
    assert int(out.item()) == -7   # nothing written
