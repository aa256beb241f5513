"""Pins of the oracle's geometric-gap sampler for the independent cascade
(models 5 and 6), independent of the oracle's own code.

* The gap draw: over all 2^32 words x, the gap is monotone in x, so each
  gap value takes an interval of words; the interval lengths (found by
  bisection on the drawn gaps) give the exact probability of every gap, which
  must be Geometric(p) -- p q^g for g < G and q^G for "none left" -- to within
  the rounding of the 32-bit word (2^-32 per boundary) and of the products.
* The RR sets realise the independent cascade: exact enumeration of all live
  worlds of a tiny hypergraph (every channel u -> v live with p_v
  independently, Section 2.1) gives Pr[u in RR(r)], which the gap sampler's
  frequencies match, for constant p and for the weighted cascade.
* Members of a star reached only through its centre are independent
  Bernoulli(p) (count Binomial, pairs p^2).
* p = 1 gives connected components, p = 0 the root alone.
"""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import hypergen
import oracle
from test_oracle_rr import TINY_EDGES, _enumerate_inclusion_f64, _tiny_thresholds_as_probs

GAPS_CONST, GAPS_WC = 5, 6


def _first_word_with_gap_at_least(q, G, g):
    """Smallest x with gap_draw(q, x, G) >= g (the draw is monotone in x)."""
    lo, hi = 0, 1 << 32
    while lo < hi:
        mid = (lo + hi) // 2
        if oracle.gap_draw(q, mid, G) >= g:
            hi = mid
        else:
            lo = mid + 1
    return lo


@pytest.mark.parametrize("p,G", [(0.3, 12), (0.01, 200), (1.0 / 3.0, 5), (1e-4, 1000), (0.999, 7)])
def test_gap_draw_is_geometric(p, G):
    q = 1.0 - p
    xs = np.random.default_rng(1).integers(0, 1 << 32, size=2000)
    gaps = [oracle.gap_draw(q, int(x), G) for x in np.sort(xs)]
    assert all(a <= b for a, b in zip(gaps, gaps[1:]))   # monotone in x
    bounds = [_first_word_with_gap_at_least(q, G, g) for g in range(G + 2)]
    for g in range(G + 1):
        prob = (bounds[g + 1] - bounds[g]) / 2.0 ** 32
        want = q ** G if g == G else p * q ** g
        assert abs(prob - want) <= 4.0 / 2 ** 32 + 1e-12 * max(want, 1e-300) * (g + 1), (g, prob, want)


@pytest.mark.slow
@pytest.mark.parametrize("model,p", [(GAPS_CONST, 0.35), (GAPS_WC, 0.0)])
def test_gap_rr_sets_match_exact_independent_cascade(model, p):
    hg = hypergen.from_lists(6, TINY_EDGES)
    g = oracle.Graph(hg, model, p)
    g.stratify()
    pv = _tiny_thresholds_as_probs(g)
    N = 20000
    for root in (0, 4):
        exact = _enumerate_inclusion_f64(hg, pv, root)
        off, mem, _ = g.generate(3, 1, 0, 0, N, roots=np.full(N, root, np.uint32))
        freq = np.bincount(mem, minlength=6) / N
        for u in range(6):
            qx = float(exact[u])
            if qx < 1e-9 or qx > 1 - 1e-9:
                assert freq[u] == round(qx)
            else:
                z = (freq[u] - qx) / np.sqrt(qx * (1 - qx) / N)
                assert abs(z) < 5, (root, u, freq[u], qx)


def test_star_members_independent_bernoulli():
    m = 40
    hg = hypergen.from_lists(m + 1, [[0, i] for i in range(1, m + 1)])
    p = 0.15
    g = oracle.Graph(hg, GAPS_CONST, p)
    g.stratify()
    pv = float(g.arrays()["thr"][0]) / 2 ** 32
    N = 20000
    off, mem, _ = g.generate(7, 0, 0, 0, N, roots=np.zeros(N, np.uint32))
    counts = np.diff(off) - 1
    pmf = stats.binom.pmf(np.arange(m + 1), m, pv)
    obs = np.bincount(counts, minlength=m + 1)
    keep = pmf * N >= 5
    o = np.append(obs[keep], obs[~keep].sum()).astype(float)
    e = np.append(pmf[keep] * N, pmf[~keep].sum() * N)
    chi = ((o - e) ** 2 / e).sum()
    assert chi < stats.chi2.ppf(1 - 1e-6, len(o) - 1)
    both = sum(1 for s in range(N) if {1, 2} <= set(mem[off[s]:off[s + 1]].tolist()))
    z = (both / N - pv * pv) / math.sqrt(pv * pv * (1 - pv * pv) / N)
    assert abs(z) < 5


def test_p_one_components_and_p_zero_root():
    hg = hypergen.tiny_hypergraph(9, 120, 70, 2, 4)
    g = oracle.Graph(hg, GAPS_CONST, 1.0)
    g.stratify()
    rows, cols = [], []
    for e in range(hg.m):
        mem = hg.he_mem[hg.he_off[e]:hg.he_off[e + 1]]
        for a in mem:
            for b in mem:
                rows.append(a)
                cols.append(b)
    A = csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(hg.n, hg.n))
    _, lab = connected_components(A, directed=False)
    for j in range(60):
        root = g.root(0, 0, 0, j)
        assert np.array_equal(g.rr_set(0, 0, 0, j), np.nonzero(lab == lab[root])[0])
    g0 = oracle.Graph(hg, GAPS_CONST, 0.0)
    g0.stratify()
    for j in range(30):
        assert np.array_equal(g0.rr_set(0, 0, 0, j), [g0.root(0, 0, 0, j)])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gap_draw_bounds_and_special_words(seed):
    """Over random (p, G): the gap lies in [0, G]; the largest word gives the
    longest gap and word 0 the shortest (t = 1 needs q^g >= 1); p = 1 (q = 0)
    makes every position live (gap 0) and p = 0 none (gap G); and the gap
    never decreases as the word grows."""
    rng = np.random.default_rng(100 + seed)
    for _ in range(300):
        p = float(rng.choice([rng.uniform(1e-6, 1e-3), rng.uniform(1e-3, 0.5), rng.uniform(0.5, 1.0)]))
        q = 1.0 - p
        G = int(rng.integers(1, 1 << int(rng.integers(1, 27))))
        xs = np.sort(rng.integers(0, 1 << 32, size=6))
        gs = [oracle.gap_draw(q, int(x), G) for x in xs]
        assert all(0 <= g <= G for g in gs)
        assert all(a <= b for a, b in zip(gs, gs[1:]))
        assert oracle.gap_draw(q, 0, G) == 0
        assert oracle.gap_draw(q, (1 << 32) - 1, G) >= gs[-1]
        assert oracle.gap_draw(0.0, int(xs[0]), G) == 0
        assert oracle.gap_draw(1.0, int(xs[0]), G) == G
