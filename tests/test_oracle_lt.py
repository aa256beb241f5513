"""Pins of the oracle's linear-threshold (LT) RR sets (Section 2.1, LT
bullet), independent of the oracle's own code.

The oracle takes LT in its live-edge form: every vertex v keeps at most one
of its c(v) channels (hyperedge, member), each with weight W_v / 2^32,
W_v = min(thr[v], floor(2^32 / c(v))) (thr = ALWAYS counting as 2^32), and an
RR set is the reverse walk along kept channels.  Checked here:

* every RR set equals the walk rebuilt with an independent Philox engine
  (PyTorch's) and an independent channel numbering;
* exact enumeration of every pick combination on tiny hypergraphs gives
  Pr[u in RR(r)], which the oracle's frequencies match (z-tests);
* the threshold process of the LT bullet itself -- thresholds lambda(v)
  uniform in [0, 1), v active once the weights of its active in-channels
  reach lambda(v) -- simulated forward with numpy gives Pr[r active | seed u]
  equal to the enumerated Pr[u in RR(r)], the reading that makes the walk a
  faithful RR set for the paper's LT model;
* special cases: on a path every RR set is an interval containing its root;
  a vertex with a single channel of weight 1 always keeps it; p = 0 and
  isolated vertices give {root}; weights above 1/c(v) are capped.
"""
import itertools

import numpy as np
import pytest

import hypergen
import oracle
from conftest import independent_coins

ALWAYS = 0xFFFFFFFF
LT_CONST, LT_WC = 2, 3
LT_SLOT = 0xFFFFFFFE   # hyperedge slot of the pick's counter
TINY_EDGES = [[0, 1, 2], [2, 3], [3, 4], [1, 4], [4, 5, 1]]


def _channels_into(hg, v):
    """Members of v's channels: hyperedges of v ascending, members in stored
    order, v itself skipped."""
    out = []
    for e in range(hg.m):
        mem = [int(x) for x in hg.he_mem[hg.he_off[e]:hg.he_off[e + 1]]]
        if v in mem:
            out.extend(u for u in mem if u != v)
    return out


def _weight(thr, c):
    w = (1 << 32) if int(thr) == ALWAYS else int(thr)
    return min(w, (1 << 32) // c) if c else 0


def _pick_table(hg, thr):
    """Per vertex: [(member, probability)] for each channel, plus the
    probability of keeping none."""
    tab = []
    for v in range(hg.n):
        ch = _channels_into(hg, v)
        W = _weight(thr[v], len(ch))
        tab.append(([(u, W / 2 ** 32) for u in ch], 1.0 - len(ch) * W / 2 ** 32))
    return tab


def _walk(root, pick):
    r, cur = {root}, root
    while pick[cur] is not None and pick[cur] not in r:
        cur = pick[cur]
        r.add(cur)
    return r


def _exact_inclusion(hg, thr):
    """Pr[u in RR(r)] for all (r, u) over every pick combination."""
    tab = _pick_table(hg, thr)
    choices = [[(u, p) for u, p in ch] + [(None, none)] for ch, none in tab]
    incl = np.zeros((hg.n, hg.n))
    for combo in itertools.product(*choices):
        pr = float(np.prod([p for _, p in combo]))
        if pr == 0.0:
            continue
        pick = [u for u, _ in combo]
        for r in range(hg.n):
            for u in _walk(r, pick):
                incl[r, u] += pr
    return incl


@pytest.mark.parametrize("model,p", [(LT_WC, 0.0), (LT_CONST, 0.15), (LT_CONST, 0.3)])
def test_lt_walks_equal_independent_reconstruction(model, p, torch_philox):
    hg = hypergen.tiny_hypergraph(31, 40, 50, 2, 6)
    g = oracle.Graph(hg, model, p)
    g.stratify()
    thr = g.arrays()["thr"]
    chans = [_channels_into(hg, v) for v in range(hg.n)]
    seed, inst, pool = 9, 4, 1
    ids = list(range(300)) + [1 << 33, (1 << 33) + 7]
    for j in ids:
        root = g.root(seed, inst, pool, j)
        x = independent_coins(torch_philox, seed, inst, pool, np.full(hg.n, j, np.uint64), LT_SLOT,
                              np.arange(hg.n), 0)
        pick = []
        for v in range(hg.n):
            C = len(chans[v])
            W = _weight(thr[v], C)
            pick.append(chans[v][int(x[v]) // W] if C and int(x[v]) < W * C else None)
        want = np.array(sorted(_walk(root, pick)), np.uint32)
        assert np.array_equal(g.rr_set(seed, inst, pool, j), want), j


@pytest.mark.slow
@pytest.mark.parametrize("model,p", [(LT_WC, 0.0), (LT_CONST, 0.15)])
def test_lt_inclusion_frequencies_match_exact_enumeration(model, p):
    hg = hypergen.from_lists(6, TINY_EDGES)
    g = oracle.Graph(hg, model, p)
    g.stratify()
    exact = _exact_inclusion(hg, g.arrays()["thr"])
    assert np.allclose(np.diag(exact), 1.0)
    N = 20000
    for root in (0, 4):
        off, mem, _ = g.generate(3, 1, 0, 0, N, roots=np.full(N, root, np.uint32))
        freq = np.bincount(mem, minlength=6) / N
        for u in range(6):
            q = float(exact[root, u])
            if q < 1e-9 or q > 1 - 1e-9:
                assert freq[u] == round(q)
            else:
                z = (freq[u] - q) / np.sqrt(q * (1 - q) / N)
                assert abs(z) < 5, (root, u, freq[u], q)


@pytest.mark.slow
def test_lt_threshold_process_matches_live_edge_walks():
    """The LT bullet's threshold process, run forward from seed {s}, activates
    r with the probability that s lies in RR(r)."""
    hg = hypergen.from_lists(6, TINY_EDGES)
    g = oracle.Graph(hg, LT_WC, 0.0)
    thr = g.arrays()["thr"]
    exact = _exact_inclusion(hg, thr)
    # in-weights p(u -> v) = (channels u -> v) * W_v / 2^32
    P = np.zeros((6, 6))
    for v in range(6):
        ch = _channels_into(hg, v)
        W = _weight(thr[v], len(ch)) / 2 ** 32
        for u in ch:
            P[u, v] += W
    rng = np.random.default_rng(5)
    N = 40000
    for s in (1, 3):
        lam = rng.random((N, 6))
        active = np.zeros((N, 6), bool)
        active[:, s] = True
        for _ in range(6):
            active |= (active.astype(float) @ P) >= lam
        freq = active.mean(axis=0)
        for r in range(6):
            q = float(exact[r, s])
            if q < 1e-9 or q > 1 - 1e-9:
                assert freq[r] == round(q)
            else:
                z = (freq[r] - q) / np.sqrt(q * (1 - q) / N)
                assert abs(z) < 5, (s, r, freq[r], q)


def test_lt_special_cases():
    # a path 0 - 1 - ... - 29: every RR set is an interval containing its root
    n = 30
    hg = hypergen.from_lists(n, [[i, i + 1] for i in range(n - 1)])
    g = oracle.Graph(hg, LT_WC, 0.0)
    g.stratify()
    lens = []
    for j in range(400):
        r = g.rr_set(2, 0, 0, j)
        root = g.root(2, 0, 0, j)
        assert root in r and np.array_equal(r, np.arange(r[0], r[-1] + 1))
        lens.append(r.size)
    assert max(lens) > 2   # walks do continue past the first step
    # a single channel of weight 1 is always kept: star 0 - {1..5} with p = 1
    hg = hypergen.from_lists(6, [[0, i] for i in range(1, 6)])
    g = oracle.Graph(hg, LT_CONST, 1.0)
    g.stratify()
    for j in range(200):
        r = g.rr_set(0, 0, 0, j)
        root = g.root(0, 0, 0, j)
        if root != 0:
            assert 0 in r and r.size >= 2   # a leaf always keeps its channel from the hub
    # weights are capped at 1/c(v): with p = 1 the hub (c = 5) keeps a channel
    # every time (5 channels of weight 1/5 each, up to rounding)
    hub = [g.rr_set(0, 0, 0, j, root=0) for j in range(200)]
    assert sum(r.size >= 2 for r in hub) == 200
    # p = 0 and isolated vertices give {root}
    hg = hypergen.from_lists(5, [[0, 1, 2]])
    for model, p in ((LT_CONST, 0.0), (LT_WC, 0.0)):
        g = oracle.Graph(hg, model, p)
        g.stratify()
        for j in range(50):
            root = g.root(0, 0, 0, j)
            r = g.rr_set(0, 0, 0, j)
            if model == LT_CONST or root >= 3:
                assert np.array_equal(r, [root])


def test_lt_estimator_unbiased_on_tiny_graph():
    """n * Lambda(S) / theta over LT RR sets estimates the LT spread of S,
    computed exactly by enumeration (Equation (1) under the LT model)."""
    hg = hypergen.from_lists(6, TINY_EDGES)
    g = oracle.Graph(hg, LT_WC, 0.0)
    g.stratify()
    exact = _exact_inclusion(hg, g.arrays()["thr"])
    theta = 32768   # whole ladder blocks: every vertex is a root theta / n times up to one per block
    off, mem, _ = g.generate(1, 0, 0, 0, theta)
    for S in ([1], [4, 0], [2, 5]):
        # exact spread: sum over roots of Pr[S meets RR(r)] -- for LT walks a
        # union bound is not exact, so enumerate again for the set
        tab = _pick_table(hg, g.arrays()["thr"])
        choices = [[(u, p) for u, p in ch] + [(None, none)] for ch, none in tab]
        spread = 0.0
        for combo in itertools.product(*choices):
            pr = float(np.prod([p for _, p in combo]))
            if pr == 0.0:
                continue
            pick = [u for u, _ in combo]
            spread += pr * sum(bool(_walk(r, pick) & set(S)) for r in range(6))
        cov = oracle.coverage(6, off, mem, np.array(S, np.uint32), theta)
        est = 6 * cov / theta
        # each RR set contributes a {0, 1} indicator times n: variance <= n^2 / 4 / theta
        assert abs(est - spread) < 5 * 6 * 0.5 / np.sqrt(theta), (S, est, spread)
        assert exact.shape == (6, 6)
