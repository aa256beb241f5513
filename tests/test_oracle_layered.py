"""Pins of the oracle's stratified-setting RR sets (Section 3.1.1,
"Activation probability", "Sampling strategy"; Algorithm 3's per-layer
draws), independent of the oracle's own code.

* Layer tables: A(v) split by w(v,u) (layer 1 the largest), ascending ids in
  a layer, rebuilt with Python sets and sorting.
* Counts and selection on a star whose centre's layers are reached only
  through the centre: per layer the number of members in RR(centre) follows
  Binomial(n, p) for n <= 20 and the truncated Poisson(P) above, each member
  is equally likely, and two members of a Binomial layer appear together with
  probability p^2 (chi-square / z-tests), with P(L_i) = 1 / (i ln(l + 1)) and
  p = min(1, P / n).
* Exact enumeration: with every layer at most 20 members the Binomial count
  plus uniform selection is the same distribution as an independent coin per
  member (Lemma 3), so all 2^C pair worlds of a tiny hypergraph give exact
  inclusion probabilities Pr[u in RR(r)], which the oracle's frequencies
  match.
* Special cases: a single-member top layer has P = 1 / ln 2 > 1 (the paper's
  Lemma 1 claims the layer probabilities sum to at most 1, but
  H_l >= ln(l + 1)), so its member is always selected.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

import hypergen
import oracle

LAYERED = 4


def _layers_python(hg):
    """Per vertex: [[layer 1 members ascending], [layer 2 ...], ...]."""
    w = [dict() for _ in range(hg.n)]
    for e in range(hg.m):
        mem = [int(x) for x in hg.he_mem[hg.he_off[e]:hg.he_off[e + 1]]]
        for v in mem:
            for u in mem:
                if u != v:
                    w[v][u] = w[v].get(u, 0) + 1
    out = []
    for v in range(hg.n):
        by = {}
        for u, c in w[v].items():
            by.setdefault(c, []).append(u)
        out.append([sorted(by[c]) for c in sorted(by, reverse=True)])
    return out


def _unpack(layers):
    nb_off, nb, ly_off, ly_end = layers
    out = []
    for v in range(len(nb_off) - 1):
        base, ls = int(nb_off[v]), []
        lo = 0
        for i in range(int(ly_off[v]), int(ly_off[v + 1])):
            hi = int(ly_end[i])
            ls.append([int(x) for x in nb[base + lo:base + hi]])
            lo = hi
        out.append(ls)
    return out


def _p_member(i, l, n):
    return min(1.0, 1.0 / (i * math.log(l + 1.0)) / n)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_layer_tables_match_python(seed):
    hg = hypergen.tiny_hypergraph(seed, 80, 120, 2, 7)
    g = oracle.Graph(hg, LAYERED, 0.0)
    st = g.stratify()
    got = _unpack(g.layers())
    want = _layers_python(hg)
    assert got == want
    assert [len(x) for x in want] == list(st["l"])


def _star(layer_sizes):
    """Centre 0; layer t (t = 0, 1, ...) has layer_sizes[t] members, each in
    (len(layer_sizes) - t) copies of the hyperedge {0, member}; members share
    no other hyperedge, so RR(0) minus the centre is exactly the centre's
    selections."""
    edges, members, nxt = [], [], 1
    L = len(layer_sizes)
    for t, size in enumerate(layer_sizes):
        ms = list(range(nxt, nxt + size))
        nxt += size
        members.append(ms)
        for u in ms:
            edges.extend([[0, u]] * (L - t))
    return hypergen.from_lists(nxt, edges), members


def test_layer_counts_selection_and_independence():
    sizes = [3, 8, 20, 25]            # three Binomial layers, one Poisson layer
    hg, members = _star(sizes)
    g = oracle.Graph(hg, LAYERED, 0.0)
    g.stratify()
    l = len(sizes)
    N = 40000
    off, mem, _ = g.generate(11, 2, 0, 0, N, roots=np.zeros(N, np.uint32))
    counts = np.zeros((N, l), np.int64)
    hits = np.zeros(hg.n, np.int64)
    pair = 0
    lay_of = np.full(hg.n, -1)
    for t, ms in enumerate(members):
        lay_of[ms] = t
    for s in range(N):
        r = mem[off[s]:off[s + 1]]
        r = r[r != 0]
        np.add.at(counts[s], lay_of[r], 1)
        hits[r] += 1
        pair += int(members[1][0] in r and members[1][1] in r)
    for t, n in enumerate(sizes):
        i = t + 1
        p = _p_member(i, l, n)
        if n <= 20:
            pmf = stats.binom.pmf(np.arange(n + 1), n, p)
        else:
            lam = 1.0 / (i * math.log(l + 1.0))
            pmf = stats.poisson.pmf(np.arange(n + 1), lam)
            pmf[-1] += 1.0 - pmf.sum()
        obs = np.bincount(counts[:, t], minlength=n + 1)
        keep = pmf * N >= 5
        exp = pmf[keep] * N
        o = obs[keep].astype(float)
        rest_o, rest_e = obs[~keep].sum(), pmf[~keep].sum() * N
        if rest_e > 0:
            o, exp = np.append(o, rest_o), np.append(exp, rest_e)
        chi = ((o - exp) ** 2 / exp).sum()
        assert chi < stats.chi2.ppf(1 - 1e-6, len(o) - 1), (t, obs, pmf * N)
        # every member of the layer equally likely
        h = hits[members[t]]
        if h.sum() > 0 and n > 1:
            e = h.sum() / n
            assert (((h - e) ** 2) / e).sum() < stats.chi2.ppf(1 - 1e-6, n - 1), (t, h)
    # two members of a Binomial layer together: p^2 (independent coins, Lemma 3)
    p1 = _p_member(2, l, sizes[1])
    q = p1 * p1
    z = (pair / N - q) / math.sqrt(q * (1 - q) / N)
    assert abs(z) < 5, (pair / N, q)


def test_single_member_top_layer_always_selected():
    # l = 1 and n(L_1) = 1: P(L_1) = 1 / ln 2 > 1, clamped to 1
    hg = hypergen.from_lists(2, [[0, 1]])
    g = oracle.Graph(hg, LAYERED, 0.0)
    g.stratify()
    for j in range(100):
        assert np.array_equal(g.rr_set(0, 0, 0, j, root=0), [0, 1])
    # the paper's Lemma 1 bound does not hold: sum_i P(L_i) = H_l / ln(l + 1) >= 1
    for l in range(1, 50):
        assert sum(1.0 / (i * math.log(l + 1.0)) for i in range(1, l + 1)) >= 1.0


def _exact_layered_inclusion(hg, root):
    """Pr[u in RR(root)] over every world of independent pair coins (u -> v
    live with p of u's layer in A(v)); valid when every layer has at most 20
    members (Binomial count + uniform selection = independent coins)."""
    lay = _layers_python(hg)
    pairs, probs = [], []
    for v in range(hg.n):
        l = len(lay[v])
        for t, ms in enumerate(lay[v]):
            p = _p_member(t + 1, l, len(ms))
            for u in ms:
                pairs.append((u, v))
                probs.append(p)
    C = len(pairs)
    incl = np.zeros(hg.n)
    for bits in range(1 << C):
        pr = 1.0
        for c in range(C):
            pr *= probs[c] if (bits >> c) & 1 else 1.0 - probs[c]
        if pr == 0.0:
            continue
        reach, grow = {root}, True
        while grow:
            grow = False
            for c in range(C):
                if (bits >> c) & 1:
                    u, v = pairs[c]
                    if v in reach and u not in reach:
                        reach.add(u)
                        grow = True
        for u in reach:
            incl[u] += pr
    return incl


@pytest.mark.slow
def test_inclusion_frequencies_match_exact_enumeration():
    hg = hypergen.from_lists(5, [[0, 1, 2], [1, 2], [2, 3], [3, 4], [0, 1]])   # 14 ordered pairs
    g = oracle.Graph(hg, LAYERED, 0.0)
    g.stratify()
    N = 30000
    for root in (0, 3):
        exact = _exact_layered_inclusion(hg, root)
        off, mem, _ = g.generate(5, 0, 1, 0, N, roots=np.full(N, root, np.uint32))
        freq = np.bincount(mem, minlength=hg.n) / N
        for u in range(hg.n):
            q = float(exact[u])
            if q < 1e-9 or q > 1 - 1e-9:
                assert freq[u] == round(q)
            else:
                z = (freq[u] - q) / np.sqrt(q * (1 - q) / N)
                assert abs(z) < 5, (root, u, freq[u], q)
