"""Pins of the oracle's random source (Philox4x32-10, SC'11) and coin keying.

The oracle's Philox is checked against two independent open-source
implementations present on this machine (PyTorch's ATen engine and rocRAND's
engine), on random and on extreme (counter, key) records.  The coin keying is
then checked through the RR-set tests, which recompute every coin with the
independent engine."""
import numpy as np
import pytest

import oracle
from conftest import run_philox_filter, independent_coins


def _records(count, seed):
    rng = np.random.default_rng(seed)
    ctr = rng.integers(0, 2 ** 32, size=(count, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, size=(count, 2), dtype=np.uint64).astype(np.uint32)
    # extremes: all zeros, all ones, single bits
    ctr[0] = 0
    key[0] = 0
    ctr[1] = 0xFFFFFFFF
    key[1] = 0xFFFFFFFF
    for b in range(32):
        ctr[2 + b] = [1 << b, 0, 0, 0]
        key[2 + b] = [0, 1 << b]
    return ctr, key


@pytest.mark.parametrize("which", ["torch", "rocrand"])
def test_philox_matches_independent_engines(which, request):
    exe = request.getfixturevalue("torch_philox" if which == "torch" else "rocrand_philox")
    ctr, key = _records(200_000, 7)
    ours = oracle.philox_batch(ctr, key)
    theirs = run_philox_filter(exe, ctr, key)
    assert ours.shape == theirs.shape
    mismatch = np.nonzero(np.any(ours != theirs, axis=1))[0]
    assert mismatch.size == 0, f"first mismatching record {mismatch[:5]}"


def test_single_call_matches_batch():
    ctr, key = _records(64, 3)
    batch = oracle.philox_batch(ctr, key)
    for i in range(64):
        assert np.array_equal(oracle.philox(ctr[i], key[i]), batch[i])


def test_coin_keying_matches_independent_engine(torch_philox):
    rng = np.random.default_rng(11)
    n = 5000
    j = rng.integers(0, 2 ** 39, size=n, dtype=np.uint64)
    he = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64)
    v = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64)
    pos = rng.integers(0, 2 ** 26, size=n, dtype=np.uint64)
    for pool in (0, 1):
        ref = independent_coins(torch_philox, 12345, 77, pool, j, he, v, pos)
        ours = np.array([oracle.coin(12345, 77, pool, int(j[i]), int(he[i]), int(v[i]), int(pos[i]))
                         for i in range(n)], dtype=np.uint32)
        assert np.array_equal(ours, ref)


def test_coins_uniform_and_pool_independent():
    """Coins of the two pools are distinct streams; each is uniform (chi^2)."""
    rng = np.random.default_rng(5)
    n = 40_000
    j = rng.integers(0, 10 ** 6, size=n)
    he = rng.integers(0, 10 ** 6, size=n)
    c0 = np.array([oracle.coin(0, 0, 0, int(j[i]), int(he[i]), 3, 0) for i in range(n)], np.uint64)
    c1 = np.array([oracle.coin(0, 0, 1, int(j[i]), int(he[i]), 3, 0) for i in range(n)], np.uint64)
    assert np.mean(c0 == c1) < 1e-3
    for c in (c0, c1):
        hist = np.bincount((c >> np.uint64(28)).astype(np.int64), minlength=16)
        chi2 = float(((hist - n / 16) ** 2 / (n / 16)).sum())
        assert chi2 < 45.0   # 15 dof, p ~ 1e-4
