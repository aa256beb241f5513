"""Pins of the oracle's sample-size control (Section 4, Algorithm 4).

* ln C(n,k) against the log-gamma closed form and exact big-integer binomials.
* theta_max / theta_0 / ladder rounds for the three synthetic workloads against
  values computed independently from the OPIM-C formula (the reading of the
  garbled Lemma 6 / Equation (13)).
* Equation (12) as a lower confidence bound and the Lemma 5 / OPIM-C upper
  bound as an upper confidence bound: on Binomial coverages with a known mean
  their failure rates stay below e^-a.
"""
import math

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("n,k", [(1000, 10), (100_000, 50), (1_000_000, 100), (30, 30), (5, 1)])
def test_lnC_matches_closed_forms(n, k):
    s = oracle.schedule(n, k, 0.1, 1.0)
    lg = math.lgamma(n + 1) - math.lgamma(k + 1) - math.lgamma(n - k + 1)
    assert s["lnC"] == pytest.approx(lg, rel=1e-10, abs=1e-9)
    if n <= 100_000:
        assert s["lnC"] == pytest.approx(math.log(math.comb(n, k)), rel=1e-10, abs=1e-9)


def _opimc_theta_max(n, k, eps, ell):
    # written from the OPIM-C statement with exact binomials (independent of the oracle's sum)
    t = 1 - 1 / math.e
    l6 = math.log(6) + ell * math.log(n)
    lnc = math.log(math.comb(n, k))
    return 2 * n * (t * math.sqrt(l6) + math.sqrt(t * (lnc + l6))) ** 2 / (eps ** 2 * k)


@pytest.mark.parametrize("n,k,eps,tmax,t0", [
    (1000, 10, 0.5, 5.322e4, 133.1),          # tiny workload
    (100_000, 50, 0.1, 1.44e8, 721),          # mid workload
    (1_000_000, 100, 0.1, 1.57e9, 1574),      # large workload
])
def test_schedule_values(n, k, eps, tmax, t0):
    s = oracle.schedule(n, k, eps, 1.0)
    assert s["theta_max"] == pytest.approx(_opimc_theta_max(n, k, eps, 1.0), rel=1e-9)
    assert s["theta_max"] == pytest.approx(tmax, rel=3e-3)
    assert s["theta0"] == pytest.approx(t0, rel=3e-3)
    assert s["theta0"] == pytest.approx(s["theta_max"] * eps ** 2 * k / n, rel=1e-12)
    th1 = s["theta1"]
    assert th1 >= max(s["theta0"], 256) and (th1 == 256 or th1 / 2 < s["theta0"])
    assert th1 & (th1 - 1) == 0
    i_max = s["i_max"]
    assert th1 * 2 ** (i_max - 1) >= s["theta_max"] > (th1 * 2 ** (i_max - 2) if i_max > 1 else 0)
    assert s["a"] == pytest.approx(math.log(3 * i_max) + math.log(n), rel=1e-12)
    assert s["delta"] == pytest.approx(1 / n, rel=1e-12)


def test_schedule_rejects_bad_arguments():
    for args in [(10, 0, 0.1, 1), (10, 11, 0.1, 1), (10, 2, 0.0, 1), (10, 2, 1.0, 1), (10, 2, 0.1, 0)]:
        with pytest.raises(ValueError):
            oracle.schedule(*args)


def test_lower_bound_special_values():
    a = 7.3
    assert oracle.sigma_lower(0.0, a, 100, 50) == pytest.approx(0.0, abs=1e-12)   # exactly 0 analytically
    assert oracle.sigma_lower(5 * a / 18, a, 100, 50) == 0.0
    # with a -> 0 the bound tends to the plain estimate n * Lambda / theta
    assert oracle.sigma_lower(40.0, 1e-12, 1000, 200) == pytest.approx(200.0, rel=1e-5)
    assert oracle.sigma_upper(40.0, 1, 1e-12, 1000, 200) == pytest.approx(200.0, rel=1e-5)
    # the greedy factor 1/(1-(1-1/k)^k) with k = 2 is 4/3
    assert oracle.sigma_upper(30.0, 2, 1e-12, 1, 1) == pytest.approx(40.0, rel=1e-5)
    xs = np.linspace(5 * a / 18, 500, 200)
    lows = [oracle.sigma_lower(x, a, 1, 1) for x in xs]
    assert np.all(np.diff(lows) >= 0)


@pytest.mark.parametrize("q,theta", [(0.02, 2000), (0.3, 500), (0.7, 300)])
def test_bounds_are_confidence_bounds(q, theta):
    a = math.log(1 / 0.05)          # nominal failure probability 5%
    rng = np.random.default_rng(int(q * 1000) + theta)
    X = rng.binomial(theta, q, size=20000)
    mean = theta * q
    low = np.array([oracle.sigma_lower(float(x), a, 1.0, 1.0) for x in X])
    up = np.array([oracle.sigma_upper(float(x), 1, a, 1.0, 1.0) for x in X])
    assert np.mean(low > mean) <= 0.05
    assert np.mean(up < mean) <= 0.05
    assert np.mean(low <= mean) > 0.9 and np.mean(up >= mean) > 0.9
