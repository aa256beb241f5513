"""Host logic of the serving loop (no GPU): arrival process, query draws,
latency percentiles."""
import numpy as np

from paper_2406_01911_amd import serving


def test_poisson_arrivals():
    a = serving.poisson_arrivals(20000, 50.0, seed=3)
    assert np.all(np.diff(a) > 0) and a[0] > 0
    gaps = np.diff(np.concatenate([[0.0], a]))
    # exponential gaps of mean 1/qps: mean within 3 standard errors
    assert abs(gaps.mean() - 0.02) < 3 * 0.02 / np.sqrt(gaps.size)
    # coefficient of variation of an exponential is 1
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05
    assert np.array_equal(a, serving.poisson_arrivals(20000, 50.0, seed=3))


def test_draw_queries():
    q = serving.draw_queries(500, 16, seed=1)
    assert q == serving.draw_queries(500, 16, seed=1)
    assert {x["k"] for x in q} == {10, 50, 200}
    assert all(0 <= x["graph"] < 16 and x["instance"] == x["graph"] and x["eps"] == 0.1 for x in q)


def test_latency_summary_nearest_rank():
    lat = np.arange(1, 101) / 1000.0          # 1..100 ms
    s = serving.latency_summary(lat)
    assert s["p50_ms"] == 50.0 and s["p99_ms"] == 99.0 and s["max_ms"] == 100.0
    assert abs(s["mean_ms"] - 50.5) < 1e-9
    s1 = serving.latency_summary([0.007])
    assert s1["p50_ms"] == s1["p99_ms"] == 7.0
    assert serving.latency_summary([])["p50_ms"] is None
