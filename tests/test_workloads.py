"""CPU checks of the seeded input generators shared by the oracle, the GPU
tests and the benchmark: each is reproducible from its seed and draws the
distribution it states (the models of the paper's Appendix A, the start
vector of its usage example, and the serving stream's Poisson arrivals)."""
import numpy as np
import pytest
from scipy import stats

import workloads as wl


def test_every_generator_is_reproducible_and_seed_dependent():
    draws = [lambda s: wl.xxz_fields(16, 3.0, s), lambda s: wl.tv_onsite(16, s),
             lambda s: wl.qrem_energies(10, s), lambda s: wl.start_vector(100, s),
             lambda s: wl.qsun_draws(3, 13, s)["A"]]
    for f in draws:
        assert np.array_equal(f(4), f(4))
        assert not np.array_equal(f(4), f(5))
    a, b = wl.serving_stream(30, 2, 1.0), wl.serving_stream(30, 2, 1.0)
    assert a == b and a != wl.serving_stream(30, 3, 1.0)


def test_uniform_fields_and_onsite_energies():
    for W in (1.0, 3.0, 5.0):
        h = np.concatenate([wl.xxz_fields(24, W, s) for s in range(400)])
        assert h.min() >= -W and h.max() <= W
        assert stats.kstest(h, stats.uniform(-W, 2 * W).cdf).pvalue > 1e-3
    e = np.concatenate([wl.tv_onsite(26, s) for s in range(400)])
    assert stats.kstest(e, stats.uniform(-2.0, 4.0).cdf).pvalue > 1e-3


def test_qrem_energies_are_gaussian_with_variance_L_over_2():
    for L in (10, 14):
        E = wl.qrem_energies(L, 7)
        n, var = E.size, L / 2.0
        assert n == 1 << L
        # mean 0 and variance L/2 within five standard errors; normal shape
        assert abs(E.mean()) < 5 * np.sqrt(var / n)
        assert abs(E.var() / var - 1) < 5 * np.sqrt(2.0 / n)
        assert stats.kstest(E, stats.norm(0.0, np.sqrt(var)).cdf).pvalue > 1e-6


def test_quantum_sun_draws():
    N, L = 3, 13
    d = wl.qsun_draws(N, L, 11, zeta=0.2, h=1.0, w=0.5)
    assert d["A"].shape == (1 << N, 1 << N)
    assert np.all(np.abs(d["u"] - np.arange(L)) <= 0.2)
    assert d["n_of_j"].dtype == np.int32
    assert d["n_of_j"].min() >= 0 and d["n_of_j"].max() < N
    assert np.all((d["h"] >= 0.5) & (d["h"] <= 1.5))
    A = np.concatenate([wl.qsun_draws(N, L, s)["A"].ravel() for s in range(200)])
    assert stats.kstest(A, stats.norm().cdf).pvalue > 1e-3


def test_start_vector_is_uniform_and_independent_of_the_model_draws():
    x = wl.start_vector(20000, 0)
    assert x.min() >= 0.0 and x.max() < 1.0
    assert stats.kstest(x, stats.uniform().cdf).pvalue > 1e-3
    # a start vector and fields drawn with the same seed come from separate streams
    h = wl.xxz_fields(64, 1.0, 0)
    assert not np.allclose(wl.start_vector(64, 0), (h + 1.0) / 2.0)


@pytest.mark.parametrize("mean_gap", [0.5, 2.0])
def test_serving_stream_has_poisson_arrivals_and_uniform_mix(mean_gap):
    n = 20000
    st = wl.serving_stream(n, 9, mean_gap)
    t = np.array([r["t_arrive"] for r in st])
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    gaps = np.diff(t)
    # exponential gaps: mean as asked, coefficient of variation 1
    assert abs(gaps.mean() / mean_gap - 1) < 0.03
    assert abs(gaps.std() / gaps.mean() - 1) < 0.03
    assert stats.kstest(gaps / mean_gap, stats.expon().cdf).pvalue > 1e-3
    for key, values in (("L", (14, 16, 18)), ("W", (1.0, 3.0, 5.0))):
        col = np.array([r[key] for r in st])
        assert set(col.tolist()) == set(values)
        for v in values:
            assert abs(np.mean(col == v) - 1 / 3) < 0.02
    assert len({r["seed"] for r in st}) == n
