"""GPU parity of the KPM density of states (Sec. 4.1 eq. dos_kpm, App. B):
moments with given vectors and with the library's own counter-based draws
against the oracle, and solves whose window and maxdos target come from the
KPM estimate (same target and filter order as the oracle, pairs as dense)."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense, kpm, lanczos, polfed
from oracle import filter as flt
from tests.test_gpu_parity import OPS, ctx, dev, host, make_op, pk, say  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _scale(H):
    lo, hi = lanczos.spectral_extremes(H)
    return flt.rescale(*lanczos.padded_bounds(lo, hi, 1e-3))


@pytest.mark.parametrize("case", [OPS[0], OPS[4], OPS[7], ("qrem", 10)],
                         ids=lambda c: "-".join(map(str, c)))
def test_kpm_moments_given_vectors(pk, ctx, case):
    say(f"kpm moments {case}")
    if case[0] == "qrem":
        from oracle import models
        E = wl.qrem_energies(case[1], 1)
        op, H = pk.Operator.qrem(ctx, case[1], E, 1.0), models.qrem(case[1], E, 1.0)
    else:
        op, H = make_op(pk, ctx, *case)
    E_c, dE = _scale(H)
    R = np.random.default_rng(4).standard_normal((op.D, 3))
    ref = kpm.moments(H, E_c, dE, R, 90)
    got = pk.kpm_moments(op, E_c, dE, 90, 3, dev(R.T))
    assert np.max(np.abs(got - ref)) <= 1e-11 * op.D


def test_kpm_moments_library_draws(pk, ctx):
    """The library's own vectors (r = NULL) are the splitmix64 draws the
    oracle reproduces from the generator's definition."""
    say("kpm moments library draws")
    op, H = make_op(pk, ctx, *OPS[0])
    E_c, dE = _scale(H)
    got = pk.kpm_moments(op, E_c, dE, 50, 4, None, seed=12345)
    ref = kpm.moments(H, E_c, dE, wl.splitmix_vectors(op.D, 4, 12345), 50)
    assert np.max(np.abs(got - ref)) <= 1e-11 * op.D


@pytest.mark.parametrize("case", [("qrem", 12, 30), ("xxz", 12, 20)])
def test_solve_with_kpm_dos_matches_oracle(pk, ctx, case):
    """kpm_moments = 64, kpm_vectors = 20: the library's maxdos target and
    filter order equal the oracle's with the same draws, and the pairs are
    the dense ones."""
    say(f"solve with kpm dos {case}")
    kind, L, n_ev = case
    if kind == "qrem":
        from oracle import models
        E = wl.qrem_energies(L, 5)
        op, H = pk.Operator.qrem(ctx, L, E, 1.0), models.qrem(L, E, 1.0)
    else:
        op, H = make_op(pk, ctx, "xxz", L, L // 2, 1.0, 0, True)
    lo, hi = lanczos.spectral_extremes(H)
    x0 = wl.start_vector(op.D, 0)
    ref = polfed.polfed(H, x0, n_ev, 0.0, "maxdos", bounds=(lo, hi),
                        kpm_vectors=wl.splitmix_vectors(op.D, 20, 0x4B504D), kpm_moments=64)
    evals, evecs, res, rep, status = pk.solve(op, dev(x0), n_ev, 0.0, "maxdos",
                                              kpm_moments=64, kpm_vectors=20,
                                              E_min=lo, E_max=hi)
    assert status == "OK"
    say(f"   lambda={rep['lambda']:.6f} (oracle {ref['lam']:.6f}) K={rep['K']} "
        f"(oracle {ref['plan']['K']})")
    assert abs(rep["lambda"] - ref["lam"]) <= 1e-9 * max(1.0, abs(ref["lam"]))
    assert rep["K"] == ref["plan"]["K"]
    Er, _ = dense.nearest_eigenpairs(H, rep["lambda"], n_ev)
    Ev = host(evals)
    assert np.max(np.abs(Ev - Er) / np.maximum(np.abs(Er), 1.0)) <= 1e-10
    assert host(res).max() <= 1e-8
