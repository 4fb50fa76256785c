"""GPU parity of the quantum random energy model (eq. qrem of App. A) and
the maxdos target (Sec. 5.4): operator application, the fused Clenshaw step
(whole vectors at small L, sampled rows at full size with every tile shape),
moments, the filter, bounds and full solves against dense diagonalization."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense, lanczos, models, polfed
from oracle import filter as flt
from tests.test_gpu_parity import ctx, dev, host, pk, say  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def qrem_case(pk, ctx, L, seed, G=1.0):
    E = wl.qrem_energies(L, seed)
    return pk.Operator.qrem(ctx, L, E, G), E


@pytest.mark.parametrize("L", [2, 3, 6, 7, 10, 13, 16])
def test_qrem_apply_matches_oracle(pk, ctx, L):
    say(f"qrem apply L={L}")
    op, E = qrem_case(pk, ctx, L, L)
    H = models.qrem(L, E, 1.0)
    x = np.random.default_rng(1).standard_normal(op.D)
    y = host(op.apply(dev(x)))
    ref = H @ x
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("L", [4, 11, 15])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("final", [False, True])
def test_qrem_clenshaw_step_matches_oracle(pk, ctx, L, prec, final):
    say(f"qrem step L={L} {prec} final={final}")
    op, E = qrem_case(pk, ctx, L, 7)
    H = models.qrem(L, E, 1.0)
    rng = np.random.default_rng(9)
    v, b1, b2 = (rng.standard_normal(op.D) for _ in range(3))
    dt = torch.float64 if prec == "fp64" else torch.float32
    if prec == "fp32":
        v, b1, b2 = (x.astype(np.float32).astype(np.float64) for x in (v, b1, b2))
    E_c, dE, a_i = 0.3, 9.5, 0.0123
    f = 0.5 if final else 1.0
    ref = a_i * v + f * 2.0 * (H @ b1 - E_c * b1) / dE - b2
    tb2 = dev(b2, dt)
    pk.clenshaw_step(op, E_c, dE, a_i, dev(v, dt), dev(b1, dt), tb2,
                     pk.FP64 if prec == "fp64" else pk.FP32, final)
    got = host(tb2).astype(np.float64)
    tol = 1e-14 if prec == "fp64" else 2e-6
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))


@pytest.mark.parametrize("L,tb", [(20, 10), (20, 11), (20, 12), (21, 12), (24, 11), (24, 12)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_qrem_full_size_step_sampled_rows(pk, ctx, L, tb, prec):
    """Full-size steps with tiles of 2^10 to 2^12 rows: sampled rows of
    a v + 2 H~ b1 - b2 against the oracle's row-by-row eq. (qrem)."""
    say(f"qrem sampled step L={L} tile bits {tb} {prec}")
    op, E = qrem_case(pk, ctx, L, 3)
    assert op.set_kernel(pk.FP64 if prec == "fp64" else pk.FP32, tb) == tb
    rng = np.random.default_rng(5)
    v, b1, b2 = (rng.standard_normal(op.D) for _ in range(3))
    dt = torch.float64 if prec == "fp64" else torch.float32
    Eh = E
    if prec == "fp32":
        v, b1, b2 = (x.astype(np.float32).astype(np.float64) for x in (v, b1, b2))
        Eh = E.astype(np.float32).astype(np.float64)
    E_c, dE, a_i = -0.2, 31.0, 0.0173
    tb2 = dev(b2, dt)
    pk.clenshaw_step(op, E_c, dE, a_i, dev(v, dt), dev(b1, dt), tb2,
                     pk.FP64 if prec == "fp64" else pk.FP32)
    got = host(tb2).astype(np.float64)
    rows = np.unique(np.concatenate([rng.integers(0, op.D, 6000), np.arange(300),
                                     np.arange(op.D - 300, op.D)]))
    Hb = models.qrem_rows_apply(L, Eh, 1.0, rows, b1)
    ref = a_i * v[rows] + 2.0 * (Hb - E_c * b1[rows]) / dE - b2[rows]
    tol = 1e-13 if prec == "fp64" else 3e-6
    assert np.max(np.abs(got[rows] - ref)) <= tol * np.max(np.abs(ref))


def test_qrem_moments_and_bounds(pk, ctx):
    say("qrem moments and bounds")
    op, E = qrem_case(pk, ctx, 12, 4)
    H = models.qrem(12, E, 1.0)
    t1, t2 = op.moments()
    r1, r2 = flt.trace_moments(H)
    assert abs(t1 - r1) <= 1e-12 * max(1, abs(r1)) and abs(t2 - r2) <= 1e-12 * abs(r2)
    lo, hi = pk.bounds(op, dev(wl.start_vector(op.D, 0)))
    rlo, rhi = lanczos.spectral_extremes(H)
    assert abs(lo - rlo) <= 1e-8 * (rhi - rlo) and abs(hi - rhi) <= 1e-8 * (rhi - rlo)


def test_qrem_filter_matches_oracle(pk, ctx):
    say("qrem filter")
    op, E = qrem_case(pk, ctx, 12, 6)
    H = models.qrem(12, E, 1.0)
    lo, hi = lanczos.spectral_extremes(H)
    E_c, dE = flt.rescale(*lanczos.padded_bounds(lo, hi, 1e-3))
    a = flt.coefficients(0.05, 400)
    x = wl.start_vector(op.D, 3)
    ref = flt.apply_filter(H, E_c, dE, a, x)
    w = host(pk.filter_apply(op, E_c, dE, a, dev(x)))
    assert np.linalg.norm(w - ref) / np.linalg.norm(ref) <= 8 * 401 * 2.2e-16


@pytest.mark.parametrize("L,n_ev,s", [(10, 20, 1), (12, 30, 1), (12, 30, 4), (14, 40, 1)])
def test_qrem_solve_at_maxdos_matches_dense(pk, ctx, L, n_ev, s):
    say(f"qrem solve L={L} n_ev={n_ev} s={s} at maxdos")
    op, E = qrem_case(pk, ctx, L, 2)
    H = models.qrem(L, E, 1.0)
    X0 = np.stack([wl.start_vector(op.D, c) for c in range(s)])
    x0 = dev(X0[0]) if s == 1 else dev(X0)
    evals, evecs, res, rep, status = pk.solve(op, x0, n_ev, 0.0, "maxdos")
    assert status == "OK"
    tr1, _ = flt.trace_moments(H)
    assert abs(rep["lambda"] - tr1) <= 1e-12 * max(1.0, abs(tr1))
    Ev, U, R = host(evals), host(evecs), host(res)
    Er, Ur = dense.nearest_eigenpairs(H, rep["lambda"], n_ev)
    rel = np.abs(Ev - Er) / np.maximum(np.abs(Er), 1.0)
    say(f"   K={rep['K']} iters={rep['iters']} rel={rel.max():.1e} res={R.max():.1e}")
    assert rel.max() <= 1e-10 and R.max() <= 1e-8
    assert np.linalg.norm(H @ U - U * Ev, axis=0).max() <= 1e-8
    assert np.min(np.abs(np.sum(U * Ur, axis=0))) >= 1 - 1e-8


def test_offset_target_matches_oracle(pk, ctx):
    say("qrem offset target")
    op, E = qrem_case(pk, ctx, 10, 8)
    H = models.qrem(10, E, 1.0)
    evals, evecs, res, rep, status = pk.solve(op, dev(wl.start_vector(op.D, 1)), 10, 0.4,
                                              "offset")
    assert status == "OK"
    tr1, _ = flt.trace_moments(H)
    lam = polfed.target_energy("offset", 0.4, rep["E_min"], rep["E_max"], tr1)
    assert abs(rep["lambda"] - lam) <= 1e-12 * max(1.0, abs(lam))
    Er, _ = dense.nearest_eigenpairs(H, rep["lambda"], 10)
    assert np.max(np.abs(host(evals) - Er) / np.maximum(np.abs(Er), 1.0)) <= 1e-10


def test_qrem_invalid(pk, ctx):
    say("qrem invalid")
    with pytest.raises(pk.PolfedError):
        pk.Operator.qrem(ctx, 1, np.zeros(2), 1.0)
    with pytest.raises(pk.PolfedError):
        pk.Operator.qrem(ctx, 4, np.full(16, np.nan), 1.0)
    op, _ = qrem_case(pk, ctx, 6, 0)
    with pytest.raises(pk.PolfedError):
        op.materialize_csr()


@pytest.mark.parametrize("s", [1, 4])
def test_qrem_many_pairs_device_eigensolvers(pk, ctx, s):
    """300 pairs of QREM L=11: the Rayleigh-Ritz matrix (n = 360) and the
    Lanczos matrix (M > 256) go through the device eigensolvers."""
    say(f"qrem L=11 300 pairs s={s}")
    op, E = qrem_case(pk, ctx, 11, 9)
    H = models.qrem(11, E, 1.0)
    X0 = np.stack([wl.start_vector(op.D, c) for c in range(s)])
    x0 = dev(X0[0]) if s == 1 else dev(X0)
    evals, evecs, res, rep, status = pk.solve(op, x0, 300, 0.0, "maxdos")
    assert status == "OK"
    assert rep["iters"] >= 256 and rep["n_want"] >= 256
    Ev, U, R = host(evals), host(evecs), host(res)
    Er, Ur = dense.nearest_eigenpairs(H, rep["lambda"], 300)
    rel = np.abs(Ev - Er) / np.maximum(np.abs(Er), 1.0)
    say(f"   K={rep['K']} iters={rep['iters']} rel={rel.max():.1e} res={R.max():.1e}")
    assert rel.max() <= 1e-10 and R.max() <= 1e-8
    assert np.linalg.norm(H @ U - U * Ev, axis=0).max() <= 1e-8
    assert np.min(np.abs(np.sum(U * Ur, axis=0))) >= 1 - 1e-8


@pytest.mark.parametrize("L,s,k,prec", [(12, 4, 0, "fp64"), (13, 3, 6, "fp64"), (14, 2, 4, "fp32"),
                                        (11, 5, 5, "fp64")])
def test_qrem_block_step_matches_oracle(pk, ctx, L, s, k, prec):
    """Block Lanczos step on QREM: the filter of the whole block runs on the
    multi-column hypercube step (chunks of 4, 2, 1 columns)."""
    say(f"qrem block step L={L} s={s} k={k} {prec}")
    op, E = qrem_case(pk, ctx, L, 11)
    H = models.qrem(L, E, 1.0)
    D = op.D
    lo, hi = lanczos.spectral_extremes(H)
    E_c, dE = flt.rescale(*lanczos.padded_bounds(lo, hi, 1e-3))
    K = 120 if prec == "fp64" else 60
    a = flt.coefficients(0.03, K)

    def P(X):
        return flt.apply_filter(H, E_c, dE, a, X)
    X0 = np.stack([wl.start_vector(D, 70 + c) for c in range(s)], 1)
    V = np.zeros((D, k + 2 * s))
    V[:, :s] = lanczos.orthonormal_start_block(X0)
    for j in range(k // s):
        _, _, Vn = lanczos.block_lanczos_step(P, V, j * s, s)
        V[:, (j + 1) * s:(j + 2) * s] = Vn
    A_ref, B_ref, Vn_ref = lanczos.block_lanczos_step(P, V, k, s)
    tV = dev(V.T)
    tA = torch.zeros((s, s), dtype=torch.float64, device="cuda:0")
    tB = torch.zeros((s, s), dtype=torch.float64, device="cuda:0")
    pk.block_lanczos_step(op, E_c, dE, a, tV, k, s, tA, tB, pk.FP64 if prec == "fp64" else pk.FP32)
    eps = 2.2e-16 if prec == "fp64" else 1.2e-7
    tol = 8 * (K + 1) * eps
    assert np.max(np.abs(host(tA).T - A_ref)) <= tol
    assert np.max(np.abs(host(tB).T - B_ref)) <= tol
    Vn = host(tV)[k + s:k + 2 * s].T
    assert np.max(np.abs(Vn - Vn_ref)) <= 4 * s * tol / np.min(np.diag(B_ref))


def test_qrem_block_solve_graph_replay(pk, ctx):
    """The multi-column QREM filter recorded once as a HIP graph and replayed
    every block step gives the dense pairs."""
    say("qrem block solve graph replay")
    op, E = qrem_case(pk, ctx, 12, 2)
    H = models.qrem(12, E, 1.0)
    X0 = np.stack([wl.start_vector(op.D, c) for c in range(4)])
    evals, evecs, res, rep, status = pk.solve(op, dev(X0), 30, 0.0, "maxdos", graph=1)
    assert status == "OK"
    Er, _ = dense.nearest_eigenpairs(H, rep["lambda"], 30)
    assert np.max(np.abs(host(evals) - Er) / np.maximum(np.abs(Er), 1.0)) <= 1e-10
    assert host(res).max() <= 1e-8
