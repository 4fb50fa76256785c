"""GPU parity of block Lanczos (Sec. 2.2 with the filter of Sec. 4.3): one
block step through the C ABI against the oracle's block step (A_j, B_{j+1}
and the next block), and block solves against dense diagonalization."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense, lanczos, polfed
from oracle import filter as flt
from tests.test_gpu_parity import OPS, ctx, dev, host, make_op, pk, say  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _filter(H, K):
    lo, hi = lanczos.spectral_extremes(H)
    E_c, dE = flt.rescale(*lanczos.padded_bounds(lo, hi, 1e-3))
    lam_t = (0.5 * (lo + hi) + 0.1 * (hi - lo) - E_c) / dE
    return E_c, dE, flt.coefficients(lam_t, K)


STEP_CASES = [(OPS[0], 2, 0), (OPS[0], 4, 8), (OPS[4], 3, 6), (OPS[6], 8, 16),
              (OPS[2], 5, 0), (OPS[7], 3, 6), (OPS[8], 4, 4),
              (("xxz", 16, 8, 3.0, 3, True), 16, 16)]


@pytest.mark.parametrize("case,s,k", STEP_CASES,
                         ids=lambda c: "-".join(map(str, c)) if isinstance(c, tuple) else str(c))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_block_lanczos_step_matches_oracle(pk, ctx, case, s, k, prec):
    say(f"block step {case} s={s} k={k} {prec}")
    op, H = make_op(pk, ctx, *case)
    D = op.D
    K = 200 if prec == "fp64" else 60
    E_c, dE, a = _filter(H, K)

    def P(X):
        return flt.apply_filter(H, E_c, dE, a, X)
    # basis of k + s columns from the oracle's own block steps
    X0 = np.stack([wl.start_vector(D, 40 + c) for c in range(s)], 1)
    V = np.zeros((D, k + 2 * s))
    V[:, :s] = lanczos.orthonormal_start_block(X0)
    for j in range(k // s):
        _, _, Vn = lanczos.block_lanczos_step(P, V, j * s, s)
        V[:, (j + 1) * s:(j + 2) * s] = Vn
    A_ref, B_ref, Vn_ref = lanczos.block_lanczos_step(P, V, k, s)
    tV = dev(V.T)
    tA = torch.zeros((s, s), dtype=torch.float64, device="cuda:0")
    tB = torch.zeros((s, s), dtype=torch.float64, device="cuda:0")
    pk.block_lanczos_step(op, E_c, dE, a, tV, k, s, tA, tB,
                          pk.FP64 if prec == "fp64" else pk.FP32)
    A = host(tA).T
    Bn = host(tB).T
    Vn = host(tV)[k + s:k + 2 * s].T
    # the Clenshaw error is relative to ||P|| <= 1; FP32 also perturbs the
    # orthogonalized block by that much relative to its smallest singular value
    eps = 2.2e-16 if prec == "fp64" else 1.2e-7
    tol = 8 * (K + 1) * eps
    assert np.max(np.abs(A - A_ref)) <= tol
    assert np.max(np.abs(Bn - B_ref)) <= tol
    assert np.count_nonzero(np.tril(Bn, -1)) == 0 and np.all(np.diag(Bn) > 0)
    cond = np.min(np.diag(B_ref))
    assert np.max(np.abs(Vn - Vn_ref)) <= 4 * s * tol / cond
    # the new block is orthonormal and orthogonal to the basis, always to
    # FP64 rounding (the orthogonalization is FP64 in either precision)
    Vall = host(tV).T
    assert np.max(np.abs(Vall.T @ Vall - np.eye(k + 2 * s))) <= 1e-12
    say(f"   max |dA|={np.max(np.abs(A - A_ref)):.1e} |dB|={np.max(np.abs(Bn - B_ref)):.1e} "
        f"|dV|={np.max(np.abs(Vn - Vn_ref)):.1e} min diag B={cond:.2e}")


def test_block_lanczos_step_rejects_bad_shapes(pk, ctx):
    say("block step invalid")
    op, H = make_op(pk, ctx, *OPS[0])
    tV = torch.zeros((12, op.D), dtype=torch.float64, device="cuda:0")
    tA = torch.zeros((4, 4), dtype=torch.float64, device="cuda:0")
    for k, s in [(2, 4), (0, 0), (0, 65), (op.D - 4, 4)]:
        with pytest.raises(pk.PolfedError):
            pk.block_lanczos_step(op, 0.0, 10.0, [1.0, 0.5], tV, k, s, tA, tA)


def _check_block_solve(pk, op, H, n_ev, s, seed=0, **kw):
    E_min, E_max = lanczos.spectral_extremes(H)
    lam = polfed.target_energy("normalized", 0.5, E_min, E_max)
    X0 = np.stack([wl.start_vector(op.D, seed + c) for c in range(s)])
    evals, evecs, res, rep, status = pk.solve(op, dev(X0), n_ev, lam, "absolute", **kw)
    E, U, R = host(evals), host(evecs), host(res)
    Er, Ur = dense.nearest_eigenpairs(H, lam, n_ev)
    rel = np.abs(E - Er) / np.maximum(np.abs(Er), 1.0)
    ov = np.abs(np.sum(U * Ur, axis=0))
    true_res = np.linalg.norm(H @ U - U * E, axis=0)
    say(f"   s={s} K={rep['K']} iters={rep['iters']} checks={rep['checks']} "
        f"restarts={rep['restarts']} rel={rel.max():.1e} res={R.max():.1e}")
    assert status == "OK"
    assert rel.max() <= 1e-10
    assert R.max() <= 1e-8 and true_res.max() <= 1e-8
    assert np.max(np.abs(true_res - R)) <= 1e-10
    assert ov.min() >= 1 - 1e-8
    assert rep["iters"] % s == 0
    return rep


SOLVE_CASES = [(OPS[0], 20, 2), (OPS[0], 20, 4), (OPS[4], 20, 4), (OPS[7], 20, 3),
               (("xxz", 14, 7, 3.0, 3, True), 50, 8), (OPS[2], 10, 2), (OPS[5], 15, 5),
               (OPS[3], 30, 16)]


@pytest.mark.parametrize("case,n_ev,s", SOLVE_CASES,
                         ids=lambda c: "-".join(map(str, c)) if isinstance(c, tuple) else str(c))
def test_block_solve_matches_dense(pk, ctx, case, n_ev, s):
    say(f"block solve {case} n_ev={n_ev} s={s}")
    op, H = make_op(pk, ctx, *case)
    _check_block_solve(pk, op, H, n_ev, s)


@pytest.mark.parametrize("graph", [1, 2])
def test_block_solve_fp32_and_graph(pk, ctx, graph):
    say(f"block solve fp32 graph={graph}")
    op, H = make_op(pk, ctx, *OPS[0])
    _check_block_solve(pk, op, H, 20, 4, precision=pk.FP32, graph=graph)


def test_block_solve_graph_matches_direct(pk, ctx):
    say("block solve fp64 graph vs direct")
    op, H = make_op(pk, ctx, *OPS[0])
    r1 = _check_block_solve(pk, op, H, 20, 4, graph=1)
    r2 = _check_block_solve(pk, op, H, 20, 4, graph=2)
    assert r1["iters"] == r2["iters"]


def test_block_solve_fp32_fallback(pk, ctx):
    say("block solve fp32 forced fallback")
    op, H = make_op(pk, ctx, *OPS[0])
    rep = _check_block_solve(pk, op, H, 20, 4, precision=pk.FP32, refine_max=-1)
    assert rep["fp32_fallback"] == 1


def test_block_solve_small_space(pk, ctx):
    """D = 70: the block Krylov space reaches most of the whole space
    (M_max = 64 with s = 4)."""
    say("block solve small space")
    op, H = make_op(pk, ctx, "xxz", 8, 4, 2.0, 5, True)
    _check_block_solve(pk, op, H, 6, 4)


def _two_block_operator(pk, ctx, d1=12, d2=300, seed=3):
    """Block-diagonal CSR: a dense random symmetric d1 x d1 block and a
    sparse random symmetric d2 x d2 block with spectra that interleave."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    A1 = rng.standard_normal((d1, d1))
    A1 = (A1 + A1.T) / np.sqrt(2 * d1) * 2.0
    A2 = sp.random(d2, d2, density=0.05, random_state=seed, data_rvs=rng.standard_normal)
    A2 = (A2 + A2.T) * 0.5 + sp.diags(rng.uniform(-2.0, 2.0, d2))
    H = sp.block_diag([sp.csr_matrix(A1), A2]).tocsr()
    H.sort_indices()
    op = pk.Operator.csr(ctx, d1 + d2, H.indptr, H.indices, H.data)
    return op, H


@pytest.mark.parametrize("s", [1, 4])
def test_breakdown_restart_reaches_the_other_block(pk, ctx, s):
    """A start supported on the 12-dimensional invariant block exhausts its
    Krylov space before convergence (Lanczos breakdown); the restart with a
    random direction must reach the other block, and the pairs nearest the
    target, from both blocks, must all be found."""
    say(f"breakdown restart s={s}")
    op, H = _two_block_operator(pk, ctx)
    D = op.D
    rng = np.random.default_rng(9)
    X0 = np.zeros((s, D))
    X0[:, :12] = rng.standard_normal((s, 12))
    lam = 0.1
    x0 = dev(X0[0]) if s == 1 else dev(X0)
    evals, evecs, res, rep, status = pk.solve(op, x0, 10, lam, "absolute")
    assert status == "OK"
    E, U = host(evals), host(evecs)
    Er, Ur = dense.nearest_eigenpairs(H, lam, 10)
    say(f"   iters={rep['iters']} restarts={rep['restarts']} "
        f"max rel={np.max(np.abs(E - Er) / np.maximum(np.abs(Er), 1.0)):.1e}")
    assert rep["restarts"] >= 1
    assert np.max(np.abs(E - Er) / np.maximum(np.abs(Er), 1.0)) <= 1e-10
    assert np.linalg.norm(H @ U - U * E, axis=0).max() <= 1e-8
    # the pairs come from both blocks
    w1 = np.linalg.norm(U[:12], axis=0)
    assert np.any(w1 > 0.99) and np.any(w1 < 0.01)


def test_block_start_must_have_full_rank(pk, ctx):
    say("block start rank deficient")
    op, H = make_op(pk, ctx, *OPS[0])
    x = wl.start_vector(op.D, 0)
    X0 = np.stack([x, 2.0 * x])
    with pytest.raises(pk.PolfedError) as e:
        pk.solve(op, dev(X0), 10, 0.5, "normalized")
    assert "full rank" in str(e.value)


def test_block_mode_rejected_by_batch_and_serving(pk, ctx):
    say("block mode rejected in batch")
    op, H = make_op(pk, ctx, *OPS[0])
    x0 = dev(wl.start_vector(op.D, 0))
    with pytest.raises(pk.PolfedError) as e:
        pk.solve_batch([op], [x0], 10, 0.5, "normalized", block_size=2)
    assert "block" in str(e.value)
    with pk.Server(ctx, 1 << 30, 4) as srv:
        with pytest.raises(pk.PolfedError) as e:
            srv.submit(op, x0, 10, 0.5, "normalized", block_size=2)
        assert "block" in str(e.value)


def test_block_solve_equals_oracle_block_solve(pk, ctx):
    """The oracle's filtered block Lanczos and the device path return the
    same pairs from the same start block."""
    say("block solve vs oracle block solve")
    op, H = make_op(pk, ctx, *OPS[0])
    X0 = np.stack([wl.start_vector(op.D, c) for c in range(4)], 1)
    ref = polfed.polfed(H, X0, 20, 0.5, "normalized")
    evals, evecs, res, rep, status = pk.solve(op, dev(X0.T), 20, 0.5, "normalized")
    assert status == "OK"
    E = host(evals)
    assert np.max(np.abs(E - ref["E"]) / np.maximum(np.abs(ref["E"]), 1.0)) <= 1e-10
    ov = np.abs(np.sum(host(evecs) * ref["U"], axis=0))
    assert ov.min() >= 1 - 1e-8
