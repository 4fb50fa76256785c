"""GPU parity of the J1-J2 and J1-J2-J3 chains (App. A eqs. j1j2, j1j2j3)
and of the optimized mapping (Sec. 5.6): operator application against the
oracle, the optimized CSR step equal to the generic one to the last bit,
and a solve against dense diagonalization."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense, lanczos, models, polfed
from tests.test_gpu_parity import ctx, dev, host, pk, say  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

COUPLINGS = {2: ([1.0, 0.5], [1.0, 1.0]), 3: ([1.0, 0.5, 0.3], [1.0, 1.0, 0.8])}


def chain(pk, ctx, L, R, periodic=True, seed=0):
    Js, Ds = COUPLINGS[R]
    h = wl.xxz_fields(L, 1.0, seed)
    op = pk.Operator.spin_chain(ctx, L, L // 2, Js, Ds, h, periodic)
    H, _ = models.spin_chain(L, L // 2, Js, Ds, h, periodic)
    return op, H


@pytest.mark.parametrize("L,R,periodic", [(12, 2, True), (12, 3, True), (13, 2, False),
                                          (11, 3, False)])
def test_spin_chain_apply_matches_oracle(pk, ctx, L, R, periodic):
    say(f"spin chain apply L={L} R={R} periodic={periodic}")
    op, H = chain(pk, ctx, L, R, periodic)
    x = np.random.default_rng(1).standard_normal(op.D)
    y = host(op.apply(dev(x)))
    ref = H @ x
    assert np.max(np.abs(y - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("R,n_values", [(2, 2), (3, 3)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_optimized_mapping_step_is_bitwise_equal(pk, ctx, R, n_values, prec):
    """The value table returns the same numbers in the same order of
    operations, so the optimized step equals the generic one exactly."""
    say(f"optimized mapping R={R} {prec}")
    L = 14
    op, H = chain(pk, ctx, L, R)
    rng = np.random.default_rng(3)
    dt = torch.float64 if prec == "fp64" else torch.float32
    p = pk.FP64 if prec == "fp64" else pk.FP32
    v, b1, b2 = (dev(rng.standard_normal(op.D), dt) for _ in range(3))
    ref = b2.clone()
    pk.clenshaw_step(op, 0.2, 9.0, 0.013, v, b1, ref, p)
    assert op.optimize_mapping() == n_values
    got = b2.clone()
    pk.clenshaw_step(op, 0.2, 9.0, 0.013, v, b1, got, p)
    assert torch.equal(got, ref)
    # and both agree with the oracle
    f = 2.0 * (H @ host(b1).astype(np.float64) - 0.2 * host(b1)) / 9.0
    want = 0.013 * host(v) + f - host(b2)
    tol = 1e-14 if prec == "fp64" else 2e-6
    assert np.max(np.abs(host(got) - want)) <= tol * np.max(np.abs(want))


def test_single_value_mapping_on_materialized_xxz(pk, ctx):
    say("optimized mapping, one value")
    h = wl.xxz_fields(12, 3.0, 0)
    op = pk.Operator.xxz(ctx, 12, 6, 1.0, 1.0, h, True)
    op.materialize_csr().set_storage(pk.CSR)
    x = dev(np.random.default_rng(2).standard_normal(op.D))
    ref = op.apply(x).clone()
    assert op.optimize_mapping() == 1
    assert torch.equal(op.apply(x), ref)


def test_many_values_leave_the_operator_unchanged(pk, ctx):
    say("optimized mapping, many values")
    import scipy.sparse as sp
    rng = np.random.default_rng(4)
    A = sp.random(500, 500, density=0.02, random_state=4, data_rvs=rng.standard_normal)
    A = (A + A.T).tocsr()
    A.sort_indices()
    op = pk.Operator.csr(ctx, 500, A.indptr, A.indices, A.data)
    x = rng.standard_normal(500)
    assert op.optimize_mapping() == 257
    y = host(op.apply(dev(x)))
    assert np.max(np.abs(y - A @ x)) <= 1e-12 * np.max(np.abs(A @ x))


@pytest.mark.parametrize("R", [2, 3])
def test_spin_chain_solve_matches_dense(pk, ctx, R):
    say(f"spin chain solve R={R}")
    op, H = chain(pk, ctx, 14, R, True, seed=2)
    assert op.optimize_mapping() == R
    lo, hi = lanczos.spectral_extremes(H)
    lam = polfed.target_energy("normalized", 0.5, lo, hi)
    evals, evecs, res, rep, status = pk.solve(op, dev(wl.start_vector(op.D, 0)), 20, lam,
                                              "absolute")
    assert status == "OK"
    Er, Ur = dense.nearest_eigenpairs(H, lam, 20)
    E, U = host(evals), host(evecs)
    assert np.max(np.abs(E - Er) / np.maximum(np.abs(Er), 1.0)) <= 1e-10
    assert host(res).max() <= 1e-8
    assert np.min(np.abs(np.sum(U * Ur, axis=0))) >= 1 - 1e-8
