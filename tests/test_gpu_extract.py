"""GPU parity of the extraction step (Sec. 4.3) and of the MFMA products it
runs on: u_j = V t_j, Rayleigh-Ritz with H on their span, residual norms,
against the oracle's rayleigh_ritz; and the two tall products (C = A B,
C -= A B, G = A^T B) element by element against NumPy's FP64 products at
sizes that span several 64 x 64 tiles, a ragged last tile, inner dimensions
that are not multiples of the 32-wide staging chunk, and the split of the
long dimension over workgroups."""
import numpy as np
import pytest

import workloads as wl  # noqa: F401
from oracle import lanczos
from tests.test_gpu_parity import ctx, dev, host, make_op, pk, say  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS = 2.220446049250313e-16


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("D,m,n", [(1, 1, 1), (63, 5, 3), (1000, 33, 65), (4097, 64, 64),
                                   (70001, 300, 130), (5000, 1, 200)])
@pytest.mark.parametrize("subtract", [False, True])
def test_gemm_nn_matches_numpy(pk, ctx, D, m, n, subtract):
    say(f"gemm nn D={D} m={m} n={n} subtract={subtract}")
    A = _rand((D, m), 1)
    B = _rand((m, n), 2)
    C0 = _rand((D, n), 3)
    ref = C0 - A @ B if subtract else A @ B
    # column-major matrices are passed as their transposes (row-major tensors)
    tA, tB, tC = dev(A.T.copy()), dev(B.T.copy()), dev(C0.T.copy())
    pk.gemm_nn(ctx, tA, tB, tC, subtract)
    got = host(tC).T
    bound = (np.abs(A) @ np.abs(B)) * (m + 2) * EPS + (np.abs(C0) * EPS if subtract else 0)
    assert np.all(np.abs(got - ref) <= bound + 1e-300)


@pytest.mark.parametrize("D,n1,n2", [(1, 1, 1), (5000, 16, 16), (2048 * 3 + 5, 65, 129),
                                     (33333, 70, 3), (200000, 120, 120), (10, 300, 2)])
def test_gemm_tn_matches_numpy(pk, ctx, D, n1, n2):
    say(f"gemm tn D={D} n1={n1} n2={n2}")
    A = _rand((D, n1), 4)
    B = _rand((D, n2), 5)
    ref = A.T @ B
    G = torch.zeros((n2, n1), dtype=torch.float64, device="cuda:0")
    pk.gemm_tn(ctx, dev(A.T.copy()), dev(B.T.copy()), G)
    got = host(G).T
    # the sum over D in any order: |error| <= (D + 2) eps sum |a b|
    bound = (np.abs(A).T @ np.abs(B)) * (D + 2) * EPS
    assert np.all(np.abs(got - ref) <= bound)
    # deterministic: the split sums are added in a fixed order
    G2 = torch.zeros_like(G)
    pk.gemm_tn(ctx, dev(A.T.copy()), dev(B.T.copy()), G2)
    assert torch.equal(G, G2)


def test_gemm_rejects_bad_arguments(pk, ctx):
    say("gemm argument checks")
    A = torch.zeros((3, 10), dtype=torch.float64, device="cuda:0")
    with pytest.raises(pk.PolfedError):
        pk._check(pk._lib.polfed_gemm_nn(ctx.handle, 10, 3, 2, pk._ptr(A), 5, pk._ptr(A), 3,
                                         pk._ptr(A), 10, 0))  # lda < D
    with pytest.raises(pk.PolfedError):
        pk._check(pk._lib.polfed_gemm_tn(ctx.handle, 10, 3, 2, pk._ptr(A), 10, pk._ptr(A), 10,
                                         pk._ptr(A), 2))  # ldg < n1


def _orthonormal(rows, cols, seed):
    q, r = np.linalg.qr(_rand((rows, cols), seed))
    return q * np.sign(np.diag(r))


def _sign_fix(U):
    idx = np.argmax(np.abs(U), axis=0)
    return U * np.sign(U[idx, np.arange(U.shape[1])])


@pytest.mark.parametrize("case,m,n", [(("xxz", 12, 6, 1.0, 0, True), 80, 30),
                                      (("xxz", 16, 8, 3.0, 3, True), 150, 97),
                                      (("qsun", 3, 7, 0), 70, 64)],
                         ids=["xxz12", "xxz16", "qsun"])
def test_extract_matches_oracle_rayleigh_ritz(pk, ctx, case, m, n):
    """Element by element: energies, residuals and the rotated Ritz vectors
    (signs fixed by the largest component) against the oracle's
    rayleigh_ritz(H, V T) (Sec. 4.3)."""
    say(f"extract {case} m={m} n={n}")
    op, H = make_op(pk, ctx, *case)
    D = op.D
    V = _orthonormal(D, m, 7)
    T = _orthonormal(m, n, 8)
    E_ref, U_ref, res_ref = lanczos.rayleigh_ritz(H, V @ T)
    E, U2, R = pk.extract(op, dev(V.T.copy()), dev(T.T.copy()))
    E, U2, R = host(E), host(U2).T, host(R)
    scale = max(1.0, np.max(np.abs(E_ref)))
    assert np.max(np.abs(E - E_ref)) <= 1e-12 * scale
    assert np.max(np.abs(R - res_ref)) <= 1e-12 * scale
    # nondegenerate Ritz values: each vector is unique up to its sign
    gap = np.min(np.diff(E_ref))
    assert gap > 1e-6 * scale
    err = np.max(np.abs(_sign_fix(U2) - _sign_fix(U_ref)))
    assert err <= 1e-12 * scale / gap, (err, gap)
