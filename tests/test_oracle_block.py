"""Pins of the oracle's block Lanczos (Sec. 2.2, Sec. 4.3) against what the
mathematics fixes: a Krylov space that fills the whole space reproduces the
spectrum, H_L is the projection V^T A V, the block residual identity of eq.
blocklan_criterion, the degenerate-eigenvalue property of block Krylov
spaces, the reduction to Lanczos at s = 1, and the filtered solve against
dense diagonalization."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense, lanczos, models, polfed


def _sym(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    return A + A.T


def test_full_krylov_space_reproduces_spectrum():
    """m s = D: the block Krylov space is the whole space, so H_L is similar
    to A and has its eigenvalues."""
    A = _sym(12, 1)
    X0 = np.random.default_rng(2).standard_normal((12, 3))
    T, V, _ = lanczos.block_lanczos(lambda X: A @ X, X0, 4)
    assert np.max(np.abs(np.sort(np.linalg.eigvalsh(T)) - np.linalg.eigvalsh(A))) < 1e-12
    Vm = V[:, :12]
    assert np.max(np.abs(Vm.T @ Vm - np.eye(12))) < 1e-13


def test_lanczos_matrix_is_the_projection():
    """H_L = V^T A V over the first m blocks, block tridiagonal (a transposed
    or misplaced off-diagonal block fails this)."""
    A = _sym(60, 3)
    X0 = np.random.default_rng(4).standard_normal((60, 4))
    T, V, _ = lanczos.block_lanczos(lambda X: A @ X, X0, 6)
    Vm = V[:, :24]
    assert np.max(np.abs(Vm.T @ A @ Vm - T)) < 1e-11 * np.linalg.norm(A, 2)
    assert np.count_nonzero(T[8:, :4]) == 0 and np.count_nonzero(T[:4, 8:]) == 0


def test_block_residual_identity():
    """||A psi_j - theta_j psi_j|| = ||B_{m+1} tau_mj|| for psi_j = V t_j
    (eq. blocklan_criterion), checked against brute-force residuals."""
    A = _sym(80, 5)
    X0 = np.random.default_rng(6).standard_normal((80, 3))
    T, V, B_last = lanczos.block_lanczos(lambda X: A @ X, X0, 5)
    theta, Y, est = lanczos.block_ritz(T, B_last)
    Psi = V[:, :15] @ Y
    brute = np.linalg.norm(A @ Psi - Psi * theta, axis=0)
    assert np.max(np.abs(brute - est)) < 1e-10 * np.linalg.norm(A, 2)
    assert np.min(est) > 1e-6  # a genuine, non-trivial test


def test_block_krylov_sees_degenerate_eigenvalue_twice():
    """A single start vector spans one direction of a degenerate
    eigenspace; a block of two spans both (Sec. 2.2).  The single-vector run
    stops at 16 steps, before rounding errors have grown the second
    direction into view."""
    rng = np.random.default_rng(7)
    ev = np.concatenate([np.linspace(0.0, 1.0, 40), [2.0, 2.0]])
    Q, _ = np.linalg.qr(rng.standard_normal((42, 42)))
    A = Q @ np.diag(ev) @ Q.T
    X0 = rng.standard_normal((42, 2))
    T2, _, _ = lanczos.block_lanczos(lambda X: A @ X, X0, 12)
    th2 = np.sort(np.linalg.eigvalsh(T2))
    assert abs(th2[-1] - 2.0) < 1e-8 and abs(th2[-2] - 2.0) < 1e-8
    T1, _, _ = lanczos.block_lanczos(lambda X: A @ X, X0[:, :1], 16)
    th1 = np.sort(np.linalg.eigvalsh(T1))
    assert abs(th1[-1] - 2.0) < 1e-8 and th1[-2] < 1.0 + 1e-8


def test_block_size_one_is_lanczos():
    """s = 1: A_j = alpha_j and B_{j+1} = beta_{j+1} of the scalar
    recurrence."""
    A = _sym(50, 8)
    x0 = np.random.default_rng(9).standard_normal(50)
    T, _, B_last = lanczos.block_lanczos(lambda X: A @ X, x0[:, None], 10)
    V = np.zeros((50, 11))
    V[:, 0] = x0 / np.linalg.norm(x0)
    al, be = [], [0.0]
    for k in range(10):
        a, b, w = lanczos.lanczos_step(lambda v: A @ v, V, k, be[k])
        al.append(a)
        be.append(b)
        V[:, k + 1] = w / b
    assert np.max(np.abs(np.diag(T) - al)) < 1e-12
    assert np.max(np.abs(np.diag(T, -1) - be[1:10])) < 1e-12
    assert abs(B_last[0, 0] - be[10]) < 1e-12


def test_block_step_unique_qr():
    """B_{j+1} is upper triangular with a positive diagonal and
    W_orth = V_{j+1} B_{j+1}."""
    A = _sym(40, 10)
    V = np.zeros((40, 8))
    V[:, :4] = lanczos.orthonormal_start_block(np.random.default_rng(11).standard_normal((40, 4)))
    Aj, Bn, Vn = lanczos.block_lanczos_step(lambda X: A @ X, V, 0, 4)
    assert np.allclose(np.tril(Bn, -1), 0) and np.all(np.diag(Bn) > 0)
    W = A @ V[:, :4]
    W_orth = W - V[:, :4] @ (V[:, :4].T @ W)
    assert np.max(np.abs(Vn @ Bn - W_orth)) < 1e-12 * np.linalg.norm(A, 2)
    assert np.max(np.abs(Aj - V[:, :4].T @ A @ V[:, :4])) < 1e-12 * np.linalg.norm(A, 2)


@pytest.mark.parametrize("s", [2, 4])
def test_filtered_block_lanczos_vs_dense(s):
    """Workload: XXZ L=12, J=Delta=1, h ~ U[-1,1] seed 0, 20 pairs at
    normalized energy 0.5, start block of s seeded normal columns."""
    H, _ = models.xxz(12, 6, 1.0, 1.0, wl.xxz_fields(12, 1.0, 0))
    X0 = np.stack([wl.start_vector(924, c) for c in range(s)], 1)
    out = polfed.polfed(H, X0, 20, 0.5, "normalized")
    Er, Ur = dense.nearest_eigenpairs(H, out["lam"], 20)
    assert np.max(np.abs(out["E"] - Er) / np.maximum(np.abs(Er), 1.0)) <= 1e-10
    assert np.max(out["res"]) <= 1e-8
    assert np.min(np.abs(np.sum(out["U"] * Ur, axis=0))) >= 1 - 1e-8
    assert out["iters"] % s == 0
