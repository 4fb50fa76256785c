"""Lanczos pieces of POLFED: spectral bounds, the filtered Lanczos iteration
with full reorthogonalization, and the eigenpair extraction.
TEST INFRASTRUCTURE ONLY.

Paper: Sec. 2.1 (eqs. lanczos_recurrence, lan_eigvecs, lan_criterion; full
reorthogonalization), Sec. 2.2 (block Lanczos: eqs.
block_lanczos_reocurrence, blocklan_criterion), Sec. 4.3 (filtered (block)
Lanczos, extraction u_i = V t_i, E_i = <u_i|H|u_i>, residual norms) and
Sec. 3.2 (E_min, E_max by Lanczos).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def spectral_extremes(H, tol: float = 1e-13):
    """E_min, E_max of symmetric H (Sec. 3.2: by Lanczos; here ARPACK's
    implicitly restarted Lanczos, dense eigvalsh for tiny matrices)."""
    D = H.shape[0]
    if D <= 2000:
        ev = np.linalg.eigvalsh(H.toarray())
        return float(ev[0]), float(ev[-1])
    v0 = np.ones(D) / math.sqrt(D)
    lo = spla.eigsh(H, k=1, which="SA", tol=tol, v0=v0,
                    return_eigenvectors=False)[0]
    hi = spla.eigsh(H, k=1, which="LA", tol=tol, v0=v0,
                    return_eigenvectors=False)[0]
    return float(lo), float(hi)


def padded_bounds(E_min: float, E_max: float, pad: float):
    """Widen [E_min, E_max] symmetrically by pad * (E_max - E_min) so that the
    rescaled spectrum stays inside [-1, 1] (the paper is silent; Lanczos
    extremes lie inside the spectrum)."""
    w = E_max - E_min
    return E_min - pad * w, E_max + pad * w


def lanczos_step(apply_op, V: np.ndarray, k: int, beta_k: float):
    """One Lanczos step (eq. lanczos_recurrence) with full reorthogonalization
    by classical Gram-Schmidt applied twice (Sec. 2.1: reorthogonalize at each
    step against all stored vectors).  V[:, :k+1] are the basis vectors.
    Returns (alpha_k, beta_{k+1}, w) where w is not yet normalized."""
    v = V[:, k]
    w = apply_op(v)
    alpha = float(v @ w)
    w = w - alpha * v
    if k > 0:
        w = w - beta_k * V[:, k - 1]
    Vk = V[:, :k + 1]
    for _ in range(2):
        w = w - Vk @ (Vk.T @ w)
    beta = float(np.linalg.norm(w))
    return alpha, beta, w


def ritz(alpha, beta_inner):
    """Eigenpairs of the tridiagonal Lanczos matrix H_L (diagonal alpha,
    off-diagonal beta_inner)."""
    if len(alpha) == 1:
        return np.array(alpha, dtype=np.float64), np.ones((1, 1))
    return sla.eigh_tridiagonal(np.asarray(alpha), np.asarray(beta_inner))


def rayleigh_ritz(H, U: np.ndarray):
    """Subspace Rayleigh-Ritz with H on the orthonormal block U:
    G = U^T H U, G = Z diag(E) Z^T, rotate U -> U Z; residuals
    ||H u_i - E_i u_i||.  Reduces to the paper's per-vector Rayleigh quotients
    (Sec. 4.3) when the Ritz vectors of P(H~) are already eigenvectors of H."""
    HU = H @ U
    G = U.T @ HU
    G = 0.5 * (G + G.T)
    E, Z = np.linalg.eigh(G)
    U2 = U @ Z
    HU2 = HU @ Z
    res = np.linalg.norm(HU2 - U2 * E, axis=0)
    return E, U2, res


def select_nearest(E: np.ndarray, res: np.ndarray, lam: float, n_ev: int,
                   tol_resid: float):
    """Indices of the accepted pairs (residual <= tol_resid) among the n_ev
    Ritz pairs nearest to lam, ordered by (|E - lam|, E), up to the first
    nearest pair that is not accepted yet: an unconverged pair nearer to
    lam than an accepted one is not skipped, so n_ev indices come back only
    when the n_ev nearest pairs are all accepted."""
    order = np.lexsort((E, np.abs(E - lam)))[:n_ev]
    ok = res[order] <= tol_resid
    run = len(order) if np.all(ok) else int(np.argmin(ok))
    return order[:run]


def complete(E_sel: np.ndarray, lam: float, theta_min: float, P_at, E_c: float,
             dE: float) -> bool:
    """True when no eigenvalue of H nearer to lam than the farthest selected
    one can be missing: P(H~) is largest around lambda~, so if P stays above
    the smallest converged Ritz value theta_min over the whole interval
    |E - lam| <= max |E_sel - lam|, every eigenvalue in it belongs to the
    converged top of the spectrum of P(H~)."""
    d = float(np.max(np.abs(E_sel - lam))) / dE
    lam_t = (lam - E_c) / dE
    pts = np.clip(np.array([lam_t - d, lam_t + d]), -1.0, 1.0)
    return bool(np.min(P_at(pts)) >= theta_min)


def filtered_lanczos(H, apply_P, x0: np.ndarray, lam: float, n_ev: int,
                     n_want: int, M_alloc: int, P_at, E_c: float, dE: float,
                     tol_P: float = 1e-10, tol_resid: float = 1e-8,
                     M_max: int | None = None):
    """Lanczos on the filtered operator P(H~) (Sec. 4.3 with block size 1).

    Every `check` steps the tridiagonal H_L is diagonalized; once the n_want
    largest Ritz values of P(H~) satisfy |b_{m+1} t_mj| <= tol_P (eq.
    lan_criterion) their Ritz vectors u = V t are extracted, refined by
    Rayleigh-Ritz with H, and the n_ev pairs nearest lam with
    ||H u - E u|| <= tol_resid are returned -- provided none can be missing
    (`complete`); otherwise n_want grows and the iteration goes on.

    Returns dict(E, U, res, iters, alpha, beta, V)."""
    D = x0.shape[0]
    if M_max is None:
        M_max = min(D, 4 * M_alloc)
    M_max = min(M_max, D)
    n_want = min(n_want, M_max)
    cap = min(M_alloc, M_max)
    V = np.zeros((D, cap + 1))
    V[:, 0] = x0 / np.linalg.norm(x0)
    alpha, beta = [], [0.0]
    check_every = max(10, int(math.ceil(0.05 * M_alloc)))
    next_check = min(n_want, M_max)
    k = 0
    rng = np.random.default_rng(12345)
    while True:
        a, b, w = lanczos_step(apply_P, V, k, beta[k])
        alpha.append(a)
        k += 1
        if k + 1 > V.shape[1]:
            grow = min(M_max, int(math.ceil(1.25 * (V.shape[1] - 1))) + 1)
            V = np.concatenate([V, np.zeros((D, grow + 1 - V.shape[1]))], 1)
        if b <= 1e-14 * max(1.0, abs(a)) and k < M_max:
            # invariant subspace: continue with a fresh random direction
            r = rng.standard_normal(D)
            for _ in range(2):
                r = r - V[:, :k] @ (V[:, :k].T @ r)
            w, b_next = r / np.linalg.norm(r), 0.0
            beta.append(b_next)
            V[:, k] = w
        else:
            beta.append(b)
            V[:, k] = w / b
        if k >= next_check or k >= M_max:
            theta, Y = ritz(alpha, beta[1:k])
            top = np.argsort(theta)[::-1][:n_want]
            resP = np.abs(beta[k] * Y[k - 1, top])
            if np.all(resP <= tol_P * max(1.0, float(np.max(np.abs(theta))))) \
                    or k >= M_max:
                U = V[:, :k] @ Y[:, top]
                E, U2, res = rayleigh_ritz(H, U)
                sel = select_nearest(E, res, lam, n_ev, tol_resid)
                ok = len(sel) >= n_ev and complete(
                    E[sel], lam, float(np.min(theta[top])), P_at, E_c, dE)
                if ok or k >= M_max:
                    return {"E": E[sel], "U": U2[:, sel], "res": res[sel],
                            "iters": k, "alpha": np.array(alpha),
                            "beta": np.array(beta), "V": V[:, :k + 1]}
                if len(sel) >= n_ev and not ok:
                    n_want = min(M_max, n_want + max(10, n_want // 5))
            next_check = k + check_every


# ------------------------------------------------------- block Lanczos ----

def orthonormal_start_block(X0: np.ndarray) -> np.ndarray:
    """The start block V_1: QR of the D x s matrix X0 (Sec. 2.2), with the
    signs fixed so that R has a positive diagonal."""
    Q, R = np.linalg.qr(X0)
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * sgn


def block_lanczos_step(apply_op, V: np.ndarray, k: int, s: int):
    """One block Lanczos step with full reorthogonalization (Sec. 2.2, Sec.
    4.3).  V[:, :k+s] holds the orthonormal blocks V_1..V_j, the current one
    being V_j = V[:, k:k+s].  W = A V_j; the diagonal block is the projection
    A_j = V_j^T W; W is orthogonalized against all stored blocks (classical
    Gram-Schmidt, two passes); QR of the result gives the next block and the
    off-diagonal block B_{j+1}.  The QR is taken with a non-negative diagonal
    of B_{j+1}, which makes it unique for a block of full rank.
    Returns (A_j, B_next, V_next)."""
    Vj = V[:, k:k + s]
    W = apply_op(Vj)
    A = Vj.T @ W
    Q = V[:, :k + s]
    for _ in range(2):
        W = W - Q @ (Q.T @ W)
    Vn, Bn = np.linalg.qr(W)
    sgn = np.where(np.diag(Bn) < 0, -1.0, 1.0)
    return A, sgn[:, None] * Bn, Vn * sgn


def block_lanczos_matrix(As, Bs) -> np.ndarray:
    """Block tridiagonal H_L (Sec. 2.2): diagonal blocks A_1..A_m
    (symmetrized: symmetric in exact arithmetic), B_{j+1} below the diagonal
    block j and B_{j+1}^T above it, for j < m."""
    m = len(As)
    s = As[0].shape[0]
    T = np.zeros((m * s, m * s))
    for j in range(m):
        T[j * s:(j + 1) * s, j * s:(j + 1) * s] = 0.5 * (As[j] + As[j].T)
        if j + 1 < m:
            T[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s] = Bs[j]
            T[j * s:(j + 1) * s, (j + 1) * s:(j + 2) * s] = Bs[j].T
    return T


def block_lanczos(apply_op, X0: np.ndarray, m: int):
    """m block steps from the start block X0.  Returns (H_L, V, B_last):
    V holds the m + 1 blocks, B_last = B_{m+1}."""
    D, s = X0.shape
    V = np.zeros((D, (m + 1) * s))
    V[:, :s] = orthonormal_start_block(X0)
    As, Bs = [], []
    for j in range(m):
        A, Bn, Vn = block_lanczos_step(apply_op, V, j * s, s)
        As.append(A)
        Bs.append(Bn)
        V[:, (j + 1) * s:(j + 2) * s] = Vn
    return block_lanczos_matrix(As, Bs), V, Bs[-1]


def block_ritz(T: np.ndarray, B_last: np.ndarray):
    """Eigenpairs (theta_j, t_j) of H_L and the residual estimates
    ||B_{m+1} tau_mj|| of eq. blocklan_criterion, tau_mj being the last block
    of s components of t_j."""
    s = B_last.shape[0]
    theta, Y = np.linalg.eigh(T)
    est = np.linalg.norm(B_last @ Y[-s:, :], axis=0)
    return theta, Y, est


def filtered_block_lanczos(H, apply_P, X0: np.ndarray, lam: float, n_ev: int,
                           n_want: int, M_alloc: int, P_at, E_c: float,
                           dE: float, tol_P: float = 1e-10,
                           tol_resid: float = 1e-8, M_max: int | None = None):
    """Block Lanczos on the filtered operator P(H~) (Sec. 4.3, block size s =
    number of columns of X0).  Checks (eq. blocklan_criterion) come at whole
    blocks; the extraction, selection and completeness test are those of
    filtered_lanczos.  A block that loses rank stops the iteration with an
    error (cases that reach it are tested against the dense solver only).

    Returns dict(E, U, res, iters)."""
    D, s = X0.shape
    if M_max is None:
        M_max = min(D, 4 * M_alloc)
    M_max = (min(M_max, D - s) // s) * s
    n_want = min(n_want, M_max)
    V = np.zeros((D, M_max + s))
    V[:, :s] = orthonormal_start_block(X0)
    As, Bs = [], []
    check_every = max(10, int(math.ceil(0.05 * M_alloc)))
    check_every = -(-check_every // s) * s
    next_check = min(-(-n_want // s) * s, M_max)
    k = 0
    while True:
        A, Bn, Vn = block_lanczos_step(apply_P, V, k, s)
        if np.min(np.abs(np.diag(Bn))) <= 1e-13:
            raise RuntimeError("block Lanczos: the next block lost rank")
        As.append(A)
        Bs.append(Bn)
        V[:, k + s:k + 2 * s] = Vn
        k += s
        if k >= next_check or k >= M_max:
            T = block_lanczos_matrix(As, Bs)
            theta, Y, est = block_ritz(T, Bs[-1])
            top = np.argsort(theta)[::-1][:n_want]
            if np.all(est[top] <= tol_P * max(1.0, float(np.max(np.abs(theta))))) \
                    or k >= M_max:
                U = V[:, :k] @ Y[:, top]
                E, U2, res = rayleigh_ritz(H, U)
                sel = select_nearest(E, res, lam, n_ev, tol_resid)
                ok = len(sel) >= n_ev and complete(
                    E[sel], lam, float(np.min(theta[top])), P_at, E_c, dE)
                if ok or k >= M_max:
                    return {"E": E[sel], "U": U2[:, sel], "res": res[sel],
                            "iters": k}
                if len(sel) >= n_ev and not ok:
                    n_want = min(M_max, n_want + max(10, n_want // 5))
            next_check = k + check_every
