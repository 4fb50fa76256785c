"""Chebyshev delta filter, its Clenshaw evaluation, the Gaussian density of
states and the choice of the polynomial order K.  TEST INFRASTRUCTURE ONLY.

Paper sections: 3.2 (polynomial spectral filtering, eqs. chebyshev_definition,
rescaledMatrix, transformation, transformationCoefficients), 4.1 (eq.
dos_gaussian), 4.2 (eqs. Nev, condition_for_K, K_approx) and 4.4 (eq.
clenshaw_chebyshev_prod).
"""
from __future__ import annotations

import math

import numpy as np

# Cutoff of the filter (Sec. 3.2 fixes it only as "slightly above the secondary
# peaks").  Near the target the normalized filter behaves as sinc(z) with
# z = (K+1/2) * dist / sqrt(1 - lambda~^2), so the empirical constant 2.655 of
# eq. K_approx corresponds to Omega = sin(2.655)/2.655.
OMEGA_DEFAULT = math.sin(2.655) / 2.655


def rescale(E_min: float, E_max: float):
    """eq. rescaledMatrix: E_c = (E_max + E_min)/2, dE = (E_max - E_min)/2."""
    return 0.5 * (E_max + E_min), 0.5 * (E_max - E_min)


def chebyshev_T(n_max: int, x) -> np.ndarray:
    """T_0..T_{n_max} at x by the three-term recurrence (eq.
    chebyshev_definition).  Returns shape (n_max+1,) + x.shape."""
    x = np.asarray(x, dtype=np.float64)
    T = np.empty((n_max + 1,) + x.shape)
    T[0] = 1.0
    if n_max >= 1:
        T[1] = x
    for n in range(1, n_max):
        T[n + 1] = 2.0 * x * T[n] - T[n - 1]
    return T


def coefficients(lam_t: float, K: int) -> np.ndarray:
    """Filter coefficients a_n = c_n / chi, n = 0..K (eqs. transformation and
    transformationCoefficients): c_n = sqrt(4 - 3 delta_{n0}) T_n(lambda~),
    chi = sum_n c_n T_n(lambda~) so that P(lambda~) = 1."""
    T = chebyshev_T(K, lam_t)
    c = 2.0 * T
    c[0] = 1.0
    chi = float(np.sum(c * T))
    return c / chi


def filter_value(x, lam_t: float, K: int) -> np.ndarray:
    """P^K_{lambda~}(x) as the plain sum (1/chi) sum_n c_n T_n(x)."""
    a = coefficients(lam_t, K)
    T = chebyshev_T(K, x)
    return np.tensordot(a, T, axes=(0, 0))


def clenshaw_scalar(a: np.ndarray, x: float) -> float:
    """eq. clenshaw_chebyshev: b_{K+1} = b_{K+2} = 0,
    b_k = a_k + 2 x b_{k+1} - b_{k+2}, S = a_0 + x b_1 - b_2."""
    K = len(a) - 1
    b1 = b2 = 0.0
    for k in range(K, 0, -1):
        b1, b2 = a[k] + 2.0 * x * b1 - b2, b1
    return a[0] + x * b1 - b2


def apply_filter(H, E_c: float, dE: float, a: np.ndarray, v: np.ndarray):
    """P(H~) v by the matrix Clenshaw recurrence (eq. clenshaw_chebyshev_prod):
        b_{K+1} = b_{K+2} = 0,  b_i = a_i v + 2 H~ b_{i+1} - b_{i+2}  (i = K..1),
        P(H~) v = a_0 v + H~ b_1 - b_2,
    with H~ x = (H x - E_c x)/dE (eq. rescaledMatrix).  K sparse mat-vecs."""
    def Ht(x):
        return (H @ x - E_c * x) / dE
    K = len(a) - 1
    b1 = np.zeros_like(v)
    b2 = np.zeros_like(v)
    for i in range(K, 0, -1):
        b_new = a[i] * v + 2.0 * Ht(b1) - b2
        b2 = b1
        b1 = b_new
    return a[0] * v + Ht(b1) - b2


def trace_moments(H):
    """Exact Tr H / D and Tr H^2 / D of a symmetric sparse H
    (Tr H^2 = sum_ij H_ij^2)."""
    D = H.shape[0]
    tr1 = float(H.diagonal().sum())
    tr2 = float(H.multiply(H).sum())
    return tr1 / D, tr2 / D


def gaussian_dos(E_t, D: int, mu_t: float, Gamma_t: float):
    """eq. dos_gaussian: rho(E~) = D/(sqrt(2 pi) Gamma~)
    exp(-(E~ - mu~)^2 / (2 Gamma~^2)), normalized to D in rescaled units."""
    E_t = np.asarray(E_t, dtype=np.float64)
    return D / (math.sqrt(2.0 * math.pi) * Gamma_t) * np.exp(
        -(E_t - mu_t) ** 2 / (2.0 * Gamma_t ** 2))


def window_halfwidth(n_ev: int, rho_at_target: float) -> float:
    """eq. Nev: delta = N_ev / (2 rho(lambda~))."""
    return n_ev / (2.0 * rho_at_target)


def K_approx(lam_t: float, delta: float) -> float:
    """eq. K_approx: K = 2.655 sqrt(1 - lambda~^2) / delta."""
    return 2.655 * math.sqrt(max(0.0, 1.0 - lam_t * lam_t)) / delta


def _meets_cutoff(K: int, lam_t: float, delta: float, omega: float) -> bool:
    pts = np.clip(np.array([lam_t - delta, lam_t + delta]), -1.0, 1.0)
    return bool(np.min(filter_value(pts, lam_t, K)) >= omega)


def choose_K(lam_t: float, delta: float, omega: float = OMEGA_DEFAULT,
             K_cap: int = 10_000_000) -> int:
    """Order K from eq. condition_for_K: the largest K with
    P^K(lambda~ +- delta) >= Omega, found by bisection started from the bracket
    [K_approx/2, 2 K_approx] (Sec. 4.2); the bracket is widened if the
    estimate is off."""
    K0 = K_approx(lam_t, delta)
    lo = max(1, int(math.floor(K0 / 2)))
    hi = max(lo + 1, int(math.ceil(2 * K0)))
    while lo > 1 and not _meets_cutoff(lo, lam_t, delta, omega):
        lo = max(1, lo // 2)
    if not _meets_cutoff(lo, lam_t, delta, omega):
        return 1
    while _meets_cutoff(hi, lam_t, delta, omega):
        lo, hi = hi, 2 * hi
        if hi > K_cap:
            return K_cap
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if _meets_cutoff(mid, lam_t, delta, omega):
            lo = mid
        else:
            hi = mid
    return lo


def expected_krylov_dim(howmany: int, blocksize: int, eta: float) -> int:
    """Krylov allocation estimate `expectedkrylovdim` of Sec. 5.5:
    ceil((20.427 * blocksize + 1.696 * howmany) * eta)."""
    return int(math.ceil((20.427 * blocksize + 1.696 * howmany) * eta))
