"""Kernel polynomial method for the density of states (Sec. 4.1 eq.
dos_kpm and App. B).  TEST INFRASTRUCTURE ONLY.

  rho_KPM(x) = [mu_0 g_0 + 2 sum_{n=1}^{N-1} mu_n g_n T_n(x)] / (pi sqrt(1 - x^2)),
  mu_n = Tr T_n(H~) ~ (1/R) sum_r <r| T_n(H~) |r>,
with the Jackson kernel g_n (App. B eq. kernels_jackson_and_lorenz) and
random vectors whose components have zero mean and unit variance.
"""
from __future__ import annotations

import numpy as np


def jackson(N: int) -> np.ndarray:
    """Jackson damping factors g_0..g_{N-1} for N moments."""
    n = np.arange(N, dtype=np.float64)
    a = np.pi / (N + 1)
    return ((N - n + 1) * np.cos(a * n) + np.sin(a * n) / np.tan(a)) / (N + 1)


def moments(H, E_c: float, dE: float, R: np.ndarray, N: int) -> np.ndarray:
    """mu_0..mu_{N-1} estimated with the columns of R (D x R_count): the
    three-term recurrence t_0 = r, t_1 = H~ r, t_{n+1} = 2 H~ t_n - t_{n-1},
    mu_n = mean over r of <r|t_n>, with H~ = (H - E_c)/dE."""
    def Ht(x):
        return (H @ x - E_c * x) / dE
    R = np.asarray(R, dtype=np.float64)
    if R.ndim == 1:
        R = R[:, None]
    mu = np.zeros(N)
    t_prev = R.copy()
    mu[0] = np.mean(np.sum(R * t_prev, axis=0))
    if N == 1:
        return mu
    t = Ht(R)
    mu[1] = np.mean(np.sum(R * t, axis=0))
    for n in range(2, N):
        t_next = 2.0 * Ht(t) - t_prev
        t_prev, t = t, t_next
        mu[n] = np.mean(np.sum(R * t, axis=0))
    return mu


def density(mu: np.ndarray, x) -> np.ndarray:
    """rho_KPM(x) of eq. dos_kpm with the Jackson kernel, for |x| < 1."""
    mu = np.asarray(mu, dtype=np.float64)
    N = len(mu)
    g = jackson(N)
    x = np.asarray(x, dtype=np.float64)
    th = np.arccos(np.clip(x, -1.0, 1.0))
    n = np.arange(1, N)
    s = mu[0] * g[0] + 2.0 * np.sum((mu[1:] * g[1:])[:, None] * np.cos(np.outer(n, th)), axis=0)
    return s / (np.pi * np.sqrt(1.0 - x * x))


def maxdos_point(mu: np.ndarray, lo: float = -1.0, hi: float = 1.0,
                 n_grid: int = 4096) -> float:
    """The rescaled energy of maximal rho_KPM among the Chebyshev nodes
    x_j = cos(pi (j + 1/2) / n_grid) that lie in [lo, hi].  Near x = +-1 the
    factor 1/sqrt(1 - x^2) magnifies the noise of stochastic moments, so the
    caller keeps the search inside the spectrum."""
    x = np.cos(np.pi * (np.arange(n_grid) + 0.5) / n_grid)
    x = x[(x >= lo) & (x <= hi)]
    return float(x[np.argmax(density(mu, x))])


def search_interval(E_min: float, E_max: float, E_c: float, dE: float):
    """The maxdos search interval in rescaled coordinates: the spectrum
    [E_min, E_max] without 5% of its width at each end."""
    w = E_max - E_min
    return (E_min + 0.05 * w - E_c) / dE, (E_max - 0.05 * w - E_c) / dE
