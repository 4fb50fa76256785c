"""The POLFED workflow (Sec. 4.6 of the paper), plain FP64 on the CPU.
TEST INFRASTRUCTURE ONLY.

  1. spectral bounds E_min, E_max (Lanczos) and rescaling (eq. rescaledMatrix)
  2. density of states near the target (Gaussian, eq. dos_gaussian, with the
     mean and width taken from the exact traces Tr H / D, Tr H^2 / D)
  3. order K from eq. condition_for_K, bracketed by eq. K_approx
  4. Lanczos on P(H~) with the Clenshaw filter (eq. clenshaw_chebyshev_prod)
  5. periodic convergence checks (eq. lan_criterion)
  6. extraction u = V t, energies, residual norms.
"""
from __future__ import annotations

import math

import numpy as np

from . import filter as flt
from . import kpm
from . import lanczos as lz


def target_energy(kind: str, target: float, E_min: float, E_max: float,
                  mean: float | None = None):
    """Absolute target energy lambda.
    'absolute'  : lambda = target;
    'rescaled'  : target is lambda~ in the rescaled coordinates of the
                  (unpadded) bounds (Sec. 5.4, the (:rescaled, eps) mode);
    'normalized': target = (lambda - E_min)/(E_max - E_min) in [0, 1] (the
                  convention of the workload definitions; 0.5 is the middle);
    'maxdos'    : the maximum of the estimated density of states (Sec. 5.4,
                  :maxdos); for the Gaussian estimate of eq. dos_gaussian that
                  is its mean, mean = Tr H / D (target is ignored);
    'offset'    : target = eta in [-1, 1] moves from the maxdos point toward
                  the upper (eta > 0) or lower (eta < 0) spectral edge,
                  linearly in the rescaled coordinates (Sec. 5.4,
                  (:offset, eta))."""
    if kind == "absolute":
        return float(target)
    if kind == "rescaled":
        E_c, dE = flt.rescale(E_min, E_max)
        return E_c + target * dE
    if kind == "normalized":
        return E_min + target * (E_max - E_min)
    if kind in ("maxdos", "offset"):
        if mean is None:
            raise ValueError("maxdos/offset targets need the mean energy")
        if kind == "maxdos":
            return float(mean)
        E_c, dE = flt.rescale(E_min, E_max)
        em = (mean - E_c) / dE
        eta = float(target)
        e = em + eta * (1.0 - em) if eta >= 0 else em + eta * (1.0 + em)
        return E_c + e * dE
    raise ValueError(kind)


def buffer_size(n_ev: int) -> int:
    """Extra pairs converged beyond N_ev so that the N_ev nearest to the
    target are all among them."""
    return max(10, int(math.ceil(0.2 * n_ev)))


def plan(H, lam: float, n_window: int, E_min: float, E_max: float,
         pad: float = 1e-3, omega: float = flt.OMEGA_DEFAULT,
         K: int | None = None, kpm_mu=None):
    """Steps 1-3: rescaling, the DOS at the target (Gaussian, or KPM from the
    moments kpm_mu of H~ when given), window half-width delta for n_window
    eigenvalues, order K and the filter coefficients."""
    D = H.shape[0]
    lo, hi = lz.padded_bounds(E_min, E_max, pad)
    E_c, dE = flt.rescale(lo, hi)
    lam_t = (lam - E_c) / dE
    m1, m2 = flt.trace_moments(H)
    mu_t = (m1 - E_c) / dE
    Gamma_t = math.sqrt(max(m2 - m1 * m1, 0.0)) / dE
    if kpm_mu is None:
        rho = float(flt.gaussian_dos(lam_t, D, mu_t, Gamma_t))
    else:
        rho = float(kpm.density(kpm_mu, np.array([lam_t]))[0])
    delta = flt.window_halfwidth(n_window, rho)
    if K is None:
        K = flt.choose_K(lam_t, delta, omega)
    a = flt.coefficients(lam_t, K)
    return {"E_c": E_c, "dE": dE, "lam_t": lam_t, "mu_t": mu_t,
            "Gamma_t": Gamma_t, "rho": rho, "delta": delta, "K": int(K),
            "a": a}


def polfed(H, x0: np.ndarray, n_ev: int, target: float,
           target_kind: str = "absolute", pad: float = 1e-3,
           omega: float = flt.OMEGA_DEFAULT, eta: float = 1.5,
           K: int | None = None, tol_P: float = 1e-10,
           tol_resid: float = 1e-8, bounds=None, kpm_vectors=None,
           kpm_moments: int = 0):
    """N_ev eigenpairs of H nearest the target.  Returns a dict with E (sorted
    by distance to lambda), U (columns), res, and the plan.  A vector x0
    runs Lanczos; a D x s matrix x0 runs block Lanczos with block size s (the
    shape of the start selects the variant)."""
    if bounds is None:
        E_min, E_max = lz.spectral_extremes(H)
    else:
        E_min, E_max = bounds
    tr1, _ = flt.trace_moments(H)
    mu = None
    if kpm_vectors is not None:
        # KPM DOS (Sec. 4.1): moments of H~ in the padded rescaling of the plan
        E_c, dE = flt.rescale(*lz.padded_bounds(E_min, E_max, pad))
        mu = kpm.moments(H, E_c, dE, kpm_vectors, kpm_moments)
    if mu is not None and target_kind in ("maxdos", "offset"):
        em = E_c + kpm.maxdos_point(mu, *kpm.search_interval(E_min, E_max, E_c, dE)) * dE
        lam = target_energy(target_kind, target, E_min, E_max, em)
    else:
        lam = target_energy(target_kind, target, E_min, E_max, tr1)
    n_want = n_ev + buffer_size(n_ev)
    # the window is sized for all n_want pairs, so that the n_ev nearest sit
    # well inside the main lobe of the filter
    p = plan(H, lam, n_want, E_min, E_max, pad, omega, K, mu)

    def apply_P(v):
        return flt.apply_filter(H, p["E_c"], p["dE"], p["a"], v)

    def P_at(x_t):
        return flt.filter_value(x_t, p["lam_t"], p["K"])

    s = 1 if x0.ndim == 1 else x0.shape[1]
    M_alloc = flt.expected_krylov_dim(n_want, s, eta)
    if x0.ndim == 1:
        out = lz.filtered_lanczos(H, apply_P, x0, lam, n_ev, n_want, M_alloc,
                                  P_at, p["E_c"], p["dE"],
                                  tol_P=tol_P, tol_resid=tol_resid)
    else:
        out = lz.filtered_block_lanczos(H, apply_P, x0, lam, n_ev, n_want,
                                        M_alloc, P_at, p["E_c"], p["dE"],
                                        tol_P=tol_P, tol_resid=tol_resid)
    out.update({"lam": lam, "E_min": E_min, "E_max": E_max, "plan": p,
                "M_alloc": M_alloc})
    return out
