"""Pins of the oracle's kernel polynomial method (Sec. 4.1 eq. dos_kpm, App.
B): exact traces reproduce sum_k T_n(E~_k) (with T_n from the cosine form),
the density integrates to D, the Jackson kernel's closed values, a single
level reconstructs as a peak at its energy, and stochastic moments approach
the exact ones."""
import math

import numpy as np

import workloads as wl
from oracle import kpm, lanczos, models
from oracle import filter as flt


def _rescaled_case():
    H, _ = models.xxz(10, 5, 1.0, 1.0, wl.xxz_fields(10, 2.0, 1))
    lo, hi = lanczos.spectral_extremes(H)
    E_c, dE = flt.rescale(*lanczos.padded_bounds(lo, hi, 1e-3))
    Et = (np.linalg.eigvalsh(H.toarray()) - E_c) / dE
    return H, E_c, dE, Et


def test_exact_trace_moments():
    """r_i = sqrt(D) e_i for i < D: (1/D) sum_i D <e_i|T_n|e_i> = Tr T_n(H~)
    exactly, to compare with sum_k cos(n arccos E~_k)."""
    H, E_c, dE, Et = _rescaled_case()
    D = H.shape[0]
    mu = kpm.moments(H, E_c, dE, np.sqrt(D) * np.eye(D), 60)
    ref = np.array([np.sum(np.cos(n * np.arccos(Et))) for n in range(60)])
    assert np.max(np.abs(mu - ref)) < 1e-9 * D


def test_density_integrates_to_dimension():
    """Gauss-Chebyshev quadrature integrates T_n/(pi sqrt(1-x^2)) exactly,
    so the integral of rho_KPM over [-1, 1] is mu_0 g_0 = D."""
    H, E_c, dE, Et = _rescaled_case()
    D = H.shape[0]
    mu = kpm.moments(H, E_c, dE, np.sqrt(D) * np.eye(D), 80)
    M = 400
    x = np.cos(np.pi * (np.arange(M) + 0.5) / M)
    integral = np.sum(kpm.density(mu, x) * np.sqrt(1 - x * x)) * np.pi / M
    assert abs(integral - D) < 1e-9 * D


def test_jackson_kernel_values():
    g = kpm.jackson(100)
    assert abs(g[0] - 1.0) < 1e-15
    assert np.all(np.diff(g) < 0) and 0 < g[-1] < 1e-3
    # N = 1: the kernel is the single factor 1
    assert abs(kpm.jackson(1)[0] - 1.0) < 1e-15


def test_single_level_is_a_peak_at_its_energy():
    """A 1 x 1 'Hamiltonian' at E~ = 0.3: the damped expansion of a delta
    peaks at 0.3 (within the grid spacing near that point)."""
    import scipy.sparse as sp
    H = sp.csr_matrix(np.array([[0.3]]))
    mu = kpm.moments(H, 0.0, 1.0, np.ones((1, 1)), 128)
    assert np.allclose(mu, np.cos(np.arange(128) * math.acos(0.3)))
    assert abs(kpm.maxdos_point(mu, n_grid=20000) - 0.3) < 2e-3


def test_stochastic_moments_approach_exact():
    H, E_c, dE, Et = _rescaled_case()
    D = H.shape[0]
    exact = kpm.moments(H, E_c, dE, np.sqrt(D) * np.eye(D), 40)
    rng = np.random.default_rng(0)
    R = rng.standard_normal((D, 400))
    est = kpm.moments(H, E_c, dE, R, 40)
    # standard error of a trace estimate with Gaussian vectors: sqrt(2 Tr T_n^2 / R)
    se = np.sqrt(2.0 * D / 400)
    assert np.max(np.abs(est - exact)) < 5 * se


def test_polfed_with_kpm_dos_vs_dense():
    """The KPM DOS sets the window and, with the maxdos target, the target
    itself; the pairs are still the dense ones nearest the target."""
    from oracle import dense, polfed
    H = models.qrem(10, wl.qrem_energies(10, 2), 1.0)
    D = H.shape[0]
    R = np.random.default_rng(3).standard_normal((D, 20))
    out = polfed.polfed(H, wl.start_vector(D, 2), 20, 0.0, "maxdos", kpm_vectors=R,
                        kpm_moments=64)
    Er, _ = dense.nearest_eigenpairs(H, out["lam"], 20)
    assert np.max(np.abs(out["E"] - Er) / np.maximum(np.abs(Er), 1.0)) <= 1e-10
    # the KPM maximum lies near the Gaussian one for this near-Gaussian DOS
    tr1, tr2 = flt.trace_moments(H)
    assert abs(out["lam"] - tr1) < 0.1 * math.sqrt(tr2 - tr1 * tr1)


def test_splitmix_draws_have_unit_variance_and_differ_per_vector():
    R = wl.splitmix_vectors(20000, 3, 7)
    assert np.all(np.abs(R.mean(axis=0)) < 0.03)
    assert np.all(np.abs(R.var(axis=0) - 1.0) < 0.03)
    assert np.all(np.abs(R) < np.sqrt(3.0))
    assert abs(np.corrcoef(R[:, 0], R[:, 1])[0, 1]) < 0.03
