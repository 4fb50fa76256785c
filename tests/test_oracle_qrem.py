"""Pins of the oracle's quantum random energy model (eq. qrem of App. A) and
of the maxdos / offset targets (Sec. 5.4): a Kronecker-product construction,
the closed-form spectrum of the transverse field alone, the trace moments,
the peak of the Gaussian DOS estimate, and a full POLFED solve at the DOS
maximum against dense diagonalization."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import dense, models, polfed
from oracle import filter as flt
from tests import kron_models as km


def test_qrem_equals_kronecker_construction():
    L, G = 6, 0.7
    E = wl.qrem_energies(L, 3)
    H = models.qrem(L, E, G).toarray()
    ref = np.diag(E)
    for i in range(L):
        ref = ref - G * km.site_op(2.0 * km.SX, i, L)
    assert np.array_equal(H, ref)


@pytest.mark.parametrize("L", [5, 8])
def test_transverse_field_spectrum(L):
    """E = 0: H = -Gamma sum_i sigma^x_i has eigenvalues -Gamma (L - 2k) with
    multiplicity binom(L, k)."""
    G = 1.3
    H = models.qrem(L, np.zeros(1 << L), G).toarray()
    ev = np.linalg.eigvalsh(H)
    ref = np.sort(np.concatenate([np.full(math.comb(L, k), -G * (L - 2 * k))
                                  for k in range(L + 1)]))
    assert np.max(np.abs(ev - ref)) < 1e-12


def test_qrem_trace_moments_closed_form():
    """Tr H / D = mean E; Tr H^2 / D = mean E^2 + L Gamma^2 (L off-diagonal
    entries of magnitude Gamma per row)."""
    L, G = 10, 1.0
    E = wl.qrem_energies(L, 5)
    tr1, tr2 = flt.trace_moments(models.qrem(L, E, G))
    assert abs(tr1 - E.mean()) < 1e-12
    assert abs(tr2 - (np.mean(E * E) + L * G * G)) < 1e-10


def test_qrem_energy_statistics():
    """The draws have mean 0 and standard deviation sqrt(L/2) (App. A)."""
    E = wl.qrem_energies(16, 0)
    assert abs(E.mean()) < 5 * math.sqrt(8.0) / math.sqrt(E.size)
    assert abs(E.std() / math.sqrt(8.0) - 1.0) < 0.01


def test_maxdos_is_the_peak_of_the_gaussian_estimate():
    H = models.qrem(10, wl.qrem_energies(10, 1), 1.0)
    tr1, tr2 = flt.trace_moments(H)
    E_min, E_max = -20.0, 20.0
    lam = polfed.target_energy("maxdos", 0.0, E_min, E_max, tr1)
    E_c, dE = flt.rescale(E_min, E_max)
    mu_t, G_t = (tr1 - E_c) / dE, math.sqrt(tr2 - tr1 * tr1) / dE
    x = np.linspace(-1, 1, 200001)
    peak = x[np.argmax(flt.gaussian_dos(x, H.shape[0], mu_t, G_t))]
    assert abs((lam - E_c) / dE - peak) <= 1e-5


def test_offset_target_interpolates_between_maxdos_and_edges():
    E_min, E_max, mean = -10.0, 30.0, 4.0
    E_c, dE = flt.rescale(E_min, E_max)
    at = lambda eta: (polfed.target_energy("offset", eta, E_min, E_max, mean) - E_c) / dE
    em = (mean - E_c) / dE
    assert abs(at(0.0) - em) < 1e-15
    assert abs(at(1.0) - 1.0) < 1e-15 and abs(at(-1.0) + 1.0) < 1e-15
    assert abs(at(0.5) - 0.5 * (em + 1.0)) < 1e-15
    assert abs(at(-0.25) - (em - 0.25 * (1.0 + em))) < 1e-15


def test_polfed_qrem_at_maxdos_vs_dense():
    """Workload: QREM L=10, Gamma=1, energies seed 2, 20 pairs at the DOS
    maximum."""
    H = models.qrem(10, wl.qrem_energies(10, 2), 1.0)
    out = polfed.polfed(H, wl.start_vector(1024, 2), 20, 0.0, "maxdos")
    tr1, _ = flt.trace_moments(H)
    assert abs(out["lam"] - tr1) < 1e-15
    Er, Ur = dense.nearest_eigenpairs(H, out["lam"], 20)
    assert np.max(np.abs(out["E"] - Er) / np.maximum(np.abs(Er), 1.0)) <= 1e-10
    assert np.max(out["res"]) <= 1e-8
