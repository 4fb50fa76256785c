"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms
printed in the paper, textbook spectra, a brute-force Kronecker construction of
the same operators, identities of Chebyshev sums, and full dense
diagonalization.  No GPU is used.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import basis, dense, lanczos, models, polfed
from oracle import filter as flt
from tests import kron_models as km


@pytest.fixture(scope="module")
def consts(golden_dir):
    with open(os.path.join(golden_dir, "paper_constants.json")) as f:
        return json.load(f)


# ---------------------------------------------------------------- basis ----

@pytest.mark.parametrize("L,N", [(1, 0), (1, 1), (6, 3), (10, 3), (12, 6),
                                 (13, 5), (16, 8)])
def test_sector_is_the_set_of_N_subsets(L, N):
    st = basis.sector_states(L, N)
    assert len(st) == math.comb(L, N)
    ref = sorted(sum(1 << p for p in c)
                 for c in itertools.combinations(range(L), N))
    assert st.tolist() == ref


def test_sector_dimensions_match_paper(consts):
    vals = consts["sector_dimension_halffilling"]["values"]
    for L_str, D in vals.items():
        L = int(L_str)
        assert math.comb(L, L // 2) == D
        if L <= 24:
            assert len(basis.sector_states(L, L // 2)) == D


def test_rank_unrank_roundtrip():
    st = basis.sector_states(14, 7)
    r = np.arange(len(st))
    assert np.array_equal(basis.rank(st, basis.unrank(st, r)), r)
    with pytest.raises(ValueError):
        basis.rank(st, [0b1])


# --------------------------------------------------------------- models ----

@pytest.mark.parametrize("L,N,periodic", [(8, 4, True), (8, 3, True),
                                          (7, 3, False), (6, 2, True)])
def test_xxz_equals_kronecker_construction(L, N, periodic):
    h = wl.xxz_fields(L, 2.0, 11)
    H, st = models.xxz(L, N, 1.3, 0.7, h, periodic)
    ref = km.project(km.xxz_full(L, 1.3, 0.7, h, periodic),
                     km.sector_list(L, N))
    assert np.max(np.abs(H.toarray() - ref)) < 1e-14


@pytest.mark.parametrize("L,N,periodic", [(8, 4, True), (8, 3, True),
                                          (7, 3, True), (7, 2, False)])
def test_tv_equals_jordan_wigner_kronecker(L, N, periodic):
    eps = wl.tv_onsite(L, 5)
    H, st = models.tv(L, N, 0.9, 1.4, eps, periodic)
    ref = km.project(km.tv_full(L, 0.9, 1.4, eps, periodic),
                     km.sector_list(L, N))
    assert np.max(np.abs(H.toarray() - ref)) < 1e-14


def test_qsun_equals_kronecker_construction():
    N, L = 2, 4
    q = wl.qsun_draws(N, L, 3)
    H = models.qsun(N, L, q["A"], 1.0, 1.0, 0.75, q["u"], q["n_of_j"], q["h"])
    Hdot = models.qsun_dot(q["A"], 1.0)
    g = 1.0 * 0.75 ** q["u"]
    ref = km.qsun_full(N, L, Hdot, g, q["n_of_j"], q["h"])
    assert np.max(np.abs(H.toarray() - ref)) < 1e-14


def test_models_are_symmetric():
    H, _ = models.xxz(12, 6, 1.0, 1.0, wl.xxz_fields(12, 1.0, 0))
    assert models.is_symmetric(H)
    H, _ = models.tv(12, 5, 1.0, 1.0, wl.tv_onsite(12, 0))
    assert models.is_symmetric(H)
    q = wl.qsun_draws(3, 6, 0)
    H = models.qsun(3, 6, q["A"], 1.0, 1.0, 0.75, q["u"], q["n_of_j"], q["h"])
    assert models.is_symmetric(H, 1e-15)


def test_xxz_offdiagonal_count_closed_form(consts):
    tot = consts["xxz_offdiag_per_row_halffilling_pbc"]["total_offdiag_nnz"]
    for L_str, n_off in tot.items():
        L = int(L_str)
        H, _ = models.xxz(L, L // 2, 1.0, 1.0, wl.xxz_fields(L, 1.0, 0))
        off = H - sp.diags(H.diagonal())
        off.eliminate_zeros()
        assert off.nnz == n_off
        assert off.nnz == len(_) * L * L // (2 * (L - 1))


def test_qsun_nnz_per_row(consts):
    N, L = 3, 13
    q = wl.qsun_draws(N, L, 0)
    H = models.qsun(N, L, q["A"], 1.0, 1.0, 0.75, q["u"], q["n_of_j"], q["h"])
    per_row = np.diff(H.indptr)
    assert np.all(per_row == consts["qsun_nnz_per_row"]["value_N3_L13"])


@pytest.mark.parametrize("L,N", [(10, 5), (12, 6), (10, 4), (9, 4)])
def test_xx_chain_is_free_fermions(L, N):
    """Delta = 0, h = 0: Jordan-Wigner gives free fermions with dispersion
    J cos k; the spin ring maps to a fermion ring that is periodic for odd N
    and antiperiodic for even N."""
    J = 1.0
    H, _ = models.xxz(L, N, J, 0.0, np.zeros(L))
    phi = 0.0 if N % 2 == 1 else 0.5
    eps = J * np.cos(2 * np.pi * (np.arange(L) + phi) / L)
    ref = sorted(sum(eps[list(c)]) for c in itertools.combinations(range(L), N))
    assert np.allclose(np.sort(dense.spectrum(H)), ref, atol=1e-12)


@pytest.mark.parametrize("L,N", [(10, 5), (10, 4), (9, 4)])
def test_tv_without_interaction_is_free_fermions(L, N):
    """V = 0, eps = 0: sums of N distinct -2t cos(2 pi m / L) (the fermion
    ring is periodic whatever N; the Jordan-Wigner sign makes it so)."""
    t = 0.8
    H, _ = models.tv(L, N, t, 0.0, np.zeros(L))
    eps = -2 * t * np.cos(2 * np.pi * np.arange(L) / L)
    ref = sorted(sum(eps[list(c)]) for c in itertools.combinations(range(L), N))
    assert np.allclose(np.sort(dense.spectrum(H)), ref, atol=1e-12)


@pytest.mark.parametrize("L", [6, 9, 12])
def test_single_magnon_dispersion(L):
    """One up spin in an XXZ ring: E(k) = J Delta (L - 4)/4 + J cos k."""
    J, Delta = 1.1, 0.6
    H, _ = models.xxz(L, 1, J, Delta, np.zeros(L))
    ref = J * Delta * (L - 4) / 4 + J * np.cos(2 * np.pi * np.arange(L) / L)
    assert np.allclose(np.sort(dense.spectrum(H)), np.sort(ref), atol=1e-13)


def test_heisenberg_four_site_ring(consts):
    H, _ = models.xxz(4, 2, 1.0, 1.0, np.zeros(4))
    e0 = consts["heisenberg_ring4_ground_energy_per_J"]["value"]
    assert abs(dense.spectrum(H)[0] - e0) < 1e-13


def test_qsun_decoupled_limit():
    """g0 = 0: eigenvalues are eig(H_dot) + sum_j h_j m_j, m_j = +-1/2."""
    N, L = 3, 5
    q = wl.qsun_draws(N, L, 7)
    H = models.qsun(N, L, q["A"], 1.0, 0.0, 0.75, q["u"], q["n_of_j"], q["h"])
    ed = np.linalg.eigvalsh(models.qsun_dot(q["A"], 1.0))
    ms = [np.dot(q["h"], np.array(m)) for m in
          itertools.product((-0.5, 0.5), repeat=L)]
    ref = np.sort(np.add.outer(ed, ms).ravel())
    assert np.allclose(np.sort(dense.spectrum(H)), ref, atol=1e-13)


def test_qsun_dot_normalization():
    """Hilbert-Schmidt norm of R_dot is one on average (App. A):
    E[Tr R'^2] = n (n + 1) for R' = (A + A^T)/sqrt 2."""
    n_dot = 1 << 8
    vals = []
    for seed in range(6):
        A = np.random.default_rng(seed).standard_normal((n_dot, n_dot))
        Hd = models.qsun_dot(A, 1.0)
        vals.append(np.trace(Hd @ Hd) / n_dot)
    assert abs(np.mean(vals) - 1.0) < 0.02


# ------------------------------------------------------- filter and K ----

def test_chebyshev_recurrence_is_cos():
    th = np.linspace(0.01, np.pi - 0.01, 37)
    T = flt.chebyshev_T(200, np.cos(th))
    k = np.arange(201)[:, None]
    assert np.max(np.abs(T - np.cos(k * th[None, :]))) < 1e-12


def _dirichlet(K, u):
    u = np.asarray(u, dtype=np.float64)
    out = np.empty_like(u)
    small = np.abs(np.sin(u / 2)) < 1e-12
    out[small] = 2 * K + 1
    out[~small] = np.sin((K + 0.5) * u[~small]) / np.sin(u[~small] / 2)
    return out


@pytest.mark.parametrize("lam_t,K", [(0.0, 10), (0.3, 57), (-0.62, 200),
                                     (0.5, 1000)])
def test_filter_closed_form(lam_t, K):
    """sum_n c_n T_n(cos t) = [D_K(t - phi) + D_K(t + phi)]/2 with the
    Dirichlet kernel D_K(u) = sin((K+1/2)u)/sin(u/2) and phi = arccos lam~,
    so P(cos t) = [D_K(t-phi) + D_K(t+phi)] / [D_K(0) + D_K(2 phi)]."""
    phi = math.acos(lam_t)
    th = np.linspace(0.0, np.pi, 301)
    ref = (_dirichlet(K, th - phi) + _dirichlet(K, th + phi)) / (
        _dirichlet(K, np.array([0.0]))[0] + _dirichlet(K, np.array([2 * phi]))[0])
    got = flt.filter_value(np.cos(th), lam_t, K)
    assert np.max(np.abs(got - ref)) < 1e-11
    assert abs(float(flt.filter_value(lam_t, lam_t, K)) - 1.0) < 1e-13


def test_clenshaw_scalar_equals_direct_sum():
    rng = np.random.default_rng(0)
    for K in (1, 5, 64, 999):
        a = rng.standard_normal(K + 1)
        for x in (-1.0, -0.37, 0.0, 0.81, 1.0):
            direct = float(np.dot(a, flt.chebyshev_T(K, x)))
            assert abs(flt.clenshaw_scalar(a, x) - direct) < 1e-10 * max(
                1.0, np.sum(np.abs(a)))


def test_matrix_clenshaw_on_diagonal_operator():
    """With H = diag(E) the filtered vector is P(E~_i) v_i exactly."""
    rng = np.random.default_rng(1)
    E = rng.uniform(-3.0, 5.0, 400)
    E_c, dE = flt.rescale(-3.0001, 5.0001)
    lam_t, K = 0.21, 150
    a = flt.coefficients(lam_t, K)
    v = rng.standard_normal(400)
    w = flt.apply_filter(sp.diags(E).tocsr(), E_c, dE, a, v)
    phi, th = math.acos(lam_t), np.arccos((E - E_c) / dE)
    P = (_dirichlet(K, th - phi) + _dirichlet(K, th + phi)) / (
        _dirichlet(K, np.array([0.0]))[0] + _dirichlet(K, np.array([2 * phi]))[0])
    assert np.max(np.abs(w - P * v)) < 1e-11


@pytest.mark.parametrize("lam_t", [0.0, 0.3, -0.5])
@pytest.mark.parametrize("delta", [1e-3, 1e-4])
def test_K_bisection_matches_semi_analytic_rule(lam_t, delta, consts):
    K = flt.choose_K(lam_t, delta)
    c = consts["K_approx_coefficient"]["value"]
    K0 = c * math.sqrt(1 - lam_t ** 2) / delta
    assert abs(K - K0) <= 3
    # K is the largest order whose window edges stay at or above the cutoff
    pts = np.array([lam_t - delta, lam_t + delta])
    assert np.min(flt.filter_value(pts, lam_t, K)) >= flt.OMEGA_DEFAULT
    assert np.min(flt.filter_value(pts, lam_t, K + 1)) < flt.OMEGA_DEFAULT


def test_omega_lies_between_side_lobes():
    """The cutoff sits above the first positive side lobe of sinc and below
    the main lobe (Sec. 3.2)."""
    z = np.linspace(4.0, 9.0, 20001)
    lobe = np.max(np.sin(z) / z)
    assert lobe < flt.OMEGA_DEFAULT < 1.0


def test_expected_krylov_dim(consts):
    c = consts["expectedkrylovdim"]
    assert flt.expected_krylov_dim(100, 1, 1.5) == math.ceil(
        (c["per_block"] + c["per_eigenpair"] * 100) * 1.5) == 286
    assert flt.expected_krylov_dim(50, 4, 1.0) == math.ceil(
        c["per_block"] * 4 + c["per_eigenpair"] * 50)


def test_trace_moments_are_spectral_moments():
    H, _ = models.xxz(10, 5, 1.0, 1.0, wl.xxz_fields(10, 3.0, 2))
    ev = dense.spectrum(H)
    m1, m2 = flt.trace_moments(H)
    assert abs(m1 - ev.mean()) < 1e-12
    assert abs(m2 - np.mean(ev ** 2)) < 1e-12


def test_gaussian_dos_normalization():
    x = np.linspace(-3, 3, 600001)
    rho = flt.gaussian_dos(x, 1000, 0.05, 0.2)
    assert abs(np.trapezoid(rho, x) - 1000) < 1e-3


# -------------------------------------------------------------- Lanczos ----

def test_lanczos_basis_orthonormal_and_relation():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((300, 300))
    A = A + A.T

    def op(v):
        return A @ v
    m = 60
    V = np.zeros((300, m + 1))
    V[:, 0] = rng.standard_normal(300)
    V[:, 0] /= np.linalg.norm(V[:, 0])
    al, be = [], [0.0]
    for k in range(m):
        a, b, w = lanczos.lanczos_step(op, V, k, be[k])
        al.append(a)
        be.append(b)
        V[:, k + 1] = w / b
    assert np.max(np.abs(V.T @ V - np.eye(m + 1))) < 1e-13
    T = np.diag(al) + np.diag(be[1:m], 1) + np.diag(be[1:m], -1)
    R = A @ V[:, :m] - V[:, :m] @ T
    R[:, m - 1] -= be[m] * V[:, m]
    assert np.max(np.abs(R)) < 1e-11 * np.linalg.norm(A, 2)


def test_spectral_extremes_match_dense():
    H, _ = models.xxz(14, 7, 1.0, 1.0, wl.xxz_fields(14, 1.0, 0))
    lo, hi = lanczos.spectral_extremes(H)
    ev = dense.spectrum(H)
    assert abs(lo - ev[0]) < 1e-10 and abs(hi - ev[-1]) < 1e-10


def _check_vs_dense(H, out, n_ev):
    Er, Ur = dense.nearest_eigenpairs(H, out["lam"], n_ev)
    assert len(out["E"]) == n_ev
    rel = np.abs(out["E"] - Er) / np.maximum(np.abs(Er), 1.0)
    assert np.max(rel) <= 1e-10
    assert np.max(out["res"]) <= 1e-8
    ov = np.abs(np.sum(out["U"] * Ur, axis=0))
    assert np.min(ov) >= 1 - 1e-8


def test_polfed_xxz_L12_vs_dense():
    """Workload: XXZ L=12, J=Delta=1, h ~ U[-1,1] seed 0, 20 pairs at
    normalized energy 0.5."""
    H, _ = models.xxz(12, 6, 1.0, 1.0, wl.xxz_fields(12, 1.0, 0))
    out = polfed.polfed(H, wl.start_vector(H.shape[0], 0), 20, 0.5,
                        "normalized")
    _check_vs_dense(H, out, 20)


def test_polfed_result_independent_of_start_vector():
    H, _ = models.xxz(12, 6, 1.0, 1.0, wl.xxz_fields(12, 1.0, 0))
    o1 = polfed.polfed(H, wl.start_vector(924, 1), 20, 0.5, "normalized")
    o2 = polfed.polfed(H, wl.start_vector(924, 2), 20, 0.5, "normalized")
    assert np.max(np.abs(o1["E"] - o2["E"])) < 1e-10


def test_polfed_tv_and_qsun_vs_dense():
    H, _ = models.tv(12, 6, 1.0, 1.0, wl.tv_onsite(12, 1))
    out = polfed.polfed(H, wl.start_vector(H.shape[0], 1), 20, 0.5,
                        "normalized")
    _check_vs_dense(H, out, 20)
    q = wl.qsun_draws(3, 7, 2)
    H = models.qsun(3, 7, q["A"], 1.0, 1.0, 0.75, q["u"], q["n_of_j"], q["h"])
    out = polfed.polfed(H, wl.start_vector(H.shape[0], 2), 20, 0.5,
                        "normalized")
    _check_vs_dense(H, out, 20)


def test_polfed_off_center_target():
    H, _ = models.xxz(12, 6, 1.0, 1.0, wl.xxz_fields(12, 3.0, 4))
    out = polfed.polfed(H, wl.start_vector(924, 4), 15, 0.3, "rescaled")
    _check_vs_dense(H, out, 15)


# --------------------------------------- planted mistakes must be caught ----

def test_planted_coefficient_mistake_is_caught(monkeypatch):
    """A wrong c_0 (2 instead of 1) in the oracle breaks the closed-form pin."""
    orig = flt.coefficients

    def bad(lam_t, K):
        a = orig(lam_t, K)
        a = a.copy()
        a[0] *= 2.0
        return a / (1.0 + a[0] / 2 - a[0] / 2)
    monkeypatch.setattr(flt, "coefficients", bad)
    with pytest.raises(AssertionError):
        test_filter_closed_form(0.3, 57)


def test_planted_boundary_sign_mistake_is_caught(monkeypatch):
    """Dropping the Jordan-Wigner string breaks the free-fermion pin for even
    particle number."""
    monkeypatch.setattr(models, "fermion_hop_sign",
                        lambda s, a, b: np.ones(len(s)))
    with pytest.raises(AssertionError):
        test_tv_without_interaction_is_free_fermions(10, 4)


def test_select_nearest_does_not_skip_an_unconverged_nearer_pair():
    """The selection takes the n_ev Ritz pairs nearest lambda and returns only
    their leading accepted run: a nearer pair that has not converged yet
    stops it (a farther accepted pair never takes its place); equal
    distances are ordered by E."""
    from oracle import lanczos
    E = np.array([0.1, -0.05, 0.3, 0.2, -0.1])
    res = np.array([1e-9, 1e-6, 1e-9, 1e-9, 1e-9])
    assert lanczos.select_nearest(E, res, 0.0, 3, 1e-8).tolist() == []
    res[1] = 1e-9
    assert lanczos.select_nearest(E, res, 0.0, 3, 1e-8).tolist() == [1, 4, 0]
    res[0] = 1e-7  # the third nearest (0.1) unconverged: the run stops there
    assert lanczos.select_nearest(E, res, 0.0, 4, 1e-8).tolist() == [1, 4]
    res[0] = 1e-9
    assert lanczos.select_nearest(E, res, 0.0, 10, 1e-8).tolist() == [1, 4, 0, 3, 2]
