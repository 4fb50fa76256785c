"""Pins of the oracle's row-by-row helpers (models.xxz_rows_apply,
tv_rows_apply, qrem_rows_apply) against the whole oracle matrices on every
row.  The helpers are the reference of the full-size step tests, where the
whole matrix is not built; a wrong bond, boundary term, sign or diagonal in a
helper fails here.  The matrices themselves are pinned in
test_oracle_pins.py (dense spectra, free fermions, the t-V/XXZ mapping)."""
import numpy as np
import pytest

import workloads as wl
from oracle import basis, models


def _all_rows_equal(ref, got):
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("L,N", [(8, 4), (9, 3), (11, 5), (12, 6), (13, 7), (16, 8)])
@pytest.mark.parametrize("periodic", [True, False])
def test_xxz_rows_apply_equals_matrix_on_all_rows(L, N, periodic):
    h = wl.xxz_fields(L, 3.0, L)
    J, Delta = 1.3, 0.7
    H, st = models.xxz(L, N, J, Delta, h, periodic)
    x = np.random.default_rng(L).standard_normal(H.shape[0])
    rows = np.arange(H.shape[0])
    _all_rows_equal(H @ x, models.xxz_rows_apply(L, N, J, Delta, h, periodic, st, rows, x))
    # an unsorted subset with repeats gives the same rows
    sub = np.random.default_rng(1).integers(0, H.shape[0], 300)
    _all_rows_equal((H @ x)[sub],
                    models.xxz_rows_apply(L, N, J, Delta, h, periodic, st, sub, x))


@pytest.mark.parametrize("L,N", [(8, 4), (9, 4), (10, 3), (12, 6), (13, 6), (16, 8)])
@pytest.mark.parametrize("periodic", [True, False])
def test_tv_rows_apply_equals_matrix_on_all_rows(L, N, periodic):
    """Odd and even particle numbers: the periodic hop's Jordan-Wigner sign
    is (-1)^(N-1), so both signs of the boundary term are covered."""
    eps = wl.tv_onsite(L, L)
    t, V = 1.1, 0.9
    H, st = models.tv(L, N, t, V, eps, periodic)
    x = np.random.default_rng(L + 1).standard_normal(H.shape[0])
    rows = np.arange(H.shape[0])
    _all_rows_equal(H @ x, models.tv_rows_apply(L, N, t, V, eps, periodic, st, rows, x))


@pytest.mark.parametrize("L", [4, 8, 11, 14])
def test_qrem_rows_apply_equals_matrix_on_all_rows(L):
    E = wl.qrem_energies(L, L)
    Gamma = 0.8
    H = models.qrem(L, E, Gamma)
    x = np.random.default_rng(L).standard_normal(H.shape[0])
    rows = np.arange(H.shape[0])
    _all_rows_equal(H @ x, models.qrem_rows_apply(L, E, Gamma, rows, x))


def test_rows_helpers_catch_a_planted_boundary_mistake():
    """A helper that drops the periodic bond differs from the periodic matrix
    on the rows that bond touches: the comparison above can see such a
    mistake."""
    L, N = 10, 5
    h = wl.xxz_fields(L, 1.0, 0)
    H, st = models.xxz(L, N, 1.0, 1.0, h, True)
    x = np.random.default_rng(0).standard_normal(H.shape[0])
    rows = np.arange(H.shape[0])
    wrong = models.xxz_rows_apply(L, N, 1.0, 1.0, h, False, st, rows, x)
    assert np.max(np.abs(wrong - H @ x)) > 1e-3
    eps = wl.tv_onsite(L, 0)
    Ht, stt = models.tv(L, N, 1.0, 1.0, eps, True)
    wrong = models.tv_rows_apply(L, N, -1.0, 1.0, eps, True, stt, rows, x)
    assert np.max(np.abs(wrong - Ht @ x)) > 1e-3


def test_tv_rows_apply_at_full_config_size_matches_a_direct_row_sum():
    """At the t-V configuration's size (L = 26, N = 13, D = 10,400,600) a few
    rows against a direct per-row sum over the model's terms written with
    Python integers (no NumPy bit tricks): hops with their Jordan-Wigner
    string counted site by site."""
    L, N = 26, 13
    st = basis.sector_states(L, N)
    eps = wl.tv_onsite(L, 0)
    x = np.random.default_rng(2).standard_normal(len(st))
    rows = np.array([0, 1, 77, 123456, 5_000_000, len(st) - 1])
    got = models.tv_rows_apply(L, N, 1.0, 1.0, eps, True, st, rows, x)
    for k, r in enumerate(rows):
        s = int(st[r])
        occ = [(s >> i) & 1 for i in range(L)]
        val = sum(eps[i] * occ[i] for i in range(L)) * x[r]
        for i in range(L):
            j = (i + 1) % L
            val += 1.0 * occ[i] * occ[j] * x[r]
            for (a, b) in ((i, j), (j, i)):
                if occ[a] == 1 and occ[b] == 0:
                    src = s ^ (1 << a) ^ (1 << b)
                    # c^dag_a c_b |src>: c_b passes the occupied sites below b
                    # of src, c^dag_a those below a of src without b
                    n = sum((src >> q) & 1 for q in range(b))
                    n += sum(((src ^ (1 << b)) >> q) & 1 for q in range(a))
                    sign = -1.0 if n % 2 else 1.0
                    val += -1.0 * sign * x[int(np.searchsorted(st, src))]
        assert abs(got[k] - val) <= 1e-12 * max(1.0, abs(val))
