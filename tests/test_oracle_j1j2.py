"""Pins of the oracle's J1-J2 and J1-J2-J3 chains (App. A eqs. j1j2,
j1j2j3): a Kronecker-product construction, the reduction to the XXZ chain,
SU(2) symmetry at Delta = 1 without fields, and the off-diagonal count."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import models
from tests import kron_models as km


@pytest.mark.parametrize("R,periodic", [(2, True), (3, True), (2, False), (3, False)])
def test_spin_chain_equals_kronecker_construction(R, periodic):
    L, N = 8, 4
    Js, Ds = [1.0, 0.5, 0.3][:R], [1.0, 0.7, 1.3][:R]
    h = wl.xxz_fields(L, 1.0, 2)
    H, st = models.spin_chain(L, N, Js, Ds, h, periodic)
    ref = km.project(km.spin_chain_full(L, Js, Ds, h, periodic), st)
    assert np.max(np.abs(H.toarray() - ref)) < 1e-14


def test_range_one_is_the_xxz_chain():
    L, N = 12, 6
    h = wl.xxz_fields(L, 3.0, 0)
    H1, _ = models.spin_chain(L, N, [1.0], [1.0], h, True)
    H2, _ = models.xxz(L, N, 1.0, 1.0, h, True)
    assert abs(H1 - H2).max() == 0.0


def test_su2_multiplets_without_fields():
    """Delta_r = 1, h = 0: H commutes with total S^2, so the Sz = 0 sector
    (L = 10) holds every multiplet and the Sz = 1 sector each of those with
    S >= 1: its spectrum is a sub-multiset of the Sz = 0 spectrum."""
    L = 10
    H0, _ = models.spin_chain(L, L // 2, [1.0, 0.5], [1.0, 1.0], np.zeros(L), True)
    H1, _ = models.spin_chain(L, L // 2 + 1, [1.0, 0.5], [1.0, 1.0], np.zeros(L), True)
    e0 = np.linalg.eigvalsh(H0.toarray())
    e1 = np.linalg.eigvalsh(H1.toarray())
    assert len(e0) - len(e1) == math.comb(L, L // 2) - math.comb(L, L // 2 + 1)
    # every Sz = 1 level appears among the Sz = 0 levels
    assert np.max(np.min(np.abs(e1[:, None] - e0[None, :]), axis=1)) < 1e-10


def test_offdiagonal_count_closed_form():
    """Each bond (i, i + r) flips the rows whose two bits differ: over the
    sector that is 2 binom(L - 2, N - 1) rows per bond."""
    L, N = 12, 6
    H, _ = models.spin_chain(L, N, [1.0, 0.5, 0.25], [1.0, 1.0, 1.0], np.zeros(L), True)
    off = H.nnz - H.shape[0]
    assert off == 3 * L * 2 * math.comb(L - 2, N - 1)
