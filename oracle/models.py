"""Model Hamiltonians as SciPy CSR matrices, built straight from the model
equations of the paper's Appendix A.  TEST INFRASTRUCTURE ONLY.

Bit convention: site j = 1..L is bit j-1; up spin / occupied site = 1.
S^z = (n - 1/2), S^x S^x + S^y S^y = (S^+ S^- + S^- S^+)/2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis


def _bit(s: np.ndarray, i: int) -> np.ndarray:
    return (s >> i) & 1


def _bonds(L: int, periodic: bool):
    bonds = [(i, i + 1) for i in range(L - 1)]
    if periodic:
        if L < 3:
            raise ValueError("periodic chain needs L >= 3")
        bonds.append((L - 1, 0))
    return bonds


def xxz(L: int, N: int, J: float, Delta: float, h, periodic: bool = True):
    """Random-field XXZ chain, eq. (xxz) of App. A:
        H = J sum_i (S^x_i S^x_{i+1} + S^y_i S^y_{i+1} + Delta S^z_i S^z_{i+1})
            + sum_i h_i S^z_i
    in the sector with N up spins.  Returns (H_csr, states)."""
    h = np.asarray(h, dtype=np.float64)
    assert h.shape == (L,)
    states = basis.sector_states(L, N)
    D = len(states)
    rows = np.arange(D, dtype=np.int64)
    diag = np.zeros(D)
    for i in range(L):
        diag += h[i] * (_bit(states, i) - 0.5)
    r_list, c_list, v_list = [rows], [rows], [None]
    for (i, j) in _bonds(L, periodic):
        bi, bj = _bit(states, i), _bit(states, j)
        diag += J * Delta * (bi - 0.5) * (bj - 0.5)
        flip = bi != bj
        partner = states[flip] ^ ((1 << i) | (1 << j))
        r_list.append(rows[flip])
        c_list.append(basis.rank(states, partner))
        v_list.append(np.full(int(flip.sum()), 0.5 * J))
    v_list[0] = diag
    H = sp.coo_matrix((np.concatenate(v_list),
                       (np.concatenate(r_list), np.concatenate(c_list))),
                      shape=(D, D)).tocsr()
    H.sum_duplicates()
    return H, states


def _occupied_below(s: np.ndarray, site: int) -> np.ndarray:
    return np.bitwise_count(s & ((1 << site) - 1)).astype(np.int64)


def spin_chain(L: int, N: int, Js, Deltas, h, periodic: bool = True):
    """Spin-1/2 chain with couplings of range r = 1..R, eqs. (j1j2) and
    (j1j2j3) of App. A (R = 2, 3; R = 1 is eq. (xxz)):
        H = sum_r J_r sum_i (S^x_i S^x_{i+r} + S^y_i S^y_{i+r} + Delta_r S^z_i S^z_{i+r})
            + sum_i h_i S^z_i
    in the sector with N up spins; periodic bonds wrap around (needs L > 2R).
    Returns (H_csr, states)."""
    h = np.asarray(h, dtype=np.float64)
    Js = [float(x) for x in Js]
    Deltas = [float(x) for x in Deltas]
    assert h.shape == (L,) and len(Js) == len(Deltas) >= 1
    assert not periodic or L > 2 * len(Js)
    states = basis.sector_states(L, N)
    D = len(states)
    rows = np.arange(D, dtype=np.int64)
    diag = np.zeros(D)
    for i in range(L):
        diag += h[i] * (_bit(states, i) - 0.5)
    r_list, c_list, v_list = [rows], [rows], [None]
    for r, (J, Dl) in enumerate(zip(Js, Deltas), start=1):
        for i in range(L):
            j = i + r
            if j >= L:
                if not periodic:
                    continue
                j -= L
            bi, bj = _bit(states, i), _bit(states, j)
            diag += J * Dl * (bi - 0.5) * (bj - 0.5)
            flip = bi != bj
            partner = states[flip] ^ ((1 << i) | (1 << j))
            r_list.append(rows[flip])
            c_list.append(basis.rank(states, partner))
            v_list.append(np.full(int(flip.sum()), 0.5 * J))
    v_list[0] = diag
    H = sp.coo_matrix((np.concatenate(v_list),
                       (np.concatenate(r_list), np.concatenate(c_list))),
                      shape=(D, D)).tocsr()
    H.sum_duplicates()
    return H, states


def fermion_hop_sign(s: np.ndarray, a: int, b: int) -> np.ndarray:
    """Sign of c^dag_a c_b |s> for states with site b occupied and site a empty,
    Jordan-Wigner ordering by site index: c_b picks up (-1)^(#occupied below b),
    then c^dag_a picks up (-1)^(#occupied below a) in the state without b."""
    after = s ^ (1 << b)
    n = _occupied_below(s, b) + _occupied_below(after, a)
    return 1.0 - 2.0 * (n & 1)


def tv(L: int, N: int, t: float, V: float, eps, periodic: bool = True):
    """Spinless fermions with nearest-neighbour hopping and interaction:
        H = -t sum_i (c^dag_i c_{i+1} + h.c.) + V sum_i n_i n_{i+1}
            + sum_i eps_i n_i
    in the sector with N particles (not a model of the paper; the fermion
    signs come from the Jordan-Wigner string).  Returns (H_csr, states)."""
    eps = np.asarray(eps, dtype=np.float64)
    assert eps.shape == (L,)
    states = basis.sector_states(L, N)
    D = len(states)
    rows = np.arange(D, dtype=np.int64)
    diag = np.zeros(D)
    for i in range(L):
        diag += eps[i] * _bit(states, i)
    r_list, c_list, v_list = [rows], [rows], [None]
    for (i, j) in _bonds(L, periodic):
        bi, bj = _bit(states, i), _bit(states, j)
        diag += V * bi * bj
        # c^dag_i c_j on states with j occupied, i empty; and the reverse
        for (a, b) in ((i, j), (j, i)):
            sel = (_bit(states, b) == 1) & (_bit(states, a) == 0)
            src = states[sel]
            dst = src ^ ((1 << a) | (1 << b))
            r_list.append(basis.rank(states, dst))
            c_list.append(rows[sel])
            v_list.append(-t * fermion_hop_sign(src, a, b))
    v_list[0] = diag
    H = sp.coo_matrix((np.concatenate(v_list),
                       (np.concatenate(r_list), np.concatenate(c_list))),
                      shape=(D, D)).tocsr()
    H.sum_duplicates()
    return H, states


def qsun_dot(A: np.ndarray, gamma: float) -> np.ndarray:
    """H_dot = gamma * R'/sqrt(2^N + 1) with R' = (A + A^T)/sqrt(2), App. A
    (quantum sun paragraph): the explicit normalization factor, not a numerical
    one."""
    n = A.shape[0]
    Rp = (A + A.T) / np.sqrt(2.0)
    return gamma * Rp / np.sqrt(n + 1.0)


def qsun(N: int, L: int, A, gamma: float, g0: float, alpha: float, u, n_of_j,
         h):
    """Quantum sun, eq. (qsun) of App. A, full 2^(N+L) space:
        H = H_dot (x) I + g0 sum_j alpha^{u_j} S^x_{n(j)} S^x_j + sum_j h_j S^z_j
    Dot spins occupy the high bits (the dot is the first tensor factor),
    dot spin k is bit L+k, outer spin j = 1..L is bit j-1.  Returns H_csr."""
    A = np.asarray(A, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    n_of_j = np.asarray(n_of_j, dtype=np.int64)
    h = np.asarray(h, dtype=np.float64)
    n_dot = 1 << N
    assert A.shape == (n_dot, n_dot) and u.shape == (L,) and h.shape == (L,)
    Hdot = qsun_dot(A, gamma)
    D = 1 << (N + L)
    idx = np.arange(D, dtype=np.int64)
    d = idx >> L
    o = idx & ((1 << L) - 1)
    r_list, c_list, v_list = [], [], []
    # H_dot (x) I: row (d, o) couples to (d', o) with H_dot[d, d']
    for dp in range(n_dot):
        r_list.append(idx)
        c_list.append((np.int64(dp) << L) | o)
        v_list.append(Hdot[d, dp])
    # outer fields
    diag_f = np.zeros(D)
    for j in range(L):
        diag_f += h[j] * (_bit(idx, j) - 0.5)
    r_list.append(idx)
    c_list.append(idx)
    v_list.append(diag_f)
    # rays: S^x_{n(j)} S^x_j = (1/4) sigma^x sigma^x flips both spins
    for j in range(L):
        g = g0 * alpha ** u[j]
        mask = (1 << (L + int(n_of_j[j]))) | (1 << j)
        r_list.append(idx)
        c_list.append(idx ^ mask)
        v_list.append(np.full(D, 0.25 * g))
    H = sp.coo_matrix((np.concatenate(v_list),
                       (np.concatenate(r_list), np.concatenate(c_list))),
                      shape=(D, D)).tocsr()
    H.sum_duplicates()
    return H


def qrem(L: int, E, Gamma: float):
    """Quantum random energy model, eq. (qrem) of App. A, full 2^L space:
        H = sum_alpha E_alpha |alpha><alpha| - Gamma sum_i sigma^x_i,
    sigma^x_i flipping bit i of the state index.  Returns H_csr."""
    E = np.asarray(E, dtype=np.float64)
    D = 1 << L
    assert E.shape == (D,)
    idx = np.arange(D, dtype=np.int64)
    rows = [idx]
    cols = [idx]
    vals = [E]
    for i in range(L):
        rows.append(idx)
        cols.append(idx ^ (1 << i))
        vals.append(np.full(D, -float(Gamma)))
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(D, D)).tocsr()
    H.sum_duplicates()
    return H


def qrem_rows_apply(L: int, E, Gamma: float, rows: np.ndarray, x: np.ndarray):
    """(H x)[r] of eq. (qrem) for the listed rows only, for checks at sizes
    where the whole matrix is not built."""
    rows = np.asarray(rows, dtype=np.int64)
    out = np.asarray(E, dtype=np.float64)[rows] * x[rows]
    for i in range(L):
        out -= float(Gamma) * x[rows ^ (1 << i)]
    return out


def xxz_rows_apply(L: int, N: int, J: float, Delta: float, h, periodic: bool,
                   states: np.ndarray, rows: np.ndarray, x: np.ndarray):
    """(H x)[r] for the listed rows only, straight from eq. (xxz), for checks
    at sizes where the whole matrix is not built.  `states` is the full
    ascending sector list (basis.sector_states)."""
    h = np.asarray(h, dtype=np.float64)
    s = states[rows]
    diag = np.zeros(len(rows))
    for i in range(L):
        diag += h[i] * (_bit(s, i) - 0.5)
    out = np.zeros(len(rows))
    for (i, j) in _bonds(L, periodic):
        bi, bj = _bit(s, i), _bit(s, j)
        diag += J * Delta * (bi - 0.5) * (bj - 0.5)
        flip = bi != bj
        partner = s[flip] ^ ((1 << i) | (1 << j))
        out[flip] += 0.5 * J * x[basis.rank(states, partner)]
    return out + diag * x[rows]


def tv_rows_apply(L: int, N: int, t: float, V: float, eps, periodic: bool,
                  states: np.ndarray, rows: np.ndarray, x: np.ndarray):
    """(H x)[r] of the t-V Hamiltonian (see `tv`) for the listed rows only,
    for checks at sizes where the whole matrix is not built.  Row state s
    receives c^dag_a c_b from the state s' = s with a and b exchanged when s
    has a occupied and b empty; the amplitude is -t times the Jordan-Wigner
    sign of that hop acting on s'.  `states` is the full ascending sector
    list (basis.sector_states)."""
    eps = np.asarray(eps, dtype=np.float64)
    s = states[rows]
    diag = np.zeros(len(rows))
    for i in range(L):
        diag += eps[i] * _bit(s, i)
    out = np.zeros(len(rows))
    for (i, j) in _bonds(L, periodic):
        diag += V * _bit(s, i) * _bit(s, j)
        for (a, b) in ((i, j), (j, i)):
            sel = (_bit(s, a) == 1) & (_bit(s, b) == 0)
            src = s[sel] ^ ((1 << a) | (1 << b))
            out[sel] += -t * fermion_hop_sign(src, a, b) * x[basis.rank(states, src)]
    return out + diag * x[rows]


def is_symmetric(H, tol: float = 0.0) -> bool:
    diff = (H - H.T).tocsr()
    if diff.nnz == 0:
        return True
    return float(np.max(np.abs(diff.data))) <= tol
