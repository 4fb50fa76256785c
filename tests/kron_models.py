"""Brute-force model Hamiltonians from Kronecker products of single-site
matrices, for tiny chains.  Used only to pin the oracle's bit-manipulation
builders: a different construction of the same operators.

Single-site basis: index 0 = down / empty, index 1 = up / occupied.  The
operator on site i (bit i of the state index) is
kron(I_{2^(L-1-i)}, op, I_{2^i}).
"""
import numpy as np

I2 = np.eye(2)
SP = np.array([[0.0, 0.0], [1.0, 0.0]])       # S^+ = |1><0|
SM = SP.T                                       # S^-
SZ = np.diag([-0.5, 0.5])
SX = 0.5 * (SP + SM)
ANNIH = np.array([[0.0, 1.0], [0.0, 0.0]])     # a = |0><1|
ZSTR = np.diag([1.0, -1.0])                     # (-1)^n


def site_op(op, i, L):
    return np.kron(np.kron(np.eye(1 << (L - 1 - i)), op), np.eye(1 << i))


def sector_list(L, N):
    return [s for s in range(1 << L) if bin(s).count("1") == N]


def project(Hfull, states):
    idx = np.asarray(states, dtype=np.int64)
    return Hfull[np.ix_(idx, idx)]


def bonds(L, periodic):
    b = [(i, i + 1) for i in range(L - 1)]
    if periodic:
        b.append((L - 1, 0))
    return b


def xxz_full(L, J, Delta, h, periodic=True):
    D = 1 << L
    H = np.zeros((D, D))
    for (i, j) in bonds(L, periodic):
        H += J * 0.5 * (site_op(SP, i, L) @ site_op(SM, j, L)
                        + site_op(SM, i, L) @ site_op(SP, j, L))
        H += J * Delta * site_op(SZ, i, L) @ site_op(SZ, j, L)
    for i in range(L):
        H += h[i] * site_op(SZ, i, L)
    return H


def spin_chain_full(L, Js, Deltas, h, periodic=True):
    """Couplings of range r = 1..R, full 2^L space, from Kronecker products."""
    D = 1 << L
    H = np.zeros((D, D))
    for r, (J, Dl) in enumerate(zip(Js, Deltas), start=1):
        for i in range(L):
            j = i + r
            if j >= L:
                if not periodic:
                    continue
                j -= L
            H += J * 0.5 * (site_op(SP, i, L) @ site_op(SM, j, L)
                            + site_op(SM, i, L) @ site_op(SP, j, L))
            H += J * Dl * site_op(SZ, i, L) @ site_op(SZ, j, L)
    for i in range(L):
        H += h[i] * site_op(SZ, i, L)
    return H


def fermion_c(i, L):
    """Jordan-Wigner annihilator: string of (-1)^n over sites below i."""
    op = np.eye(1)
    for k in range(L - 1, -1, -1):
        if k > i:
            f = I2
        elif k == i:
            f = ANNIH
        else:
            f = ZSTR
        op = np.kron(op, f)
    return op


def tv_full(L, t, V, eps, periodic=True):
    D = 1 << L
    H = np.zeros((D, D))
    c = [fermion_c(i, L) for i in range(L)]
    n = [ci.T @ ci for ci in c]
    for (i, j) in bonds(L, periodic):
        H += -t * (c[i].T @ c[j] + c[j].T @ c[i])
        H += V * n[i] @ n[j]
    for i in range(L):
        H += eps[i] * n[i]
    return H


def qsun_full(N, L, Hdot, g, n_of_j, h):
    """Dot = first tensor factor (high bits), outer spin j = bit j."""
    Dd = 1 << N
    H = np.kron(Hdot, np.eye(1 << L))
    tot = N + L
    for j in range(L):
        H += g[j] * site_op(SX, L + int(n_of_j[j]), tot) @ site_op(SX, j, tot)
        H += h[j] * site_op(SZ, j, tot)
    assert H.shape == (Dd << L, Dd << L)
    return H
