"""Sector basis of an L-site spin-1/2 (or spinless-fermion) chain with fixed
magnetization / particle number.  TEST INFRASTRUCTURE ONLY.

Convention (the paper leaves it open, App. A names only the U(1) sector):
site j = 1..L is bit j-1 of the state integer; an up spin / occupied site is a
set bit.  The sector with N set bits has dimension binom(L, N) (App. A, U(1)
quantum sun paragraph), and its states are listed in ascending integer order.
The rank of a state is its position in that list.
"""
from __future__ import annotations

import numpy as np


def sector_states(L: int, N: int) -> np.ndarray:
    """All L-bit integers with exactly N set bits, ascending (int64)."""
    if not (0 <= N <= L <= 40):
        raise ValueError("need 0 <= N <= L <= 40")
    everything = np.arange(1 << L, dtype=np.int64)
    keep = np.bitwise_count(everything) == N
    return everything[keep]


def rank(states_sorted: np.ndarray, s) -> np.ndarray:
    """Position of each state of `s` in the ascending sector list.
    Raises if a state is not in the sector."""
    s = np.asarray(s, dtype=np.int64)
    r = np.searchsorted(states_sorted, s)
    r_clip = np.minimum(r, len(states_sorted) - 1)
    if len(states_sorted) == 0 or np.any(states_sorted[r_clip] != s):
        raise ValueError("state outside the sector")
    return r


def unrank(states_sorted: np.ndarray, r) -> np.ndarray:
    return states_sorted[np.asarray(r, dtype=np.int64)]
