"""Dense reference: the plain definition of the result POLFED computes -- the
N_ev eigenpairs of H with the smallest |E - lambda| (Sec. 4.6 problem
statement) -- by full diagonalization.  TEST INFRASTRUCTURE ONLY; for
dimensions up to a few thousand."""
from __future__ import annotations

import numpy as np


def nearest_eigenpairs(H, lam: float, n_ev: int):
    """Returns (E, U) ordered by (|E - lam|, E), U with unit columns."""
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    E, U = np.linalg.eigh(Hd)
    order = np.lexsort((E, np.abs(E - lam)))[:n_ev]
    return E[order], U[:, order]


def spectrum(H) -> np.ndarray:
    Hd = H.toarray() if hasattr(H, "toarray") else np.asarray(H)
    return np.linalg.eigvalsh(Hd)
