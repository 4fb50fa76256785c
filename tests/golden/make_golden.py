"""Writes the stored expected values under tests/golden/ from the CPU oracle
only.  Run from the repository root:  python tests/golden/make_golden.py"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wl  # noqa: E402
from oracle import dense, lanczos, models, polfed  # noqa: E402


def xxz_l12():
    """Random-field XXZ L=12, PBC, J=1, Delta=1, h ~ U[-1,1] (seed 0),
    Sz=0 sector (dim 924), 20 pairs nearest normalized energy 0.5."""
    L, W, seed, n_ev = 12, 1.0, 0, 20
    h = wl.xxz_fields(L, W, seed)
    H, _ = models.xxz(L, L // 2, 1.0, 1.0, h)
    E_min, E_max = lanczos.spectral_extremes(H)
    lam = polfed.target_energy("normalized", 0.5, E_min, E_max)
    E, _ = dense.nearest_eigenpairs(H, lam, n_ev)
    p = polfed.plan(H, lam, n_ev + polfed.buffer_size(n_ev), E_min, E_max)
    return {"workload": "xxz L=12 N=6 J=1 Delta=1 W=1 seed=0 periodic",
            "fields": h.tolist(), "E_min": E_min, "E_max": E_max,
            "lambda": lam, "n_ev": n_ev, "eigenvalues_nearest": E.tolist(),
            "plan": {"K": p["K"], "lam_t": p["lam_t"], "delta": p["delta"],
                     "E_c": p["E_c"], "dE": p["dE"]},
            "source": "oracle.dense (numpy eigh) and oracle.polfed.plan"}


if __name__ == "__main__":
    out = xxz_l12()
    with open(os.path.join(HERE, "xxz_L12_eps05.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote xxz_L12_eps05.json")
