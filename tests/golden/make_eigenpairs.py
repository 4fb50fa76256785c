"""Writes golden eigenpairs of the two mid-size workloads from the CPU oracle
only (its plain POLFED: ARPACK bounds, Gaussian-DOS plan, SciPy CSR Clenshaw
filter, Lanczos with full reorthogonalization, Rayleigh-Ritz with H).

  xxz20   random-field XXZ chain L=20, periodic, J=1, Delta=1, W=3, seed 0,
          Sz=0 (D=184,756), 100 pairs nearest normalized energy 0.5
          (App. A eq. xxz; the problem statement of Sec. 4.6)
  qsun    quantum sun N=3 (GOE dot, gamma=1) + L=13 outer spins, g0=1,
          alpha=0.75, seed 0 (D=65,536), 50 pairs nearest normalized
          energy 0.5 (App. A eq. qsun)

The start vector is the seeded U[0,1) draw of workloads.start_vector (Sec.
5.2).  Each file holds the target lambda (absolute), the bounds, the plan's K,
the eigenvalues sorted by (|E - lambda|, E) and their residuals ||Hu - Eu||.
Eigenvectors are not stored (they are recomputed from H where needed).

Run from the repository root (CPU hours for xxz20, tens of minutes for qsun):
    python tests/golden/make_eigenpairs.py xxz20
    python tests/golden/make_eigenpairs.py qsun
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as wl  # noqa: E402
from oracle import lanczos, models, polfed  # noqa: E402


def _solve(H, x0, n_ev, workload, extra):
    t0 = time.time()
    E_min, E_max = lanczos.spectral_extremes(H)
    lam = polfed.target_energy("normalized", 0.5, E_min, E_max)
    out = polfed.polfed(H, x0, n_ev, lam, "absolute", bounds=(E_min, E_max))
    E = np.asarray(out["E"])
    order = np.lexsort((E, np.abs(E - lam)))
    res = np.asarray(out["res"])[order]
    E = E[order]
    # residuals recomputed straight from H, independent of the extraction
    U = out["U"][:, order]
    res_direct = np.linalg.norm(H @ U - U * E, axis=0)
    g = {"workload": workload, "D": int(H.shape[0]), "n_ev": n_ev,
         "E_min": E_min, "E_max": E_max, "lambda": lam,
         "K": out["plan"]["K"], "iters": int(out["iters"]),
         "eigenvalues_nearest": E.tolist(), "residuals": res.tolist(),
         "residuals_direct": res_direct.tolist(),
         "cpu_seconds": round(time.time() - t0, 1),
         "source": "oracle.polfed.polfed (tests/golden/make_eigenpairs.py)"}
    g.update(extra)
    return g


def xxz20():
    L, W, seed, n_ev = 20, 3.0, 0, 100
    h = wl.xxz_fields(L, W, seed)
    H, _ = models.xxz(L, L // 2, 1.0, 1.0, h)
    x0 = wl.start_vector(H.shape[0], seed)
    return _solve(H, x0, n_ev, "xxz L=20 N=10 J=1 Delta=1 W=3 seed=0 periodic, "
                  "x0 = workloads.start_vector(D, 0)", {"fields": h.tolist()})


def qsun():
    N, L, seed, n_ev = 3, 13, 0, 50
    q = wl.qsun_draws(N, L, seed)
    H = models.qsun(N, L, q["A"], 1.0, 1.0, 0.75, q["u"], q["n_of_j"], q["h"])
    x0 = wl.start_vector(H.shape[0], seed)
    return _solve(H, x0, n_ev, "quantum sun N=3 gamma=1 + L=13, g0=1, alpha=0.75, seed=0, "
                  "x0 = workloads.start_vector(D, 0)", {})


if __name__ == "__main__":
    which = sys.argv[1]
    name = {"xxz20": "xxz_L20_W3_eps05.json", "qsun": "qsun_N3_L13_eps05.json"}[which]
    g = {"xxz20": xxz20, "qsun": qsun}[which]()
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(g, f, indent=1)
    print("wrote", name, "in", g["cpu_seconds"], "s; max residual", max(g["residuals"]))
