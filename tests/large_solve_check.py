"""A complete solve of the random-field XXZ workload at a large chain length
on the GPU, checked on the host with the oracle's CSR matrix (App. A eq.
xxz; the problem statement of Sec. 4.6).  Not a pytest module: a full solve
at L = 22 takes minutes, so it runs on its own:

    python tests/large_solve_check.py --L 22 --precision auto

Prints one JSON line: solve time, eigenpairs/s, the plan and the checks
(residual ||Hu - Eu|| of every returned pair computed with the oracle's
matrix, orthonormality of the returned vectors, the ordering by distance
from the target, and the library's own completeness status)."""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, default=22)
    ap.add_argument("--W", type=float, default=3.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--n-ev", type=int, default=100)
    ap.add_argument("--precision", choices=["auto", "fp64", "fp32"], default="auto")
    args = ap.parse_args()
    import torch

    import paper_2605_10191_amd as pk
    import workloads as wl
    from oracle import models

    L, N = args.L, args.L // 2
    prec = {"auto": pk.AUTO, "fp64": pk.FP64, "fp32": pk.FP32}[args.precision]
    ctx = pk.Context(0)
    h = wl.xxz_fields(L, args.W, args.seed)
    op = pk.Operator.xxz(ctx, L, N, 1.0, 1.0, h, True)
    x0 = torch.tensor(wl.start_vector(op.D, args.seed), device=ctx.torch_device)
    print(f"solve XXZ L={L} D={op.D} n_ev={args.n_ev} precision={args.precision}: start",
          flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, U, R, rep, status = pk.solve(op, x0, args.n_ev, 0.5, "normalized", precision=prec,
                                     allow_partial=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"solve done in {dt:.1f}s status={status} K={rep['K']} iters={rep['iters']}",
          flush=True)
    E = ev.cpu().numpy()
    Uh = U.cpu().numpy()  # D x n_ev (column-major pairs)
    del U
    H, _ = models.xxz(L, N, 1.0, 1.0, h)
    res = np.linalg.norm(H @ Uh - Uh * E, axis=0)
    ortho = float(np.max(np.abs(Uh.T @ Uh - np.eye(len(E))))) if len(E) else None
    lam = rep["lambda"]
    ordered = bool(np.array_equal(np.lexsort((E, np.abs(E - lam))), np.arange(len(E))))
    out = {"workload": f"XXZ L={L} periodic J=1 Delta=1 W={args.W} seed {args.seed}, "
                       f"Sz=0 (D={op.D}), {args.n_ev} pairs at normalized energy 0.5",
           "precision_requested": args.precision,
           "precision_used": {pk.FP64: "fp64", pk.FP32: "fp32_bulk+fp64_refine"}.get(
               rep["precision"], rep["precision"]),
           "status": status, "n_found": int(len(E)), "solve_s": round(dt, 1),
           "eigenpairs_per_s": round(len(E) / dt, 4) if status == "OK" else None,
           "K": rep["K"], "iters": rep["iters"], "refine_sweeps": rep["refine_sweeps"],
           "fp32_fallback": rep["fp32_fallback"],
           "t_filter": round(rep["t_filter"], 1), "t_reorth": round(rep["t_reorth"], 1),
           "t_check": round(rep["t_check"], 1), "t_extract": round(rep["t_extract"], 1),
           "t_refine": round(rep["t_refine"], 1), "filter_GBps": round(rep["filter_GBps"], 1),
           "lambda": lam,
           "max_resid_oracle_csr": float(res.max()) if len(res) else None,
           "max_resid_reported": float(R.max().item()) if len(E) else None,
           "orthonormality_max_dev": ortho, "ordered_by_distance": ordered,
           "checks_pass": bool(status == "OK" and len(E) == args.n_ev and res.max() <= 1e-8
                               and ortho <= 1e-8 and ordered)}
    print(json.dumps(out), flush=True)
    return 0 if out["checks_pass"] else 1


if __name__ == "__main__":
    sys.exit(main())
