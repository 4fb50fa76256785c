"""Seeded synthetic inputs for the POLFED workloads.

This module only draws random numbers.  It holds none of the method's arithmetic
(no Hamiltonian, filter or Lanczos step): the raw draws are handed unchanged to
both the CPU oracle and the GPU library, which each build their own operators.

Distributions follow the models of the paper's Appendix A:
* random-field XXZ chain, eq. (xxz): fields h_i ~ U[-W, W];
* quantum sun, eq. (qsun): GOE seed matrix A with i.i.d. standard normal
  entries, exponents u_j = j + U[-zeta, zeta] (j counted from 0), dot spin n(j)
  uniform over the N dot spins, fields h_j ~ U[h - w, h + w];
* spinless t-V fermions (not in the paper): on-site energies eps_i ~ U[-2, 2];
* quantum random energy model, eq. (qrem): one Gaussian energy per basis state,
  mean 0 and standard deviation sqrt(L/2);
* start vector: U[0, 1) entries, as in the paper's usage example (Sec. 5.2);
* KPM probe vectors (Sec. 4.1, App. B) with zero-mean, unit-variance entries,
  drawn by the published splitmix64 generator from a counter, so that the
  library, which draws its own probe vectors on the device, and the oracle see
  the same vectors.
"""
from __future__ import annotations

import numpy as np

# Stream offsets keep the start vector independent of the model draws that
# share a seed.
_X0_STREAM = 1_000_003


def xxz_fields(L: int, W: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-W, W, L)


def tv_onsite(L: int, seed: int, width: float = 2.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-width, width, L)


def qsun_draws(N: int, L: int, seed: int, zeta: float = 0.2,
               h: float = 1.0, w: float = 0.5) -> dict:
    rng = np.random.default_rng(seed)
    n_dot = 1 << N
    A = rng.standard_normal((n_dot, n_dot))
    u = np.arange(L, dtype=np.float64) + rng.uniform(-zeta, zeta, L)
    n_of_j = rng.integers(0, N, L).astype(np.int32)
    hj = rng.uniform(h - w, h + w, L)
    return {"A": A, "u": u, "n_of_j": n_of_j, "h": hj}


def qrem_energies(L: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, np.sqrt(L / 2.0), 1 << L)


def start_vector(D: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed + _X0_STREAM)
    return rng.random(D)


def serving_stream(n_req: int, seed: int, mean_gap_s: float,
                   Ls=(14, 16, 18), Ws=(1.0, 3.0, 5.0)) -> list:
    """Poisson arrivals: exponential gaps with the given mean.  Each request
    draws its chain length and disorder strength uniformly, and carries its own
    realization seed."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(mean_gap_s, n_req)
    t = np.cumsum(gaps) - gaps[0]
    Lc = rng.choice(np.asarray(Ls), n_req)
    Wc = rng.choice(np.asarray(Ws), n_req)
    return [{"t_arrive": float(t[i]), "L": int(Lc[i]), "W": float(Wc[i]),
             "seed": int(seed * 100003 + i)} for i in range(n_req)]


def splitmix_vectors(D: int, R: int, seed: int) -> np.ndarray:
    """D x R KPM probe vectors from the published splitmix64 generator
    (Steele, Lea and Flood, 2014): for vector c the counter i + 1 is mixed
    from the state seed + c + golden * (i + 1); u = (z >> 11) / 2^53 on
    [0, 1), entries sqrt(3) (2u - 1) (zero mean, unit variance)."""
    M = (1 << 64) - 1
    golden = 0x9E3779B97F4A7C15
    out = np.empty((D, R))
    i = np.arange(1, D + 1, dtype=np.uint64)
    for c in range(R):
        with np.errstate(over="ignore"):
            z = (np.uint64((seed + c) & M) + np.uint64(golden) * i)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
        u = (z >> np.uint64(11)).astype(np.float64) * (2.0 / 9007199254740992.0) - 1.0
        out[:, c] = np.sqrt(3.0) * u
    return out
