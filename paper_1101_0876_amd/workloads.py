"""Seeded synthetic workloads (job lists) for the batch and serving paths.

Holds no arithmetic of the method: it only draws lattice sizes, q, inverse
temperatures (around the exact transition point beta_c = ln(1 + sqrt q),
Eq. 2), starts, seeds and sweep counts with numpy.
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

ORDERED, RANDOM = 0, 1


def beta_c(q: int) -> float:
    return math.log1p(math.sqrt(q))


def batch_jobs(n: int = 1024, sweeps: int = 500, seed: int = 1101) -> List[Dict]:
    """Batched replicas: L = 2^U{7..12}, q = U{3..12}, beta = beta_c(q) U[0.98, 1.02],
    random start, job i seeded i+1, `sweeps` sweeps each."""
    rng = np.random.default_rng(seed)
    Ls = 2 ** rng.integers(7, 13, size=n)
    qs = rng.integers(3, 13, size=n)
    f = rng.uniform(0.98, 1.02, size=n)
    return [dict(L=int(L), q=int(q), seed=i + 1, start=RANDOM, beta=beta_c(int(q)) * float(x), nsweeps=sweeps)
            for i, (L, q, x) in enumerate(zip(Ls, qs, f))]


def serve_jobs(n: int = 1000, rate: float = 200.0, seed: int = 1101, sweep_scale: float = 1.0) -> List[Dict]:
    """Served jobs: Poisson arrivals at `rate` per second; L = 2^U{8..13},
    q = U{3..15}, start ordered or random with probability 1/2, a beta ramp of
    P = U{8..32} points linear over [0.98, 1.02] beta_c(q) (heating from the
    ordered start: beta descending; cooling from the random start: ascending),
    S = round(10^U[3, 5] * sweep_scale) sweeps split evenly over the points
    (remainder to the last); job j seeded j+1."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    Ls = 2 ** rng.integers(8, 14, size=n)
    qs = rng.integers(3, 16, size=n)
    starts = rng.integers(0, 2, size=n)
    points = rng.integers(8, 33, size=n)
    sweeps = np.round(10 ** rng.uniform(3, 5, size=n) * sweep_scale).astype(np.int64)
    jobs = []
    for j in range(n):
        q, P, S = int(qs[j]), int(points[j]), max(int(sweeps[j]), int(points[j]))
        grid = beta_c(q) * (0.98 + 0.04 * np.arange(P) / max(P - 1, 1))
        betas = grid[::-1] if starts[j] == ORDERED else grid
        per = [S // P] * P
        per[-1] += S - sum(per)
        jobs.append(dict(arrival=float(arrivals[j]), L=int(Ls[j]), q=q, seed=j + 1, start=int(starts[j]),
                         betas=[float(b) for b in betas], sweeps=per))
    return jobs
