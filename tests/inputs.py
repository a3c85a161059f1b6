"""Seeded synthetic inputs shared by the oracle-side and GPU-side tests.

Holds no arithmetic of the method: only lattice shapes, seeds, temperatures and
random configurations drawn with numpy.
"""
from __future__ import annotations

import math

import numpy as np


def beta_c(q: int) -> float:
    """Exact transition point of the square-lattice Potts model (Eq. 2): T_c = 1/ln(1+sqrt q)."""
    return math.log1p(math.sqrt(q))


def random_lattice(L: int, q: int, seed: int) -> np.ndarray:
    """Uniform random L x L lattice of values 0..q-1 (uint8)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, q, size=(L, L), dtype=np.uint8)


def random_words(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)


# (L, q, seed, start, beta, sweeps) cases spanning several tiles and ragged tails
PARITY_CASES = [
    (4, 2, 1, 1, 0.7, 20),
    (8, 3, 7, 1, beta_c(3), 20),
    (12, 9, 3, 0, 1.02 * beta_c(9), 15),
    (20, 6, 11, 1, beta_c(6), 12),
    (64, 9, 1, 1, 1.02 * math.log(4.0), 40),
    (100, 15, 5, 1, beta_c(15), 10),
    (132, 256, 2, 1, 0.3, 6),
    (256, 6, 9, 0, beta_c(6), 10),
    (260, 12, 4, 1, 0.98 * beta_c(12), 8),
    (1024, 6, 1, 1, beta_c(6), 4),
]
