"""Exact equilibrium references for small Potts lattices, independent of the
oracle: brute-force enumeration (tests/native/enum_dos.c) and a row transfer
matrix.  Used to pin the oracle's Markov chain statistically."""
from __future__ import annotations

import itertools
import math
import subprocess
from typing import Dict, Tuple

import numpy as np


def enum_dos(native_bin, L: int, q: int) -> Dict[Tuple[int, int], int]:
    exe = native_bin("enum_dos.c")
    out = subprocess.run([exe, str(L), str(q)], capture_output=True, text=True, check=True).stdout
    dos = {}
    for line in out.strip().splitlines():
        e, m, c = (int(v) for v in line.split())
        dos[(e, m)] = c
    return dos


def dos_averages(dos, beta: float, N: int, q: int) -> Dict[str, float]:
    """Boltzmann averages with weight exp(beta * e_sat) (H = -e_sat, Eq. 1)."""
    emax = max(e for e, _ in dos)
    z = e1 = e2 = e4 = m1 = m2 = 0.0
    for (e, nmax), c in dos.items():
        w = c * math.exp(beta * (e - emax))
        m = (q * nmax / N - 1.0) / (q - 1.0)
        z += w
        e1 += w * e
        e2 += w * e * e
        e4 += w * float(e) ** 4
        m1 += w * m
        m2 += w * m * m
    return {"E": e1 / z, "E2": e2 / z, "E4": e4 / z, "m": m1 / z, "m2": m2 / z}


def transfer_matrix_moments(L: int, q: int, beta: float) -> Dict[str, float]:
    """<e_sat> and <e_sat^2> of the L x L periodic Potts model from the row
    transfer matrix T(a,b) = exp(beta*(h(a)/2 + h(b)/2 + v(a,b))), where h counts
    satisfied bonds inside a row and v between two rows.  Z = Tr T^L; the
    moments come from the exact derivatives of Tr T^L with respect to beta."""
    rows = np.array(list(itertools.product(range(q), repeat=L)), dtype=np.int64)
    h = (rows == np.roll(rows, -1, axis=1)).sum(axis=1).astype(np.float64)
    v = (rows[:, None, :] == rows[None, :, :]).sum(axis=2).astype(np.float64)
    energy = 0.5 * h[:, None] + 0.5 * h[None, :] + v
    shift = energy.max()
    T = np.exp(beta * (energy - shift))
    T1 = T * energy
    T2 = T * energy * energy
    powers = [np.eye(len(rows))]
    for _ in range(L):
        powers.append(powers[-1] @ T)
    Z = np.trace(powers[L])
    d1 = L * np.trace(T1 @ powers[L - 1])
    d2 = L * np.trace(T2 @ powers[L - 1])
    for k in range(L - 1):
        d2 += L * np.trace(T1 @ powers[k] @ T1 @ powers[L - 2 - k])
    return {"E": d1 / Z, "E2": d2 / Z}


def binned(series: np.ndarray, nbins: int = 50):
    """Mean and its standard error from the spread of nbins consecutive block means."""
    x = np.asarray(series, dtype=np.float64)
    n = (len(x) // nbins) * nbins
    blocks = x[:n].reshape(nbins, -1).mean(axis=1)
    return float(x[:n].mean()), float(blocks.std(ddof=1) / math.sqrt(nbins))
