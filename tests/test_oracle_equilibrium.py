"""Pins the oracle's whole Markov chain (neighbour indexing, colour order, random
words, acceptance) to exact equilibrium: long oracle runs must reproduce
Boltzmann averages obtained without the oracle.

  * 4x4, q=3: full enumeration of 3^16 configurations (brute force)
  * 8x8, q=2: row transfer matrix; the q=2 Potts model is the Ising model at
    half the coupling (Sec. 4, footnote on J_Potts = 2 J_Ising)
  * the two exact methods agree with each other on 4x4 (q=2 and q=3)
"""
import math

import numpy as np
import pytest

from tests.exact import binned, dos_averages, enum_dos, transfer_matrix_moments
from tests.inputs import beta_c


@pytest.fixture(scope="module")
def dos_4x4_q3(native_bin):
    return enum_dos(native_bin, 4, 3)


def test_enumeration_counts(dos_4x4_q3):
    assert sum(dos_4x4_q3.values()) == 3**16
    # ground states: the q uniform lattices, 32 satisfied bonds, N_max = 16
    assert dos_4x4_q3[(32, 16)] == 3
    assert max(e for e, _ in dos_4x4_q3) == 32


@pytest.mark.parametrize("q", [2, 3])
def test_transfer_matrix_agrees_with_enumeration(native_bin, q, dos_4x4_q3):
    dos = dos_4x4_q3 if q == 3 else enum_dos(native_bin, 4, 2)
    for beta in (0.3, 1.0, 1.7):
        a = dos_averages(dos, beta, 16, q)
        b = transfer_matrix_moments(4, q, beta)
        assert b["E"] == pytest.approx(a["E"], rel=1e-10)
        assert b["E2"] == pytest.approx(a["E2"], rel=1e-10)


def _oracle_series(oracle_lib, L, q, beta, seed, n, burn=2000):
    spins = oracle_lib.init(L, q, seed, 1)
    thr = oracle_lib.threshold_table(beta)
    oracle_lib.sweeps(spins, q, seed, 0, burn, thr, record=False)
    rec = oracle_lib.sweeps(spins, q, seed, burn, n, thr)
    e = rec[:, 0].astype(np.float64)
    nmax = rec[:, 1:].max(axis=1).astype(np.float64)
    m = (q * nmax / (L * L) - 1.0) / (q - 1.0)
    return e, m


@pytest.mark.parametrize("beta", [0.5, beta_c(3), 1.6])
def test_4x4_q3_matches_enumeration(oracle_lib, dos_4x4_q3, beta):
    exact = dos_averages(dos_4x4_q3, beta, 16, 3)
    e, m = _oracle_series(oracle_lib, 4, 3, beta, seed=17, n=200_000)
    for name, series, want in (("E", e, exact["E"]), ("E2", e * e, exact["E2"]),
                               ("E4", e**4, exact["E4"]), ("m", m, exact["m"])):
        mean, err = binned(series, 100)
        assert abs(mean - want) < 5 * err + 1e-12, (name, mean, want, err)
        # the run must be precise enough to catch a wrong chain
        assert err < 0.01 * abs(want) + 1e-3, (name, err)


@pytest.mark.parametrize("beta", [0.6, beta_c(2), 1.2])
def test_8x8_q2_matches_transfer_matrix(oracle_lib, beta):
    exact = transfer_matrix_moments(8, 2, beta)
    e, _ = _oracle_series(oracle_lib, 8, 2, beta, seed=3, n=200_000)
    for name, series, want in (("E", e, exact["E"]), ("E2", e * e, exact["E2"])):
        mean, err = binned(series, 100)
        assert abs(mean - want) < 5 * err, (name, mean, want, err)
        assert err < 0.005 * want


def test_energy_at_transition_q3(oracle_lib):
    """Self-dual energy at beta_c (Eq. 6 with e_d = e_o for q <= 4):
    e(beta_c) -> -(1 + 1/sqrt q) as L grows; at L = 32 the finite-size shift is
    a few per cent at most."""
    q, L = 3, 32
    e, _ = _oracle_series(oracle_lib, L, q, beta_c(q), seed=5, n=6000, burn=1000)
    mean = -e.mean() / (L * L)
    assert mean == pytest.approx(-(1 + 1 / math.sqrt(q)), rel=0.03)
