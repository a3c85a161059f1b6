"""Pins the oracle's heat-bath update (Sec. 7: other single-spin-flip
algorithms) to what it must compute, without the oracle's own formula:

  * the exact probability of every new value, read off the oracle's draw by
    binary search over the 32-bit word, equals the Boltzmann conditional
    exp(beta n(k)) / sum_v exp(beta n(v)) to within the table's quantization
  * a worked example fixes the ranking convention (neighbour values in order
    of first appearance among up, down, left, right, then the rest ascending)
  * long runs reproduce the Boltzmann averages of the 4x4 q=3 lattice by
    full enumeration, and the 8x8 q=2 ones from the transfer matrix
  * a half sweep uses counter word 3 = colour + 4 and the word w[2b]
"""
import itertools
import math

import numpy as np
import pytest

from tests.exact import binned, dos_averages, enum_dos, transfer_matrix_moments
from tests.inputs import beta_c


def _ranking(nb, q):
    seen, out = set(), []
    for v in nb:
        if v not in seen:
            seen.add(v)
            out.append(v)
    return out + [v for v in range(q) if v not in seen]


def _exact_probabilities(oracle_lib, q, nb, thr):
    """P(k) = #{w : draw(w) = k} / 2^32.  The draw's rank position is
    nondecreasing in w, so the boundaries follow by binary search."""
    rank = _ranking(nb, q)
    pos = {v: i for i, v in enumerate(rank)}

    def position(w):
        return pos[oracle_lib.heatbath_site(q, nb, w, thr)]

    starts = []
    for i in range(q):
        lo, hi = 0, 2**32  # smallest w with position(w) >= i
        while lo < hi:
            mid = (lo + hi) // 2
            if position(mid) >= i:
                hi = mid
            else:
                lo = mid + 1
        starts.append(lo)
    starts.append(2**32)
    return {rank[i]: (starts[i + 1] - starts[i]) / 2**32 for i in range(q)}


NEIGHBOURHOODS = [(0, 0, 0, 0), (0, 1, 0, 1), (2, 1, 2, 0), (0, 1, 2, 3), (1, 1, 1, 0), (3, 3, 1, 1)]


@pytest.mark.parametrize("q", [2, 3, 5, 9])
@pytest.mark.parametrize("beta", [0.0, 0.4, 1.3, 3.0])
def test_conditional_distribution_is_boltzmann(oracle_lib, q, beta):
    thr = oracle_lib.threshold_table(beta)
    for nb in NEIGHBOURHOODS:
        nb = tuple(v % q for v in nb)
        p = _exact_probabilities(oracle_lib, q, nb, thr)
        n = [sum(1 for u in nb if u == v) for v in range(q)]
        z = sum(math.exp(beta * n[v]) for v in range(q))
        for v in range(q):
            want = math.exp(beta * n[v]) / z
            # each weight is floored to an integer out of a total >= 2^32
            assert abs(p[v] - want) < (q + 2) * 2.0**-31, (nb, v, p[v], want)


def test_ranking_convention_worked_example(oracle_lib):
    """q = 5, neighbours (up, down, left, right) = (3, 1, 3, 0), beta = 0:
    counts n(3) = 2, n(1) = n(0) = 1, n_max = 2; weights D[0] = 2^32 for 3 and
    D[d] = 2^32 - 1 for the rest; ranking 3, 1, 0, 2, 4; Z = 5 * 2^32 - 4.
    w = 2^31 gives r = floor(Z / 2) = 5 * 2^31 - 2, which falls in the third
    value's interval [2^33 - 1, 3 * 2^32 - 2): k = 0 (an ascending ranking
    would give 2)."""
    thr = oracle_lib.threshold_table(0.0)
    assert list(thr) == [2**32 - 1] * 4
    nb = (3, 1, 3, 0)
    assert oracle_lib.heatbath_site(5, nb, 2**31, thr) == 0
    assert oracle_lib.heatbath_site(5, nb, 0, thr) == 3
    assert oracle_lib.heatbath_site(5, nb, 2**32 - 1, thr) == 4
    # the first word past 3's interval: r = 2^32 needs w = ceil(2^64 / Z)
    w1 = -(-(2**64) // (5 * 2**32 - 4))
    assert oracle_lib.heatbath_site(5, nb, w1 - 1, thr) == 3
    assert oracle_lib.heatbath_site(5, nb, w1, thr) == 1


def test_half_sweep_layout(oracle_lib):
    L, q, seed, t = 12, 7, (5 << 32) | 9, 2**32 + 11
    thr = oracle_lib.threshold_table(0.8)
    base = oracle_lib.init(L, q, 3, 1)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for colour in (0, 1):
        s = base.copy()
        oracle_lib.heatbath_half_sweep(s, q, seed, t, colour, thr)
        for y in range(L):
            for x in range(L):
                if (x + y) & 1 != colour:
                    assert s[y, x] == base[y, x]
                    continue
                w = oracle_lib.philox4x32_10([t & 0xFFFFFFFF, y * (L // 4) + x // 4, t >> 32, colour + 4], key)
                nb = (base[(y - 1) % L, x], base[(y + 1) % L, x], base[y, (x - 1) % L], base[y, (x + 1) % L])
                assert s[y, x] == oracle_lib.heatbath_site(q, nb, int(w[2 * ((x >> 1) & 1)]), thr)


@pytest.fixture(scope="module")
def dos_4x4_q3(native_bin):
    return enum_dos(native_bin, 4, 3)


def _series(oracle_lib, L, q, beta, seed, n, burn=1000):
    spins = oracle_lib.init(L, q, seed, 1)
    thr = oracle_lib.threshold_table(beta)
    oracle_lib.heatbath_sweeps(spins, q, seed, 0, burn, thr, record=False)
    rec = oracle_lib.heatbath_sweeps(spins, q, seed, burn, n, thr)
    e = rec[:, 0].astype(np.float64)
    nmax = rec[:, 1:].max(axis=1).astype(np.float64)
    return e, (q * nmax / (L * L) - 1.0) / (q - 1.0)


@pytest.mark.parametrize("beta", [0.5, beta_c(3), 1.6])
def test_4x4_q3_heatbath_matches_enumeration(oracle_lib, dos_4x4_q3, beta):
    exact = dos_averages(dos_4x4_q3, beta, 16, 3)
    e, m = _series(oracle_lib, 4, 3, beta, seed=23, n=150_000)
    for name, series, want in (("E", e, exact["E"]), ("E2", e * e, exact["E2"]), ("m", m, exact["m"])):
        mean, err = binned(series, 100)
        assert abs(mean - want) < 5 * err + 1e-12, (name, mean, want, err)
        assert err < 0.01 * abs(want) + 1e-3, (name, err)


@pytest.mark.parametrize("beta", [0.6, beta_c(2)])
def test_8x8_q2_heatbath_matches_transfer_matrix(oracle_lib, beta):
    exact = transfer_matrix_moments(8, 2, beta)
    e, _ = _series(oracle_lib, 8, 2, beta, seed=4, n=150_000)
    for name, series, want in (("E", e, exact["E"]), ("E2", e * e, exact["E2"])):
        mean, err = binned(series, 100)
        assert abs(mean - want) < 5 * err, (name, mean, want, err)
