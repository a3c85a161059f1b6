"""Pins the oracle's simple-cubic lattice (Sec. 7: the checkerboard update in
three dimensions) without its own code paths:

  * the six-entry table against exp in 60-digit decimal
  * exact detailed balance of the six-neighbour Metropolis decision, with the
    proposal and acceptance probabilities read off by binary search
  * a half sweep equals a numpy re-derivation: neighbours by np.roll, random
    words from Philox at the documented counter (t_lo, chunk, t_hi, colour+8)
  * the random start's counter layout, brute-force observables (3N bonds)
  * beta = 0: every bond is satisfied with probability 1/q on average;
    beta = infinity quench never loses a satisfied bond

No exact equilibrium reference exists at L >= 4 (the smallest lattice of the
layout has 64 sites), so the chain is pinned locally (the exact single-site
kernel) and through its wiring; see the 2D pins for global checks of the
same sweep structure.
"""
from decimal import Decimal, getcontext

import numpy as np
import pytest

getcontext().prec = 60
ALWAYS6 = [2**32 - 1] * 6


@pytest.mark.parametrize("beta", [0.0, 0.1, 0.4433, 0.5505, 1.0, 3.0, 30.0])
def test_table6_is_floor_of_exact_weight(oracle_lib, beta):
    thr = oracle_lib.threshold_table6(beta)
    for d in range(1, 7):
        exact = (-(Decimal(beta) * d)).exp() * Decimal(2) ** 32
        want = min(int(exact), 2**32 - 1)
        assert abs(int(thr[d - 1]) - want) <= 1, (beta, d)


def _proposal_count(oracle_lib, q, k):
    """Number of 32-bit words proposing k: read off the decision with a saturated table."""
    nb = [0] * 6

    def prop(w):
        return oracle_lib.site_update3d(q, 0, nb, w, 0, ALWAYS6)

    def first(v):  # first word proposing >= v
        lo, hi = 0, 2**32
        while lo < hi:
            mid = (lo + hi) // 2
            if prop(mid) >= v:
                hi = mid
            else:
                lo = mid + 1
        return lo

    return (first(k + 1) if k + 1 < q else 2**32) - first(k)


def _transition(oracle_lib, q, a, b, nb, thr, w_prop):
    """P(a -> b) for b != a: proposal probability times the accepted fraction
    of acceptance words (binary search for the first rejecting word)."""
    lo, hi = 0, 2**32
    while lo < hi:
        mid = (lo + hi) // 2
        if oracle_lib.site_update3d(q, a, nb, w_prop, mid, thr) == b:
            lo = mid + 1
        else:
            hi = mid
    return _proposal_count(oracle_lib, q, b) / 2**32 * (lo / 2**32)


NEIGHBOURHOODS = [(0, 0, 0, 0, 0, 0), (0, 1, 0, 1, 0, 1), (1, 1, 1, 1, 0, 2), (2, 0, 1, 1, 0, 0), (0, 1, 2, 0, 1, 2)]


@pytest.mark.parametrize("q", [2, 3, 4])
@pytest.mark.parametrize("beta", [0.3, 0.5505, 1.2])
def test_six_neighbour_detailed_balance(oracle_lib, q, beta):
    thr = oracle_lib.threshold_table6(beta)
    # a word proposing each value (the middle of its interval)
    words = {}
    for w in range(0, 2**32, 2**32 // 64):
        words.setdefault(oracle_lib.site_update3d(q, 0, [0] * 6, w, 0, ALWAYS6), w)
    for nb in NEIGHBOURHOODS:
        nb = [v % q for v in nb]
        n = [sum(1 for u in nb if u == v) for v in range(q)]
        for a in range(q):
            for b in range(q):
                if a == b:
                    continue
                pab = _transition(oracle_lib, q, a, b, nb, thr, words[b])
                pba = _transition(oracle_lib, q, b, a, nb, thr, words[a])
                lhs, rhs = np.exp(beta * n[a]) * pab, np.exp(beta * n[b]) * pba
                # the floor of thr[d-1] costs up to 1/thr[d-1] relative; proposals 2^-32
                d = abs(n[a] - n[b])
                rel = (2.0 / int(thr[d - 1]) if d else 0.0) + 4e-9
                assert abs(lhs - rhs) <= rel * max(lhs, rhs) + 2**-31, (nb, a, b, lhs, rhs)


def _words(oracle_lib, L, x, y, z, seed, c0, c2, c3):
    key = [seed & 0xFFFFFFFF, seed >> 32]
    return oracle_lib.philox4x32_10([c0, ((z * L + y) * L + x) // 4, c2, c3], key)


@pytest.mark.parametrize("colour", [0, 1])
def test_half_sweep_wiring(oracle_lib, colour):
    L, q, seed, t = 8, 5, (2 << 32) | 41, 2**32 + 6
    thr = oracle_lib.threshold_table6(0.7)
    rng = np.random.default_rng(3)
    base = rng.integers(0, q, size=(L, L, L), dtype=np.uint8)
    s = base.copy()
    oracle_lib.half_sweep3d(s, q, seed, t, colour, thr)
    nbs = [np.roll(base, -1, axis=2), np.roll(base, 1, axis=2), np.roll(base, -1, axis=1),
           np.roll(base, 1, axis=1), np.roll(base, -1, axis=0), np.roll(base, 1, axis=0)]
    for z in range(L):
        for y in range(L):
            for x in range(L):
                if (x + y + z) & 1 != colour:
                    assert s[z, y, x] == base[z, y, x]
                    continue
                w = _words(oracle_lib, L, x, y, z, seed, t & 0xFFFFFFFF, t >> 32, colour + 8)
                b = (x >> 1) & 1
                nb = [int(a[z, y, x]) for a in nbs]
                want = oracle_lib.site_update3d(q, int(base[z, y, x]), nb, int(w[2 * b]), int(w[2 * b + 1]), thr)
                assert s[z, y, x] == want, (x, y, z)


def test_random_start_layout(oracle_lib):
    L, q, seed = 8, 7, 99
    s = oracle_lib.init3d(L, q, seed, 1)
    for (x, y, z) in [(0, 0, 0), (3, 1, 2), (7, 7, 7), (5, 0, 6)]:
        w = _words(oracle_lib, L, x, y, z, seed, 0, 0, 10)
        assert s[z, y, x] == (int(w[x & 3]) * q) >> 32
    assert not oracle_lib.init3d(L, q, seed, 0).any()


def test_observables_brute_force(oracle_lib):
    L, q = 8, 4
    s = np.random.default_rng(8).integers(0, q, size=(L, L, L), dtype=np.uint8)
    e, hist = oracle_lib.observables3d(s, q)
    want = sum(int((s == np.roll(s, -1, axis=a)).sum()) for a in range(3))
    assert e == want
    assert np.array_equal(hist, np.bincount(s.ravel(), minlength=q))


def test_infinite_temperature_bond_probability(oracle_lib):
    L, q, n = 8, 4, 400
    s = oracle_lib.init3d(L, q, 2, 0)
    rec = oracle_lib.sweeps3d(s, q, 2, 0, n, oracle_lib.threshold_table6(0.0))
    e = rec[50:, 0] / (3 * L**3)
    # bonds satisfied with probability 1/q; 1536 bonds per record
    assert abs(e.mean() - 1.0 / q) < 5 * np.sqrt((1 / q) * (1 - 1 / q) / 1536 / (n - 50)) * 3


def test_quench_never_loses_bonds(oracle_lib):
    L, q = 8, 3
    s = oracle_lib.init3d(L, q, 4, 1)
    rec = oracle_lib.sweeps3d(s, q, 4, 0, 30, oracle_lib.threshold_table6(40.0))
    assert np.all(np.diff(rec[:, 0]) >= 0)
    assert np.all(rec[:, 1:].sum(axis=1) == L**3)


@pytest.mark.parametrize("start", [0, 1])
def test_window_matches_full_cube(oracle_lib, start):
    """The window restriction reproduces the full chain on its exact interior,
    including windows that wrap around every axis."""
    L, q, seed, n, beta = 16, 5, 17, 2, 0.6
    thr = oracle_lib.threshold_table6(beta)
    full = oracle_lib.init3d(L, q, seed, start)
    oracle_lib.sweeps3d(full, q, seed, 0, n, thr, record=False)
    r = 2 * n
    for (x0, y0, z0, d) in [(0, 0, 0, 12), (11, 13, 9, 12), (3, 0, 14, 16)]:
        win = oracle_lib.window3d(L, q, seed, start, n, thr, x0, y0, z0, d)
        idx = [(c0 + np.arange(r, d - r)) % L for c0 in (z0, y0, x0)]
        assert np.array_equal(win[r:d - r, r:d - r, r:d - r], full[np.ix_(*idx)])
