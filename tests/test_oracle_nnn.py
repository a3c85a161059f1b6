"""Pins of the oracle's first-plus-second-neighbour chain (Sec. 7: nine
independent sub-lattices), against what the mathematics fixes:

  * the table entries are the floors of the exact Boltzmann weights (50-digit
    decimal exp), with the always-accept entry exactly where dE <= 0;
  * one trial accepts with probability min(1, exp(-beta dE)) to 2^-32, with dE
    counted by brute force from the two neighbour groups (a swap of the
    groups, a dropped j2 or a wrong sign fails);
  * detailed balance of single trials;
  * the nine colour classes are independent sets of the coupling graph;
  * a colour pass equals the site rule applied to neighbourhoods gathered by
    numpy, with the contract's Philox words, and touches nothing else;
  * bond counts against a brute-force count;
  * equilibrium energies of a 12 x 12 Ising (q = 2) lattice against the exact
    transfer matrix, for a ferromagnetic and a frustrating j2.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

TWO32 = 1 << 32


def exact_floor(beta, de):
    getcontext().prec = 50
    return int((Decimal(-beta) * Decimal(de)).exp() * Decimal(TWO32))


@pytest.mark.parametrize("beta,j2", [(0.0, 0.5), (0.3, 0.5), (0.7, -0.4), (1.1, 1.0), (2.0, 0.25), (0.45, 2.0)])
def test_table_is_floor_of_exact_weight(oracle_lib, beta, j2):
    thr = oracle_lib.nnn_table(beta, j2)
    for d1 in range(-4, 5):
        for d2 in range(-4, 5):
            de = d1 + j2 * d2
            got = int(thr[(d1 + 4) * 9 + (d2 + 4)])
            if de <= 0:
                assert got == TWO32, (d1, d2)
            else:
                want = min(exact_floor(beta, Decimal(d1) + Decimal(repr(j2)) * d2), TWO32 - 1)
                assert abs(got - want) <= 1, (d1, d2, got, want)


def _accepted_fraction(oracle_lib, q, s, k, nb1, nb2, thr):
    """Fraction of acceptance words that accept the proposal k (the decision is
    monotone in the word: binary search for the first rejecting word)."""
    w_prop = -(-k * TWO32 // q)  # smallest word giving floor(w q / 2^32) = k
    assert (w_prop * q) >> 32 == k
    lo, hi = 0, TWO32  # first rejecting word in [lo, hi]
    while lo < hi:
        mid = (lo + hi) // 2
        if oracle_lib.nnn_site_update(q, s, nb1, nb2, w_prop, mid, thr) == k:
            lo = mid + 1
        else:
            hi = mid
    return lo / TWO32


def _counts(v, nb):
    return sum(1 for x in nb if x == v)


@pytest.mark.parametrize("beta,j2", [(0.4, 0.5), (0.9, -0.6), (1.3, 1.7)])
def test_single_trial_acceptance(oracle_lib, beta, j2):
    rng = np.random.default_rng(11)
    q = 4
    thr = oracle_lib.nnn_table(beta, j2)
    for _ in range(60):
        nb1 = rng.integers(0, q, 4)
        nb2 = rng.integers(0, q, 4)
        s, k = (int(x) for x in rng.choice(q, 2, replace=False))
        de = (_counts(s, nb1) - _counts(k, nb1)) + j2 * (_counts(s, nb2) - _counts(k, nb2))
        p = _accepted_fraction(oracle_lib, q, s, k, nb1, nb2, thr)
        assert abs(p - min(1.0, math.exp(-beta * de))) <= 2.0 / TWO32, (nb1, nb2, s, k)


def test_detailed_balance(oracle_lib):
    rng = np.random.default_rng(5)
    beta, j2, q = 0.8, 0.35, 3
    thr = oracle_lib.nnn_table(beta, j2)
    for _ in range(40):
        nb1 = rng.integers(0, q, 4)
        nb2 = rng.integers(0, q, 4)
        s, k = (int(x) for x in rng.choice(q, 2, replace=False))
        e = lambda v: -(_counts(v, nb1) + j2 * _counts(v, nb2))
        p_sk = _accepted_fraction(oracle_lib, q, s, k, nb1, nb2, thr)
        p_ks = _accepted_fraction(oracle_lib, q, k, s, nb1, nb2, thr)
        # pi(s) P(s->k) = pi(k) P(k->s), pi ~ exp(-beta E); rounding 2^-32 each
        lhs = math.exp(-beta * e(s)) * p_sk
        rhs = math.exp(-beta * e(k)) * p_ks
        assert abs(lhs - rhs) <= 4e-9 * max(lhs, rhs) + 2 * 2.0**-32


def test_nine_colours_are_independent_sets():
    L = 12
    colour = lambda x, y: 3 * (y % 3) + (x % 3)
    for y in range(L):
        for x in range(L):
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    if dx or dy:
                        assert colour((x + dx) % L, (y + dy) % L) != colour(x, y)
    counts = np.bincount([colour(x, y) for y in range(L) for x in range(L)], minlength=9)
    assert np.all(counts == L * L // 9)


@pytest.mark.parametrize("colour", range(9))
def test_colour_pass_wiring(oracle_lib, colour):
    L, q, seed, t, beta, j2 = 24, 5, 7, 3, 0.6, 0.45
    thr = oracle_lib.nnn_table(beta, j2)
    rng = np.random.default_rng(colour)
    before = rng.integers(0, q, (L, L), dtype=np.uint8)
    after = before.copy()
    oracle_lib.nnn_colour_pass(after, q, seed, t, colour, thr)
    r = lambda dy, dx: np.roll(np.roll(before, -dy, axis=0), -dx, axis=1)  # value at (y+dy, x+dx)
    near = [r(0, 1), r(0, -1), r(1, 0), r(-1, 0)]
    diag = [r(-1, -1), r(-1, 1), r(1, -1), r(1, 1)]
    key = [seed & 0xFFFFFFFF, seed >> 32]
    moved = 0
    for y in range(L):
        for x in range(L):
            if 3 * (y % 3) + (x % 3) != colour:
                assert after[y, x] == before[y, x]
                continue
            w = oracle_lib.philox4x32_10([t & 0xFFFFFFFF, y * (L // 6) + x // 6, t >> 32, 16 + colour], key)
            b = (x // 3) & 1
            want = oracle_lib.nnn_site_update(q, int(before[y, x]), [n[y, x] for n in near], [n[y, x] for n in diag],
                                              int(w[2 * b]), int(w[2 * b + 1]), thr)
            assert after[y, x] == want, (x, y)
            moved += want != before[y, x]
    assert moved > 0


def test_each_block_serves_two_sites_per_colour():
    """The counter layout: within one colour pass every Philox block (row y,
    segment x // 6) serves exactly two sites, with the two word pairs."""
    L = 36
    for colour in range(9):
        cy, cx = divmod(colour, 3)
        seen = {}
        for y in range(cy, L, 3):
            for x in range(cx, L, 3):
                seen.setdefault(y * (L // 6) + x // 6, []).append((x // 3) & 1)
        assert all(sorted(v) == [0, 1] for v in seen.values())
        assert len(seen) == (L // 3) * (L // 3) // 2


def test_observables_brute_force(oracle_lib):
    L, q = 24, 4
    s = np.random.default_rng(3).integers(0, q, (L, L), dtype=np.uint8)
    e1, e2, hist = oracle_lib.nnn_observables(s, q)
    roll = lambda dy, dx: np.roll(np.roll(s, -dy, axis=0), -dx, axis=1)
    assert e1 == int((s == roll(0, 1)).sum() + (s == roll(1, 0)).sum())
    assert e2 == int((s == roll(1, 1)).sum() + (s == roll(1, -1)).sum())
    assert np.array_equal(hist, np.bincount(s.ravel(), minlength=q))


def test_sweep_is_nine_passes_then_record(oracle_lib):
    L, q, seed = 12, 3, 9
    thr = oracle_lib.nnn_table(0.5, 0.3)
    a = oracle_lib.init(L, q, seed, 1)
    b = a.copy()
    rec = oracle_lib.nnn_sweeps(a, q, seed, 4, 2, thr)
    for t in (4, 5):
        for c in range(9):
            oracle_lib.nnn_colour_pass(b, q, seed, t, c, thr)
        e1, e2, hist = oracle_lib.nnn_observables(b, q)
        assert list(rec[t - 4]) == [e1, e2, *hist]
    assert np.array_equal(a, b)


def _transfer_matrix_energies(L, K1, K2):
    """Exact <e1>, <e2> (per bond) of the L x L periodic q = 2 Potts lattice
    with nearest couplings K1 and diagonal couplings K2, from the row-to-row
    transfer matrix over the 2^L row states."""
    n = 1 << L
    a = np.arange(n, dtype=np.int64)
    bits = (a[:, None] >> np.arange(L)) & 1
    pop = np.array([bin(i).count("1") for i in range(n)], dtype=np.int64)
    rot_up = ((a >> 1) | ((a & 1) << (L - 1)))           # bit i <- bit i+1
    rot_dn = (((a << 1) & (n - 1)) | (a >> (L - 1)))     # bit i <- bit i-1
    h = (bits == np.roll(bits, -1, axis=1)).sum(axis=1).astype(np.float64)
    v = (L - pop[a[:, None] ^ a[None, :]]).astype(np.float64)
    d = (2 * L - pop[a[:, None] ^ rot_up[None, :]] - pop[a[:, None] ^ rot_dn[None, :]]).astype(np.float64)
    H1 = (h[:, None] + h[None, :]) / 2 + v
    expo = K1 * H1 + K2 * d
    T = np.exp(expo - expo.max())
    T2 = T @ T
    T4 = T2 @ T2
    T8 = T4 @ T4
    Tm = T8 @ T2 @ T  # T^(L-1) for L = 12
    Z = float(np.sum(Tm * T.T))
    E1 = L * float(np.sum(Tm * (T * H1).T)) / Z
    E2 = L * float(np.sum(Tm * (T * d).T)) / Z
    return E1 / (2 * L * L), E2 / (2 * L * L)


@pytest.mark.parametrize("beta,j2", [(0.3, 0.5), (0.35, -0.4)])
def test_equilibrium_energies_transfer_matrix(oracle_lib, beta, j2):
    L, q, seed, burn, n = 12, 2, 17, 400, 6000
    want1, want2 = _transfer_matrix_energies(L, beta, beta * j2)
    s = oracle_lib.init(L, q, seed, 1)
    rec = oracle_lib.nnn_sweeps(s, q, seed, 0, burn + n, oracle_lib.nnn_table(beta, j2))[burn:]
    for col, want in ((0, want1), (1, want2)):
        x = rec[:, col] / (2 * L * L)
        blocks = x.reshape(60, -1).mean(axis=1)
        err = blocks.std(ddof=1) / math.sqrt(len(blocks))
        assert abs(x.mean() - want) < 5 * err + 1e-4, (col, x.mean(), want, err)
