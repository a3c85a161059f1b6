"""Invariants, special cases and the random-word layout of the oracle.

  * e_sat and N_v by brute force (numpy) equal the oracle's (Eq. 1, Eq. 7)
  * ordered start: every bond satisfied, N_max = N
  * records: sum N_v = N, 0 <= e_sat <= 2N
  * chunking: n sweeps in one call == n calls of one sweep
  * visiting order inside a colour is irrelevant (checkerboard, Sec. 3)
  * beta = 0: every proposal is accepted, so a half sweep writes the proposal
    words' values -- this fixes the counter layout, word choice and colour order
  * beta = inf quench: satisfied bonds never decrease
  * the window restriction equals the full chain on its exact interior
"""
import numpy as np
import pytest

from tests.inputs import beta_c, random_lattice


def _numpy_observables(s, q):
    e = int((s == np.roll(s, -1, axis=1)).sum() + (s == np.roll(s, -1, axis=0)).sum())
    return e, np.bincount(s.ravel(), minlength=q).astype(np.int64)


@pytest.mark.parametrize("L,q", [(4, 2), (8, 3), (12, 256), (20, 7)])
def test_observables_brute_force(oracle_lib, L, q):
    s = random_lattice(L, q, seed=L * q)
    e, hist = oracle_lib.observables(s, q)
    e2, hist2 = _numpy_observables(s, q)
    assert e == e2 and np.array_equal(hist, hist2)


def test_q2_ising_identity(oracle_lib):
    """q=2: e_sat = (2N + sum_<ij> sigma_i sigma_j)/2 with sigma = +-1 (Sec. 4)."""
    L = 16
    for seed in range(5):
        s = random_lattice(L, 2, seed)
        sigma = 2 * s.astype(np.int64) - 1
        bonds = int((sigma * np.roll(sigma, -1, 1)).sum() + (sigma * np.roll(sigma, -1, 0)).sum())
        e, _ = oracle_lib.observables(s, 2)
        assert 2 * e == 2 * L * L + bonds


@pytest.mark.parametrize("q", [2, 9, 256])
def test_ordered_start(oracle_lib, q):
    L = 16
    s = oracle_lib.init(L, q, 5, 0)
    assert not s.any()
    e, hist = oracle_lib.observables(s, q)
    assert e == 2 * L * L and hist[0] == L * L and hist[1:].sum() == 0


@pytest.mark.parametrize("q", [2, 3, 9, 256])
def test_random_start_layout_and_uniformity(oracle_lib, q):
    L, seed = 64, 12345
    s = oracle_lib.init(L, q, seed, 1)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for y in (0, 1, 31, 63):
        for x in (0, 1, 2, 3, 4, 61, 63):
            w = oracle_lib.philox4x32_10([0, y * (L // 4) + x // 4, 0, 2], key)
            assert s[y, x] == (int(w[x & 3]) * q) >> 32
    counts = np.bincount(s.ravel(), minlength=q)
    assert counts.size == q
    exp = L * L / q
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < (q - 1) + 6 * np.sqrt(2 * (q - 1))


@pytest.mark.parametrize("colour", [0, 1])
@pytest.mark.parametrize("t", [0, 7, 2**32 + 3])
def test_beta_zero_writes_proposals(oracle_lib, colour, t):
    L, q, seed = 16, 5, (3 << 32) | 77
    thr = oracle_lib.threshold_table(0.0)
    base = random_lattice(L, q, seed=9)
    s = base.copy()
    oracle_lib.half_sweep(s, q, seed, t, colour, thr)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for y in range(L):
        for x in range(L):
            if (x + y) & 1 != colour:
                assert s[y, x] == base[y, x]
                continue
            w = oracle_lib.philox4x32_10([t & 0xFFFFFFFF, y * (L // 4) + x // 4, t >> 32, colour], key)
            b = (x >> 1) & 1
            if int(w[2 * b + 1]) == 2**32 - 1:  # the one rejecting word
                continue
            assert s[y, x] == (int(w[2 * b]) * q) >> 32


def test_records_and_chunking(oracle_lib):
    L, q, seed, beta = 12, 6, 21, beta_c(6)
    thr = oracle_lib.threshold_table(beta)
    a = oracle_lib.init(L, q, seed, 1)
    rec = oracle_lib.sweeps(a, q, seed, 0, 10, thr)
    assert np.all(rec[:, 1:].sum(axis=1) == L * L)
    assert np.all((rec[:, 0] >= 0) & (rec[:, 0] <= 2 * L * L))
    b = oracle_lib.init(L, q, seed, 1)
    parts = [oracle_lib.sweeps(b, q, seed, t, 1, thr) for t in range(10)]
    assert np.array_equal(a, b)
    assert np.array_equal(rec, np.concatenate(parts))
    e, hist = oracle_lib.observables(a, q)
    assert rec[-1, 0] == e and np.array_equal(rec[-1, 1:], hist)


def test_visiting_order_irrelevant(oracle_lib):
    L, q, seed = 16, 4, 8
    thr = oracle_lib.threshold_table(0.8)
    base = random_lattice(L, q, seed=2)
    rng = np.random.default_rng(0)
    for colour in (0, 1):
        ref = base.copy()
        oracle_lib.half_sweep(ref, q, seed, 3, colour, thr)
        for _ in range(3):
            s = base.copy()
            oracle_lib.half_sweep(s, q, seed, 3, colour, thr, order=rng.permutation(L * L))
            assert np.array_equal(s, ref)


def test_zero_temperature_quench_never_loses_bonds(oracle_lib):
    L, q, seed = 32, 5, 4
    s = oracle_lib.init(L, q, seed, 1)
    prev, _ = oracle_lib.observables(s, q)
    for t in range(20):
        for colour in (0, 1):
            oracle_lib.half_sweep(s, q, seed, t, colour, [0, 0, 0, 0])
            e, _ = oracle_lib.observables(s, q)
            assert e >= prev
            prev = e
    assert prev > 2 * L * L * 0.5


@pytest.mark.parametrize("start", [0, 1])
def test_window_matches_full_lattice(oracle_lib, start):
    L, q, seed, n = 32, 7, 13, 3
    thr = oracle_lib.threshold_table(0.9)
    full, _ = oracle_lib.run(L, q, seed, start, 0.9, n)
    for (x0, y0, h, w) in [(0, 0, 20, 24), (25, 27, 16, 16), (10, 3, 32, 32)]:
        win = oracle_lib.window(L, q, seed, start, n, thr, x0, y0, h, w)
        r = 2 * n
        ys = (y0 + np.arange(r, h - r)) % L
        xs = (x0 + np.arange(r, w - r)) % L
        assert np.array_equal(win[r:h - r, r:w - r], full[np.ix_(ys, xs)])


@pytest.mark.parametrize("args", [(3, 2), (6, 2), (8, 1), (8, 257), (0, 3)])
def test_rejects_bad_shapes(oracle_lib, args):
    L, q = args
    with pytest.raises(ValueError):
        oracle_lib.init(L, q, 1, 1) if L > 0 else oracle_lib.init(4, q, 1, 5)


def test_sweep_is_colour0_then_colour1(oracle_lib):
    """One MCS updates all sites of colour 0 ((x+y) even), then colour 1 (Sec. 3)."""
    L, q, seed = 16, 3, 31
    for thr in ([0, 0, 0, 0], oracle_lib.threshold_table(1.1)):
        a = random_lattice(L, q, seed=5)
        b = a.copy()
        oracle_lib.sweeps(a, q, seed, 4, 1, thr, record=False)
        oracle_lib.half_sweep(b, q, seed, 4, 0, thr)
        oracle_lib.half_sweep(b, q, seed, 4, 1, thr)
        assert np.array_equal(a, b)
        c = random_lattice(L, q, seed=5)
        oracle_lib.half_sweep(c, q, seed, 4, 1, thr)
        oracle_lib.half_sweep(c, q, seed, 4, 0, thr)
        assert not np.array_equal(a, c)
