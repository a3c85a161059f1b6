"""First plus second neighbours through the C ABI (potts_nnn_*) against the
oracle's nine-colour chain: spins and every per-sweep record {e1, e2, hist}
bit-exact, caller tables, the record ring, the largest lattice, and the
argument checks."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def potts():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_0876_amd as p

    p.load()
    return p


CASES = [
    # L, q, seed, start, beta, j2, sweeps
    (12, 2, 1, 1, 0.3, 0.5, 8),        # one 12-byte block per row, wrap on both sides
    (24, 3, 2, 1, 0.7, -0.4, 6),       # frustrating second neighbours
    (36, 9, 3, 0, 1.0, 0.5, 5),
    (48, 256, 4, 1, 2.0, 1.0, 4),
    (60, 17, 5, 1, 1.2, 0.25, 4),
    (96, 100, 6, 1, 9.0, 0.5, 3),      # entries 0 for every dE > 0
    (120, 7, 7, 1, 0.0, 0.5, 3),       # beta = 0
    (600, 5, 8, 1, 0.9, 0.3, 3),
    (3084, 4, 9, 1, 0.8, 0.5, 1),      # 9.5 M sites: 257 blocks per row, more than one per thread
]


@pytest.mark.parametrize("kernel", [1, 2])
@pytest.mark.parametrize("L,q,seed,start,beta,j2,n", CASES)
def test_sweeps_match_oracle(potts, oracle_lib, L, q, seed, start, beta, j2, n, kernel):
    _say(f"nnn L={L} q={q} beta={beta} j2={j2} n={n} kernel={kernel}")
    s = oracle_lib.init(L, q, seed, start)
    rec = oracle_lib.nnn_sweeps(s, q, seed, 0, n, oracle_lib.nnn_table(beta, j2))
    with potts.NnnLattice(L, q, seed, start) as lat:
        lat.tune(kernel)
        lat.sweep(beta, j2, n)
        assert lat.t == n
        assert np.array_equal(lat.records(0, n), rec)
        assert np.array_equal(lat.spins(), s)
        e1, e2, hist = oracle_lib.nnn_observables(s, q)
        obs = lat.observables()
        assert (obs["e1"], obs["e2"], obs["t"]) == (e1, e2, n) and np.array_equal(obs["hist"], hist)


@pytest.mark.parametrize("L,q,seed", [(12, 3, 1), (36, 256, 2)])
def test_initial_conditions(potts, oracle_lib, L, q, seed):
    for start in (0, 1):
        with potts.NnnLattice(L, q, seed, start) as lat:
            assert np.array_equal(lat.spins(), oracle_lib.init(L, q, seed, start))


def test_caller_tables_and_split_calls(potts, oracle_lib):
    """Arbitrary tables (zeros, 2^32 and values in between, in no order), a
    change of (beta, j2) between calls, and calls split at any point."""
    L, q, seed = 48, 6, 12
    rng = np.random.default_rng(4)
    odd = rng.integers(0, 1 << 32, 81, dtype=np.uint64)
    odd[rng.integers(0, 81, 20)] = 0
    odd[rng.integers(0, 81, 20)] = 1 << 32
    t1, t2 = oracle_lib.nnn_table(0.6, 0.5), oracle_lib.nnn_table(0.9, -0.3)
    s = oracle_lib.init(L, q, seed, 1)
    r = [oracle_lib.nnn_sweeps(s, q, seed, 0, 2, t1), oracle_lib.nnn_sweeps(s, q, seed, 2, 3, odd),
         oracle_lib.nnn_sweeps(s, q, seed, 5, 2, t2)]
    with potts.NnnLattice(L, q, seed, 1) as lat:
        lat.sweep(0.6, 0.5, 1)
        lat.sweep(0.6, 0.5, 1)
        lat.sweep_thr(odd, 3)
        lat.sweep(0.9, -0.3, 2)
        assert np.array_equal(lat.records(0, 7), np.concatenate(r))
        assert np.array_equal(lat.spins(), s)


def test_record_ring(potts):
    with potts.NnnLattice(12, 3, 1, 1) as lat:
        lat.sweep(0.5, 0.5, 4100)
        with pytest.raises(potts.PottsError):
            lat.records(4, 1)
        with pytest.raises(potts.PottsError):
            lat.records(4099, 2)
        r = lat.records(5, 4095)
        assert np.all(r[:, 2:].sum(axis=1) == 144)
        obs = lat.observables()
        assert list(r[-1]) == [obs["e1"], obs["e2"], *obs["hist"]]


@pytest.mark.parametrize("L,q", [(16380, 3), (16392, 200)])
def test_row_class_limit(potts, oracle_lib, L, q):
    """The largest lattice the row-class kernel takes (three rows of 16380
    bytes in LDS) against the per-colour kernel, and the first one past it
    (automatic choice: per colour, row-class refused) against the oracle."""
    seed, beta, j2 = 5, 0.9, 0.4
    _say(f"nnn row-class limit L={L} q={q}")
    with potts.NnnLattice(L, q, seed, 1) as a:
        if L <= 16380:
            a.tune(1)
        else:
            with pytest.raises(potts.PottsError):
                a.tune(1)
        a.sweep(beta, j2, 1)
        got = a.spins()
        rec = a.records(0, 1)
    if L <= 16380:
        with potts.NnnLattice(L, q, seed, 1) as b:
            b.tune(2)
            b.sweep(beta, j2, 1)
            assert np.array_equal(b.records(0, 1), rec)
            assert np.array_equal(b.spins(), got)
        return
    s = oracle_lib.init(L, q, seed, 1)
    assert np.array_equal(oracle_lib.nnn_sweeps(s, q, seed, 0, 1, oracle_lib.nnn_table(beta, j2)), rec)
    assert np.array_equal(s, got)


# the largest lattice: L % 12 == 0 with L^2/4 below 2^32 (17.2 GB)
L_MAX = 131064


def test_maximum_lattice_frozen_ground_state(potts):
    """q = 256, beta = 9, j2 = 0.5 from the ordered start: a proposal k != 0
    costs dE = 4 + 0.5 * 4 = 6 (table entry 0), k = 0 changes nothing, so each
    record is e1 = e2 = 2N, N_0 = N: the record sums at their largest."""
    L, q, n = L_MAX, 256, 1
    _say(f"nnn maximum lattice L={L}")
    N = L * L
    with potts.NnnLattice(L, q, 3, 0) as lat:
        lat.sweep(9.0, 0.5, n)
        rec = lat.records(0, n)
    assert rec[0, 0] == 2 * N and rec[0, 1] == 2 * N and rec[0, 2] == N and not rec[0, 3:].any()


def test_rejects_bad_arguments(potts):
    with potts.NnnLattice(12, 3, 1, 1) as lat:
        for k in (-1, 3):
            with pytest.raises(potts.PottsError):
                lat.tune(k)
    for L, q in [(18, 3), (8, 3), (24, 1), (24, 257)]:
        with pytest.raises(potts.PottsError):
            potts.NnnLattice(L, q, 1, 1)
    with potts.NnnLattice(12, 3, 1, 1) as lat:
        with pytest.raises(potts.PottsError):
            lat.sweep(-1.0, 0.5, 1)
        with pytest.raises(potts.PottsError):
            lat.sweep(1.0, float("inf"), 1)
        with pytest.raises(potts.PottsError):
            lat.sweep(1.0, 0.5, -1)
        bad = np.zeros(81, dtype=np.uint64)
        bad[5] = (1 << 32) + 1
        with pytest.raises(potts.PottsError):
            lat.sweep_thr(bad, 1)
        lat.sweep(1.0, 0.5, 0)
        assert lat.t == 0
