"""The multi-sweep tile kernel (kernel 5: several sweeps per launch on LDS
tiles whose halos are recomputed) through the C ABI, bit for bit against the
oracle: spins and every per-sweep record, for every comparison-mode and
histogram class of q, tile shapes from the smallest (16 x 2, one sweep per
launch) to the largest that fits (256 x 32, eight sweeps), lattices smaller
than one tile with its halo, sweep counts that leave a partial last launch,
calls that change beta, a record ring shorter than the run, caller-owned
buffers (whose lattice must be current after every call), and switches to and
from the other kernels in the middle of a chain."""
import math

import numpy as np
import pytest

from tests.inputs import beta_c

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def potts():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_0876_amd as p

    p.load()
    return p


def _say(*args):
    print(*args, flush=True)


# L, q, seed, start, beta, sweeps, (tx, ty, sweeps per launch) or None (automatic)
CASES = [
    (16, 3, 1, 1, 1.2, 7, None),
    (48, 9, 2, 1, beta_c(9), 9, (16, 2, 1)),
    (64, 16, 3, 0, beta_c(16), 10, (32, 8, 3)),
    (96, 17, 4, 1, beta_c(17), 11, (32, 16, 8)),
    (160, 64, 5, 1, beta_c(64), 6, (32, 32, 2)),
    (256, 65, 6, 1, beta_c(65), 5, (256, 32, 4)),
    (528, 6, 7, 1, beta_c(6), 13, (16, 16, 5)),
    (512, 129, 8, 0, beta_c(129), 4, (128, 16, 8)),
    (1040, 256, 9, 1, beta_c(256), 5, None),
    (1024, 9, 10, 1, 1.02 * math.log(4.0), 17, None),
]


@pytest.mark.parametrize("L,q,seed,start,beta,n,shape", CASES)
def test_tiles_match_oracle(potts, oracle_lib, L, q, seed, start, beta, n, shape):
    _say(f"tiles L={L} q={q} seed={seed} start={start} n={n} shape={shape}")
    want_spins, want_rec = oracle_lib.run(L, q, seed, start, beta, n)
    with potts.Lattice(L, q, seed, start) as lat:
        lat.tune(kernel=5)
        if shape:
            lat.tune_tiles(*shape)
        lat.sweep(beta, n)
        got_rec = lat.records(0, n)
        got_spins = lat.spins()
        meas = lat.measure()
    assert np.array_equal(got_rec, want_rec)
    assert np.array_equal(got_spins, want_spins)
    assert meas["e_sat"] == want_rec[-1, 0] and np.array_equal(meas["hist"], want_rec[-1, 1:])


def test_tiles_calls_beta_changes_and_ring(potts, oracle_lib):
    """Calls of 1, 3, 8 and 5 sweeps at three temperatures, including caller
    tables with zero thresholds (the 64-bit acceptance table), on a ring of 8
    slots."""
    L, q, seed = 192, 7, 11
    tables = [oracle_lib.threshold_table(beta_c(q)), oracle_lib.threshold_table(0.9 * beta_c(q)),
              np.array([3, 0, 7, 0], dtype=np.uint32), oracle_lib.threshold_table(beta_c(q))]
    calls = [1, 3, 8, 5]
    s = oracle_lib.init(L, q, seed, 1)
    recs, t = [], 0
    for thr, n in zip(tables, calls):
        recs.append(oracle_lib.sweeps(s, q, seed, t, n, thr))
        t += n
    want = np.concatenate(recs)
    with potts.Lattice.from_torch(L, q, seed, 1, records_capacity=8) as lat:
        lat.tune(kernel=5)
        lat.tune_tiles(64, 16, 3)
        for thr, n in zip(tables, calls):
            lat.sweep_thr(thr, n)
        assert lat.t == t
        assert np.array_equal(lat.records(t - 7, 7), want[-7:])
        assert np.array_equal(lat.spins(), s)


def test_tiles_caller_buffers_current_after_each_call(potts, oracle_lib):
    """Caller-owned buffers: the lattice is in the caller's first buffer after
    every call, whether the call made an odd or an even number of launches,
    and a write into it between calls is where the next call starts."""
    import torch

    L, q, seed, beta = 128, 5, 13, beta_c(5)
    thr = oracle_lib.threshold_table(beta)
    s = oracle_lib.init(L, q, seed, 1)
    t = 0
    with potts.Lattice.from_torch(L, q, seed, 1) as lat:
        lat.tune(kernel=5)
        lat.tune_tiles(32, 8, 2)
        a, _, _ = lat._keep
        for n in (3, 4, 1):  # 2, 2 and 1 launches
            lat.sweep(beta, n)
            oracle_lib.sweeps(s, q, seed, t, n, thr, record=False)
            t += n
            torch.cuda.synchronize()
            assert np.array_equal(a.cpu().numpy().reshape(L, L), s), n
        s[:] = np.random.default_rng(5).integers(0, q, (L, L), dtype=np.uint8)
        a.copy_(torch.from_numpy(s.reshape(-1)).to(a.device))
        torch.cuda.synchronize()
        lat.sweep(beta, 3)
        oracle_lib.sweeps(s, q, seed, t, 3, thr, record=False)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy().reshape(L, L), s)


def test_tiles_switch_kernels_mid_chain(potts, oracle_lib):
    """Tile sweeps interleaved with the colour-split, strip and chunk kernels
    and with heat-bath sweeps on one state: the same chain as the oracle's."""
    L, q, seed, beta = 256, 6, 17, beta_c(6)
    thr = oracle_lib.threshold_table(beta)
    s = oracle_lib.init(L, q, seed, 1)
    t, recs = 0, []
    plan = [(5, 3, "m"), (0, 2, "m"), (5, 4, "m"), (1, 1, "m"), (0, 2, "h"), (5, 5, "m"), (2, 1, "m"), (5, 2, "h"),
            (5, 3, "m")]
    with potts.Lattice(L, q, seed, 1) as lat:
        for kernel, n, kind in plan:
            lat.tune(kernel=kernel)
            if kind == "m":
                lat.sweep(beta, n)
                recs.append(oracle_lib.sweeps(s, q, seed, t, n, thr))
            else:
                lat.sweep_heatbath(beta, n)
                recs.append(oracle_lib.heatbath_sweeps(s, q, seed, t, n, thr))
            t += n
        assert np.array_equal(lat.records(0, t), np.concatenate(recs))
        assert np.array_equal(lat.spins(), s)


def test_tiles_large_lattice(potts, oracle_lib):
    """L = 2048 (the Table 2 size) in the automatic tile shape: every site and
    record after 9 sweeps (two full launches and a partial one)."""
    L, q, seed, start, beta, n = 2048, 6, 21, 1, beta_c(6), 9
    _say(f"tiles large L={L}")
    want_spins, want_rec = oracle_lib.run(L, q, seed, start, beta, n)
    with potts.Lattice(L, q, seed, start) as lat:
        lat.tune(kernel=5)
        lat.sweep(beta, n)
        assert np.array_equal(lat.records(0, n), want_rec)
        assert np.array_equal(lat.spins(), want_spins)


def test_tiles_reject_bad_shapes(potts):
    with potts.Lattice(96, 3, 1, 1) as lat:
        for shape in [(24, 8, 2), (64, 8, 2), (32, 10, 2), (32, 9, 2), (32, 8, 9), (-16, 8, 2), (256, 256, 8)]:
            with pytest.raises(potts.PottsError):
                lat.tune_tiles(*shape)
        lat.tune_tiles(32, 8, 2)
    with potts.Lattice(20, 3, 1, 1) as lat:
        with pytest.raises(potts.PottsError):
            lat.tune(kernel=5)
