"""GPU parity of the persistent band kernel (kernel 7): workgroups keep bands
of whole rows of the colour-split lattice in LDS for up to 64 sweeps per
cooperative launch and trade their edge rows after every half sweep.  Spins
and every record must equal the oracle's, bit for bit, for every band shape,
q class, table form, launch split and buffer ownership."""
import math

import numpy as np
import pytest

from tests.inputs import beta_c

pytestmark = pytest.mark.gpu


def _say(*args):
    print(*args, flush=True)


@pytest.fixture(scope="module")
def potts():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_0876_amd as p

    p.load()
    return p


# band shapes from 2 rows to the automatic ones, 256 / 512 / 1024 lanes, one
# and several items per lane, rows of 16-byte items not a power of two
# (L = 96, 3072), every q class (q <= 16 packed flags, q <= 64 lane-private
# counters, shared bins beyond, q > 128), both starts, odd sweep counts
@pytest.mark.parametrize("L,q,seed,start,beta,n,rows,block", [
    (64, 2, 1, 1, 0.7, 9, 2, 256),
    (96, 3, 4, 0, beta_c(3), 20, 4, 256),
    (128, 9, 3, 1, 1.02 * beta_c(9), 15, 8, 256),
    (256, 17, 6, 1, beta_c(17), 7, 8, 256),
    (512, 6, 2, 0, beta_c(6), 5, 16, 512),
    (1024, 65, 8, 1, 0.9 * beta_c(65), 3, 8, 256),
    (1024, 256, 9, 1, 0.3, 3, 16, 512),
    (1024, 9, 5, 1, beta_c(9), 4, 32, 1024),
    (2048, 6, 1, 1, beta_c(6), 4, 0, 0),
    (3072, 4, 5, 1, beta_c(4), 2, 12, 1024),
    (4096, 6, 2, 1, beta_c(6), 2, 0, 0),
])
def test_band_kernel_matches_oracle(potts, oracle_lib, L, q, seed, start, beta, n, rows, block):
    _say(f"band L={L} q={q} seed={seed} start={start} n={n} rows={rows} block={block}")
    want_spins, want_rec = oracle_lib.run(L, q, seed, start, beta, n)
    with potts.Lattice(L, q, seed, start) as lat:
        lat.tune(kernel=7)
        lat.tune_band(rows, block)
        lat.sweep(beta, n)
        assert np.array_equal(lat.records(0, n), want_rec)
        assert np.array_equal(lat.spins(), want_spins)


def test_band_kernel_across_launches_and_calls(potts, oracle_lib):
    """Runs of more than one launch (64 sweeps each), split over calls of
    uneven length, against the oracle."""
    L, q, seed, beta = 128, 5, 21, 0.95 * beta_c(5)
    _say(f"band launches L={L} q={q}")
    s = oracle_lib.init(L, q, seed, 1)
    want = oracle_lib.sweeps(s, q, seed, 0, 150, oracle_lib.threshold_table(beta))
    with potts.Lattice(L, q, seed, 1) as lat:
        lat.tune(kernel=7)
        lat.tune_band(4, 256)
        for n in (70, 3, 77):
            lat.sweep(beta, n)
        assert lat.t == 150
        assert np.array_equal(lat.records(0, 150), want)
        assert np.array_equal(lat.spins(), s)


def test_band_kernel_with_a_short_ring(potts, oracle_lib):
    """A record ring shorter than a launch: launches shrink to the ring, which
    then keeps the last capacity - 1 sweeps."""
    L, q, seed, beta = 256, 6, 7, beta_c(6)
    _say(f"band ring L={L}")
    s = oracle_lib.init(L, q, seed, 1)
    want = oracle_lib.sweeps(s, q, seed, 0, 45, oracle_lib.threshold_table(beta))
    with potts.Lattice(L, q, seed, 1) as lat:
        lat.reserve_records(16)
        lat.tune(kernel=7)
        lat.sweep(beta, 45)
        assert np.array_equal(lat.records(30, 15), want[30:])
        assert np.array_equal(lat.spins(), s)


def test_band_kernel_with_zero_thresholds(potts, oracle_lib):
    """A caller table with zero entries takes the 64-bit table form."""
    L, q, seed = 256, 4, 3
    thr = [2**31, 2**30, 0, 0]
    s = oracle_lib.init(L, q, seed, 1)
    want = oracle_lib.sweeps(s, q, seed, 0, 11, thr)
    with potts.Lattice(L, q, seed, 1) as lat:
        lat.tune(kernel=7)
        lat.sweep_thr(thr, 11)
        assert np.array_equal(lat.records(0, 11), want)
        assert np.array_equal(lat.spins(), s)


def test_band_kernel_on_caller_buffers(potts, oracle_lib):
    """Caller-owned buffers hold the row-major lattice after every call, and
    the kernels in between see writes made through them."""
    import torch

    L, q, seed, beta = 512, 9, 11, beta_c(9)
    _say(f"band torch buffers L={L}")
    thr = oracle_lib.threshold_table(beta)
    s = oracle_lib.init(L, q, seed, 1)
    want = oracle_lib.sweeps(s, q, seed, 0, 6, thr)
    with potts.Lattice.from_torch(L, q, seed, 1) as lat:
        lat.tune(kernel=7)
        lat.sweep(beta, 6)
        torch.cuda.synchronize()
        buf = lat._keep[0].cpu().numpy().reshape(L, L)
        assert np.array_equal(buf, s)
        assert np.array_equal(lat.records(0, 6), want)


def test_band_kernel_equals_colour_split_kernel(potts):
    """The band kernel and the streaming colour-split kernel (kernel 4) give
    the same chain on a lattice of the automatic band range, with kernels
    switched between calls."""
    L, q, seed, beta = 4096, 9, 1, 1.02 * math.log(4.0)
    _say(f"band vs colour-split L={L}")
    out = []
    for plan in ((4, 4, 4), (7, 7, 7), (7, 4, 7)):
        with potts.Lattice(L, q, seed, potts.RANDOM) as lat:
            for k, n in zip(plan, (5, 64, 7)):
                lat.tune(kernel=k)
                lat.sweep(beta, n)
            out.append((lat.spins(), lat.records(0, 76)))
    for spins, rec in out[1:]:
        assert np.array_equal(spins, out[0][0])
        assert np.array_equal(rec, out[0][1])


def test_band_kernel_reports_an_expired_wait(potts, oracle_lib, monkeypatch):
    """A wait bound set too short (1 us, from the host) makes neighbour waits
    expire; every workgroup still exits, the next read reports EDEVICE, and
    the state sweeps correctly again once the bound is restored."""
    L, q, seed, beta = 2048, 6, 4, beta_c(6)
    _say(f"band expired wait L={L}")
    s0 = oracle_lib.init(L, q, seed, 1)
    monkeypatch.setenv("POTTS_BAND_WAIT_US", "1")
    with potts.Lattice(L, q, seed, 1) as lat:
        lat.tune(kernel=7)
        lat.sweep(beta, 64)
        try:
            rec = lat.records(0, 64)
        except potts.PottsError:
            rec = None
        if rec is not None:  # every wait happened to be met at once: then the result is exact
            want = oracle_lib.sweeps(s0.copy(), q, seed, 0, 64, oracle_lib.threshold_table(beta))
            assert np.array_equal(rec, want)
        monkeypatch.delenv("POTTS_BAND_WAIT_US")
        s = s0.copy()
        want = oracle_lib.sweeps(s, q, seed, 0, 3, oracle_lib.threshold_table(beta))
        lat.set_spins(s0, 0)
        lat.sweep(beta, 3)
        assert np.array_equal(lat.records(0, 3), want)
        assert np.array_equal(lat.spins(), s)


def test_band_kernel_rejects_shapes_it_cannot_take(potts):
    with potts.Lattice(80, 3, 1, 0) as lat:  # L % 32 != 0
        with pytest.raises(potts.PottsError):
            lat.tune(kernel=7)
    with potts.Lattice(1024, 3, 1, 0) as lat:
        for rows, block in ((3, 256), (6, 256), (8, 128), (8, 32), (0, 256)):
            with pytest.raises(potts.PottsError):
                lat.tune_band(rows, block)
        lat.tune_band(8, 0)


def test_band_kernel_on_two_streams_at_once(potts, oracle_lib):
    """Two lattices of the band range sweep on two streams at the same time
    (their cooperative launches queued together): both chains equal the
    oracle's."""
    import torch

    q, beta, n = 6, beta_c(6), 8
    _say("band two streams L=2048 and L=4096")
    jobs = [(2048, 3), (4096, 4)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    lats = [potts.Lattice.on_stream(L, q, seed, potts.RANDOM, stream=st) for (L, seed), st in zip(jobs, streams)]
    try:
        for lat in lats:
            lat.tune(kernel=7)
        for lat in lats:  # both queued before either is waited for
            lat.sweep(beta, n)
        torch.cuda.synchronize()
        for (L, seed), lat in zip(jobs, lats):
            s = oracle_lib.init(L, q, seed, 1)
            want = oracle_lib.sweeps(s, q, seed, 0, n, oracle_lib.threshold_table(beta))
            assert np.array_equal(lat.records(0, n), want)
            assert np.array_equal(lat.spins(), s)
    finally:
        for lat in lats:
            lat.close()


@pytest.mark.parametrize("L,n", [(2048, 3000), (4096, 1000)])
def test_band_kernel_long_chain_equals_colour_split_kernel(potts, L, n):
    """Thousands of edge-row exchanges (2 x n half sweeps between every pair
    of neighbouring bands): the band kernel's chain, every record and the
    final lattice, equals the streaming colour-split kernel's, so no half
    sweep read a stale edge row."""
    q, seed, beta = 6, 12, beta_c(6)
    _say(f"band long chain L={L} n={n}")
    out = []
    for kernel in (4, 7):
        with potts.Lattice(L, q, seed, potts.RANDOM) as lat:
            lat.reserve_records(n + 1)
            lat.tune(kernel=kernel)
            lat.sweep(beta, n)
            out.append((lat.spins(), lat.records(0, n)))
    assert np.array_equal(out[1][1], out[0][1])
    assert np.array_equal(out[1][0], out[0][0])


def test_band_kernel_with_checkpoints_ramps_and_heat_bath(potts, oracle_lib, tmp_path):
    """The band path (the automatic choice at L = 2048) inside a chain that
    also checkpoints and resumes, and interleaves heat-bath sweeps (which run
    on the same colour-split copy): spins and records equal the oracle's."""
    L, q, seed = 2048, 7, 5
    b1, b2 = beta_c(7), 1.05 * beta_c(7)
    _say(f"band chain with checkpoint and heat bath L={L}")
    s = oracle_lib.init(L, q, seed, 1)
    want = [oracle_lib.sweeps(s, q, seed, 0, 5, oracle_lib.threshold_table(b1)),
            oracle_lib.heatbath_sweeps(s, q, seed, 5, 2, oracle_lib.threshold_table(b2)),
            oracle_lib.sweeps(s, q, seed, 7, 4, oracle_lib.threshold_table(b2))]
    want = np.concatenate(want)
    path = str(tmp_path / "band.ckpt")
    with potts.Lattice(L, q, seed, 1) as lat:
        lat.sweep(b1, 5)
        lat.save(path)
    with potts.Lattice.load_checkpoint(path) as lat:
        assert lat.t == 5
        lat.sweep_heatbath(b2, 2)
        lat.sweep(b2, 4)
        assert np.array_equal(lat.records(5, 6), want[5:])
        assert np.array_equal(lat.spins(), s)


def test_band_kernel_ramp_equals_colour_split_ramp(potts):
    """potts_ramp over the band path: the per-point statistics equal those of
    the same ramp on the streaming colour-split kernel."""
    L, q, seed = 4096, 6, 8
    betas = [0.98 * beta_c(6), beta_c(6), 1.02 * beta_c(6)]
    _say(f"band ramp L={L}")
    out = []
    for kernel in (4, 0):
        with potts.Lattice(L, q, seed, potts.ORDERED) as lat:
            lat.tune(kernel=kernel)
            out.append(lat.ramp(betas, 30, 40))
    assert out[0] == out[1]


def test_band_kernel_seeded_shapes_equal_colour_split_kernel(potts):
    """Seeded draws of lattice size (multiples of 32 from 64 to 4096, many
    not powers of two: rows of an odd number of items, edge rows that end
    inside a wave), band height, lanes, q, start and temperature: each band
    chain equals the streaming colour-split kernel's, every record and the
    final lattice."""
    rng = np.random.default_rng(20261203)
    done = 0
    for _ in range(400):
        if done == 14:
            break
        L = 32 * int(rng.integers(2, 129))
        rows = int(rng.choice([2, 4, 6, 8, 10, 12, 16, 20, 24, 32]))
        block = int(rng.choice([256, 512, 1024]))
        q = int(rng.choice([2, 3, 5, 9, 16, 17, 40, 64, 65, 200]))
        start = int(rng.integers(0, 2))
        beta = float(rng.uniform(0.9, 1.1)) * beta_c(q)
        n = int(rng.integers(1, 90))
        seed = 100 + done
        out = []
        for kernel in (7, 4):
            with potts.Lattice(L, q, seed, start) as lat:
                try:
                    lat.tune(kernel=kernel)
                    if kernel == 7:
                        lat.tune_band(rows, block)
                except potts.PottsError:
                    break  # a shape this lattice cannot take: draw again
                if kernel == 7:
                    _say(f"band seeded L={L} rows={rows} block={block} q={q} start={start} n={n}")
                lat.sweep(beta, n)
                out.append((lat.spins(), lat.records(0, n)))
        if len(out) < 2:
            continue
        assert np.array_equal(out[0][1], out[1][1]), (L, rows, block, q, n)
        assert np.array_equal(out[0][0], out[1][0]), (L, rows, block, q, n)
        done += 1
    assert done == 14
