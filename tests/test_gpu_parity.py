"""GPU parity: the HIP sweep through the C ABI against the CPU oracle, bit for bit
on spins and integer records, to 1e-12 relative on derived FP64 statistics."""
import math
import os

import numpy as np
import pytest

from tests.inputs import PARITY_CASES, beta_c, random_lattice

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


@pytest.mark.parametrize("L,q,seed,start,beta,n", PARITY_CASES)
def test_sweeps_match_oracle(potts, oracle_lib, L, q, seed, start, beta, n):
    _say(f"parity L={L} q={q} seed={seed} start={start} beta={beta} n={n}")
    want_spins, want_rec = oracle_lib.run(L, q, seed, start, beta, n)
    with potts.Lattice(L, q, seed, start) as lat:
        assert np.array_equal(lat.spins(), oracle_lib.init(L, q, seed, start))
        lat.sweep(beta, n)
        got_rec = lat.records(0, n)
        got_spins = lat.spins()
        obs = lat.observables()
        meas = lat.measure()
    assert np.array_equal(got_spins, want_spins)
    assert np.array_equal(got_rec, want_rec)
    assert obs["e_sat"] == want_rec[-1, 0] and np.array_equal(obs["hist"], want_rec[-1, 1:])
    assert meas["e_sat"] == obs["e_sat"] and np.array_equal(meas["hist"], obs["hist"])
    assert obs["nmax"] == want_rec[-1, 1:].max()


@pytest.mark.parametrize("q", [2, 3, 16, 17, 255, 256])
@pytest.mark.parametrize("start", [0, 1])
def test_init_matches_oracle(potts, oracle_lib, q, start):
    L = 68
    _say(f"init L={L} q={q} start={start}")
    with potts.Lattice(L, q, 77, start) as lat:
        assert np.array_equal(lat.spins(), oracle_lib.init(L, q, 77, start))
        m = lat.measure()
    e, hist = oracle_lib.observables(oracle_lib.init(L, q, 77, start), q)
    assert m["e_sat"] == e and np.array_equal(m["hist"], hist) and m["t"] == 0


def test_beta_schedule_and_chunked_calls(potts, oracle_lib):
    L, q, seed = 48, 9, 5
    schedule = [(beta_c(9) * 0.98, 3), (beta_c(9), 1), (beta_c(9) * 1.02, 4), (0.0, 2), (9.0, 2)]
    _say(f"schedule L={L} q={q}")
    s = oracle_lib.init(L, q, seed, 1)
    want = []
    t = 0
    for beta, n in schedule:
        want.append(oracle_lib.sweeps(s, q, seed, t, n, oracle_lib.threshold_table(beta)))
        t += n
    with potts.Lattice(L, q, seed, 1) as lat:
        for beta, n in schedule:
            lat.sweep(beta, n)
        assert lat.t == t
        assert np.array_equal(lat.records(0, t), np.concatenate(want))
        assert np.array_equal(lat.spins(), s)


def test_caller_threshold_table(potts, oracle_lib):
    L, q, seed = 16, 4, 3
    thr = [2**31, 2**30, 12345, 0]
    s = oracle_lib.init(L, q, seed, 1)
    want = oracle_lib.sweeps(s, q, seed, 0, 5, thr)
    with potts.Lattice(L, q, seed, 1) as lat:
        lat.sweep_thr(thr, 5)
        assert np.array_equal(lat.records(0, 5), want)
        assert np.array_equal(lat.spins(), s)


def test_set_spins_and_resume(potts, oracle_lib, tmp_path):
    L, q, seed, beta = 40, 7, 12, 1.1
    base = random_lattice(L, q, seed=8)
    s = base.copy()
    want = oracle_lib.sweeps(s, q, seed, 1000, 6, oracle_lib.threshold_table(beta))
    with potts.Lattice(L, q, seed, 0) as lat:
        lat.set_spins(base, 1000)
        lat.sweep(beta, 3)
        path = str(tmp_path / "ck.bin")
        lat.save(path)
        lat.sweep(beta, 3)
        assert np.array_equal(lat.records(1000, 6), want)
        assert np.array_equal(lat.spins(), s)
        with pytest.raises(potts.PottsError):
            lat.records(999, 1)
    with potts.Lattice.load_checkpoint(path) as lat2:
        assert lat2.t == 1003
        lat2.sweep(beta, 3)
        assert np.array_equal(lat2.spins(), s)
        assert np.array_equal(lat2.records(1003, 3), want[3:])


def test_set_spins_rejects_values_ge_q(potts):
    with potts.Lattice(8, 3, 1, 0) as lat:
        bad = np.zeros((8, 8), dtype=np.uint8)
        bad[3, 3] = 3
        with pytest.raises(potts.PottsError):
            lat.set_spins(bad, 0)


@pytest.mark.parametrize("asked,slots", [(6, 8), (8, 8), (2, 2)])
def test_record_ring_wraps(potts, oracle_lib, asked, slots):
    """The ring keeps a power-of-two number of slots (>= the capacity asked
    for); the last slots - 1 records survive any chunking of the sweeps."""
    import torch

    q, seed, beta, n = 5, 2, 0.9, 23
    # records cleared per sweep (chunk kernel), written whole (resident), folded
    # from partial records (strip, colour-split)
    for kernel, L in ((2, 16), (3, 16), (1, 32), (4, 32)):
        _, want = oracle_lib.run(L, q, seed, 1, beta, n)
        lat = potts.Lattice.from_torch(L, q, seed, 1, records_capacity=asked)
        with lat:
            lat.tune(kernel=kernel)
            for chunk in (4, 1, 7, 11):
                lat.sweep(beta, chunk)
            torch.cuda.synchronize()
            assert np.array_equal(lat.records(n - slots + 1, slots - 1), want[n - slots + 1:])
            with pytest.raises(potts.PottsError):
                lat.records(n - slots, 1)
            with pytest.raises(potts.PottsError):
                lat.records(n - 1, 2)


def test_torch_buffers_and_stream(potts, oracle_lib):
    import torch

    L, q, seed, beta, n = 64, 9, 1, 1.02 * math.log(4.0), 25
    want_spins, want_rec = oracle_lib.run(L, q, seed, 1, beta, n)
    stream = torch.cuda.Stream()
    lat = potts.Lattice.from_torch(L, q, seed, 1, stream=stream)
    with lat:
        lat.sweep(beta, n)
        ptr = lat.device_ptr()  # may queue work on the stream: synchronize after it
        stream.synchronize()
        a, _, _ = lat._keep
        assert ptr == a.data_ptr()
        assert np.array_equal(a.cpu().numpy().reshape(L, L), want_spins)
        assert np.array_equal(lat.records(0, n), want_rec)


def test_colour_split_copy_stays_in_step(potts, oracle_lib):
    """Single colour-split sweeps keep the lattice split into colour planes
    between calls; every read (spins, measure, device pointer), a switch to
    other kernels and set_spins must see and continue the same chain."""
    import torch

    L, q, seed, beta = 512, 7, 29, beta_c(7)
    thr = oracle_lib.threshold_table(beta)
    s = oracle_lib.init(L, q, seed, 1)
    t = 0

    def oracle_sweeps(n):
        nonlocal t
        oracle_lib.sweeps(s, q, seed, t, n, thr, record=False)
        t += n

    with potts.Lattice.from_torch(L, q, seed, 1) as lat:
        lat.tune(kernel=4)
        for n in (1, 1, 2):
            lat.sweep(beta, n)
            oracle_sweeps(n)
        assert np.array_equal(lat.spins(), s)
        lat.sweep(beta, 1)
        oracle_sweeps(1)
        e, hist = oracle_lib.observables(s, q)
        m = lat.measure()
        assert m["e_sat"] == e and np.array_equal(m["hist"], hist)
        lat.sweep(beta, 1)
        oracle_sweeps(1)
        a, b, _ = lat._keep
        ptr = lat.device_ptr()
        torch.cuda.synchronize()
        cur = a if ptr == a.data_ptr() else b
        assert np.array_equal(cur[:L * L].cpu().numpy().reshape(L, L), s)
        for kernel, n in ((1, 2), (4, 1), (2, 1), (0, 3)):
            lat.tune(kernel=kernel)
            lat.sweep(beta, n)
            oracle_sweeps(n)
        lat.sweep(beta, 1)
        oracle_sweeps(1)
        # overwrite the lattice mid-chain and continue from a new counter
        s[:] = np.random.default_rng(3).integers(0, q, (L, L), dtype=np.uint8)
        t = 40
        lat.set_spins(s, t)
        lat.sweep(beta, 2)
        oracle_sweeps(2)
        assert lat.t == t
        assert np.array_equal(lat.spins(), s)


def test_caller_buffer_holds_the_lattice_between_calls(potts, oracle_lib):
    """Caller-owned buffers on the colour-split path: after every sweep call the
    caller's dev_spins tensor holds the row-major lattice (read directly, with
    no library call), and a configuration the caller writes into it between
    calls is where the next sweep starts."""
    import torch

    L, q, seed, beta = 512, 6, 9, beta_c(6)
    thr = oracle_lib.threshold_table(beta)
    s = oracle_lib.init(L, q, seed, 1)
    stream = torch.cuda.Stream()
    with potts.Lattice.from_torch(L, q, seed, 1, stream=stream) as lat:
        lat.tune(kernel=4)
        a, _, _ = lat._keep
        for n, t in ((3, 0), (1, 3)):
            lat.sweep(beta, n)
            stream.synchronize()
            oracle_lib.sweeps(s, q, seed, t, n, thr, record=False)
            assert np.array_equal(a[:L * L].cpu().numpy().reshape(L, L), s), t
        w = np.random.default_rng(5).integers(0, q, (L, L), dtype=np.uint8)
        with torch.cuda.stream(stream):
            a[:L * L].copy_(torch.from_numpy(w.ravel()).to(a.device, non_blocking=False))
        lat.sweep(beta, 2)
        stream.synchronize()
        rec = oracle_lib.sweeps(w, q, seed, 4, 2, thr)
        assert np.array_equal(a[:L * L].cpu().numpy().reshape(L, L), w)
        assert np.array_equal(lat.records(4, 2), rec)
        assert np.array_equal(lat.spins(), w)


def test_device_pointer_writes_reach_the_next_sweep(potts, oracle_lib):
    """A library-owned state keeps its colour-split copy between calls; a
    configuration written through potts_device_spins between calls is where
    the next sweep starts."""
    import ctypes

    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    hip.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
    L, q, seed, beta = 512, 5, 13, beta_c(5)
    thr = oracle_lib.threshold_table(beta)
    with potts.Lattice(L, q, seed, 1) as lat:
        lat.sweep(beta, 2)
        ptr = lat.device_ptr()
        assert hip.hipStreamSynchronize(ctypes.c_void_p(lat.stream_ptr())) == 0
        w = np.random.default_rng(6).integers(0, q, (L, L), dtype=np.uint8)
        assert hip.hipMemcpy(ctypes.c_void_p(ptr), w.ctypes.data_as(ctypes.c_void_p), L * L, 1) == 0
        assert hip.hipDeviceSynchronize() == 0
        lat.sweep(beta, 3)
        rec = oracle_lib.sweeps(w, q, seed, 2, 3, thr)
        assert np.array_equal(lat.records(2, 3), rec)
        assert np.array_equal(lat.spins(), w)


@pytest.mark.parametrize("window", [(0, 200), (150, 400), (7, 8)])
def test_derived_stats_match_oracle(potts, oracle_lib, window):
    from oracle.stats import derived

    L, q, seed, beta, n = 32, 6, 4, beta_c(6), 400
    _, rec = oracle_lib.run(L, q, seed, 1, beta, n)
    t0, t1 = window
    with potts.Lattice(L, q, seed, 1) as lat:
        lat.sweep(beta, n)
        got = lat.stats(t0, t1 - t0, beta)
    want = derived(rec[t0:t1, 0].tolist(), rec[t0:t1, 1:].max(axis=1).tolist(), L * L, q, beta)
    for k in ("e", "C", "V_L", "m", "chi"):
        assert got[k] == pytest.approx(want[k], rel=1e-12, abs=1e-300), k


@pytest.mark.parametrize("start,torch_buffers", [(1, False), (0, True)])
def test_large_lattice_sampled_windows(potts, oracle_lib, start, torch_buffers):
    """L = 32768 (the single-large-lattice workload, both of its starts; the
    ordered one on torch-owned buffers and stream, as the benchmark builds
    it): sampled windows against the oracle's window restriction, plus
    whole-lattice invariants."""
    L, q, seed, beta, n = 32768, 6, 1, beta_c(6), 2
    _say(f"large L={L} q={q} n={n} start={start}")
    thr = oracle_lib.threshold_table(beta)
    make = potts.Lattice.from_torch if torch_buffers else potts.Lattice
    with make(L, q, seed, start) as lat:
        lat.tune(kernel=0)
        lat.sweep(beta, n)
        rec = lat.records(0, n)
        spins = lat.spins()
        meas = lat.measure()
    N = L * L
    assert np.all(rec[:, 1:].sum(axis=1) == N)
    assert np.all((rec[:, 0] >= 0) & (rec[:, 0] <= 2 * N))
    assert meas["e_sat"] == rec[-1, 0] and np.array_equal(meas["hist"], rec[-1, 1:])
    r = 2 * n
    for (x0, y0) in [(0, 0), (L - 20, L - 13), (12345, 777), (L // 2, L - 30), (4096, 0)]:
        h = w = 48
        win = oracle_lib.window(L, q, seed, start, n, thr, x0, y0, h, w)
        ys = (y0 + np.arange(r, h - r)) % L
        xs = (x0 + np.arange(r, w - r)) % L
        assert np.array_equal(win[r:h - r, r:w - r], spins[np.ix_(ys, xs)]), (x0, y0)


# the largest lattices: L = 65520 is the largest the strip kernel takes (just
# below 4 GiB); L = 65536 (4 GiB, e_sat up to 2^33) runs on the chunk kernel
MAX_LATTICES = [65520, 65536]


@pytest.mark.parametrize("L", MAX_LATTICES)
def test_maximum_lattice_frozen_ground_state(potts, L):
    """q = 256 at beta = 9 from the ordered start: every proposal costs dE = 4,
    whose threshold floor(exp(-36) 2^32) is 0, so the lattice never changes:
    each record is e_sat = 2N, N_0 = N, and the window statistics are e = -2,
    C = 0, V_L = 2/3, m = 1, chi = 0 (Eq. 7, Eq. 9) -- through the exact
    integer moments at their largest values."""
    q, n = 256, 3
    _say(f"maximum lattice L={L} q={q} ordered beta=9")
    N = L * L
    with potts.Lattice.from_torch(L, q, 5, 0, records_capacity=4) as lat:
        lat.sweep(9.0, n)
        rec = lat.records(0, n)
        s = lat.stats(0, n, 9.0)
        r = lat.reweight(0, n, 9.0, [9.0, 9.5])
    assert np.all(rec[:, 0] == 2 * N) and np.all(rec[:, 1] == N) and not rec[:, 2:].any()
    assert s["e"] == -2.0 and s["C"] == 0.0 and s["m"] == 1.0 and s["chi"] == 0.0
    assert s["V_L"] == pytest.approx(2.0 / 3.0, rel=1e-15)
    for x in r:
        assert x["e"] == -2.0 and x["C"] == 0.0 and x["m"] == 1.0 and x["chi"] == 0.0
        assert x["V_L"] == pytest.approx(2.0 / 3.0, rel=1e-15)


@pytest.mark.parametrize("L", MAX_LATTICES)
def test_maximum_lattice_sampled_windows(potts, oracle_lib, L):
    """A random start and one sweep: windows at the corners (the lattice's
    last bytes included), the last rows and the last columns against the
    oracle's window restriction."""
    import torch

    q, seed, beta, n = 7, 21, beta_c(7), 1
    _say(f"maximum lattice L={L} q={q} random windows")
    thr = oracle_lib.threshold_table(beta)
    with potts.Lattice.from_torch(L, q, seed, 1, records_capacity=4) as lat:
        lat.sweep(beta, n)
        rec = lat.records(0, n)
        a, b, _ = lat._keep
        cur = (a if lat.device_ptr() == a.data_ptr() else b)[:L * L].view(L, L)
        torch.cuda.synchronize()
        assert int(rec[0, 1:].sum()) == L * L
        r, h, w = 2 * n, 24, 24
        for (x0, y0) in [(0, 0), (L - 12, L - 12), (L - 20, L - 20), (40000, L - 20), (L - 20, 50000),
                         (65000 % L, 1)]:
            win = oracle_lib.window(L, q, seed, 1, n, thr, x0, y0, h, w)
            ys = torch.tensor((y0 + np.arange(r, h - r)) % L, device=cur.device)
            xs = torch.tensor((x0 + np.arange(r, w - r)) % L, device=cur.device)
            got = cur.index_select(0, ys).index_select(1, xs).cpu().numpy()
            assert np.array_equal(win[r:h - r, r:w - r], got), (x0, y0)


def test_oracle_observables_of_large_lattice(potts, oracle_lib):
    L, q, seed, beta = 8192, 15, 3, beta_c(15)
    with potts.Lattice(L, q, seed, 0) as lat:
        lat.sweep(beta, 3)
        rec = lat.records(2, 1)
        spins = lat.spins()
    e, hist = oracle_lib.observables(np.ascontiguousarray(spins), q)
    assert rec[0, 0] == e and np.array_equal(rec[0, 1:], hist)


# q at the edges of the kernels' comparison modes (<=16, <=128, <=256) and of
# the lane-private histogram (<=32); L with power-of-two and other row widths;
# every kernel that takes the shape: 1 strip (any L % 16 == 0), 3 LDS-resident
# (L <= 256), 4 colour-split (L % 32 == 0)
Q_EDGE_SHAPES = [(48, 16), (48, 17), (80, 32), (80, 33), (96, 64), (96, 65), (96, 128), (112, 129), (208, 256),
                 (1040, 9), (64, 2), (128, 3), (16, 7), (224, 256), (1056, 9), (320, 33)]
Q_EDGE_CASES = [(L, q, k) for (L, q) in Q_EDGE_SHAPES for k in (1, 3, 4)
                if not (k == 3 and L > 256) and not (k == 4 and L % 32)]


@pytest.mark.parametrize("L,q,kernel", Q_EDGE_CASES)
def test_kernel_q_edges(potts, oracle_lib, L, q, kernel):
    seed, beta, n = 6, 0.9, 7
    _say(f"q-edge L={L} q={q} kernel={kernel}")
    want_spins, want_rec = oracle_lib.run(L, q, seed, 1, beta, n)
    with potts.Lattice(L, q, seed, 1) as lat:
        lat.tune(kernel=kernel)
        lat.sweep(beta, n)
        assert np.array_equal(lat.records(0, n), want_rec)
        assert np.array_equal(lat.spins(), want_spins)


def test_resident_long_run_plain_method(potts, oracle_lib):
    """The plain-method workload (q=9, L=64, random start, seed 1,
    beta = 1.02 ln 4, 1000 sweeps) in full, on the default (LDS-resident) path."""
    L, q, seed, beta, n = 64, 9, 1, 1.02 * math.log(4.0), 1000
    want_spins, want_rec = oracle_lib.run(L, q, seed, 1, beta, n)
    with potts.Lattice(L, q, seed, 1) as lat:
        lat.sweep(beta, n)
        assert np.array_equal(lat.records(0, n), want_rec)
        assert np.array_equal(lat.spins(), want_spins)


def test_resident_chunked_launches(potts, oracle_lib):
    """More sweeps than one resident launch holds (4096) and a ring smaller
    than the run."""
    L, q, seed, beta, n = 16, 3, 8, 1.0, 5000
    want_spins, want_rec = oracle_lib.run(L, q, seed, 0, beta, n)
    lat = potts.Lattice.from_torch(L, q, seed, 0, records_capacity=1000)
    with lat:
        lat.sweep(beta, n)
        assert np.array_equal(lat.records(n - 999, 999), want_rec[n - 999:])
        assert np.array_equal(lat.spins(), want_spins)


@pytest.mark.parametrize("L", [64, 96, 256, 1024])
def test_launch_shape_does_not_change_results(potts, oracle_lib, L):
    """Random numbers are keyed by (seed, site, sweep): every kernel, strip
    height and grid size must give the same bits."""
    q, seed, beta, n = 9, 11, 1.4, 6
    want_spins, want_rec = oracle_lib.run(L, q, seed, 1, beta, n)
    shapes = [(2, 0, 0), (1, 0, 0), (1, 2, 1), (1, 2, 7), (1, 4, 0), (1, 8, 3), (1, 16, 64), (1, 32, 0),
              (3, 0, 0), (4, 0, 0), (4, 2, 1), (4, 8, 3), (4, 16, 0), (4, 32, 5)]
    for kernel, rows, groups in shapes:
        if rows and L % rows:
            continue
        if kernel == 3 and L > 256:
            continue
        _say(f"shape L={L} kernel={kernel} rows={rows} groups={groups}")
        with potts.Lattice(L, q, seed, 1) as lat:
            lat.tune(kernel, rows, groups)
            lat.sweep(beta, n)
            assert np.array_equal(lat.records(0, n), want_rec), (kernel, rows, groups)
            assert np.array_equal(lat.spins(), want_spins), (kernel, rows, groups)


@pytest.mark.parametrize("L,q,start", [(512, 6, 1), (1056, 16, 0), (96, 9, 1), (512, 40, 1)])
def test_occupancy_does_not_change_results(potts, oracle_lib, L, q, start):
    """The colour-split kernel asked for 8 waves per SIMD (q <= 16; other q
    keep the default variant) gives the same bits, alone and switched
    mid-chain."""
    seed, beta, n = 31, beta_c(q), 5
    want_spins, want_rec = oracle_lib.run(L, q, seed, start, beta, n)
    with potts.Lattice(L, q, seed, start) as lat:
        if L % 32 == 0:
            lat.tune(kernel=4)
        lat.tune_occupancy(8)
        lat.sweep(beta, 3)
        lat.tune_occupancy(0)
        lat.sweep(beta, 1)
        lat.tune_occupancy(8)
        lat.sweep(beta, 1)
        assert np.array_equal(lat.records(0, n), want_rec)
        assert np.array_equal(lat.spins(), want_spins)
        with pytest.raises(potts.PottsError):
            lat.tune_occupancy(4)


@pytest.mark.parametrize("L,q,K", [(512, 6, 8), (1056, 40, 4), (96, 9, 3)])
def test_graph_replay_does_not_change_results(potts, oracle_lib, L, q, K):
    """Colour-split sweeps replayed from a captured graph of K sweeps (whole
    graphs first, the remainder launched directly), across calls, a change
    of beta and of occupancy, with a ring shorter than the run."""
    seed = 17
    betas = [beta_c(q), 0.95 * beta_c(q), beta_c(q)]
    calls = [2 * K + 3, 2 * K, K - 1]
    s = oracle_lib.init(L, q, seed, 1)
    t, recs = 0, []
    for b, n in zip(betas, calls):
        recs.append(oracle_lib.sweeps(s, q, seed, t, n, oracle_lib.threshold_table(b)))
        t += n
    want = np.concatenate(recs)
    import torch

    stream = torch.cuda.Stream()  # a stream that can be captured
    with potts.Lattice.from_torch(L, q, seed, 1, stream=stream, records_capacity=64) as lat:
        if L % 32 == 0:
            lat.tune(kernel=4)
        lat.tune_graph(K)
        for i, (b, n) in enumerate(zip(betas, calls)):
            if i == 2 and q <= 16:
                lat.tune_occupancy(8)
            lat.sweep(b, n)
        assert lat.t == t
        n = min(t, 40)  # the last records the 64-slot ring still holds
        assert np.array_equal(lat.records(t - n, n), want[-n:])
        assert np.array_equal(lat.spins(), s)
    with potts.Lattice(20, 3, 1, 1) as lat:
        with pytest.raises(potts.PottsError):
            lat.tune_graph(-1)


def test_tune_rejects_bad_shapes(potts):
    with potts.Lattice(20, 3, 1, 1) as lat:
        with pytest.raises(potts.PottsError):
            lat.tune(kernel=1)  # 20 % 16 != 0
        with pytest.raises(potts.PottsError):
            lat.tune(kernel=3)  # 20 % 16 != 0
        with pytest.raises(potts.PottsError):
            lat.tune(kernel=4)
        with pytest.raises(potts.PottsError):
            lat.tune(kernel=5)
        with pytest.raises(potts.PottsError):
            lat.tune(kernel=0, strip_rows=3)
    with potts.Lattice(48, 3, 1, 1) as lat:
        with pytest.raises(potts.PottsError):
            lat.tune(kernel=4)  # 48 % 32 != 0


@pytest.mark.parametrize("L,start", [(64, 0), (64, 1), (512, 1), (100, 0)])
def test_ramp_matches_oracle(potts, oracle_lib, L, start):
    """Temperature ramp (protocol of Sec. 3): heating from the ordered state with
    beta descending, cooling from the random state with beta ascending; state
    carried over; derived statistics of each point's measurement window."""
    from oracle.stats import derived

    q, seed, t_equil, t_meas = 9, 1, 10, 25
    k = np.arange(6)
    betas = beta_c(q) * (0.98 + 0.04 * k / 5)
    if start == 0:
        betas = betas[::-1]
    _say(f"ramp L={L} start={start}")
    s = oracle_lib.init(L, q, seed, start)
    t, want = 0, []
    for b in betas:
        rec = oracle_lib.sweeps(s, q, seed, t, t_equil + t_meas, oracle_lib.threshold_table(b))
        t += t_equil + t_meas
        w = rec[t_equil:]
        want.append(derived(w[:, 0].tolist(), w[:, 1:].max(axis=1).tolist(), L * L, q, float(b)))
    lat = potts.Lattice.from_torch(L, q, seed, start, records_capacity=4)
    with lat:
        got = lat.ramp(betas, t_equil, t_meas)
        assert np.array_equal(lat.spins(), s)
        assert lat.t == t
    for g, w in zip(got, want):
        assert g["n"] == t_meas
        for key in ("e", "C", "V_L", "m", "chi"):
            assert g[key] == pytest.approx(w[key], rel=1e-12, abs=1e-300), key


def test_ramp_rejects_bad_arguments(potts):
    with potts.Lattice(16, 3, 1, 1) as lat:
        with pytest.raises(potts.PottsError):
            lat.ramp([1.0], 5, 0)
        with pytest.raises(potts.PottsError):
            lat.ramp([1.0, -1.0], 5, 5)
        with pytest.raises(potts.PottsError):
            lat.ramp([], 5, 5)
