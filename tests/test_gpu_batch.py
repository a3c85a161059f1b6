"""Batches through the C ABI (potts_batch_*): every job must give the bits the
oracle gives for it alone, whatever the mix, graph capture or tuning."""
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


# resident (L <= 256), colour-split (L >= 512, L % 32 == 0) and strip
# (L % 32 == 16) jobs, every comparison class, zero thresholds (beta = 9),
# uneven sweep counts, both starts
MIX = [
    dict(L=16, q=3, seed=11, start=1, beta=1.0, nsweeps=9),
    dict(L=64, q=9, seed=12, start=0, beta=1.02 * math.log(4.0), nsweeps=12),
    dict(L=128, q=17, seed=13, start=1, beta=1.3, nsweeps=7),
    dict(L=256, q=6, seed=14, start=1, beta=beta_c(6), nsweeps=10),
    dict(L=96, q=100, seed=15, start=1, beta=2.0, nsweeps=5),
    dict(L=48, q=200, seed=16, start=0, beta=9.0, nsweeps=6),
    dict(L=512, q=9, seed=17, start=1, beta=beta_c(9), nsweeps=11),
    dict(L=512, q=12, seed=18, start=0, beta=0.98 * beta_c(12), nsweeps=8),
    dict(L=1024, q=3, seed=19, start=1, beta=beta_c(3), nsweeps=6),
    dict(L=528, q=40, seed=20, start=1, beta=9.0, nsweeps=7),
    dict(L=512, q=130, seed=21, start=1, beta=1.1, nsweeps=4),
    dict(L=544, q=5, seed=22, start=1, beta=1.2, nsweeps=0),
    dict(L=576, q=40, seed=23, start=0, beta=9.0, nsweeps=5),     # colour-split, wide, private bins
    dict(L=512, q=100, seed=24, start=1, beta=1.0, nsweeps=6),    # colour-split, shared bins
    dict(L=560, q=7, seed=25, start=1, beta=beta_c(7), nsweeps=5),  # strip, q <= 16
]


def _oracle(oracle_lib, j, t0=0, spins=None):
    s = oracle_lib.init(j["L"], j["q"], j["seed"], j["start"]) if spins is None else spins
    rec = oracle_lib.sweeps(s, j["q"], j["seed"], t0, j["nsweeps"], oracle_lib.threshold_table(j["beta"]))
    return s, rec


@pytest.mark.parametrize("graph,tune", [(False, False), (True, False), (True, True)])
def test_batch_matches_oracle(potts, oracle_lib, graph, tune):
    from oracle.stats import derived

    _say(f"batch graph={graph} tune={tune}")
    with potts.Batch(MIX, graph=graph, tune=tune) as b:
        b.run()
        res = b.results()
        for i, j in enumerate(MIX):
            s, rec = _oracle(oracle_lib, j)
            n = j["nsweeps"]
            assert res[i]["t"] == n
            assert np.array_equal(b.spins(i), s), i
            if n:
                assert np.array_equal(b.records(i, 0, n), rec), i
                assert res[i]["e_sat"] == rec[-1, 0] and res[i]["nmax"] == rec[-1, 1:].max()
                want = derived(rec[:, 0].tolist(), rec[:, 1:].max(axis=1).tolist(), j["L"] ** 2, j["q"], j["beta"])
                for k in ("e", "C", "V_L", "m", "chi"):
                    assert res[i][k] == pytest.approx(want[k], rel=1e-12, abs=1e-300), (i, k)


def test_batch_second_run_continues(potts, oracle_lib):
    jobs = [MIX[1], MIX[6], MIX[8]]
    with potts.Batch(jobs, graph=True, tune=False) as b:
        b.run()
        b.run()
        for i, j in enumerate(jobs):
            s, rec1 = _oracle(oracle_lib, j)
            s, rec2 = _oracle(oracle_lib, j, t0=j["nsweeps"], spins=s)
            n = j["nsweeps"]
            assert np.array_equal(b.spins(i), s)
            assert np.array_equal(b.records(i, n, n), rec2)


def test_batch_equals_alone(potts):
    """Each job of the mix gives the bits of the same lattice run alone."""
    with potts.Batch(MIX, graph=True, tune=True) as b:
        b.run()
        for i, j in enumerate(MIX):
            with potts.Lattice(j["L"], j["q"], j["seed"], j["start"]) as lat:
                lat.sweep(j["beta"], j["nsweeps"])
                assert np.array_equal(lat.spins(), b.spins(i)), i
                if j["nsweeps"]:
                    assert np.array_equal(lat.records(0, j["nsweeps"]), b.records(i, 0, j["nsweeps"])), i


def test_batch_windowed_summary(potts, oracle_lib):
    from oracle.stats import derived

    j = MIX[6]
    with potts.Batch([j], graph=False, tune=False, window=4) as b:
        b.run()
        r = b.results()[0]
    _, rec = _oracle(oracle_lib, j)
    w = rec[-4:]
    want = derived(w[:, 0].tolist(), w[:, 1:].max(axis=1).tolist(), j["L"] ** 2, j["q"], j["beta"])
    assert r["n"] == 4
    for k in ("e", "C", "V_L", "m", "chi"):
        assert r[k] == pytest.approx(want[k], rel=1e-12, abs=1e-300), k


@pytest.mark.parametrize("bad", [dict(L=20), dict(L=8), dict(q=1), dict(q=257), dict(start=3),
                                 dict(nsweeps=-1), dict(beta=-1.0)])
def test_batch_rejects_bad_jobs(potts, bad):
    j = dict(MIX[0])
    j.update(bad)
    with pytest.raises(potts.PottsError):
        potts.Batch([MIX[1], j])


def test_tuner_shapes_cache_and_every_shape(potts, oracle_lib, tmp_path):
    """The tuner times strip heights per lattice size, then the workgroup shape
    (lanes per workgroup, occupancy) per kernel group, on real sweeps of the
    run; its choices persist in a JSON cache keyed by the kernels' digest,
    which a second batch reads without timing.  Every shape, forced through
    the cache, gives the oracle's bits."""
    import json

    cache = str(tmp_path / "tune.json")
    jobs = [dict(j, nsweeps=40) for j in (MIX[6], MIX[7], MIX[8], MIX[14])]
    want = [_oracle(oracle_lib, j) for j in jobs]
    digest = potts.load().potts_kernel_digest().decode()

    def check(b):
        for i, (s, rec) in enumerate(want):
            assert np.array_equal(b.records(i, 0, 40), rec), i
            assert np.array_equal(b.spins(i), s), i

    with potts.Batch(jobs, graph=True, tune=True, tune_cache=cache) as b:
        b.run()
        tuned = b.tuning()
        _say(f"tuned: {tuned}")
        check(b)
    assert "rows=" in tuned and "block=" in tuned and "waves/SIMD=" in tuned
    data = json.load(open(cache))
    assert data["kernel_hash"] == digest
    assert set(data["rows"]) == {"packed/0/512", "packed/0/1024", "strip/0/560"}
    assert set(data["shapes"]) == {"packed/0", "strip/0"}
    with potts.Batch(jobs, graph=True, tune=False, tune_cache=cache) as b:
        b.run()
        assert "(cached)" in b.tuning() and "block=" in b.tuning()
        check(b)
    for shape in ([128, 0], [256, 8], [128, 8], [256, 0]):
        with open(cache, "w") as f:
            json.dump({"kernel_hash": digest, "rows": {"packed/0/512": 2, "packed/0/1024": 32, "strip/0/560": 8},
                       "shapes": {"packed/0": shape, "strip/0": shape}}, f)
        _say(f"forced shape {shape}")
        with potts.Batch(jobs, graph=False, tune=False, tune_cache=cache) as b:
            b.run()
            check(b)
    # a cache of other kernel sources is ignored
    with open(cache, "w") as f:
        json.dump({"kernel_hash": "other", "rows": {"packed/0/512": 4}, "shapes": {"packed/0": [128, 8]}}, f)
    with potts.Batch(jobs, graph=False, tune=False, tune_cache=cache) as b:
        b.run()
        assert "cached" not in b.tuning()
        check(b)
