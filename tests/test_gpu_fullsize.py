"""Parity at the workloads' full configurations, in the launch configurations the
benchmark times, against the oracle (run on all host cores, tests/fullsize.py).

* Single large lattice (L = 32768, q = 6, beta_c, both starts): every record
  of the first three sweeps against the oracle's observables of the oracle's
  lattice, and every site after the first and the third sweep.
* Metastability ramps (L = 8192, q = 6, 9, 12, 15, heating and cooling): the
  first two points of all eight runs, spins and per-point statistics.
* Batched replicas (1024 jobs, 500 sweeps, one graph, in-run tuning): every
  job with L <= 512 in full (all records and the final spins), and the first
  20 records of eight jobs of each larger L; the two largest jobs against
  the same job run alone.
* Serving (the 1000-job burst, sweeps x 0.01): sixteen jobs, four of each L
  from 256 to 2048, per-point statistics and final spins; the largest job
  (L = 8192) against the same ramp run alone.
"""
import math

import numpy as np
import pytest

from tests.fullsize import full_lattice, make_pool, ramp_job, wait_all
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


@pytest.mark.parametrize("start", [0, 1])
def test_large_lattice_every_site_and_record(potts, oracle_lib, start):
    """L = 32768, q = 6, beta_c, seed 1, library-owned buffers on a caller
    stream (the benchmark's configuration): a one-sweep call, then a two-sweep
    call.  The GPU lattice after each call equals the oracle's at every site;
    the three fused records equal the oracle's observables of its lattice
    after one, two and three sweeps."""
    L, q, seed, beta = 32768, 6, 1, beta_c(6)
    thr = oracle_lib.threshold_table(beta)
    _say(f"full-size large lattice L={L} q={q} start={start}")
    with make_pool() as pool:
        want, futs = {}, []
        for n in (1, 2, 3):
            want[n], f = full_lattice(pool, oracle_lib, L, q, seed, start, n, thr)
            futs += f
        lat = potts.Lattice.on_stream(L, q, seed, start)
        with lat:
            lat.sweep(beta, 1)
            got1 = lat.spins()
            lat.sweep(beta, 2)
            got3 = lat.spins()
            rec = lat.records(0, 3)
        _say("GPU done; waiting for the oracle tiles")
        wait_all(futs)
        obs = [pool.submit(oracle_lib.observables, want[n], q) for n in (1, 2, 3)]
        assert np.array_equal(got1, want[1])
        del got1
        assert np.array_equal(got3, want[3])
        del got3
        for k, f in enumerate(obs):
            e, hist = f.result()
            assert rec[k, 0] == e and np.array_equal(rec[k, 1:], hist), k


def test_ramps_all_runs_first_points(potts, oracle_lib):
    """The ramp workload (L = 8192, 64-point grid within +-2 % of beta_c(q),
    heating from the ordered start with beta descending, cooling from the
    random start with beta ascending) for q = 6, 9, 12, 15 and both
    directions: the first two points with 1 + 2 sweeps each, spins and every
    point's statistics against the oracle."""
    from oracle.stats import derived

    L, seed, t_equil, t_meas = 8192, 1, 1, 2
    runs = [(q, start) for q in (6, 9, 12, 15) for start in (0, 1)]

    def oracle_run(q, start):
        grid = beta_c(q) * (0.98 + 0.04 * np.arange(64) / 63)
        betas = (grid[::-1] if start == 0 else grid)[:2]
        s = oracle_lib.init(L, q, seed, start)
        t, pts = 0, []
        for b in betas:
            rec = oracle_lib.sweeps(s, q, seed, t, t_equil + t_meas, oracle_lib.threshold_table(b))
            t += t_equil + t_meas
            w = rec[t_equil:]
            pts.append(derived(w[:, 0].tolist(), w[:, 1:].max(axis=1).tolist(), L * L, q, float(b)))
        return betas, s, pts

    with make_pool() as pool:
        futs = {r: pool.submit(oracle_run, *r) for r in runs}
        for (q, start) in runs:
            _say(f"ramp q={q} start={start}")
            grid = beta_c(q) * (0.98 + 0.04 * np.arange(64) / 63)
            betas = (grid[::-1] if start == 0 else grid)[:2]
            with potts.Lattice(L, q, seed, start) as lat:
                got = lat.ramp(betas, t_equil, t_meas)
                spins = lat.spins()
            wbetas, ws, wpts = futs[(q, start)].result()
            assert np.array_equal(betas, wbetas)
            assert np.array_equal(spins, ws), (q, start)
            for g, w in zip(got, wpts):
                assert g["n"] == t_meas
                for key in ("e", "C", "V_L", "m", "chi"):
                    assert g[key] == pytest.approx(w[key], rel=1e-12, abs=1e-300), (q, start, key)


def test_batch_full_configuration_against_oracle(potts, oracle_lib):
    """The batched-replicas workload as the benchmark runs it (one batch, graph
    and in-run tuning): every job of L <= 512 (the LDS-resident and tiled
    kernels) in full, all 500 records and the final spins; the first 20
    records of the eight lowest-numbered jobs of each L >= 1024; populations
    and energy bounds of every job."""
    from paper_1101_0876_amd.workloads import batch_jobs

    jobs = batch_jobs()
    assert len(jobs) == 1024 and all(j["nsweeps"] == 500 for j in jobs)
    full = [i for i, j in enumerate(jobs) if j["L"] <= 512]
    head = []
    for L in (1024, 2048, 4096):
        head += [i for i, j in enumerate(jobs) if j["L"] == L][:8]
    _say(f"batch: {len(full)} jobs in full, {len(head)} jobs' first 20 records")

    def oracle_job(i, n):
        j = jobs[i]
        s = oracle_lib.init(j["L"], j["q"], j["seed"], j["start"])
        rec = oracle_lib.sweeps(s, j["q"], j["seed"], 0, n, oracle_lib.threshold_table(j["beta"]))
        return s, rec

    with make_pool() as pool:
        # the slowest oracle jobs first
        order = sorted(full, key=lambda i: -jobs[i]["L"])
        fut_full = {i: pool.submit(oracle_job, i, 500) for i in order}
        fut_head = {i: pool.submit(oracle_job, i, 20) for i in head}
        with potts.Batch(jobs, graph=True, tune=True) as b:
            b.run()
            _say(f"batch ran: {b.tuning()}")
            res = b.results()
            for i, (r, j) in enumerate(zip(res, jobs)):
                assert r["t"] == 500
                last = b.records(i, 499, 1)
                assert int(last[0, 1:].sum()) == j["L"] ** 2, i
                assert r["e_sat"] == last[0, 0] and 0 <= r["e_sat"] <= 2 * j["L"] ** 2
            got_full = {i: (b.spins(i), b.records(i, 0, 500)) for i in full}
            got_head = {i: b.records(i, 0, 20) for i in head}
            # the two largest jobs, all 500 sweeps, against the same job run alone
            for i in sorted(range(len(jobs)), key=lambda i: (jobs[i]["L"], i))[-2:]:
                j = jobs[i]
                _say(f"alone job {i}: L={j['L']} q={j['q']}")
                with potts.Lattice(j["L"], j["q"], j["seed"], j["start"]) as lat:
                    lat.sweep(j["beta"], 500)
                    assert np.array_equal(lat.records(0, 500), b.records(i, 0, 500)), i
                    assert np.array_equal(lat.spins(), b.spins(i)), i
        for i in head:
            _, rec = fut_head[i].result()
            assert np.array_equal(got_head[i], rec), i
        for i in full:
            s, rec = fut_full[i].result()
            assert np.array_equal(got_full[i][1], rec), i
            assert np.array_equal(got_full[i][0], s), i


def test_serve_burst_jobs_against_oracle(potts, oracle_lib):
    """The serving workload's 1000-job burst (sweeps x 0.01) in the benchmark's
    server configuration, submitted at once: every job completes with the
    sweeps it asked for; sixteen jobs (the four cheapest of each L = 256, 512,
    1024, 2048) keep their final lattice, which, with the per-point statistics
    and the last record, equals the oracle's."""
    from paper_1101_0876_amd.workloads import serve_jobs

    jobs = serve_jobs(sweep_scale=0.01)
    cost = [j["L"] ** 2 * sum(j["sweeps"]) for j in jobs]
    sample = []
    for L in (256, 512, 1024, 2048):
        ids = sorted((i for i, j in enumerate(jobs) if j["L"] == L), key=lambda i: cost[i])
        sample += ids[:4]
    assert len(sample) == 16
    _say(f"serve burst: 1000 jobs, oracle on {sample}")
    with make_pool() as pool:
        futs = {i: pool.submit(ramp_job, oracle_lib, jobs[i]) for i in sample}
        with potts.Server(quantum=32, max_slots=256) as srv:
            tickets = [srv.submit(j["L"], j["q"], j["seed"], j["start"], j["betas"], j["sweeps"],
                                  keep_spins=(i in futs)) for i, j in enumerate(jobs)]
            srv.drain(300000)
            got = [srv.collect(t, spins=(i in futs)) for i, t in enumerate(tickets)]
        for g, j in zip(got, jobs):
            assert g["status"] == 0 and g["sweeps"] == sum(j["sweeps"])
            assert 0 <= g["e_sat"] <= 2 * j["L"] ** 2 and 0 < g["nmax"] <= j["L"] ** 2
            assert len(g["points"]) == len(j["betas"])
        # the largest job (L = 8192) against the same ramp run alone
        big = max(range(len(jobs)), key=lambda i: (jobs[i]["L"], cost[i]))
        j = jobs[big]
        _say(f"alone job {big}: L={j['L']} q={j['q']} points={len(j['betas'])}")
        with potts.Lattice(j["L"], j["q"], j["seed"], j["start"]) as lat:
            for k, (beta, n) in enumerate(zip(j["betas"], j["sweeps"])):
                lat.sweep(beta, n)
                w = max(1, (n + 1) // 2)
                want = lat.stats(lat.t - w, w, beta)
                for key in ("e", "C", "V_L", "m", "chi"):
                    assert got[big]["points"][k][key] == pytest.approx(want[key], rel=1e-14, abs=1e-300)
        for i in sample:
            s, pts, last = futs[i].result()
            g = got[i]
            assert np.array_equal(g["spins"], s), i
            assert g["e_sat"] == last[0] and g["nmax"] == last[1:].max(), i
            for k, (gp, wp) in enumerate(zip(g["points"], pts)):
                for key in ("e", "C", "V_L", "m", "chi"):
                    assert gp[key] == pytest.approx(wp[key], rel=1e-12, abs=1e-300), (i, k, key)


def test_end_to_end_run_equals_each_sample_alone(potts, oracle_lib):
    """The paper's end-to-end run as the benchmark runs it (q = 9, L = 1024,
    three samples concurrently on their own streams, T = 0.71 .. 0.73 in steps
    of 0.002, 2000 + 8000 sweeps per point, heating from the ordered start):
    every sample's per-point statistics equal those of the same ramp run alone;
    the same protocol, shortened to 20 + 30 sweeps on the first three points,
    equals the oracle's."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle.stats import derived

    L, q, samples = 1024, 9, 3
    betas = [1.0 / (0.71 + 0.002 * k) for k in range(11)]

    def run(t_tran, t_max, npts):
        lats = [potts.Lattice(L, q, s + 1, potts.ORDERED) for s in range(samples)]
        for lat in lats:
            lat.reserve_records(t_max + 2)
        with ThreadPoolExecutor(max_workers=samples) as pool:
            curves = list(pool.map(lambda lat: lat.ramp(betas[:npts], t_tran, t_max), lats))
        spins = [lat.spins() for lat in lats]
        for lat in lats:
            lat.close()
        return curves, spins

    _say("end-to-end run: 3 samples x 11 points x 10000 sweeps")
    curves, _ = run(2000, 8000, 11)
    for s in range(samples):
        with potts.Lattice(L, q, s + 1, potts.ORDERED) as lat:
            want = lat.ramp(betas, 2000, 8000)
        assert curves[s] == want, s
    # shortened protocol against the oracle
    t_tran, t_max, npts = 20, 30, 3
    curves, spins = run(t_tran, t_max, npts)
    for s in range(samples):
        o = oracle_lib.init(L, q, s + 1, 0)
        t = 0
        for k in range(npts):
            rec = oracle_lib.sweeps(o, q, s + 1, t, t_tran + t_max, oracle_lib.threshold_table(betas[k]))
            t += t_tran + t_max
            w = rec[t_tran:]
            want = derived(w[:, 0].tolist(), w[:, 1:].max(axis=1).tolist(), L * L, q, betas[k])
            for key in ("e", "C", "V_L", "m", "chi"):
                assert curves[s][k][key] == pytest.approx(want[key], rel=1e-12, abs=1e-300), (s, k, key)
        assert np.array_equal(spins[s], o), s
