"""Serving loop through the C ABI (potts_server_*): jobs submitted while others
run; each job's results must equal the oracle's and the same job run alone."""
import time

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


def _ramp(q, P, start):
    grid = beta_c(q) * (0.98 + 0.04 * np.arange(P) / max(P - 1, 1))
    return grid[::-1] if start == 0 else grid


JOBS = [
    dict(L=64, q=9, seed=1, start=1, betas=_ramp(9, 3, 1), sweeps=[9, 4, 7]),
    dict(L=512, q=6, seed=2, start=0, betas=_ramp(6, 4, 0), sweeps=[5, 5, 6, 3]),
    dict(L=256, q=12, seed=3, start=1, betas=_ramp(12, 2, 1), sweeps=[40, 11]),
    dict(L=528, q=15, seed=4, start=1, betas=_ramp(15, 3, 1), sweeps=[3, 17, 2]),
    dict(L=128, q=3, seed=5, start=0, betas=[9.0, 0.5], sweeps=[6, 6]),
    dict(L=1024, q=40, seed=6, start=1, betas=_ramp(40, 2, 1), sweeps=[4, 4]),
]


def _oracle(oracle_lib, j):
    from oracle.stats import derived

    L, q, seed = j["L"], j["q"], j["seed"]
    s = oracle_lib.init(L, q, seed, j["start"])
    t, pts = 0, []
    for b, n in zip(j["betas"], j["sweeps"]):
        rec = oracle_lib.sweeps(s, q, seed, t, n, oracle_lib.threshold_table(b))
        t += n
        w = rec[-((n + 1) // 2):]
        pts.append(derived(w[:, 0].tolist(), w[:, 1:].max(axis=1).tolist(), L * L, q, float(b)))
    return s, pts, rec[-1]


def _check(got, want_spins, want_pts, want_last):
    assert got["status"] == 0
    assert np.array_equal(got["spins"], want_spins)
    assert got["e_sat"] == want_last[0] and got["nmax"] == want_last[1:].max()
    for g, w in zip(got["points"], want_pts):
        for k in ("e", "C", "V_L", "m", "chi"):
            assert g[k] == pytest.approx(w[k], rel=1e-12, abs=1e-300), k


@pytest.mark.parametrize("cfg", [dict(quantum=4), dict(quantum=32, max_slots=2), dict(quantum=8, hbm_budget=1 << 21)])
def test_served_jobs_match_oracle(potts, oracle_lib, cfg):
    with potts.Server(**cfg) as srv:
        tickets = []
        for i, j in enumerate(JOBS):
            tickets.append(srv.submit(j["L"], j["q"], j["seed"], j["start"], j["betas"], j["sweeps"], keep_spins=True))
            if i % 2:
                time.sleep(0.02)  # arrivals while earlier jobs run
        srv.drain(120000)
        done = set()
        while len(done) < len(JOBS):
            done.update(srv.wait(64, 1000))
        got = {t: srv.collect(t, spins=True) for t in tickets}
    for t, j in zip(tickets, JOBS):
        s, pts, last = _oracle(oracle_lib, j)
        _check(got[t], s, pts, last)
        g = got[t]
        assert g["t_submit"] <= g["t_admit"] <= g["t_done"]
        assert g["sweeps"] == sum(j["sweeps"])


def test_served_equals_alone(potts):
    with potts.Server(quantum=8) as srv:
        tickets = [srv.submit(j["L"], j["q"], j["seed"], j["start"], j["betas"], j["sweeps"], keep_spins=True)
                   for j in JOBS]
        srv.drain(120000)
        got = {t: srv.collect(t, spins=True) for t in tickets}
    for t, j in zip(tickets, JOBS):
        with potts.Lattice(j["L"], j["q"], j["seed"], j["start"]) as lat:
            for k, (b, n) in enumerate(zip(j["betas"], j["sweeps"])):
                lat.sweep(b, n)
                st = lat.stats(lat.t - (n + 1) // 2, (n + 1) // 2, b)
                for key in ("e", "C", "V_L", "m", "chi"):
                    assert got[t]["points"][k][key] == st[key]
            assert np.array_equal(lat.spins(), got[t]["spins"])


def test_budget_admits_one_at_a_time(potts):
    """A budget that holds one 512 x 512 job: jobs run one after the other."""
    jobs = [JOBS[1], dict(JOBS[1], seed=7), dict(JOBS[1], seed=8)]
    with potts.Server(quantum=4, hbm_budget=512 * 512 + (1 << 16)) as srv:
        tickets = [srv.submit(j["L"], j["q"], j["seed"], j["start"], j["betas"], j["sweeps"]) for j in jobs]
        srv.drain(120000)
        got = [srv.collect(t) for t in tickets]
    for a, b in zip(got, got[1:]):
        assert b["t_admit"] >= a["t_done"] - 1e-6


def test_bad_requests(potts):
    with potts.Server() as srv:
        with pytest.raises(potts.PottsError):
            srv.submit(20, 3, 1, 1, [1.0], [5])
        with pytest.raises(potts.PottsError):
            srv.submit(64, 300, 1, 1, [1.0], [5])
        with pytest.raises(potts.PottsError):
            srv.submit(64, 3, 1, 1, [1.0], [0])
        with pytest.raises(potts.PottsError):
            srv.submit(64, 3, 1, 1, [-1.0], [5])
    with potts.Server(hbm_budget=1 << 12) as srv:
        with pytest.raises(potts.PottsError):
            srv.submit(1024, 3, 1, 1, [1.0], [5])


@pytest.mark.parametrize("L,q,fault_at", [(512, 7, 30 + 25 + 13), (128, 5, 30 + 25 + 40 + 3)])
def test_served_job_resumes_after_a_failure(potts, oracle_lib, tmp_path, L, q, fault_at):
    """Recovery: a served job that writes a checkpoint after each point fails
    at sweep fault_at (an injected host-side failure, mid-point) while other
    jobs run; they finish unaffected, and the job resubmitted from its last
    checkpoint ends with the bits of the oracle's uninterrupted run.  L = 512
    runs in the strip kernel, L = 128 in the LDS-resident one."""
    job = dict(L=L, q=q, seed=41, start=1, betas=_ramp(q, 5, 1), sweeps=[30, 25, 40, 20, 35])
    ck = str(tmp_path / "job.ckpt")
    others = JOBS[:3]

    def submit(srv, j, **kw):
        return srv.submit(j["L"], j["q"], j["seed"], j["start"], j["betas"], j["sweeps"], keep_spins=True, **kw)

    with potts.Server(quantum=8, max_slots=16) as srv:
        srv.inject_fault(0, fault_at)  # attached at submission: the job cannot finish first
        bad = submit(srv, job, checkpoint=ck)
        t_others = [submit(srv, j) for j in others]
        srv.drain(120000)
        failed = srv.collect(bad, spins=True)
        assert failed["status"] == -3  # POTTS_EDEVICE
        assert fault_at - 8 < failed["sweeps"] <= fault_at
        for t, j in zip(t_others, others):
            _check(srv.collect(t, spins=True), *_oracle(oracle_lib, j))
        with pytest.raises(potts.PottsError):
            srv.inject_fault(bad, 1)  # finished jobs cannot fail again
        resumed = submit(srv, job, resume_from=ck)
        srv.drain(120000)
        got = srv.collect(resumed, spins=True)
        with pytest.raises(potts.PottsError):  # a checkpoint of another job
            srv.submit(L, q, 42, 1, job["betas"], job["sweeps"], resume_from=ck)
    assert got["sweeps"] == sum(job["sweeps"])
    _check(got, *_oracle(oracle_lib, job))


def test_server_tunes_and_persists_shapes(potts, oracle_lib, tmp_path):
    """A tuning server times the strip height of each new lattice size and the
    workgroup shape of q <= 16 on a throwaway lattice before its first job of
    that size; the choices persist, a second server reads them, and every job
    still gives the oracle's bits."""
    import json

    cache = str(tmp_path / "serve_tune.json")
    for tune in (True, False):
        with potts.Server(quantum=8, tune=tune, tune_cache=cache) as srv:
            tickets = [srv.submit(j["L"], j["q"], j["seed"], j["start"], j["betas"], j["sweeps"], keep_spins=True)
                       for j in JOBS]
            srv.drain(120000)
            got = [srv.collect(t, spins=True) for t in tickets]
            tuned = srv.tuning()
        print(f"tune={tune}: {tuned}", flush=True)
        for g, j in zip(got, JOBS):
            _check(g, *_oracle(oracle_lib, j))
        assert "rows=" in tuned and "block=" in tuned
        if not tune:
            assert "(cached)" in tuned
    data = json.load(open(cache))
    assert data["kernel_hash"] == potts.load().potts_kernel_digest().decode()
    assert {"strip/0/512", "strip/0/528", "strip/1/1024"} <= set(data["rows"])
    assert "strip/0" in data["shapes"]
