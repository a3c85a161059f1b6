"""bench.py's host-side contract, on the CPU: more than one GPU is refused with
a message, the counter traffic of a workload is reported only while the
kernel sources hash as when it was taken, the CPU baseline is the oracle
with the fields the JSON line carries, and the default line's other parts
run at their own workload sizes."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout.strip() == ""


@pytest.mark.parametrize("workload", ["large", "cubic", "nnn", "mid"])
def test_counter_traffic_follows_the_source_hash(workload, tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench

    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    for rel in bench.SOURCES_OF[workload]:
        dst = tmp_path / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_text(open(os.path.join(ROOT, rel)).read())
    good = {"kernel_hash": bench.kernel_hash(bench.SOURCES_OF[workload]), "bytes_per_launch": 1234.0}
    path = tmp_path / "profiles" / f"traffic_{workload}.json"
    path.write_text(json.dumps(good))
    assert bench.counter_traffic(workload) == 1234.0
    # a comment-only edit keeps the record, a code edit drops it
    src = tmp_path / bench.SOURCES_OF[workload][0]
    src.write_text(src.read_text() + "\n// a comment\n")
    assert bench.counter_traffic(workload) == 1234.0
    src.write_text(src.read_text() + "\nint an_extra_symbol;\n")
    assert bench.counter_traffic(workload) is None


@pytest.mark.parametrize("workload", ["large", "cubic", "nnn", "mid"])
def test_committed_counter_records_match_the_kernels(workload):
    """The committed traffic records were taken on the kernel sources as they
    stand (a header shared by every kernel counts too), so the bench lines
    report counter traffic rather than null."""
    sys.path.insert(0, ROOT)
    import bench

    assert bench.counter_traffic(workload) is not None


def test_cpu_baseline_is_the_oracle():
    sys.path.insert(0, ROOT)
    import bench

    b = bench.cpu_baseline(seconds_target=0.2)
    assert b["kind"] == "oracle" and b["cores"] == 1 and b["unit"] == "ns per spin flip"
    assert 0.1 < b["value"] < 1e4 and "L=4096" in b["sample"]


def test_default_line_extras_run_at_their_own_sizes(monkeypatch):
    """The batched, served, plain-method and ramp parts of the default line
    run at their workloads' own sizes whatever --steps and --warmup the
    driver passes, and land in the line under their own keys."""
    sys.path.insert(0, ROOT)
    import argparse

    import bench

    seen = {}

    def fake(name, out):
        def run(args):
            seen[name] = args
            return out
        return run

    monkeypatch.setattr(bench, "run_plain", fake("plain", {"value": 2.5e-4, "ms_per_step": 1.0, "steps": 20,
                                                           "config": {"workload": "plain method"}}))
    monkeypatch.setattr(bench, "run_ramp", fake("ramp", {"value": 8e-4, "wall_s": 3.0,
                                                         "config": {"workload": "metastability ramp"}}))
    monkeypatch.setattr(bench, "run_batch", fake("batch", {
        "value": 600.0, "ns_per_spin_flip": 9e-4, "untuned_jobs_per_s": 590.0,
        "plain_loop": {"jobs_per_s": 150.0, "speedup_of_batch": 4.0}, "config": {"workload": "batched replicas"}}))
    monkeypatch.setattr(bench, "run_serve", fake("serve", {
        "value": 190.0, "latency_s": {"p50": 0.08, "p99": 0.35, "max": 0.4}, "ns_per_spin_flip": 1.8e-3,
        "span_s": 5.3, "config": {"workload": "serving loop"}}))
    args = argparse.Namespace(steps=20, warmup=5, no_cpu=False, no_plain=True, tune_cache="x", ramp_sweeps=7,
                              serve_jobs=3, serve_rate=1.0, serve_scale=1.0, batch_jobs=1024)
    out = bench.run_extras(args)
    assert seen["batch"].steps == 500 and seen["batch"].no_plain is False and seen["batch"].tune_cache is None
    assert (seen["serve"].serve_jobs, seen["serve"].serve_rate, seen["serve"].serve_scale) == (1000, 200.0, 0.01)
    assert seen["plain"].steps == 20 and seen["plain"].no_cpu is True
    assert seen["ramp"].ramp_sweeps == 100
    assert args.steps == 20 and args.ramp_sweeps == 7  # the caller's arguments are left alone
    assert out["batched"]["jobs_per_s"] == 600.0 and out["batched"]["speedup_over_plain_loop"] == 4.0
    assert out["served"]["latency_s"]["p99"] == 0.35 and "x0.01" in out["served"]["note"]
    assert out["plain"]["ns_per_spin_flip"] == 2.5e-4 and out["ramp"]["ns_per_spin_flip"] == 8e-4
