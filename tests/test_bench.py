"""bench.py's host-side contract, on the CPU: more than one GPU is refused with
a message, the counter traffic of a workload is reported only while the
kernel sources hash as when it was taken, and the CPU baseline is the oracle
with the fields the JSON line carries."""
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


@pytest.mark.parametrize("workload", ["large", "cubic", "nnn"])
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


def test_cpu_baseline_is_the_oracle():
    sys.path.insert(0, ROOT)
    import bench

    b = bench.cpu_baseline(seconds_target=0.2)
    assert b["kind"] == "oracle" and b["cores"] == 1 and b["unit"] == "ns per spin flip"
    assert 0.1 < b["value"] < 1e4 and "L=4096" in b["sample"]
