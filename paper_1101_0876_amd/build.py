"""Builds the HIP library libpotts.so (gfx950) in-tree with hipcc.

Each source compiles to an object in a temporary directory, all of them at
once, and the objects link into the library.  The digest of the tuned
kernels' sources (comments and blank space ignored) is compiled in as
POTTS_KERNEL_HASH: the launch-shape cache of the batch and serving tuners
keys its entries by it.
"""
from __future__ import annotations

import hashlib
import os
import re
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["capi.hip", "kernels.hip", "strip.hip", "packed.hip", "resident.hip", "stats.hip", "batch.hip",
           "server.hip", "cubic.hip", "cubic_packed.hip", "nnn.hip", "tune_cache.hip", "heatbath_packed.hip", "noalloc.hip", "tiles.hip", "band.hip"]
# the kernels whose launch shapes the tuners pick
TUNED = ["strip.hip", "packed.hip", "sweep_row.hpp", "device.hpp", "kernels.hpp"]
LIB_PATH = os.path.join(_HERE, "libpotts.so")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wall"]
_NOISE = "is not a recognized feature for this target"


def kernel_digest() -> str:
    h = hashlib.sha256()
    for name in TUNED:
        with open(os.path.join(_HERE, "csrc", name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(line for line in res.stderr.splitlines() if _NOISE not in line)
    return res.returncode, errs


def build(verbose: bool = False) -> str:
    digest = kernel_digest()
    with tempfile.TemporaryDirectory() as tmpdir:
        jobs = []
        for src in SOURCES:
            obj = os.path.join(tmpdir, os.path.splitext(src)[0] + ".o")
            cmd = ["hipcc", *FLAGS, f'-DPOTTS_KERNEL_HASH="{digest}"', "-c", os.path.join(_HERE, "csrc", src),
                   "-o", obj]
            jobs.append((src, obj, cmd))
        if verbose:
            print(" ".join(jobs[0][2]).replace(jobs[0][0], "<source>"), f"  ({len(jobs)} sources)", flush=True)
        workers = max(1, min(len(jobs), os.cpu_count() or 1, 16))
        with ThreadPoolExecutor(workers) as pool:
            results = list(pool.map(lambda j: _run(j[2]), jobs))
        failed = [(j[0], rc, errs) for j, (rc, errs) in zip(jobs, results) if rc != 0]
        if failed:
            raise RuntimeError("hipcc failed:\n" + "\n".join(f"{src} ({rc}):\n{errs}" for src, rc, errs in failed))
        if verbose:
            for (src, _, _), (_, errs) in zip(jobs, results):
                if errs.strip():
                    print(f"{src}:\n{errs}")
        tmp = LIB_PATH + ".tmp"
        rc, errs = _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *[j[1] for j in jobs]])
        if rc != 0:
            raise RuntimeError(f"link failed ({rc}):\n{errs}")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
