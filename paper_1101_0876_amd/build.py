"""Builds the HIP library libpotts.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["capi.hip", "kernels.hip", "strip.hip", "packed.hip", "resident.hip", "stats.hip", "batch.hip", "server.hip", "cubic.hip", "cubic_packed.hip", "nnn.hip"]
LIB_PATH = os.path.join(_HERE, "libpotts.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(_HERE, "csrc", s) for s in SOURCES]
    tmp = LIB_PATH + ".tmp"
    cmd = [
        "hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-o", tmp, *srcs,
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    errs = "\n".join(line for line in res.stderr.splitlines() if noise not in line)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{errs}")
    if verbose and errs.strip():
        print(errs)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
