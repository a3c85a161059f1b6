"""Oracle runs for the full-size parity tests, spread over host threads.

The oracle is serial C called through ctypes, which releases the GIL, so a
thread pool runs independent oracle calls (windows of one lattice, separate
jobs) on all host cores while the GPU works.  Nothing here computes any part
of the method: it only tiles the oracle's window restriction and its
per-job runs.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def workers() -> int:
    """Host threads for oracle work: the machine's cores, at most 16."""
    return max(1, min(16, os.cpu_count() or 1))


def make_pool() -> ThreadPoolExecutor:
    return ThreadPoolExecutor(max_workers=workers())


def full_lattice(pool, oracle_lib, L, q, seed, start, nsweeps, thr, tile=1024):
    """The oracle's whole L x L lattice after nsweeps sweeps from the initial
    condition, assembled from tile x tile blocks, each the exact interior of an
    oracle window with a margin of 2 * nsweeps sites on every side.  Returns
    (array, futures); the array is complete once every future is done."""
    assert L % tile == 0
    m = 2 * nsweeps
    out = np.empty((L, L), dtype=np.uint8)

    def block(y0, x0):
        w = oracle_lib.window(L, q, seed, start, nsweeps, thr, (x0 - m) % L, (y0 - m) % L, tile + 2 * m,
                              tile + 2 * m)
        out[y0:y0 + tile, x0:x0 + tile] = w[m:m + tile, m:m + tile]

    futs = [pool.submit(block, y0, x0) for y0 in range(0, L, tile) for x0 in range(0, L, tile)]
    return out, futs


def wait_all(futs) -> None:
    for f in futs:
        f.result()


def ramp_job(oracle_lib, job):
    """A served job on the oracle: its beta ramp with the sweeps of each point
    (state carried over), the derived statistics of the last ceil(n/2)
    records of each point, the final lattice and the last record."""
    from oracle.stats import derived

    L, q, seed = job["L"], job["q"], job["seed"]
    s = oracle_lib.init(L, q, seed, job["start"])
    t, pts, rec = 0, [], None
    for b, n in zip(job["betas"], job["sweeps"]):
        rec = oracle_lib.sweeps(s, q, seed, t, n, oracle_lib.threshold_table(b))
        t += n
        w = rec[-((n + 1) // 2):]
        pts.append(derived(w[:, 0].tolist(), w[:, 1:].max(axis=1).tolist(), L * L, q, float(b)))
    return s, pts, rec[-1]
