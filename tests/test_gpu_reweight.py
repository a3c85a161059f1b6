"""Temperature reweighting through the C ABI (potts_reweight) against the
oracle's decimal evaluation of the same definition on the oracle's own record
series (identical bits to the GPU's, checked elsewhere).

Tolerance 1e-11 relative: the device sums n weights and moments in FP64 in a
different order (relative error ~ n^(1/2) 2^-53 ~ 1e-14 for n <= 10^3), and the
variances subtract squares of shifted means a few standard deviations wide
(one to two more digits)."""
import math

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


CASES = [
    # L, q, seed, start, beta0, sweeps run, window (t0, n), ring capacity
    (64, 9, 1, 1, 1.02 * math.log(4.0), 1000, (0, 1000), 0),       # the plain-method run
    (256, 6, 3, 0, beta_c(6), 400, (100, 300), 0),
    (128, 3, 5, 1, beta_c(3), 100, (40, 60), 64),                  # window wraps the ring
]


@pytest.mark.parametrize("L,q,seed,start,beta0,nsw,window,cap", CASES)
def test_reweight_matches_oracle(potts, oracle_lib, L, q, seed, start, beta0, nsw, window, cap):
    from oracle.stats import reweight

    t0, n = window
    print(f"reweight L={L} q={q} window={window}", flush=True)
    s = oracle_lib.init(L, q, seed, start)
    rec = oracle_lib.sweeps(s, q, seed, 0, nsw, oracle_lib.threshold_table(beta0))[t0:t0 + n]
    betas = [beta0 * 0.99, beta0, beta0 * 1.004, beta0 * 1.02]
    with potts.Lattice.from_torch(L, q, seed, start, records_capacity=cap) as lat:
        lat.sweep(beta0, nsw)
        got = lat.reweight(t0, n, beta0, betas)
    for b, g in zip(betas, got):
        want = reweight(rec[:, 0].tolist(), rec[:, 1:].max(axis=1).tolist(), L * L, q, beta0, b)
        assert g["n"] == n
        for k in ("e", "C", "V_L", "m", "chi"):
            assert g[k] == pytest.approx(want[k], rel=1e-11, abs=1e-300), (b, k)


def test_reweight_at_beta0_equals_stats(potts):
    L, q, beta = 128, 5, beta_c(5)
    with potts.Lattice(L, q, 2, 1) as lat:
        lat.sweep(beta, 200)
        a = lat.stats(50, 150, beta)
        b = lat.reweight(50, 150, beta, [beta])[0]
    for k in ("e", "C", "V_L", "m", "chi"):
        assert b[k] == pytest.approx(a[k], rel=1e-11, abs=1e-300), k


def test_reweight_rejects_bad_arguments(potts):
    with potts.Lattice(64, 3, 1, 1) as lat:
        lat.sweep(1.0, 10)
        for args in [(0, 0, 1.0, [1.0]), (0, 5, -1.0, [1.0]), (0, 5, 1.0, [float("nan")]), (0, 5, 1.0, [])]:
            with pytest.raises(potts.PottsError):
                lat.reweight(*args)
        with pytest.raises(potts.PottsError):
            lat.reweight(5, 10, 1.0, [1.0])  # beyond the last sweep
