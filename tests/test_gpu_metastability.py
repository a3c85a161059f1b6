"""The metastability branches run through the serving loop: every sample's
per-point energy equals the oracle's statistics of the oracle's records of the
same ramp, and equals the same sample run alone through potts_ramp."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def potts():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_0876_amd as p

    p.load()
    return p


@pytest.mark.parametrize("side", ["high", "low"])
def test_branch_matches_oracle_and_alone(potts, oracle_lib, side):
    from oracle.stats import derived
    from paper_1101_0876_amd.metastability import analyse, branch

    q, L, samples, sweeps = 9, 64, 3, 40
    taus = [0.03, 0.01, 0.004]
    print(f"branch side={side}", flush=True)
    b = branch(q, L, samples, taus, sweeps, side, seed0=11)
    start = potts.RANDOM if side == "high" else potts.ORDERED
    half = sweeps // 2
    for i in range(samples):
        seed = 11 + i
        s = oracle_lib.init(L, q, seed, start)
        t = 0
        for k, beta in enumerate(b["beta"]):
            rec = oracle_lib.sweeps(s, q, seed, t, sweeps, oracle_lib.threshold_table(float(beta)))
            t += sweeps
            w = rec[sweeps - half:]
            want = derived(w[:, 0].tolist(), w[:, 1:].max(axis=1).tolist(), L * L, q, float(beta))
            assert b["e"][i, k] == pytest.approx(want["e"], rel=1e-12), (i, k)
            assert b["C"][i, k] == pytest.approx(want["C"], rel=1e-12, abs=1e-300), (i, k)
        with potts.Lattice(L, q, seed, start) as lat:
            pts = lat.ramp(b["beta"], sweeps - half, half)
        assert [p["e"] for p in pts] == list(b["e"][i])
    r = analyse(b)
    assert len(r["x"]) == len(taus) and np.all(r["x"] > 0)
