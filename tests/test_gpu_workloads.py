"""The variants' benchmark configurations, in the launch configurations the
benchmark times (the main path's workloads are in test_gpu_fullsize.py).
Heat-bath and second neighbours: the benchmark lattices' first sweeps against
the oracle.  Simple cubic: sampled windows of the benchmark cube against the
oracle."""
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


def test_heatbath_benchmark_configuration(potts, oracle_lib):
    """The heat-bath workload's lattice (L = 8192, q = 9, beta = 1.02 ln 4,
    random start, seed 1) on the path the benchmark times: the first two
    sweeps, every spin and record against the oracle."""
    import math

    L, q, seed, n = 8192, 9, 1, 2
    beta = 1.02 * math.log(4.0)
    print(f"heat-bath benchmark configuration: L={L} q={q} sweeps={n}", flush=True)
    s = oracle_lib.init(L, q, seed, 1)
    rec = oracle_lib.heatbath_sweeps(s, q, seed, 0, n, oracle_lib.threshold_table(beta))
    with potts.Lattice(L, q, seed, 1) as lat:
        lat.sweep_heatbath(beta, n)
        assert np.array_equal(lat.records(0, n), rec)
        assert np.array_equal(lat.spins(), s)


def test_second_neighbour_benchmark_configuration(potts, oracle_lib):
    """The second-neighbour workload's lattice (L = 8184, q = 9, j2 = 0.5,
    beta = 0.8, random start, seed 1) on the kernel the benchmark times: the
    first two sweeps, every spin and record against the oracle."""
    L, q, seed, n, beta, j2 = 8184, 9, 1, 2, 0.8, 0.5
    print(f"second-neighbour benchmark configuration: L={L} q={q} sweeps={n}", flush=True)
    s = oracle_lib.init(L, q, seed, 1)
    rec = oracle_lib.nnn_sweeps(s, q, seed, 0, n, oracle_lib.nnn_table(beta, j2))
    with potts.NnnLattice(L, q, seed, 1) as lat:
        lat.sweep(beta, j2, n)
        assert np.array_equal(lat.records(0, n), rec)
        assert np.array_equal(lat.spins(), s)


def test_cube_benchmark_configuration(potts, oracle_lib):
    """The simple-cubic workload's cube (L = 1024, q = 3, beta = 0.5505, random
    start, seed 1) on the kernel the benchmark times (automatic: colour-split):
    two sweeps, windows at the origin, across the periodic faces and inside
    against the oracle's window restriction, the last record against the
    observables kernel and the populations summing to N."""
    L, q, seed, beta, n = 1024, 3, 1, 0.5505, 2
    print(f"cube benchmark configuration: L={L} q={q} sweeps={n}", flush=True)
    thr = oracle_lib.threshold_table6(beta)
    with potts.Cube(L, q, seed, 1) as c:
        c.sweep(beta, n)
        rec = c.records(0, n)
        obs = c.observables()
        spins = c.spins()
    assert np.all(rec[:, 1:].sum(axis=1) == L**3)
    assert rec[-1, 0] == obs["e_sat"] and np.array_equal(rec[-1, 1:], obs["hist"])
    d, r = 16, 2 * n
    for (x0, y0, z0) in [(0, 0, 0), (L - 8, L - 8, L - 8), (L - d, 3, L - 9), (500, 511, 512), (31, 32, 33)]:
        win = oracle_lib.window3d(L, q, seed, 1, n, thr, x0, y0, z0, d)
        idx = [(c0 + np.arange(r, d - r)) % L for c0 in (z0, y0, x0)]
        assert np.array_equal(win[r:d - r, r:d - r, r:d - r], spins[np.ix_(*idx)]), (x0, y0, z0)
