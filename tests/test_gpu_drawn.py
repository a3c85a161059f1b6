"""GPU parity of the LDS-resident kernel with pre-drawn words (kernel 6, the
automatic choice for single lattices with L % 16 == 0 and L <= 64): a
generator kernel over the whole GPU draws every site's proposal and
acceptance word for a chunk of up to 1024 sweeps, and the one-workgroup
kernel reads them a few half sweeps ahead.  Spins and every record must
equal the oracle's, bit for bit, as for every other kernel."""
import math

import numpy as np
import pytest

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


# every lattice size the kernel takes, every q class (q <= 16 packed flags,
# q <= 64 lane-private counters, shared bins beyond), odd sweep counts (the
# loop body runs two sweeps), both starts
@pytest.mark.parametrize("L,q,seed,start,beta,n", [
    (16, 2, 1, 1, 0.7, 9),
    (16, 3, 4, 0, beta_c(3), 20),
    (32, 9, 3, 1, 1.02 * beta_c(9), 15),
    (48, 17, 6, 1, beta_c(17), 7),
    (64, 9, 1, 1, 1.02 * math.log(4.0), 40),
    (64, 6, 2, 0, beta_c(6), 1),
    (64, 64, 5, 1, beta_c(64), 6),
    (64, 65, 8, 1, 0.9 * beta_c(65), 5),
    (64, 256, 9, 1, 0.3, 4),
])
def test_drawn_kernel_matches_oracle(potts, oracle_lib, L, q, seed, start, beta, n):
    _say(f"drawn L={L} q={q} seed={seed} start={start} n={n}")
    want_spins, want_rec = oracle_lib.run(L, q, seed, start, beta, n)
    with potts.Lattice(L, q, seed, start) as lat:
        lat.tune(kernel=6)
        lat.sweep(beta, n)
        assert np.array_equal(lat.spins(), want_spins)
        assert np.array_equal(lat.records(0, n), want_rec)


def test_drawn_kernel_is_the_automatic_choice_and_equals_kernel_3(potts):
    """The automatic choice for L = 64 and the in-kernel draw (kernel 3) give
    the same chain: the plain method's configuration, 1000 sweeps."""
    L, q, seed, n = 64, 9, 1, 1000
    beta = 1.02 * math.log(4.0)
    _say(f"drawn vs resident L={L} q={q} n={n}")
    out = []
    for kernel in (0, 3, 6):
        with potts.Lattice(L, q, seed, potts.RANDOM) as lat:
            lat.tune(kernel=kernel)
            lat.sweep(beta, n)
            out.append((lat.spins(), lat.records(0, n)))
    for spins, rec in out[1:]:
        assert np.array_equal(spins, out[0][0])
        assert np.array_equal(rec, out[0][1])


def test_drawn_kernel_across_chunks_and_calls(potts, oracle_lib):
    """Runs longer than one generator chunk (1024 sweeps), split over calls of
    uneven length, against the oracle."""
    L, q, seed, beta = 16, 5, 21, 0.95 * beta_c(5)
    _say(f"drawn chunks L={L} q={q}")
    s = oracle_lib.init(L, q, seed, 1)
    want = oracle_lib.sweeps(s, q, seed, 0, 2100, oracle_lib.threshold_table(beta))
    with potts.Lattice(L, q, seed, 1) as lat:
        lat.reserve_records(4096)
        lat.tune(kernel=6)
        for n in (1025, 3, 1072):
            lat.sweep(beta, n)
        assert lat.t == 2100
        assert np.array_equal(lat.records(0, 2100), want)
        assert np.array_equal(lat.spins(), s)


def test_drawn_kernel_with_zero_thresholds(potts, oracle_lib):
    """A caller table with zero entries (moves that raise the energy by 3 or 4
    never accepted) takes the 64-bit table form."""
    L, q, seed = 32, 4, 3
    thr = [2**31, 2**30, 0, 0]
    s = oracle_lib.init(L, q, seed, 1)
    want = oracle_lib.sweeps(s, q, seed, 0, 11, thr)
    with potts.Lattice(L, q, seed, 1) as lat:
        lat.tune(kernel=6)
        lat.sweep_thr(thr, 11)
        assert np.array_equal(lat.records(0, 11), want)
        assert np.array_equal(lat.spins(), s)


def test_drawn_kernel_rejects_larger_lattices(potts):
    with potts.Lattice(80, 3, 1, 0) as lat:
        with pytest.raises(potts.PottsError):
            lat.tune(kernel=6)
