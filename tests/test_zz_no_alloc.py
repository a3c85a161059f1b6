"""The allocation-free entry point potts_sweep_static, through the C ABI,
against potts_sweep_thr of a state on the same row-major strip kernel: the
same lattice and every record, bit for bit, on two calls in a row (the second
on a smaller lattice with fewer states, continuing a chain at t0 > 0), so
that the static partial records left by one call cannot leak into the next.
The first case is also checked against the oracle."""
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


def _reference(potts, L, q, seed, start, thr, t_pre, n):
    """potts_sweep_thr on a state (strip kernel): the lattice after t_pre
    sweeps, then after t_pre + n, and the records of the last n sweeps."""
    with potts.Lattice(L, q, seed, start) as ref:
        ref.tune(kernel=1)
        if t_pre:
            ref.sweep_thr(thr, t_pre)
        before = ref.spins()
        ref.sweep_thr(thr, n)
        return before, ref.spins(), ref.records(t_pre, n)


def _static(potts, before, L, q, seed, thr, t0, n):
    import torch

    spins = torch.from_numpy(before.reshape(-1).copy()).to("cuda")
    rec = torch.full((n, q + 1), -1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    print(f"potts_sweep_static L={L} q={q} seed={seed} t0={t0} n={n}", flush=True)
    potts.sweep_static(spins.data_ptr(), L, q, seed, t0, thr, n, rec.data_ptr(), stream.cuda_stream)
    stream.synchronize()
    return spins.cpu().numpy().reshape(L, L), rec.cpu().numpy()


def test_static_sweeps_equal_the_state_path(potts, oracle_lib):
    cases = [
        # L, q, seed, start, beta, sweeps before, sweeps
        (528, 200, 5, potts.RANDOM, beta_c(200), 0, 6),
        (64, 3, 9, potts.ORDERED, 1.3, 3, 4),
    ]
    for k, (L, q, seed, start, beta, t_pre, n) in enumerate(cases):
        thr = potts.threshold_table(beta)
        before, want_spins, want_rec = _reference(potts, L, q, seed, start, thr, t_pre, n)
        got_spins, got_rec = _static(potts, before, L, q, seed, thr, t_pre, n)
        assert np.array_equal(got_rec, want_rec), k
        assert np.array_equal(got_spins, want_spins), k
        if k == 0:
            o_spins, o_rec = oracle_lib.run(L, q, seed, start, beta, n)
            assert np.array_equal(got_spins, o_spins)
            assert np.array_equal(got_rec, o_rec)


def test_static_sweeps_error_codes(potts):
    import torch

    thr = potts.threshold_table(math.log(1 + math.sqrt(3)))
    spins = torch.zeros(64 * 64, dtype=torch.uint8, device="cuda")
    rec = torch.zeros((2, 4), dtype=torch.int64, device="cuda")
    for args in [(spins.data_ptr(), 60, 3, 1, 0, thr, 2, rec.data_ptr()),   # L % 16 != 0
                 (spins.data_ptr(), 64, 257, 1, 0, thr, 2, rec.data_ptr()),  # q > 256
                 (spins.data_ptr(), 64, 3, 1, -1, thr, 2, rec.data_ptr()),   # t0 < 0
                 (spins.data_ptr(), 64, 3, 1, 0, thr, 2, 0),                 # no record buffer
                 (0, 64, 3, 1, 0, thr, 2, rec.data_ptr())]:                  # no lattice
        with pytest.raises(potts.PottsError):
            potts.sweep_static(*args)
    with pytest.raises(potts.PottsError):
        potts.sweep_static(spins.data_ptr(), 64, 3, 1, 2 ** 63 - 2, thr, 4, rec.data_ptr())
    # nothing to do: no error, nothing written
    potts.sweep_static(spins.data_ptr(), 64, 3, 1, 0, thr, 0, rec.data_ptr())
    torch.cuda.synchronize()
    assert int(rec.abs().sum()) == 0 and int(spins.sum()) == 0
