"""Row slabs through the C ABI (potts_slab_half_sweep): a lattice swept slab
by slab, halos refreshed before every half sweep, gives the oracle's bits for
any slab count, and at the single-large-lattice shape (L = 32768 in 8 slabs of
4096 rows) the bits of the whole-lattice sweep."""
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


@pytest.mark.parametrize("L,q,G,start,beta,n", [
    (256, 9, 1, 1, beta_c(9), 5),
    (256, 9, 2, 1, beta_c(9), 5),
    (512, 6, 4, 0, 1.1, 4),
    (384, 40, 3, 1, 9.0, 3),      # 128-row slabs, zero thresholds (wide table)
    (272, 200, 17, 1, 2.0, 3),    # 16-row slabs, q > 128
    (64, 3, 8, 1, 1.0, 7),        # 8-row slabs (items of 2 rows)
])
def test_slabs_match_oracle(potts, oracle_lib, L, q, G, start, beta, n):
    _say(f"slabs L={L} q={q} G={G} start={start} n={n}")
    s = oracle_lib.init(L, q, 31, start)
    rec = oracle_lib.sweeps(s, q, 31, 0, n, oracle_lib.threshold_table(beta))
    sl = potts.Slabs(L, q, 31, start, nslabs=G, ring_slots=8)
    sl.sweep(beta, n)
    assert np.array_equal(sl.spins(), s)
    assert np.array_equal(sl.records(0, n), rec)


def test_slabs_continue_across_calls(potts, oracle_lib):
    L, q, beta = 128, 5, beta_c(5)
    s = oracle_lib.init(L, q, 8, 1)
    rec = oracle_lib.sweeps(s, q, 8, 0, 10, oracle_lib.threshold_table(beta))
    sl = potts.Slabs(L, q, 8, 1, nslabs=4, ring_slots=4)
    for _ in range(10):
        sl.sweep(beta, 1)
    assert np.array_equal(sl.spins(), s)
    assert np.array_equal(sl.records(7, 3), rec[7:])


def test_slabs_at_full_shape(potts, oracle_lib):
    """One device's share of the single large lattice run on 8 devices:
    L = 32768, slabs of 4096 rows.  Equal bits to the whole-lattice sweep, and
    oracle windows across slab edges."""
    import torch

    L, q, seed, beta, n, G = 32768, 6, 1, beta_c(6), 2, 8
    _say(f"slabs full shape L={L} G={G} n={n}")
    sl = potts.Slabs(L, q, seed, 1, nslabs=G, ring_slots=4)
    sl.sweep(beta, n)
    torch.cuda.synchronize()
    with potts.Lattice.from_torch(L, q, seed, 1) as lat:
        lat.sweep(beta, n)
        rec = lat.records(0, n)
        a, b, _ = lat._keep
        cur = (a if lat.device_ptr() == a.data_ptr() else b).view(L, L)
        torch.cuda.synchronize()
        for g in range(G):
            assert torch.equal(cur[g * 4096:(g + 1) * 4096], sl.buf[g][1:4097]), g
    assert np.array_equal(sl.records(0, n), rec)
    thr = oracle_lib.threshold_table(beta)
    r = 2 * n
    for (x0, y0) in [(100, 4096 - 24), (L - 24, 7 * 4096 - 24), (5000, L - 24)]:
        h = w = 48
        win = oracle_lib.window(L, q, seed, 1, n, thr, x0, y0, h, w)
        for i in range(r, h - r):
            y = (y0 + i) % L
            g, yy = divmod(y, 4096)
            xs = (x0 + np.arange(r, w - r)) % L
            got = sl.buf[g][1 + yy].cpu().numpy()[xs]
            assert np.array_equal(win[i, r:w - r], got), (x0, y0, i)
