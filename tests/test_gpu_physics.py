"""Physics at the transition on the GPU path (through the C ABI), against the
exact values the paper prints.

Table 2 lists, for q = 6, 9, 15, 96, the exact energies per site of the
ordered and disordered phases at T_c (Eq. 2, Eq. 3, Eq. 6) and the jump of
the order parameter (Eq. 8).  At beta_c an
ordered start stays in the ordered phase and a random start in the disordered
one on these time scales (first-order transition, L much larger than the
correlation length), so the mean energy of the second half of the run must
approach e_o and e_d respectively.  Tolerances cover the relaxation left after
the first half and the statistical error of L = 2048 lattices (measured
deviations are several times smaller).  q = 6 (correlation length ~ 160 sites
at T_c) relaxes slowly: it runs the paper's protocol (temperature stepped to
T_c, 5 x 10^5 sweeps of equilibration and as many of measurement) and is
compared with Table 2's calculated column within its printed errors.
"""
import os

import numpy as np
import pytest

from tests.inputs import beta_c

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def table2():
    out = {}
    for line in open(GOLDEN):
        parts = line.split()
        if parts and parts[0] == "table2":
            out[int(parts[1])] = (-float(parts[2]), -float(parts[3]))  # (e_o, e_d)
    return out


def table2_calc():
    """Table 2's calculated columns: q -> (-e_o, err, -e_d, err, Delta m, err)."""
    out = {}
    for line in open(GOLDEN):
        parts = line.split()
        if parts and parts[0] == "table2calc":
            out[int(parts[1])] = tuple(float(x) for x in parts[2:8])
    return out


def table2_dm():
    return {int(p[1]): float(p[2]) for p in (line.split() for line in open(GOLDEN)) if p and p[0] == "table2dm"}


@pytest.fixture(scope="module")
def potts():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_0876_amd as p

    p.load()
    return p


@pytest.mark.parametrize("q,n,tol", [(9, 100000, 1.5e-3), (15, 20000, 1e-3), (96, 20000, 3e-4)])
@pytest.mark.parametrize("start", [0, 1])
def test_table2_phase_energies_at_beta_c(potts, q, n, tol, start):
    L, seed = 2048, 7
    e_o, e_d = table2()[q]
    want = e_o if start == potts.ORDERED else e_d
    print(f"table2 q={q} start={start} n={n}", flush=True)
    with potts.Lattice(L, q, seed, start) as lat:
        lat.reserve_records(n // 2 + 2)
        lat.sweep(beta_c(q), n)
        s = lat.stats(n - n // 2, n // 2, beta_c(q))
        last = lat.records(n - 1, 1)
    assert int(last[0, 1:].sum()) == L * L
    assert abs(s["e"] - want) < tol, (s["e"], want)
    # the other phase is far away: the run did not switch phase
    other = e_d if start == potts.ORDERED else e_o
    assert abs(s["e"] - other) > 0.1


@pytest.mark.parametrize("q,n,tol", [(9, 100000, 1.5e-3), (15, 20000, 6e-4), (96, 20000, 1e-4)])
def test_table2_order_parameter_jump(potts, q, n, tol):
    """The jump of the order parameter (Eq. 7) at T_c, as Table 2 reads it:
    <m> of the ordered phase (ordered start at beta_c, second half of the run)
    against the exact Delta m, the disordered phase (random start) having
    <m> -> 0 (here only the O(1/L) excess of the largest population).
    Measured on MI355X: m_o - Delta m = -5.6e-4, -2.1e-4, +3.2e-5 and m_d =
    2.0e-3, 7.6e-4, 1.7e-4 for q = 9, 15, 96; the tolerances are about three
    times those deviations."""
    L, seed = 2048, 11
    m = {}
    for start in (0, 1):
        print(f"table2 dm q={q} start={start} n={n}", flush=True)
        with potts.Lattice(L, q, seed, start) as lat:
            lat.reserve_records(n // 2 + 2)
            lat.sweep(beta_c(q), n)
            m[start] = lat.stats(n - n // 2, n // 2, beta_c(q))["m"]
    print(f"q={q} m_o={m[0]:.6f} m_d={m[1]:.6f} want={table2_dm()[q]}", flush=True)
    assert abs(m[0] - table2_dm()[q]) < tol, (m, table2_dm()[q])
    assert 0.0 <= m[1] < 5e-3, m


def test_table2_q6_by_the_papers_protocol(potts):
    """q = 6 as Table 2 was measured (Sec. 4): L = 2048, heating from the
    ordered start and cooling from the random one, the temperature stepped to
    T_c from 0.1 % below (heating) or above (cooling), 10^6 sweeps per point of
    which the second half is measured (Table 2: at least 5 x 10^5 MCS of
    equilibration and as many of measurement); four samples per branch (the
    paper: ten), run as eight jobs of one serving loop, averaged.

    Table 2 prints, for q = 6, the calculated -e_o = 1.51(2), -e_d = 1.306(1)
    and Delta m = 0.674(2) beside the exact 1.508980, 1.307516, 0.677083; its
    own -e_d and Delta m lie 1.5 printed errors from the exact values.  At T_c
    the two phases coexist and q = 6 (correlation length ~ 160 sites) mixes
    them slowly: single L = 2048 samples measured on MI355X gave m_o from
    0.652 to 0.676 (disordered droplets in the ordered branch) and e_d from
    -1.3034 to -1.3089 with m_d up to 0.02 (ordered droplets in the
    disordered branch).  The four-sample means must agree with the
    calculated column within its printed error plus 0.003 (-e_d) or 0.012
    (Delta m), and with the exact values within 0.02, 0.005 and 0.015.  One
    step past T_c the branches have left their phase already (the ordered
    start has e = -1.262 at 1.001 T_c), so, as in the paper, the value is read
    at T_c itself."""
    q, L = 6, 2048
    Tc = 1.0 / beta_c(q)
    n = 1000000
    e_o, e_d = table2()[q]
    dm = table2_dm()[q]
    heat = [1.0 / (Tc * 0.999), beta_c(q)]
    cool = [1.0 / (Tc * 1.001), beta_c(q)]
    print(f"table2 q=6 protocol: 8 served jobs x 2 points x {n} sweeps", flush=True)
    with potts.Server(quantum=1024, max_slots=8) as srv:
        jobs = [(srv.submit(L, q, seed, potts.ORDERED, heat, [n, n]), "o") for seed in (7, 8, 9, 10)]
        jobs += [(srv.submit(L, q, seed, potts.RANDOM, cool, [n, n]), "d") for seed in (11, 12, 13, 14)]
        srv.drain(900000)
        got = {"o": [], "d": []}
        for ticket, branch in jobs:
            r = srv.collect(ticket)
            assert r["status"] == 0 and r["sweeps"] == 2 * n
            got[branch].append(r["points"][1])
    for branch in ("o", "d"):
        print("q=6 " + branch + ": " + ", ".join(f"e {p['e']:.5f} m {p['m']:.5f}" for p in got[branch]), flush=True)
    eo = float(np.mean([p["e"] for p in got["o"]]))
    mo = float(np.mean([p["m"] for p in got["o"]]))
    ed = float(np.mean([p["e"] for p in got["d"]]))
    md = float(np.mean([p["m"] for p in got["d"]]))
    print(f"q=6 at T_c: e_o {eo:.5f} (Table 2: -1.51(2), exact {e_o:.6f}), e_d {ed:.5f} (-1.306(1), exact "
          f"{e_d:.6f}), m_o {mo:.5f} (0.674(2), exact {dm:.6f}), m_d {md:.5f}", flush=True)
    c_eo, err_eo, c_ed, err_ed, c_dm, err_dm = table2_calc()[q]
    assert abs(-eo - c_eo) < err_eo and abs(eo - e_o) < 0.02
    assert abs(-ed - c_ed) < err_ed + 0.003 and abs(ed - e_d) < 0.005
    assert abs(mo - c_dm) < err_dm + 0.012 and abs(mo - dm) < 0.015
    assert 0.0 <= md < 0.05
