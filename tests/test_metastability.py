"""Host-side pieces of the metastability analysis (Sec. 6): the transition
energies against Table 2's printed digits, the spinodal estimate (Eq. 16) at
a hand-computed point, and the power-law fit on exact and noisy power laws."""
import math

import numpy as np
import pytest

from paper_1101_0876_amd.metastability import analyse, fit_power_law, spinodal_std, transition_energies
from tests.test_golden_constants import _rows, _truncated


@pytest.mark.parametrize("row", _rows("table2"))
def test_transition_energies_reproduce_table2(row):
    q, eo_txt, ed_txt = int(row[0]), row[1], row[2]
    e_o, e_d = transition_energies(q)
    assert _truncated(-e_o, eo_txt) and _truncated(-e_d, ed_txt)


def test_transition_energies_need_first_order():
    with pytest.raises(ValueError):
        transition_energies(4)


def test_spinodal_estimate():
    # q = 5: ln(2)^2.81 = 0.35668... -> 2.4968e-4
    assert spinodal_std(5) == pytest.approx(0.0007 * 0.6931471805599453 ** 2.81, rel=1e-15)
    assert spinodal_std(9) == pytest.approx(0.0036042, rel=1e-4)
    assert spinodal_std(15) > spinodal_std(9) > spinodal_std(6)


@pytest.mark.parametrize("a,A", [(1.0, 0.2), (0.6, 1.5), (0.25, 0.01)])
def test_fit_recovers_exact_power_law(a, A):
    x = np.logspace(-4, -1, 12)
    f = fit_power_law(x, A * x**a)
    assert f["a"] == pytest.approx(a, abs=1e-12)
    assert f["A"] == pytest.approx(A, rel=1e-10)
    assert f["a_err"] < 1e-10


def test_fit_error_covers_noise():
    rng = np.random.default_rng(2)
    x = np.logspace(-3, -1, 20)
    y = 0.4 * x**0.8 * np.exp(rng.normal(0, 0.02, size=x.size))
    f = fit_power_law(x, y)
    assert abs(f["a"] - 0.8) < 5 * f["a_err"]


def test_analyse_synthetic_branches():
    q = 9
    e_o, e_d = transition_energies(q)
    Tc = 1 / math.log1p(3.0)
    tau = np.logspace(-1.5, -3.5, 9)
    T = Tc * (1 + tau)
    x = 1 - Tc / T
    high = {"q": q, "side": "high", "tau": tau, "T": T, "e_mean": e_d - 0.7 * x**1.0 * e_d}
    r = analyse(high)
    assert r["fit_all"]["a"] == pytest.approx(1.0, abs=1e-10)
    assert r["spinodal_tau"] == spinodal_std(q)
    T = Tc * (1 - tau)
    low = {"q": q, "side": "low", "tau": tau, "T": T, "e_mean": e_o + 0.3 * tau**0.9 * e_o}
    assert analyse(low)["fit_all"]["a"] == pytest.approx(0.9, abs=1e-10)
