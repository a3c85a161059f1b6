"""Pins the oracle's derived statistics (oracle/stats.py) with closed forms and an
independent floating-point evaluation."""
import math

import numpy as np
import pytest

from oracle.stats import derived


def test_constant_series():
    N, q, beta = 64, 3, 1.1
    d = derived([100] * 7, [N] * 7, N, q, beta)
    assert d["e"] == -100 / 64
    assert d["C"] == 0.0
    assert d["V_L"] == pytest.approx(2.0 / 3.0, abs=0)  # 1 - E^4/(3 E^4)
    assert d["m"] == 1.0 and d["chi"] == 0.0


def test_two_valued_series_closed_form():
    # E alternates a, b: <E> = (a+b)/2, var = ((a-b)/2)^2
    a, b, N, q, beta = 90, 110, 100, 4, 0.7
    d = derived([a, b] * 50, [N // q] * 100, N, q, beta)
    assert d["e"] == pytest.approx(-(a + b) / 2 / N, rel=1e-15)
    assert d["C"] == pytest.approx(beta**2 * ((a - b) / 2) ** 2 / N, rel=1e-15)
    e4 = (a**4 + b**4) / 2
    e2 = (a**2 + b**2) / 2
    assert d["V_L"] == pytest.approx(1 - e4 / (3 * e2**2), rel=1e-14)
    assert d["m"] == 0.0  # N_max = N/q: uniform populations


def test_against_float_evaluation():
    rng = np.random.default_rng(3)
    N, q, beta = 4096, 9, 1.4
    e = rng.integers(5000, 7000, size=1000)
    nmax = rng.integers(N // q, N, size=1000)
    d = derived(e.tolist(), nmax.tolist(), N, q, beta)
    ef = e.astype(np.float64)
    m = (q * nmax / N - 1) / (q - 1)
    assert d["e"] == pytest.approx(-ef.mean() / N, rel=1e-12)
    assert d["C"] == pytest.approx(beta**2 * ef.var() / N, rel=1e-9)
    assert d["V_L"] == pytest.approx(1 - (ef**4).mean() / (3 * (ef**2).mean() ** 2), rel=1e-12)
    assert d["m"] == pytest.approx(m.mean(), rel=1e-12)
    assert d["chi"] == pytest.approx(N * beta * m.var(), rel=1e-9)


def test_exact_where_float_cancels():
    # var/mean^2 ~ 1e-14: float64 loses the variance, exact integers do not
    big = 2**31 - 5
    e = [big, big + 1] * 500
    d = derived(e, [1] * 1000, 2**30, 6, 1.0)
    assert d["C"] == 0.25 / 2**30


# -- temperature reweighting (Sec. 7) ------------------------------------------------


def _ising4x4_all_configurations():
    """e_sat and N_max of every one of the 2^16 configurations of the 4 x 4
    periodic q = 2 lattice: an exact sample of beta = 0."""
    cfg = ((np.arange(2**16)[:, None] >> np.arange(16)) & 1).reshape(-1, 4, 4)
    e = (cfg == np.roll(cfg, -1, axis=2)).sum(axis=(1, 2)) + (cfg == np.roll(cfg, -1, axis=1)).sum(axis=(1, 2))
    ones = cfg.sum(axis=(1, 2))
    return e.tolist(), np.maximum(ones, 16 - ones).tolist()


def test_reweight_to_the_same_beta_is_the_plain_average():
    from oracle.stats import reweight

    rng = np.random.default_rng(5)
    N, q, beta = 1024, 6, 1.2
    e = rng.integers(1500, 1700, size=300).tolist()
    nmax = rng.integers(N // q, N, size=300).tolist()
    r, d = reweight(e, nmax, N, q, beta, beta), derived(e, nmax, N, q, beta)
    for k in ("e", "C", "V_L", "m", "chi"):
        assert r[k] == pytest.approx(d[k], rel=1e-14), k


@pytest.mark.parametrize("beta", [0.3, 0.8813735870195430, 1.3])
def test_reweight_of_all_configurations_gives_the_transfer_matrix_moments(beta):
    """Every configuration once is the exact beta = 0 ensemble; reweighted to
    beta it must give the canonical <E>, <E^2> of the exact row transfer
    matrix (independent of the reweighting formula)."""
    from oracle.stats import reweight
    from tests.exact import transfer_matrix_moments

    e, nmax = _ising4x4_all_configurations()
    r = reweight(e, nmax, 16, 2, 0.0, beta, digits=30)
    tm = transfer_matrix_moments(4, 2, beta)
    E = -r["e"] * 16
    assert E == pytest.approx(tm["E"], rel=1e-12)
    assert r["C"] * 16 / beta**2 + E * E == pytest.approx(tm["E2"], rel=1e-12)


def test_reweight_order_parameter_limits():
    """beta = 0: <m> over all configurations by counting (binomial sum);
    large beta: only the two ground states survive (e_sat = 2N, m = 1)."""
    from oracle.stats import reweight

    e, nmax = _ising4x4_all_configurations()
    hot = reweight(e, nmax, 16, 2, 0.0, 0.0, digits=30)
    exact_m = sum(math.comb(16, k) * (2 * max(k, 16 - k) / 16 - 1) for k in range(17)) / 2**16
    assert hot["m"] == pytest.approx(exact_m, rel=1e-14)
    cold = reweight(e, nmax, 16, 2, 0.0, 40.0, digits=30)
    assert cold["e"] == pytest.approx(-2.0, rel=1e-12)
    assert cold["m"] == pytest.approx(1.0, rel=1e-12)
    assert abs(cold["C"]) < 1e-12
