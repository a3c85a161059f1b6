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
