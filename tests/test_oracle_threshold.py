"""Pins the oracle's acceptance table against exp evaluated in 60-digit decimal
arithmetic: thr[d] = min(floor(exp(-beta d) 2^32), 2^32 - 1), d = 1..4
(Metropolis weights kept per temperature, Sec. 5)."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

from tests.inputs import beta_c

getcontext().prec = 60
TWO32 = Decimal(2) ** 32


def _exact_scaled(beta: float, d: int) -> Decimal:
    return (-(Decimal(beta) * d)).exp() * TWO32


BETAS = [0.0, 1e-12, 0.1, 0.5, beta_c(2), beta_c(3), beta_c(6), 1.02 * math.log(4.0), beta_c(9),
         beta_c(15), 2.0, 5.0, 7.0, 50.0]


@pytest.mark.parametrize("beta", BETAS)
def test_table_is_floor_of_exact_weight(oracle_lib, beta):
    thr = oracle_lib.threshold_table(beta)
    for d in range(1, 5):
        exact = _exact_scaled(beta, d)
        want = min(int(exact), 2**32 - 1)  # int() floors a positive Decimal
        frac = exact - int(exact)
        if Decimal("1e-6") < frac < 1 - Decimal("1e-6") or want == 2**32 - 1:
            assert int(thr[d - 1]) == want, (beta, d)
        else:  # the FP64 exp may round across an integer: one unit either way
            assert abs(int(thr[d - 1]) - want) <= 1
        # acceptance probability thr/2^32 is within 2^-31 of min(exp(-beta d), 1 - 2^-32)
        assert abs(Decimal(int(thr[d - 1])) - min(exact, Decimal(2**32 - 1))) < 2


def test_table_limits_and_monotonicity(oracle_lib):
    assert list(oracle_lib.threshold_table(0.0)) == [2**32 - 1] * 4
    assert list(oracle_lib.threshold_table(50.0)) == [0, 0, 0, 0]
    prev = None
    for beta in np.linspace(0, 3, 61):
        thr = [int(v) for v in oracle_lib.threshold_table(float(beta))]
        assert thr == sorted(thr, reverse=True)
        if prev is not None:
            assert all(a <= b for a, b in zip(thr, prev))
        prev = thr


@pytest.mark.parametrize("beta", [-1.0, float("nan"), float("inf")])
def test_table_rejects_bad_beta(oracle_lib, beta):
    with pytest.raises(ValueError):
        oracle_lib.threshold_table(beta)
