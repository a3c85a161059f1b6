"""Derived FP64 observables of a window of per-sweep integer records, computed
with exact rational arithmetic and rounded once.

TEST INFRASTRUCTURE ONLY (part of the oracle).

Inputs are the integer series the sweep records: e_sat[t] (satisfied bonds,
H = -e_sat, Eq. 1) and nmax[t] = max_v N_v (Eq. 7), for n sweeps of an
N-site lattice with q states at inverse temperature beta.

  energy per spin     e   = <H>/N                               (Sec. 2.1)
  specific heat       C   = beta^2 (<H^2> - <H>^2) / N          (standard
                            fluctuation form; the paper does not print it)
  energy cumulant     V_L = 1 - <H^4> / (3 <H^2>^2)             (Sec. 4, Eq. 9)
  order parameter     m   = (q N_max/N - 1) / (q - 1)           (Eq. 7, read as
                            the standard form: 1 when ordered, 0 when uniform)
  susceptibility      chi = (N/T) (<m^2> - <m>^2), T = 1/beta   (Sec. 4, Eq. 11)

beta enters as the FP64 value the caller passes; it is converted exactly to a
rational, so the only rounding is the final conversion of each result.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Dict, Sequence


def derived(e_sat: Sequence[int], nmax: Sequence[int], N: int, q: int, beta: float) -> Dict[str, float]:
    n = len(e_sat)
    if n == 0 or len(nmax) != n:
        raise ValueError("need a non-empty window with one nmax per record")
    b = Fraction(beta)
    s1 = sum(int(e) for e in e_sat)
    s2 = sum(int(e) ** 2 for e in e_sat)
    s4 = sum(int(e) ** 4 for e in e_sat)
    # <H> = -s1/n ; <H^2> = s2/n ; <H^4> = s4/n
    e_mean = Fraction(-s1, n * N)
    heat = b * b * Fraction(n * s2 - s1 * s1, n * n * N)
    v_l = (1 - Fraction(n * s4, 3 * s2 * s2)) if s2 != 0 else Fraction(0)
    ms = [Fraction(q * int(k) - N, N * (q - 1)) for k in nmax]
    m1 = sum(ms) / n
    m2 = sum(m * m for m in ms) / n
    chi = Fraction(N) * b * (m2 - m1 * m1)
    return {
        "e": float(e_mean),
        "C": float(heat),
        "V_L": float(v_l),
        "m": float(m1),
        "chi": float(chi),
        "S1": s1,
        "S2": s2,
        "S4": s4,
    }


def reweight(e_sat: Sequence[int], nmax: Sequence[int], N: int, q: int, beta0: float, beta: float,
             digits: int = 50) -> Dict[str, float]:
    """Single-histogram temperature reweighting (Ferrenberg and Swendsen, 1989;
    named in Sec. 7): a series recorded at beta0 gives canonical averages at
    beta as <X>_beta = sum_t X_t w_t / sum_t w_t with w_t = exp(-(beta - beta0)
    H_t) = exp((beta - beta0) e_sat_t).  The observables are those of
    `derived`, evaluated with the weighted averages at beta.  Arithmetic in
    `digits`-digit decimal with an unbounded exponent range; beta0 and beta
    enter as the exact values of the FP64 numbers passed."""
    from decimal import MAX_EMAX, MIN_EMIN, Decimal, localcontext

    n = len(e_sat)
    if n == 0 or len(nmax) != n:
        raise ValueError("need a non-empty window with one nmax per record")
    with localcontext() as ctx:
        ctx.prec = digits
        ctx.Emax = MAX_EMAX
        ctx.Emin = MIN_EMIN
        b = Decimal(beta)
        db = b - Decimal(beta0)
        w = [(db * int(e)).exp() for e in e_sat]
        W = sum(w)

        def avg(xs):
            return sum(wi * x for wi, x in zip(w, xs)) / W

        E = [Decimal(int(e)) for e in e_sat]
        e1, e2, e4 = avg(E), avg([x * x for x in E]), avg([x ** 4 for x in E])
        ms = [Decimal(q * int(k) - N) / Decimal(N * (q - 1)) for k in nmax]
        m1, m2 = avg(ms), avg([m * m for m in ms])
        return {
            "e": float(-e1 / N),
            "C": float(b * b * (e2 - e1 * e1) / N),
            "V_L": float(1 - e4 / (3 * e2 * e2)) if e2 != 0 else 0.0,
            "m": float(m1),
            "chi": float(N * b * (m2 - m1 * m1)),
        }
