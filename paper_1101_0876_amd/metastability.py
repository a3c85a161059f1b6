"""Binder's metastability criterion on the GPU path (Sec. 2.2, Sec. 6).

If the transition has true metastable states, the specific heat diverges at
pseudo-spinodal temperatures away from T_c (Eqs. 14-15), and the two energy
branches reach T_c with a finite slope: fitted to the power laws in the
distance to T_c of Eqs. 12-13, their exponents tend to 1 close enough to T_c.
A divergence at T_c itself would give exponents below 1.

``branch`` measures one branch as the paper does: each sample starts in the
phase that is stable on that side (ordered below T_c, random above) and is
carried through temperatures approaching T_c, sweeps split per point with the
second half of each point measured.  All samples run concurrently through the
serving loop (potts_server_*), so a branch is one batch of jobs on the GPU.
``fit_power_law`` and ``analyse`` do the host-side fits; ``spinodal_std``
gives the short-time-dynamics estimate of the lower spinodal (Eq. 16) that
marks where the crossover is expected on the high-temperature branch.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np


def beta_c(q: int) -> float:
    """Exact transition point, Eq. 2: beta_c = ln(1 + sqrt q)."""
    return math.log1p(math.sqrt(q))


def transition_energies(q: int) -> tuple:
    """(e_o, e_d): energies per site of the ordered and disordered phases at
    T_c, from the latent heat (Eq. 3, read with prefactor 2(1 + 1/sqrt q) and
    Theta = arccosh(sqrt(q)/2)) and the self-dual mean (Eq. 6:
    e_o + e_d = -2(1 + 1/sqrt q)).  Needs q > 4."""
    if q <= 4:
        raise ValueError("the transition is first order only for q > 4")
    theta = math.acosh(math.sqrt(q) / 2)
    prod, n = 1.0, 1
    while True:
        f = math.tanh(n * theta) ** 2
        prod *= f
        if 1.0 - f < 1e-17:
            break
        n += 1
    latent = 2 * (1 + 1 / math.sqrt(q)) * math.tanh(theta / 2) * prod
    mean = -(1 + 1 / math.sqrt(q))
    return mean - latent / 2, mean + latent / 2


def spinodal_std(q: int) -> float:
    """(T_c - T_sp^-)/T_c from short-time dynamics, Eq. 16:
    0.0007 (ln(1 + q - 4))^2.81."""
    return 0.0007 * math.log(q - 3) ** 2.81


def branch(q: int, L: int, samples: int, taus: Sequence[float], sweeps: int, side: str,
           seed0: int = 1, server=None) -> Dict:
    """One energy branch.  side "high": T = T_c (1 + tau), random start, beta
    ascending (cooling towards T_c); side "low": T = T_c (1 - tau), ordered
    start, beta descending (heating towards T_c).  taus are visited from the
    largest to the smallest; `sweeps` sweeps per point, the second half
    measured.  Sample i uses seed seed0 + i."""
    from . import ORDERED, RANDOM, Server

    if side not in ("high", "low"):
        raise ValueError("side is 'high' or 'low'")
    tau = np.sort(np.asarray(taus, dtype=np.float64))[::-1]
    Tc = 1.0 / beta_c(q)
    T = Tc * (1 + tau) if side == "high" else Tc * (1 - tau)
    betas = 1.0 / T
    start = RANDOM if side == "high" else ORDERED
    own = server is None
    srv = Server() if own else server
    try:
        tickets = [srv.submit(L, q, seed0 + i, start, betas, [sweeps] * len(betas)) for i in range(samples)]
        srv.drain()
        e = np.empty((samples, len(betas)))
        C = np.empty((samples, len(betas)))
        for i, t in enumerate(tickets):
            res = srv.collect(t)
            if res["status"] != 0:
                raise RuntimeError(f"sample {i} failed with code {res['status']}")
            e[i] = [p["e"] for p in res["points"]]
            C[i] = [p["C"] for p in res["points"]]
    finally:
        if own:
            srv.stop()
    return {"q": q, "L": L, "side": side, "tau": tau, "T": T, "beta": betas, "sweeps": sweeps,
            "samples": samples, "e": e, "C": C, "e_mean": e.mean(axis=0),
            "e_err": e.std(axis=0, ddof=1) / math.sqrt(samples) if samples > 1 else np.zeros(len(tau))}


def fit_power_law(x, y) -> Dict[str, float]:
    """Least-squares fit of log y = log A + a log x; returns a, A and the
    standard error of a."""
    lx, ly = np.log(np.asarray(x, dtype=np.float64)), np.log(np.asarray(y, dtype=np.float64))
    n = lx.size
    if n < 2:
        raise ValueError("need at least two points")
    X = np.vstack([lx, np.ones(n)]).T
    coef, res, _, _ = np.linalg.lstsq(X, ly, rcond=None)
    a, logA = coef
    err = float("nan")
    if n > 2:
        resid = ly - X @ coef
        s2 = float(resid @ resid) / (n - 2)
        err = math.sqrt(s2 / float(((lx - lx.mean()) ** 2).sum()))
    return {"a": float(a), "A": float(math.exp(logA)), "a_err": err}


def analyse(b: Dict) -> Dict:
    """Energy differences of a branch against the transition energies and their
    power-law fits (Eqs. 12-13): high side |(e - e_d)/e_d| against 1 - T_c/T,
    low side (e - e_o)/e_o against 1 - T/T_c; fitted over all points and
    separately on both sides of the spinodal estimate (high side only)."""
    q = b["q"]
    e_o, e_d = transition_energies(q)
    Tc = 1.0 / beta_c(q)
    T, e = b["T"], b["e_mean"]
    if b["side"] == "high":
        x, y = 1.0 - Tc / T, np.abs((e - e_d) / e_d)
    else:
        x, y = 1.0 - T / Tc, (e - e_o) / e_o
    out = {"x": x, "y": y, "fit_all": fit_power_law(x, y) if np.all(y > 0) else None}
    if b["side"] == "high":
        cut = spinodal_std(q)
        near, far = b["tau"] <= cut, b["tau"] > cut
        out["spinodal_tau"] = cut
        out["fit_near"] = fit_power_law(x[near], y[near]) if near.sum() >= 2 and np.all(y[near] > 0) else None
        out["fit_far"] = fit_power_law(x[far], y[far]) if far.sum() >= 2 and np.all(y[far] > 0) else None
    return out
