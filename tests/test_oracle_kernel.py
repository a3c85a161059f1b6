"""Pins the oracle's single-site Metropolis rule and its half sweep to the exact
transition kernel.

The per-site transition probabilities are read off the oracle's own decision
function (``oracle_site_update``) by locating, with binary search over the
32-bit words, the interval of proposal words giving each value k and the
acceptance-word cut-off for each move.  Then:

  * detailed balance  exp(beta n(a)) P(a->b) = exp(beta n(b)) P(b->a)  for every
    neighbourhood, which is what Metropolis at H = -sum delta (Eq. 1) must give,
    to within the 2^-32 quantisation of the table;
  * the outcome frequencies of the oracle's real half sweep over many sweep
    indices match those probabilities site by site (ties neighbour indexing,
    colour selection and random words to the kernel).
"""
import itertools
import math

import numpy as np
import pytest

from tests.inputs import random_lattice

ALWAYS = [2**32 - 1] * 4


def _proposal_edges(oracle_lib, q):
    """edges[k] = first 32-bit word proposing value k (edges[q] = 2^32)."""
    nb = [0, 0, 0, 0]

    def prop(w):
        # acceptance word 0 with a saturated table accepts every move
        return oracle_lib.site_update(q, 0, nb, w, 0, ALWAYS)

    edges = [0]
    for k in range(1, q):
        lo, hi = edges[-1], 2**32  # first w with prop(w) >= k
        while lo < hi:
            mid = (lo + hi) // 2
            if prop(mid) >= k:
                hi = mid
            else:
                lo = mid + 1
        edges.append(lo)
    edges.append(2**32)
    rng = np.random.default_rng(1)
    for w in rng.integers(0, 2**32, size=200):
        k = int(np.searchsorted(edges, int(w), side="right") - 1)
        assert prop(int(w)) == k
    return edges


def _accept_cut(oracle_lib, q, s, nb, w_prop, thr):
    """Number of acceptance words (out of 2^32) that accept the proposed move."""
    k = oracle_lib.site_update(q, s, nb, w_prop, 0, ALWAYS)
    if k == s:
        return 2**32
    lo, hi = 0, 2**32  # first acceptance word that rejects
    while lo < hi:
        mid = (lo + hi) // 2
        if oracle_lib.site_update(q, s, nb, w_prop, mid, thr) == s:
            hi = mid
        else:
            lo = mid + 1
    return lo


def _site_probs(oracle_lib, q, nb, thr, edges):
    """P[a][b] for one neighbourhood, exact rationals over 2^64 as floats."""
    P = np.zeros((q, q))
    for a in range(q):
        for b in range(q):
            width = edges[b + 1] - edges[b]
            if b == a:
                continue
            P[a, b] = width / 2**32 * _accept_cut(oracle_lib, q, a, nb, edges[b], thr) / 2**32
        P[a, a] = 1.0 - P[a].sum()
    return P


@pytest.mark.parametrize("q", [2, 3, 5])
@pytest.mark.parametrize("beta", [0.4, 1.3])
def test_detailed_balance_per_neighbourhood(oracle_lib, q, beta):
    thr = oracle_lib.threshold_table(beta)
    edges = _proposal_edges(oracle_lib, q)
    widths = np.diff(np.array(edges, dtype=np.float64))
    assert np.all(np.abs(widths / 2**32 - 1.0 / q) <= 1.0 / 2**32)
    neighbourhoods = list(itertools.product(range(q), repeat=4))
    if len(neighbourhoods) > 200:
        rng = np.random.default_rng(q)
        neighbourhoods = [neighbourhoods[i] for i in rng.choice(len(neighbourhoods), 200, replace=False)]
    for nb in neighbourhoods:
        P = _site_probs(oracle_lib, q, list(nb), thr, edges)
        n = [sum(1 for v in nb if v == a) for a in range(q)]
        for a in range(q):
            for b in range(a + 1, q):
                lhs = math.exp(beta * n[a]) * P[a, b]
                rhs = math.exp(beta * n[b]) * P[b, a]
                assert lhs == pytest.approx(rhs, rel=2e-7), (nb, a, b)
                assert P[a, b] > 0


def test_zero_and_infinite_temperature_rules(oracle_lib):
    q = 4
    nb = [1, 1, 2, 3]
    zero_t = [0, 0, 0, 0]
    edges = _proposal_edges(oracle_lib, q)
    # beta = inf: only moves that do not lose satisfied bonds
    for s in range(q):
        for k in range(q):
            new = oracle_lib.site_update(q, s, nb, edges[k], 0, zero_t)
            lost = nb.count(s) - nb.count(k)
            assert new == (k if lost <= 0 else s)


@pytest.mark.parametrize("colour", [0, 1])
def test_half_sweep_frequencies_match_kernel(oracle_lib, colour):
    L, q, beta, seed = 8, 3, 0.9, 99
    thr = oracle_lib.threshold_table(beta)
    edges = _proposal_edges(oracle_lib, q)
    base = random_lattice(L, q, seed=4)
    M = 6000
    counts = np.zeros((L, L, q), dtype=np.int64)
    for t in range(M):
        s = base.copy()
        oracle_lib.half_sweep(s, q, seed, t, colour, thr)
        # the other colour never changes
        mask = ((np.add.outer(np.arange(L), np.arange(L))) & 1) != colour
        assert np.array_equal(s[mask], base[mask])
        counts[np.arange(L)[:, None], np.arange(L)[None, :], s] += 1
    chi2, dof = 0.0, 0
    for y in range(L):
        for x in range(L):
            if (x + y) & 1 != colour:
                continue
            nb = [base[y, (x + 1) % L], base[y, (x - 1) % L], base[(y + 1) % L, x], base[(y - 1) % L, x]]
            P = _site_probs(oracle_lib, q, [int(v) for v in nb], thr, edges)[base[y, x]]
            exp = M * P
            chi2 += float((((counts[y, x] - exp) ** 2) / exp).sum())
            dof += q - 1
    # 64 dof; a wrong neighbour or word choice gives chi2 in the thousands
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)
