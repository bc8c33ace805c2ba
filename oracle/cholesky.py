"""Symmetry-adapted two-step Cholesky decomposition of a symmetric positive
semidefinite "two-electron integral" matrix, FP64, on the CPU (oracle, test
infrastructure only).

Paper (arXiv 2512.21909): section "Symmetry-adapted two-step CD algorithm"
(Algorithm 1: the Cholesky basis) and the CD/DF section's equation for the
second-step vectors, ``L^P_rs = sum_R K^-1_PR (R|rs)`` with ``K K^T`` the
metric ``(Q|R)`` over the basis.

What the first step computes, stated as a pivoted partial Cholesky
factorisation with restricted pivot choice.  The integrals are dense
per-irrep matrices ``V[g]`` (pairs of different irreps do not couple), so
every pair is its own shell and "computing a shell quartet" is reading
matrix entries.  The residual of irrep g after the vectors chosen so far is
``R_g = V_g - sum_p l_p l_p^T``; its diagonal is the quantity every choice
looks at.

* A pair is *active* while its residual diagonal is at least tau (the
  screening threshold); inactive pairs are zero in every later vector.
* The factorisation proceeds in rounds.  A round fixes D_max (the largest
  active residual diagonal over all irreps) and a candidate list: the at
  most Q_max active pairs with the largest diagonals among those at least
  sigma D_max (sigma: the span factor), ordered by diagonal, ties to the
  lower irrep and then the lower index.
* Within a round, pivots are taken from the candidate list only: each time
  the candidate with the largest current residual diagonal (the first in
  list order among equal ones), as long as that diagonal is at least the
  round's threshold tau_mic.  Eliminating pivot q of irrep g adds the vector
  ``l = R_g[:, q] / sqrt(R_g[q, q])`` (active rows only) and subtracts
  ``l l^T`` from R_g; the pivot's own diagonal is then exactly zero.
* After the round every pair whose diagonal fell below tau becomes inactive.
  The factorisation ends when no pair is active.

The paper does not spell out tau_mic; it is read as ``max(tau, sigma
D_max)`` with the D_max of the round (the span factor bounds both which
diagonals qualify and how far the qualified ones are decomposed).  Pinned in
``tests/test_oracle_cd.py`` by a hand-worked five-pair matrix whose pivot
order differs from greedy pivoting and from tau_mic = tau, by the Q_max = 1
reduction to textbook greedy pivoting, by the decomposition error bound, by
exact low rank and by invariance under reordering of the pairs.

Second step: for each irrep, K = the lower Cholesky factor of the metric
V[piv, piv] and L = K^-1 V[piv, :] (triangular solve), returned as the
matrix ``L[r, P]`` (pair-major, vector index fastest).

Library primitives: numpy outer products, numpy.linalg.cholesky and
scipy.linalg.solve_triangular.
"""
from __future__ import annotations

import numpy as np

__all__ = ["cd_basis", "cd_vectors", "cd_tau_mic"]


def cd_tau_mic(tau: float, sigma: float, dmax: float) -> float:
    """Threshold of the pivots taken within one round."""
    return max(tau, sigma * dmax)


def cd_basis(V: list, tau: float, sigma: float = 1e-2, qmax: int = 1000):
    """First step.  V: list of dense symmetric (n_g, n_g) matrices, one per
    irrep.  Returns (piv, diag): piv[g] = pivot indices of irrep g in the
    order they were chosen; diag[g] = the final residual diagonals of the
    pairs still active (np.nan for pairs that became inactive; their
    diagonal was then below tau)."""
    h = len(V)
    R = [np.array(v, dtype=np.float64) for v in V]           # residual matrices
    active = [np.diag(r) >= tau for r in R]
    for g in range(h):                                       # screened pairs: zero rows and columns
        R[g][~active[g], :] = 0.0
        R[g][:, ~active[g]] = 0.0
    piv = [[] for _ in range(h)]

    def diag(g, r):
        return R[g][r, r]

    while any(a.any() for a in active):
        dmax = max(float(np.diag(R[g])[active[g]].max()) for g in range(h) if active[g].any())
        ranked = sorted(((-diag(g, r), g, int(r)) for g in range(h) for r in np.flatnonzero(active[g])
                         if diag(g, r) >= sigma * dmax))
        cands = [(g, r) for _, g, r in ranked[:qmax]]
        thr = cd_tau_mic(tau, sigma, dmax)
        while True:
            g, q = max(cands, key=lambda c: diag(*c))       # max() keeps the first of equal values
            d = diag(g, q)
            if d < thr:
                break
            l = np.where(active[g], R[g][:, q], 0.0) / np.sqrt(d)
            R[g] -= np.outer(l, l)
            R[g][q, q] = 0.0
            piv[g].append(q)
        for g in range(h):
            drop = active[g] & (np.diag(R[g]) < tau)
            active[g] &= ~drop
            R[g][drop, :] = 0.0
            R[g][:, drop] = 0.0
    final = [np.where(active[g], np.diag(R[g]), np.nan) for g in range(h)]
    return [np.array(p, dtype=np.int64) for p in piv], final


def cd_vectors(V: list, piv: list) -> list:
    """Second step: L[g] of shape (n_g, npiv_g), L[g][r, P] = L^P_r."""
    from scipy.linalg import solve_triangular
    out = []
    for v, p in zip(V, piv):
        p = np.asarray(p, dtype=np.int64)
        if p.size == 0:
            out.append(np.zeros((v.shape[0], 0)))
            continue
        K = np.linalg.cholesky(v[np.ix_(p, p)])
        out.append(solve_triangular(K, v[p, :], lower=True).T.copy())
    return out
