"""Symmetry-adapted two-step Cholesky decomposition of a symmetric positive
semidefinite "two-electron integral" matrix, FP64, on the CPU (oracle, test
infrastructure only).

Paper (arXiv 2512.21909), section "Symmetry-adapted two-step CD algorithm",
Algorithm 1 (first step: the Cholesky basis) and the equation for the
vectors of the second step in the section on CD/DF integrals
(``L^P_rs = sum_R K^-1_PR (R|rs)`` with ``K K^T`` the metric ``(Q|R)`` over
the basis).  Here the integrals are given as dense per-irrep matrices
``V[g]`` (rows and columns: the basis-function pairs of irrep g; pairs of
different irreps do not couple, so the matrix is block diagonal), so
"computing a shell quartet" is reading matrix entries and every pair is its
own shell.

First step, in the paper's order and notation:

* P = pairs with Diag(r) = (r|r) >= tau, D = their diagonals;
* while P is not empty:
  - D_max = max over P; the qualified list Q = the (at most Q_max) largest
    members of P with Diag >= sigma D_max (ties: lower irrep, then lower
    index first);
  - residual columns M~_rq = (r|q) - sum over the vectors L(G_q) of
    L_r^p L_q^p for r in P of the irrep of q;
  - micro iterations: while the largest Diag over Q is >= tau_mic, take it
    as pivot q; for every r in P of the irrep of q,
    L_r^q = (M~_rq - sum over this iteration's vectors of L_r^p L_q^p) /
    sqrt(Diag(q)) and Diag(r) -= (L_r^q)^2; the vector joins L_mic(G_q);
  - L(G) gains L_mic(G); pairs with Diag < tau leave P (their entries of
    later vectors are zero).

``tau_mic`` is not spelled out in the paper; it is read as
``max(tau, sigma D_max)`` with the D_max of the current macro iteration
(the span factor bounds both which diagonals qualify and how far the
qualified ones are decomposed).  The pivot of a micro iteration is the
first maximum in Q order.  After a pivot its own diagonal is set to zero.

Second step: for each irrep, K = the lower Cholesky factor of the metric
V[piv, piv] and L = K^-1 V[piv, :] (triangular solve), returned as the
matrix ``L[r, P]`` (pair-major, vector index fastest).

Library primitives: numpy matmul, numpy.linalg.cholesky and
scipy.linalg.solve_triangular.
"""
from __future__ import annotations

import numpy as np

__all__ = ["cd_basis", "cd_vectors", "cd_tau_mic"]


def cd_tau_mic(tau: float, sigma: float, dmax: float) -> float:
    return max(tau, sigma * dmax)


def cd_basis(V: list, tau: float, sigma: float = 1e-2, qmax: int = 1000):
    """First step.  V: list of dense symmetric (n_g, n_g) matrices, one per
    irrep.  Returns (piv, diag): piv[g] = pivot indices of irrep g in the
    order they were chosen; diag[g] = the final diagonals of the pairs still
    in P (np.nan for pairs that left P, the diagonal at leaving time is
    below tau)."""
    h = len(V)
    D = [np.array(np.diag(v), dtype=np.float64) for v in V]
    inP = [d >= tau for d in D]
    vecs = [np.zeros((v.shape[0], 0)) for v in V]      # L(G): rows r, one column per vector
    piv = [[] for _ in range(h)]
    while any(m.any() for m in inP):
        dmax = max(float(D[g][inP[g]].max()) for g in range(h) if inP[g].any())
        cand = [(-D[g][r], g, r) for g in range(h) for r in np.nonzero(inP[g])[0]
                if D[g][r] >= sigma * dmax]
        cand.sort()
        Q = [(g, int(r)) for _, g, r in cand[:qmax]]
        # residual columns over P for every qualified pair
        res = {}
        for g, q in Q:
            col = V[g][:, q] - vecs[g] @ vecs[g][q, :]
            col[~inP[g]] = 0.0
            res[(g, q)] = col
        tmic = cd_tau_mic(tau, sigma, dmax)
        mic = [np.zeros((V[g].shape[0], 0)) for g in range(h)]
        while True:
            best, bq = -np.inf, None
            for g, q in Q:               # first maximum in Q order
                if D[g][q] > best:
                    best, bq = D[g][q], (g, q)
            if bq is None or best < tmic:
                break
            g, q = bq
            m = mic[g]
            col = (res[(g, q)] - m @ m[q, :]) / np.sqrt(D[g][q])
            col[~inP[g]] = 0.0
            D[g] = D[g] - col * col
            D[g][q] = 0.0
            mic[g] = np.concatenate([m, col[:, None]], axis=1)
            piv[g].append(q)
        for g in range(h):
            vecs[g] = np.concatenate([vecs[g], mic[g]], axis=1)
            leave = inP[g] & (D[g] < tau)
            inP[g] = inP[g] & ~leave
    diag = [np.where(inP[g], D[g], np.nan) for g in range(h)]
    return [np.array(p, dtype=np.int64) for p in piv], diag


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
