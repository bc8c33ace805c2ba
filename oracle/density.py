"""vvvv block of the CCSD two-body density contracted with Cholesky vectors,
FP64, on the CPU (oracle, test infrastructure only).

Paper (arXiv 2512.21909):

* Appendix "CCSD two-body density matrices": the vvvv block is
  ``Gamma_AbCd = 1/2 P_+(ab,cd) V_AbCd`` with ``V_AbEf = sum_mn tau_Mn^Ef
  lambda_Ab^Mn`` (the timing section writes the same product with a tilde on
  tau; the caller supplies that amplitude, here ``X``), and ``P_+(pq) = 1 +
  P(pq)``, the symmetric permutation operator of the one-body appendix,
  applied to the pair (ab) <-> (cd).
* Section "CCSD analytic first derivatives", eq. for Gamma^P_pr:
  ``Gamma^P_pr = sum_qs Gamma~_pqrs L~^P_qs``; for the vvvv block p = A,
  q = b, r = C, s = d, so ``G^P_ac = sum_bd Gamma_abcd L^P_bd`` -- the
  intermediate is contracted on the fly with the transformed Cholesky
  vectors and never stored (timing section, the O(O^2 V^4) term).

Closed-shell spatial orbitals: ``Y_mn^ab`` (lambda) and ``X_mn^cd`` (tau~)
are amplitude tensors with the pair symmetry ``Y_mn^ab = Y_nm^ba``.  Written
out::

    V_abcd   = sum_mn Y_mn^ab X_mn^cd
    Gamma    = (V_abcd + V_cdab) / 2
    G^P_ac   = sum_bd Gamma_abcd L^P_bd

Library primitives: einsum / matmul only; symmetry blocks of the
direct-product decomposition are the only blocking.
"""
from __future__ import annotations

import numpy as np

__all__ = ["vvvv_density_loops", "vvvv_density_full", "vvvv_density_blocks"]


def vvvv_density_loops(X: np.ndarray, Y: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Pure-Python loops for microscopic sizes.  X, Y: (o, o, v, v); L:
    (P, v, v).  Returns G: (P, v, v) with G[P, a, c]."""
    nP, v, _ = L.shape
    o = X.shape[0]
    G = np.zeros((nP, v, v))
    for P in range(nP):
        for a in range(v):
            for c in range(v):
                s = 0.0
                for b in range(v):
                    for d in range(v):
                        v1 = v2 = 0.0
                        for m in range(o):
                            for n in range(o):
                                v1 += Y[m, n, a, b] * X[m, n, c, d]
                                v2 += Y[m, n, c, d] * X[m, n, a, b]
                        s += 0.5 * (v1 + v2) * L[P, b, d]
                G[P, a, c] = s
    return G


def vvvv_density_full(X: np.ndarray, Y: np.ndarray, L: np.ndarray) -> np.ndarray:
    """The definition on full tensors: V, the P_+ symmetrisation, then the
    contraction with L over (b, d)."""
    V = np.einsum("mnab,mncd->abcd", Y, X)
    Gam = 0.5 * (V + V.transpose(2, 3, 0, 1))
    return np.einsum("abcd,Pbd->Pac", Gam, L)


def vvvv_density_blocks(sym: dict, X: dict, Y: dict, L: dict) -> dict:
    """Symmetry-blocked form.  Amplitude blocks are keyed (G, gi, ga) with
    shape (o_gi, o_gj, v_ga, v_gb); Cholesky and result blocks (gP, ga) with
    shape (v_ga, v_gc, N_gP), gc = ga ^ gP.  For the result block (gP, ga) and
    each irrep gb of b: gd = gb ^ gP, the pair irrep of (a, b) is G = ga ^ gb
    = gc ^ gd, and

        V[a, b, c, d] = sum_{gi} sum_{m in gi, n in gi^G} Y[m n a b] X[m n c d]

    is formed by one matmul per occupied block, symmetrised with the (c, d,
    a, b) block, and contracted with L[(gP, gb)][b, d, P] by a matmul."""
    h, no, nv, nc = sym["h"], sym["nocc"], sym["nvir"], sym["ncd"]
    out = {}
    for gP in range(h):
        for ga in range(h):
            gc = ga ^ gP
            out[(gP, ga)] = np.zeros((nv[ga], nv[gc], nc[gP]))
            if nc[gP] == 0:
                continue
            for gb in range(h):
                gd = gb ^ gP
                G = ga ^ gb
                V1 = np.zeros((nv[ga] * nv[gb], nv[gc] * nv[gd]))  # V_abcd
                V2 = np.zeros((nv[gc] * nv[gd], nv[ga] * nv[gb]))  # V_cdab
                for gi in range(h):
                    gj = gi ^ G
                    nmn = no[gi] * no[gj]
                    y_ab = Y[(G, gi, ga)].reshape(nmn, nv[ga] * nv[gb])
                    x_ab = X[(G, gi, ga)].reshape(nmn, nv[ga] * nv[gb])
                    y_cd = Y[(G, gi, gc)].reshape(nmn, nv[gc] * nv[gd])
                    x_cd = X[(G, gi, gc)].reshape(nmn, nv[gc] * nv[gd])
                    V1 += y_ab.T @ x_cd
                    V2 += y_cd.T @ x_ab
                Gam = 0.5 * (V1 + V2.T)  # rows (a, b), columns (c, d)
                Gam = Gam.reshape(nv[ga], nv[gb], nv[gc], nv[gd]).transpose(0, 2, 1, 3)
                Lb = L[(gP, gb)].reshape(nv[gb] * nv[gd], nc[gP])
                out[(gP, ga)] += (Gam.reshape(nv[ga] * nv[gc], nv[gb] * nv[gd]) @ Lb).reshape(
                    nv[ga], nv[gc], nc[gP])
    return out
