"""vvvv block of the spin-adapted CCSD two-body density contracted with
Cholesky vectors, FP64, on the CPU (oracle, test infrastructure only).

Paper (arXiv 2512.21909):

* Appendix "CCSD two-body density matrices": the vvvv block is
  ``Gamma_AbCd = 1/2 P_+(ab,cd) V_AbCd`` with ``V_AbEf = sum_mn tau_Mn^Ef
  lambda_Ab^Mn`` (the timing section writes the same product with a tilde on
  tau; the caller supplies that amplitude, here ``X``), and ``P_+(pq) = 1 +
  P(pq)``, the symmetric permutation operator of the one-body appendix,
  applied to the pair (ab) <-> (cd).
* Section "CCSD density matrices": for an RHF reference only the
  spin-adapted density ``Gamma~_pqrs = 2 Gamma_PqRs - Gamma_PqSr`` is used.
* Section "CCSD analytic first derivatives", eq. for Gamma^P_pr:
  ``Gamma^P_pr = sum_qs Gamma~_pqrs L~^P_qs``; for the vvvv block p = a,
  q = b, r = c, s = d, so ``G^P_ac = sum_bd Gamma~_abcd L^P_bd`` -- the
  intermediate is contracted on the fly with the transformed Cholesky
  vectors and never stored (timing section, the O(O^2 V^4) term).

Closed-shell spatial orbitals: ``Y_mn^ab`` (lambda_Ab^Mn) and ``X_mn^cd``
(tau~_Mn^Cd) are amplitude tensors in the alpha-beta labelling of the paper
(first index of each pair alpha, second beta).  Written out::

    V_abcd   = sum_mn Y_mn^ab X_mn^cd
    Gamma    = (V_abcd + V_cdab) / 2
    Gamma~   = 2 Gamma_abcd - Gamma_abdc
    G^P_ac   = sum_bd Gamma~_abcd L^P_bd

Library primitives: einsum / matmul only; symmetry blocks of the
direct-product decomposition are the only blocking.

Pins (``tests/test_oracle_density.py``): pure-Python loops, a rank-one
closed form with distinct vectors on every index (so the exchange term
``Gamma_abdc`` is visible), the identity-vector special case written as
plain matrix products, the X <-> Y and a <-> c symmetries, scaling, the
blocked form against the scattered full tensors, and an independent
derivation from spin-orbital amplitudes and the spin-orbital density
(``Gamma~`` = half the spin sum of the spin-orbital vvvv density).
"""
from __future__ import annotations

import numpy as np

__all__ = ["vvvv_density_loops", "vvvv_density_full", "vvvv_density_blocks"]


def vvvv_density_loops(X: np.ndarray, Y: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Pure-Python loops for microscopic sizes.  X, Y: (o, o, v, v); L:
    (P, v, v).  Returns G: (P, v, v) with G[P, a, c]."""
    nP, v, _ = L.shape
    o = X.shape[0]

    def V(p, q, r, s):  # V_pqrs = sum_mn Y_mn^pq X_mn^rs
        acc = 0.0
        for m in range(o):
            for n in range(o):
                acc += Y[m, n, p, q] * X[m, n, r, s]
        return acc

    def Gam(p, q, r, s):  # 1/2 P_+(pq, rs) V_pqrs
        return 0.5 * (V(p, q, r, s) + V(r, s, p, q))

    G = np.zeros((nP, v, v))
    for P in range(nP):
        for a in range(v):
            for c in range(v):
                s = 0.0
                for b in range(v):
                    for d in range(v):
                        s += (2.0 * Gam(a, b, c, d) - Gam(a, b, d, c)) * L[P, b, d]
                G[P, a, c] = s
    return G


def vvvv_density_full(X: np.ndarray, Y: np.ndarray, L: np.ndarray) -> np.ndarray:
    """The definition on full tensors: V, the P_+ symmetrisation, the
    spin adaptation, then the contraction with L over (b, d)."""
    V = np.einsum("mnab,mncd->abcd", Y, X)
    Gam = 0.5 * (V + V.transpose(2, 3, 0, 1))
    Gt = 2.0 * Gam - Gam.transpose(0, 1, 3, 2)
    return np.einsum("abcd,Pbd->Pac", Gt, L)


def vvvv_density_blocks(sym: dict, X: dict, Y: dict, L: dict) -> dict:
    """Symmetry-blocked form.  Amplitude blocks are keyed (G, gi, ga) with
    shape (o_gi, o_gj, v_ga, v_gb); Cholesky and result blocks (gP, ga) with
    shape (v_ga, v_gc, N_gP), gc = ga ^ gP.  For the result block (gP, ga) and
    each irrep gb of b: gd = gb ^ gP, the pair irrep of (a, b) is G = ga ^ gb
    = gc ^ gd, and

        V[a, b, c, d] = sum_{gi} sum_{m in gi, n in gi^G} Y[m n a b] X[m n c d]

    is formed by one matmul per occupied block (with the (c, d, a, b) block
    for the P_+ symmetrisation); the exchange partner Gamma_abdc is the same
    construction for the block (a in ga, b in gb, d in gd, c in gc), whose
    amplitude blocks are (G, gi, gd) with the last two axes swapped.  The
    spin-adapted block is contracted with L[(gP, gb)][b, d, P] by a
    matmul."""
    h, no, nv, nc = sym["h"], sym["nocc"], sym["nvir"], sym["ncd"]

    def gamma(ga, gb, gc, gd, swap_cd):
        """Gamma_abcd for a in ga, b in gb and the pair (c, d) from the
        amplitude block of irreps (gc, gd); swap_cd reads it as (d, c)."""
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
        Gam = 0.5 * (V1 + V2.T)  # rows (a, b), columns (c, d) of irreps (gc, gd)
        Gam = Gam.reshape(nv[ga], nv[gb], nv[gc], nv[gd])
        return Gam.transpose(0, 1, 3, 2) if swap_cd else Gam

    out = {}
    for gP in range(h):
        for ga in range(h):
            gc = ga ^ gP
            out[(gP, ga)] = np.zeros((nv[ga], nv[gc], nc[gP]))
            if nc[gP] == 0:
                continue
            for gb in range(h):
                gd = gb ^ gP
                direct = gamma(ga, gb, gc, gd, False)       # Gamma_abcd, axes (a, b, c, d)
                exch = gamma(ga, gb, gd, gc, True)          # Gamma_abdc, read back as (a, b, c, d)
                Gt = (2.0 * direct - exch).transpose(0, 2, 1, 3)  # (a, c, b, d)
                Lb = L[(gP, gb)].reshape(nv[gb] * nv[gd], nc[gP])
                out[(gP, ga)] += (Gt.reshape(nv[ga] * nv[gc], nv[gb] * nv[gd]) @ Lb).reshape(
                    nv[ga], nv[gc], nc[gP])
    return out
