"""O(O^3 V^3) contraction M_bi^dc = sum_mn lambda_bi^mn tau~_mn^dc, FP64, on
the CPU (oracle, test infrastructure only).

Paper (arXiv 2512.21909), the closing paragraph of the section on the
spin-adapted I_pq multipliers: the symmetric-antisymmetric algorithm is used
for every O(O^2 V^4) contraction, and a "partial" variant of it for the
O(O^3 V^3) ones, halving their cost; the example given is
``M_bi^dc = sum_mn lambda_Bi^Mn tau~_mn^dc``, where only the +/- combinations
of lambda over the pair ``M >= n`` can be formed, because lambda is not square
in its (B, i) pair.

``M`` has a plain definition, so the oracle writes that definition out
(loops, the full-tensor einsum, the symmetry-blocked sum).  The partial
algorithm is written out as well, in its own steps, as a pin of the identity
the GPU path relies on: with tau~ pair-symmetric (tau~_mn^dc = tau~_nm^cd)

    lam+_bi^(m>=n) = lam_bi^mn + lam_bi^nm   (m > n),   lam_bi^mm   (m = n)
    lam-_bi^(m>n)  = lam_bi^mn - lam_bi^nm
    tau+_(m>=n)^dc = tau~_mn^dc + tau~_mn^cd  (symmetric in d, c)
    tau-_(m>n)^dc  = tau~_mn^dc - tau~_mn^cd  (antisymmetric in d, c)
    S^dc = sum_{m>=n} lam+ tau+,   A^dc = sum_{m>n} lam- tau-
    M_bi^dc = (S^dc + A^dc) / 2,   M_bi^cd = (S^dc - A^dc) / 2

so only the d >= c columns of S and A are needed.

Blocks: ``lam[(G, gb, gm)]`` has shape (v_gb, o_gi, o_gm, o_gn) with
gi = gb ^ G, gn = gm ^ G; ``tau[(G, gm, gd)]`` (o_gm, o_gn, v_gd, v_gc);
the result ``M[(G, gb, gd)]`` (v_gb, o_gi, v_gd, v_gc).  Library primitives:
einsum / matmul only.
"""
from __future__ import annotations

import numpy as np

__all__ = ["partial_loops", "partial_full", "partial_blocks", "partial_pm_steps"]


def partial_loops(lam: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Pure-Python loops for microscopic sizes.  lam: (v, o, o, o) as
    [b, i, m, n]; tau: (o, o, v, v) as [m, n, d, c].  Returns M[b, i, d, c]."""
    v, o = lam.shape[0], lam.shape[1]
    M = np.zeros((v, o, v, v))
    for b in range(v):
        for i in range(o):
            for d in range(v):
                for c in range(v):
                    s = 0.0
                    for m in range(o):
                        for n in range(o):
                            s += lam[b, i, m, n] * tau[m, n, d, c]
                    M[b, i, d, c] = s
    return M


def partial_full(lam: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """The definition on full tensors."""
    return np.einsum("bimn,mndc->bidc", lam, tau)


def partial_blocks(sym: dict, lam: dict, tau: dict) -> dict:
    """Symmetry-blocked definition: for each pair irrep G and irreps gb (of b)
    and gd (of d), M[(G, gb, gd)] = sum over gm of the (b i, m n) block of lam
    times the (m n, d c) block of tau, one matmul per gm."""
    h, no, nv = sym["h"], sym["nocc"], sym["nvir"]
    out = {}
    for G in range(h):
        for gb in range(h):
            gi = gb ^ G
            nrow = nv[gb] * no[gi]
            for gd in range(h):
                gc = gd ^ G
                ncol = nv[gd] * nv[gc]
                acc = np.zeros((nrow, ncol))
                for gm in range(h):
                    gn = gm ^ G
                    k = no[gm] * no[gn]
                    acc += lam[(G, gb, gm)].reshape(nrow, k) @ tau[(G, gm, gd)].reshape(k, ncol)
                out[(G, gb, gd)] = acc.reshape(nv[gb], no[gi], nv[gd], nv[gc])
    return out


def partial_pm_steps(lam: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """The partial symmetric-antisymmetric algorithm on full tensors, step by
    step (see the module docstring).  Equals the definition when tau is pair
    symmetric; it is a pin of that identity, not a second reference."""
    v, o = lam.shape[0], lam.shape[1]
    ge = [(m, n) for m in range(o) for n in range(m + 1)]          # m >= n
    gt = [(m, n) for m in range(o) for n in range(m)]              # m > n
    lp = np.stack([lam[:, :, m, n] + (lam[:, :, n, m] if m != n else 0.0) for m, n in ge], axis=-1)
    lm = np.stack([lam[:, :, m, n] - lam[:, :, n, m] for m, n in gt], axis=-1) if gt else np.zeros((v, o, 0))
    tp = np.stack([tau[m, n] + tau[m, n].T for m, n in ge], axis=0)
    tm = np.stack([tau[m, n] - tau[m, n].T for m, n in gt], axis=0) if gt else np.zeros((0, v, v))
    S = np.einsum("bik,kdc->bidc", lp, tp)
    A = np.einsum("bik,kdc->bidc", lm, tm)
    M = np.empty((v, o, v, v))
    for d in range(v):
        for c in range(d + 1):
            M[:, :, d, c] = 0.5 * (S[:, :, d, c] + A[:, :, d, c])
            M[:, :, c, d] = 0.5 * (S[:, :, d, c] - A[:, :, d, c])
    return M
