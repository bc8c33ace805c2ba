"""Particle-particle ladder (PPL) terms, FP64, on the CPU (oracle).

Paper: "CCSD analytic gradients using Cholesky decomposition ... and Abelian
point-group symmetry" (arXiv 2512.21909).

* T2 ladder (section "Stationarity ... Lambda equations": the amplitude-equation
  PPL term handled with the same strategy; the term is
  ``R_ij^ab = sum_cd tau_ij^cd (ac|bd)``) with the Cholesky-decomposed
  integrals of eq. (1): ``(ac|bd) = sum_P B^P_ac B^P_bd``.
* Lambda ladder (eq. for Z in the same section):
  ``Z_ij^ab = sum_ef lambda_ij^ef W_efab`` with ``W`` from Appendix A
  (``W_AbEf = sum_P [(L^P_AE - t^P_AE) L^P_bf - sum_m t_m^b L^P_AE L^P_mf]``,
  relabelled ``A,b,E,f -> E,f,A,b``) and ``t^P_ab = sum_m t_m^a L^P_bm``
  (Appendix A).
* Symmetric-antisymmetric split (same section, eqs. for S, A and the +/-
  combinations), written out on full tensors.
* Direct-product decomposition (symmetry section): blocks whose irrep product
  is not totally symmetric are zero and are skipped.

Everything is plain FP64 NumPy: einsum / matmul as the only library
primitives, no blocking beyond the symmetry blocks, no fusion.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "t2_ladder_loops", "t2_ladder_full", "t2_ladder_blocks", "t1_dressing_full",
    "lambda_w_full", "lambda_ladder_full", "lambda_ladder_blocks",
    "t2_ladder_symantisym_full", "pair_energies_full", "denominator_update_full",
    "pair_energies_blocks", "denominator_update_blocks",
    "element_t2", "element_lambda", "rel_errors",
]


# --------------------------------------------------------------------------
# T2 ladder
# --------------------------------------------------------------------------
def t2_ladder_loops(B: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Pure-Python loops for microscopic sizes: R_ij^ab = sum_cd tau_ij^cd
    sum_P B^P_ac B^P_bd.  B: (P, v, v), tau: (o, o, v, v)."""
    nP, v, _ = B.shape
    o = tau.shape[0]
    R = np.zeros((o, o, v, v))
    for i in range(o):
        for j in range(o):
            for a in range(v):
                for b in range(v):
                    s = 0.0
                    for c in range(v):
                        for d in range(v):
                            w = 0.0
                            for P in range(nP):
                                w += B[P, a, c] * B[P, b, d]
                            s += tau[i, j, c, d] * w
                    R[i, j, a, b] = s
    return R


def t2_ladder_full(B: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Brute force with the explicit four-index integrals (ac|bd)."""
    W = np.einsum("Pac,Pbd->acbd", B, B)
    return np.einsum("ijcd,acbd->ijab", tau, W)


def t2_ladder_blocks(sym: dict, B: dict, tau: dict) -> dict:
    """Symmetry-blocked T2 ladder.  For pair irrep G and the irreps of a and
    P, the allowed irreps are gb = ga^G, gc = ga^gP, gd = gb^gP; each block of
    (ac|bd) is built from the two Cholesky blocks and contracted by matmul."""
    h, no, nv, nc = sym["h"], sym["nocc"], sym["nvir"], sym["ncd"]
    R = {}
    for G in range(h):
        for gi in range(h):
            gj = gi ^ G
            for ga in range(h):
                R[(G, gi, ga)] = np.zeros((no[gi], no[gj], nv[ga], nv[ga ^ G]))
    for G in range(h):
        for ga in range(h):
            gb = ga ^ G
            for gP in range(h):
                if nc[gP] == 0:
                    continue
                gc, gd = ga ^ gP, gb ^ gP
                # (ac|bd) for this block: (v_a, v_c, v_b, v_d), a matmul over P
                Ba, Bb = B[(gP, ga)], B[(gP, gb)]
                Wb = (Ba.reshape(-1, nc[gP]) @ Bb.reshape(-1, nc[gP]).T).reshape(
                    nv[ga], nv[gc], nv[gb], nv[gd])
                Wm = Wb.transpose(1, 3, 0, 2).reshape(nv[gc] * nv[gd], nv[ga] * nv[gb])
                for gi in range(h):
                    gj = gi ^ G
                    t = tau[(G, gi, gc)].reshape(no[gi] * no[gj], nv[gc] * nv[gd])
                    R[(G, gi, ga)] += (t @ Wm).reshape(no[gi], no[gj], nv[ga], nv[gb])
    return R


def t2_ladder_symantisym_full(B: np.ndarray, tau: np.ndarray, restricted: bool = False):
    """The symmetric-antisymmetric algorithm written out on full tensors.

    ``+/-x_cd = (x_cd +/- x_dc)/2`` for tau (over its virtual pair) and for
    W_cdab = (ac|bd) (over its first pair);  S = sum +tau +W, A = sum -tau -W,
    R = S + A.  With ``restricted`` the sums run over c >= d only, with weight
    (2 - delta_cd) for S and 2 for A (c > d), as the stored halves allow.
    Returns (R, S, A)."""
    W = np.einsum("Pac,Pbd->cdab", B, B)  # W_cdab = (ac|bd)
    tp = 0.5 * (tau + tau.transpose(0, 1, 3, 2))
    tm = 0.5 * (tau - tau.transpose(0, 1, 3, 2))
    Wp = 0.5 * (W + W.transpose(1, 0, 2, 3))
    Wm = 0.5 * (W - W.transpose(1, 0, 2, 3))
    if not restricted:
        S = np.einsum("ijcd,cdab->ijab", tp, Wp)
        A = np.einsum("ijcd,cdab->ijab", tm, Wm)
    else:
        v = tau.shape[2]
        c_idx, d_idx = np.tril_indices(v)  # c >= d
        wS = np.where(c_idx == d_idx, 1.0, 2.0)
        wA = np.where(c_idx == d_idx, 0.0, 2.0)
        S = np.einsum("ijk,kab->ijab", tp[:, :, c_idx, d_idx] * wS, Wp[c_idx, d_idx])
        A = np.einsum("ijk,kab->ijab", tm[:, :, c_idx, d_idx] * wA, Wm[c_idx, d_idx])
    return S + A, S, A


# --------------------------------------------------------------------------
# Lambda ladder
# --------------------------------------------------------------------------
def t1_dressing_full(Bvo: np.ndarray, t1: np.ndarray) -> np.ndarray:
    """Appendix A: t^P_ab = sum_m t_m^a L^P_bm.  Bvo: (P, v, o) = L^P_bm,
    t1: (o, v) = t_m^a.  Returns (P, v, v) indexed [P, a, b]."""
    return np.einsum("ma,Pbm->Pab", t1, Bvo)


def lambda_w_full(B: np.ndarray, Bvo: np.ndarray, t1: np.ndarray) -> np.ndarray:
    """W_efab literally from Appendix A, relabelled from W_AbEf:
    W_efab = sum_P [(L^P_ea - t^P_ea) L^P_fb - sum_m t_m^f L^P_ea L^P_mb],
    with L^P_mb = L^P_bm (Cholesky vectors of a symmetric matrix)."""
    tP = t1_dressing_full(Bvo, t1)
    first = np.einsum("Pea,Pfb->efab", B - tP, B)
    second = np.einsum("mf,Pea,Pbm->efab", t1, B, Bvo)
    return first - second


def lambda_ladder_full(B, Bvo, t1, lam) -> np.ndarray:
    """Z_ij^ab = sum_ef lambda_ij^ef W_efab (brute force)."""
    return np.einsum("ijef,efab->ijab", lam, lambda_w_full(B, Bvo, t1))


def lambda_ladder_blocks(sym: dict, B: dict, Bvo: dict, t1: list, lam: dict) -> dict:
    """Symmetry-blocked Lambda ladder: for pair irrep G and irreps (ga, gP),
    ge = ga^gP, gf = gb^gP; W_efab = sum_P [(B_ea - t_ea) B_fb - B_ea t_fb]
    with t^P_xy = sum_m t_m^x L^P_ym (the same Appendix-A terms, per block)."""
    h, no, nv, nc = sym["h"], sym["nocc"], sym["nvir"], sym["ncd"]

    def tP(gP, gx):
        # t^P_xy for x in irrep gx, y in gy = gx^gP: sum_m t_m^x L^P_ym, m in gx
        gy = gx ^ gP
        return np.einsum("mx,ymP->xyP", t1[gx], Bvo[(gP, gy)])

    Z = {}
    for G in range(h):
        for gi in range(h):
            for ga in range(h):
                Z[(G, gi, ga)] = np.zeros((no[gi], no[gi ^ G], nv[ga], nv[ga ^ G]))
    for G in range(h):
        for ga in range(h):
            gb = ga ^ G
            for gP in range(h):
                if nc[gP] == 0:
                    continue
                ge, gf = ga ^ gP, gb ^ gP
                Bea = B[(gP, ge)]          # (e, a, P)
                Bfb = B[(gP, gf)]          # (f, b, P)
                n = nc[gP]
                # W_efab = sum_P (B_ea - t_ea) B_fb - B_ea t_fb, each term a matmul over P
                m1 = (Bea - tP(gP, ge)).reshape(-1, n) @ Bfb.reshape(-1, n).T      # (ea, fb)
                m2 = Bea.reshape(-1, n) @ tP(gP, gf).reshape(-1, n).T              # (ea, fb)
                Wb = (m1 - m2).reshape(nv[ge], nv[ga], nv[gf], nv[gb]).transpose(0, 2, 1, 3)
                Wm = Wb.reshape(nv[ge] * nv[gf], nv[ga] * nv[gb])
                for gi in range(h):
                    gj = gi ^ G
                    lm = lam[(G, gi, ge)].reshape(no[gi] * no[gj], nv[ge] * nv[gf])
                    Z[(G, gi, ga)] += (lm @ Wm).reshape(no[gi], no[gj], nv[ga], nv[gb])
    return Z


# --------------------------------------------------------------------------
# Epilogue quantities
# --------------------------------------------------------------------------
def pair_energies_full(X: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Closed-shell pair functional e_ij = sum_ab (2 X_ij^ab - X_ij^ba) R_ij^ab."""
    return np.einsum("ijab,ijab->ij", 2.0 * X - X.transpose(0, 1, 3, 2), R)


def denominator_update_full(R: np.ndarray, eps_occ: np.ndarray, eps_vir: np.ndarray) -> np.ndarray:
    """R / D with D_ij^ab = e_i + e_j - e_a - e_b (the D of the doubles
    Lambda equation)."""
    D = (eps_occ[:, None, None, None] + eps_occ[None, :, None, None]
         - eps_vir[None, None, :, None] - eps_vir[None, None, None, :])
    return R / D


def pair_energies_blocks(sym: dict, X: dict, R: dict) -> np.ndarray:
    """The pair functional of ``pair_energies_full`` on symmetry blocks
    (no full tensor is formed): for the block (G, gi, ga) the exchange
    partner X_ij^ba sits in block (G, gi, gb), gb = ga^G, with its last two
    axes swapped.  Returns the (o_tot, o_tot) matrix e[I, J] with global
    occupied indices."""
    h, no = sym["h"], sym["nocc"]
    off = np.concatenate([[0], np.cumsum(no)]).astype(int)
    e = np.zeros((off[-1], off[-1]))
    for G in range(h):
        for gi in range(h):
            gj = gi ^ G
            for ga in range(h):
                gb = ga ^ G
                r = R[(G, gi, ga)]
                if r.size == 0:
                    continue
                xt = 2.0 * X[(G, gi, ga)] - X[(G, gi, gb)].transpose(0, 1, 3, 2)
                e[off[gi]:off[gi + 1], off[gj]:off[gj + 1]] += np.einsum("ijab,ijab->ij", xt, r)
    return e


def denominator_update_blocks(sym: dict, R: dict, eps_occ: list, eps_vir: list) -> dict:
    """``denominator_update_full`` on symmetry blocks: R / (e_i + e_j - e_a -
    e_b) with eps_occ[g], eps_vir[g] the orbital energies of irrep g."""
    h = sym["h"]
    out = {}
    for (G, gi, ga), r in R.items():
        gj, gb = gi ^ G, ga ^ G
        D = (eps_occ[gi][:, None, None, None] + eps_occ[gj][None, :, None, None]
             - eps_vir[ga][None, None, :, None] - eps_vir[gb][None, None, None, :])
        out[(G, gi, ga)] = r / D if r.size else r.copy()
    assert len(out) == h ** 3
    return out


# --------------------------------------------------------------------------
# Single elements (for sampled checks at full size)
# --------------------------------------------------------------------------
def _locate(sym, g_list, idx):
    """(irrep, local index) of a global orbital index."""
    off = 0
    for g, n in enumerate(g_list):
        if idx < off + n:
            return g, idx - off
        off += n
    raise IndexError(idx)


def element_t2(sym: dict, B: dict, tau: dict, i: int, j: int, a: int, b: int) -> float:
    """One element R_ij^ab (global orbital indices) straight from the
    definition, summing only symmetry-allowed blocks."""
    h, nc = sym["h"], sym["ncd"]
    gi, il = _locate(sym, sym["nocc"], i)
    gj, jl = _locate(sym, sym["nocc"], j)
    ga, al = _locate(sym, sym["nvir"], a)
    gb, bl = _locate(sym, sym["nvir"], b)
    G = gi ^ gj
    if ga ^ gb != G:
        return 0.0
    s = 0.0
    for gP in range(h):
        if nc[gP] == 0:
            continue
        gc = ga ^ gP
        Wab = B[(gP, ga)][al] @ B[(gP, gb)][bl].T    # (c, d)
        s += float(np.sum(tau[(G, gi, gc)][il, jl] * Wab))
    return s


def element_lambda(sym: dict, B: dict, Bvo: dict, t1: list, lam: dict, i, j, a, b) -> float:
    """One element Z_ij^ab from the Appendix-A form of W."""
    h, nc = sym["h"], sym["ncd"]
    gi, il = _locate(sym, sym["nocc"], i)
    gj, jl = _locate(sym, sym["nocc"], j)
    ga, al = _locate(sym, sym["nvir"], a)
    gb, bl = _locate(sym, sym["nvir"], b)
    G = gi ^ gj
    if ga ^ gb != G:
        return 0.0
    s = 0.0
    for gP in range(h):
        if nc[gP] == 0:
            continue
        ge, gf = ga ^ gP, gb ^ gP
        Bea = B[(gP, ge)][:, al, :]                          # (e, P)
        Bfb = B[(gP, gf)][:, bl, :]                          # (f, P)
        tea = t1[ge].T @ Bvo[(gP, ga)][al]                   # t^P_ea: (e, P)
        tfb = t1[gf].T @ Bvo[(gP, gb)][bl]                   # t^P_fb: (f, P)
        Wef = (Bea - tea) @ Bfb.T - Bea @ tfb.T
        s += float(np.sum(lam[(G, gi, ge)][il, jl] * Wef))
    return s


# --------------------------------------------------------------------------
# Error metrics
# --------------------------------------------------------------------------
def rel_errors(got: dict, ref: dict):
    """Normwise relative errors over all blocks: (max|d|/max|ref|, ||d||_F/||ref||_F)."""
    mx_d = mx_r = 0.0
    s_d = s_r = 0.0
    for k, r in ref.items():
        g = got[k]
        if r.size == 0:
            continue
        d = np.asarray(g, dtype=np.float64) - r
        mx_d = max(mx_d, float(np.max(np.abs(d))))
        mx_r = max(mx_r, float(np.max(np.abs(r))))
        s_d += float(np.sum(d * d))
        s_r += float(np.sum(r * r))
    if mx_r == 0.0:
        return (0.0 if mx_d == 0.0 else np.inf), (0.0 if s_d == 0.0 else np.inf)
    return mx_d / mx_r, np.sqrt(s_d) / np.sqrt(s_r)
