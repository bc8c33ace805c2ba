"""Seeded synthetic inputs for the Cholesky-decomposed CCSD particle-particle
ladder, in per-symmetry-block form.

This module only draws numbers. It contains none of the method's arithmetic
(no contraction, no packing, no offsets): both the CPU oracle and the HIP path
take these blocks and lay them out their own way.

Conventions (Abelian groups D2h and subgroups, irreps 0..h-1, product = XOR):

* ``sym``: dict ``h, nocc[h], nvir[h], ncd[h]`` (orbitals and Cholesky vectors
  per irrep).
* ``B[(gP, ga)]``: array ``(v_ga, v_gc, N_gP)`` holding ``B^P_ac`` with
  ``gc = ga ^ gP`` (the Cholesky vectors of the vv block, selection rule of the
  direct-product decomposition).
* ``Bvo[(gP, ga)]``: array ``(v_ga, o_gm, N_gP)`` holding ``L^P_am`` with
  ``gm = ga ^ gP`` (vo block of the same vectors, used by the T1 dressing).
* ``t1[g]``: array ``(o_g, v_g)`` holding ``t_m^e`` (only ``gm == ge``).
* amplitudes ``tau[(G, gi, ga)]`` / ``lam[...]``: array ``(o_gi, o_gj, v_ga, v_gb)``
  with ``gj = gi ^ G``, ``gb = ga ^ G`` (pair irrep ``G``).
* ``eps_occ[g]``, ``eps_vir[g]``: orbital energies per irrep.
* ``lam_vo[(G, gb, gm)]``: array ``(v_gb, o_gi, o_gm, o_gn)`` with
  ``gi = gb ^ G``, ``gn = gm ^ G``, holding a tensor ``lambda_bi^mn`` with one
  virtual and three occupied indices (pair irrep ``G`` of (b,i) and of (m,n)),
  the left operand of the O(O^3 V^3) contraction ``M_bi^dc``.

Value recipe (synthetic stand-ins for molecular data, none of which is
available): ``eps_occ ~ U[-2,-0.5]``, ``eps_vir ~ U[0.2,3]``;
``B^P_ac = N(0,1) exp(-p/60)`` with ``p`` the 0-based index inside the irrep's
vector list, symmetrised ``(G + G^T)/sqrt(2)`` off the diagonal;
``t2 = N(0,1) * 0.01 / (e_a + e_b - e_i - e_j)`` averaged with its pair
transpose so that ``t2_ij^ab = t2_ji^ba``; ``t1 ~ N(0, (1e-3)^2)``;
``tau = t2 + t1 t1``; ``lambda`` drawn like ``t2``; ``Bvo`` like ``B``;
``lam_vo ~ N(0, (1e-3)^2)`` (no permutational symmetry).

Synthetic "two-electron integral" matrices for the Cholesky decomposition
(``make_cd_matrices``): per irrep g a dense symmetric positive semidefinite
``V = W Z S S Z^T W`` over n_g basis-function pairs, ``Z ~ N(0,1)``
(n_g x n_g), ``S = diag(exp(-k / kappa))`` (an exponentially decaying
spectrum, as for Coulomb integrals) and ``W = diag(exp(-u_r))``,
``u_r ~ U[0, 9]`` (pair magnitudes spanning several orders, as Schwarz
bounds do).
Every block draws from ``numpy.random.default_rng([seed, tensor_id, ...])`` so
the values do not depend on generation order.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

__all__ = [
    "SPLIT_D2H", "largest_remainder_split", "sym_c1_small", "sym_d2h_medium",
    "sym_d2h_large", "sym_hbc_shape", "sym_serving_large", "sym_custom", "dirichlet_sym",
    "batch_syms", "make_eps", "make_B", "make_Bvo", "make_t1", "make_t2",
    "make_tau", "make_lambda", "make_problem", "make_density_problem", "make_lam_vo",
    "make_partial_problem", "make_cd_matrices", "irrep_pairs",
    "serving_stream", "TENSOR_IDS",
]

# Proportions of the 8-irrep split used by the large configurations.
SPLIT_D2H = (Fraction(20, 100), Fraction(11, 100), Fraction(15, 100), Fraction(10, 100),
             Fraction(16, 100), Fraction(9, 100), Fraction(11, 100), Fraction(8, 100))

TENSOR_IDS = {"eps_occ": 1, "eps_vir": 2, "B": 3, "Bvo": 4, "t1": 5, "t2": 6,
              "lam": 7, "Bsym": 8, "lam_vo": 9, "cd": 10}


def largest_remainder_split(total: int, weights) -> list[int]:
    """Split ``total`` by ``weights`` with exact rational largest remainder;
    ties go to the lowest index."""
    w = [Fraction(x) for x in weights]
    s = sum(w)
    if total == 0 or s == 0:
        return [0] * len(w)
    quotas = [Fraction(total) * x / s for x in w]
    base = [int(q) for q in quotas]  # floor for non-negative
    rem = total - sum(base)
    order = sorted(range(len(w)), key=lambda k: (-(quotas[k] - base[k]), k))
    for k in order[:rem]:
        base[k] += 1
    return base


def sym_custom(nocc, nvir, ncd) -> dict:
    nocc, nvir, ncd = list(map(int, nocc)), list(map(int, nvir)), list(map(int, ncd))
    h = len(nocc)
    if h not in (1, 2, 4, 8) or len(nvir) != h or len(ncd) != h:
        raise ValueError("irrep count must be 1, 2, 4 or 8 with matching lists")
    return {"h": h, "nocc": nocc, "nvir": nvir, "ncd": ncd}


def sym_c1_small() -> dict:
    """C1, o=8, v=40, 300 Cholesky vectors (the small plain FP64 case)."""
    return sym_custom([8], [40], [300])


def sym_d2h_medium(cd_reading: str = "A") -> dict:
    """8 irreps, o=20, v=200, 1500 Cholesky vectors.  Reading A puts every
    vector in the totally symmetric irrep; reading B splits them evenly."""
    nocc = [4, 2, 3, 2, 3, 2, 2, 2]
    nvir = [40, 22, 30, 20, 32, 18, 22, 16]
    if cd_reading == "A":
        ncd = [1500, 0, 0, 0, 0, 0, 0, 0]
    else:
        ncd = largest_remainder_split(1500, [1] * 8)
    return sym_custom(nocc, nvir, ncd)


def sym_d2h_large() -> dict:
    """8 irreps, o=40, v=400, 3000 Cholesky vectors split evenly."""
    return sym_custom(largest_remainder_split(40, SPLIT_D2H),
                      largest_remainder_split(400, SPLIT_D2H),
                      largest_remainder_split(3000, [1] * 8))


def sym_hbc_shape() -> dict:
    """The size of the paper's largest D2h test molecule (135 occupied, 543
    virtual orbitals, 3710 Cholesky vectors), split over the 8 irreps like
    the o=40 system (vectors evenly)."""
    return sym_custom(largest_remainder_split(135, SPLIT_D2H),
                      largest_remainder_split(543, SPLIT_D2H),
                      largest_remainder_split(3710, [1] * 8))


def sym_serving_large() -> dict:
    """The large request of the serving mix: o=30, v=300, 2500 vectors."""
    return sym_custom(largest_remainder_split(30, SPLIT_D2H),
                      largest_remainder_split(300, SPLIT_D2H),
                      largest_remainder_split(2500, [1] * 8))


def dirichlet_sym(rng: np.random.Generator) -> dict:
    """One system of the uneven batch: o ~ U[5,20], v ~ U[40,160],
    N_cd = 7.5 (o+v) rounded half up, h in {1,2,4,8}, Dirichlet(2) splits."""
    o = int(rng.integers(5, 21))
    v = int(rng.integers(40, 161))
    ncd = (15 * (o + v) + 1) // 2
    h = int(rng.choice([1, 2, 4, 8]))
    wo = rng.dirichlet([2.0] * h)
    wv = rng.dirichlet([2.0] * h)

    def frac(x):
        return Fraction(float(x)).limit_denominator(1 << 30)

    nocc = largest_remainder_split(o, [frac(x) for x in wo])
    nvir = largest_remainder_split(v, [frac(x) for x in wv])
    ncdl = largest_remainder_split(ncd, [1] * h)
    return sym_custom(nocc, nvir, ncdl)


def batch_syms(nsys: int = 64, seed: int = 0) -> list[dict]:
    """System k of the uneven batch draws its shape from seed ``[seed, k]``."""
    return [dirichlet_sym(np.random.default_rng([seed, 4, k])) for k in range(nsys)]


def irrep_pairs(h: int, G: int):
    """(gi, gj) pairs with gi ^ gj == G, gi ascending."""
    return [(g, g ^ G) for g in range(h)]


def make_eps(sym: dict, seed: int = 0):
    h = sym["h"]
    eo = [np.random.default_rng([seed, TENSOR_IDS["eps_occ"], g]).uniform(-2.0, -0.5, sym["nocc"][g])
          for g in range(h)]
    ev = [np.random.default_rng([seed, TENSOR_IDS["eps_vir"], g]).uniform(0.2, 3.0, sym["nvir"][g])
          for g in range(h)]
    return eo, ev


def _decay(n: int) -> np.ndarray:
    return np.exp(-np.arange(n, dtype=np.float64) / 60.0)


def make_B(sym: dict, seed: int = 0, symmetric: bool = True) -> dict:
    """``B^P_ac`` blocks; symmetric in (a, c) unless ``symmetric`` is False."""
    h, nv, nc = sym["h"], sym["nvir"], sym["ncd"]
    G = {}
    for gP in range(h):
        dec = _decay(nc[gP])
        for ga in range(h):
            gc = ga ^ gP
            rng = np.random.default_rng([seed, TENSOR_IDS["B"], gP, ga])
            G[(gP, ga)] = rng.standard_normal((nv[ga], nv[gc], nc[gP])) * dec
    if not symmetric:
        return G
    out = {}
    r2 = 1.0 / np.sqrt(2.0)
    for gP in range(h):
        for ga in range(h):
            gc = ga ^ gP
            g1 = G[(gP, ga)]
            g2 = G[(gP, gc)].transpose(1, 0, 2)
            blk = (g1 + g2) * r2
            if ga == gc:
                n = nv[ga]
                idx = np.arange(n)
                blk[idx, idx, :] = g1[idx, idx, :]
            out[(gP, ga)] = blk
    return out


def make_Bvo(sym: dict, seed: int = 0) -> dict:
    h, nv, no, nc = sym["h"], sym["nvir"], sym["nocc"], sym["ncd"]
    out = {}
    for gP in range(h):
        dec = _decay(nc[gP])
        for ga in range(h):
            gm = ga ^ gP
            rng = np.random.default_rng([seed, TENSOR_IDS["Bvo"], gP, ga])
            out[(gP, ga)] = rng.standard_normal((nv[ga], no[gm], nc[gP])) * dec
    return out


def make_t1(sym: dict, seed: int = 0) -> list:
    return [np.random.default_rng([seed, TENSOR_IDS["t1"], g]).standard_normal(
        (sym["nocc"][g], sym["nvir"][g])) * 1e-3 for g in range(sym["h"])]


def _pair_blocks(sym: dict, seed: int, tid: int, eps) -> dict:
    """N(0,1) * 0.01 / (e_a + e_b - e_i - e_j), averaged with the pair transpose."""
    h, no, nv = sym["h"], sym["nocc"], sym["nvir"]
    eo, ev = eps
    raw = {}
    for G in range(h):
        for gi in range(h):
            gj = gi ^ G
            for ga in range(h):
                gb = ga ^ G
                rng = np.random.default_rng([seed, tid, G, gi, ga])
                raw[(G, gi, ga)] = rng.standard_normal((no[gi], no[gj], nv[ga], nv[gb]))
    out = {}
    for G in range(h):
        for gi in range(h):
            gj = gi ^ G
            for ga in range(h):
                gb = ga ^ G
                g = 0.5 * (raw[(G, gi, ga)] + raw[(G, gj, gb)].transpose(1, 0, 3, 2))
                # grouped so that the pair transpose sees bitwise the same value
                den = ((ev[ga][None, None, :, None] + ev[gb][None, None, None, :])
                       - (eo[gi][:, None, None, None] + eo[gj][None, :, None, None]))
                out[(G, gi, ga)] = g * 0.01 / den
    return out


def make_t2(sym: dict, seed: int = 0, eps=None) -> dict:
    eps = eps if eps is not None else make_eps(sym, seed)
    return _pair_blocks(sym, seed, TENSOR_IDS["t2"], eps)


def make_tau(sym: dict, t2: dict, t1: list) -> dict:
    """tau_ij^ab = t2_ij^ab + t_i^a t_j^b (the input recipe of the amplitudes)."""
    h = sym["h"]
    out = {}
    for (G, gi, ga), blk in t2.items():
        blk = blk.copy()
        gj, gb = gi ^ G, ga ^ G
        if gi == ga and gj == gb:
            blk += np.einsum("ia,jb->ijab", t1[gi], t1[gj])
        out[(G, gi, ga)] = blk
    assert len(out) == h ** 3
    return out


def make_lambda(sym: dict, seed: int = 0, eps=None) -> dict:
    eps = eps if eps is not None else make_eps(sym, seed)
    return _pair_blocks(sym, seed, TENSOR_IDS["lam"], eps)


def make_problem(sym: dict, seed: int = 0, kind: str = "t2",
                 symmetric_B: bool = True, with_t1: bool = True) -> dict:
    """All inputs of one ladder evaluation, as blocks.

    kind = "t2": B, tau (= t2 + t1 t1), eps.
    kind = "lambda": B, lam, Bvo, t1 (zero if ``with_t1`` is False), eps.
    """
    eps = make_eps(sym, seed)
    prob = {"sym": sym, "eps_occ": eps[0], "eps_vir": eps[1],
            "B": make_B(sym, seed, symmetric_B)}
    t1 = make_t1(sym, seed)
    if not with_t1:
        t1 = [np.zeros_like(x) for x in t1]
    prob["t1"] = t1
    if kind == "t2":
        prob["X"] = make_tau(sym, make_t2(sym, seed, eps), t1)
    elif kind == "lambda":
        prob["X"] = make_lambda(sym, seed, eps)
        prob["Bvo"] = make_Bvo(sym, seed)
    else:
        raise ValueError(kind)
    prob["kind"] = kind
    return prob


def make_density_problem(sym: dict, seed: int = 0) -> dict:
    """Inputs of one vvvv two-body-density contraction, as blocks: the
    transformed Cholesky vectors ``L`` (same blocks and distribution as B),
    ``X`` = tau~ (the tau recipe) and ``Y`` = lambda (the lambda recipe)."""
    eps = make_eps(sym, seed)
    t1 = make_t1(sym, seed)
    return {"sym": sym, "kind": "density", "L": make_B(sym, seed + 7919, True),
            "X": make_tau(sym, make_t2(sym, seed, eps), t1), "Y": make_lambda(sym, seed, eps)}


def make_lam_vo(sym: dict, seed: int = 0) -> dict:
    """lambda_bi^mn blocks ``(v_gb, o_gi, o_gm, o_gn)``, N(0, (1e-3)^2)."""
    h, no, nv = sym["h"], sym["nocc"], sym["nvir"]
    out = {}
    for G in range(h):
        for gb in range(h):
            gi = gb ^ G
            for gm in range(h):
                gn = gm ^ G
                rng = np.random.default_rng([seed, TENSOR_IDS["lam_vo"], G, gb, gm])
                out[(G, gb, gm)] = 1e-3 * rng.standard_normal((nv[gb], no[gi], no[gm], no[gn]))
    return out


def make_partial_problem(sym: dict, seed: int = 0) -> dict:
    """Inputs of one O(O^3 V^3) contraction M_bi^dc = sum_mn lambda_bi^mn
    tau~_mn^dc: ``lam`` (lam_vo blocks) and ``tau`` (the tau recipe, pair
    symmetric)."""
    eps = make_eps(sym, seed)
    t1 = make_t1(sym, seed)
    return {"sym": sym, "kind": "partial", "lam": make_lam_vo(sym, seed),
            "tau": make_tau(sym, make_t2(sym, seed, eps), t1)}


def make_cd_matrices(npairs, seed: int = 0, kappa: float = 60.0) -> list:
    """Dense symmetric PSD matrices, one per irrep (see the module docstring)."""
    out = []
    for g, n in enumerate(npairs):
        rng = np.random.default_rng([seed, TENSOR_IDS["cd"], g])
        z = rng.standard_normal((n, n))
        w = np.exp(-rng.uniform(0.0, 9.0, n))
        s_ = np.exp(-np.arange(n) / kappa)
        gm = (w[:, None] * z) * s_[None, :]
        v = gm @ gm.T
        out.append(0.5 * (v + v.T))
    return out


def serving_stream(n_requests: int, rate_hz: float, seed: int = 5, p_large: float = 0.1):
    """Poisson arrival times and request shapes for the serving loop: shapes
    as in the uneven batch, plus Bernoulli(p_large) large requests."""
    rng = np.random.default_rng([seed])
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    t = np.cumsum(gaps)
    reqs = []
    for k in range(n_requests):
        if rng.random() < p_large:
            sym = sym_serving_large()
        else:
            sym = dirichlet_sym(np.random.default_rng([seed, 4, k]))
        reqs.append((float(t[k]), sym, k))
    return reqs
