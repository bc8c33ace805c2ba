"""Pins of the vvvv two-body-density oracle against things other than
itself: pure-loop brute force, a rank-one closed form with distinct vectors
on every index (the exchange term Gamma_abdc of the spin-adapted density is
visible in it), the identity-vector special case written as plain matrix
products, the X <-> Y and a <-> c symmetries the definition implies,
scaling, the symmetry-blocked form against the full tensors scattered from
the blocks, and an independent derivation from spin-orbital amplitudes: the
spin-adapted density Gamma~_pqrs = 2 Gamma_PqRs - Gamma_PqSr is half the sum
over spins of the spin-orbital density built from antisymmetrised amplitudes."""
import numpy as np
import pytest

import oracle as O
from oracle.layout import OracleLayout
import synth as S


def _rng(*k):
    return np.random.default_rng(list(k))


def _pair_sym(t):
    return 0.5 * (t + t.transpose(1, 0, 3, 2))


def test_loops_equal_definition():
    rng = _rng(31)
    o, v, n = 2, 3, 2
    X = rng.standard_normal((o, o, v, v))
    Y = rng.standard_normal((o, o, v, v))
    L = rng.standard_normal((n, v, v))
    np.testing.assert_allclose(O.vvvv_density_full(X, Y, L), O.vvvv_density_loops(X, Y, L),
                               rtol=1e-13, atol=1e-13)


def test_rank_one_closed_form():
    """Y_mn^ab = y_mn u_a r_b and X_mn^cd = x_mn w_c z_d (four different
    vectors): V_abcd = s u_a r_b w_c z_d with s = sum_mn y_mn x_mn, so

      G^P_ac = s [u_a w_c (r.L^P z) + w_a u_c (z.L^P r)]
             - s/2 [u_a z_c (r.L^P w) + w_a r_c (z.L^P u)]

    (first bracket: 2 Gamma_abcd; second: Gamma_abdc)."""
    rng = _rng(32)
    o, v, n = 3, 5, 2
    y, x = rng.standard_normal((o, o)), rng.standard_normal((o, o))
    u, r, w, z = (rng.standard_normal(v) for _ in range(4))
    L = rng.standard_normal((n, v, v))
    Y = np.einsum("mn,a,b->mnab", y, u, r)
    X = np.einsum("mn,c,d->mncd", x, w, z)
    s = float(np.sum(y * x))

    def q(p, t):
        return np.array([p @ L[P] @ t for P in range(n)])

    expect = (s * (np.einsum("a,c,P->Pac", u, w, q(r, z)) + np.einsum("a,c,P->Pac", w, u, q(z, r)))
              - 0.5 * s * (np.einsum("a,c,P->Pac", u, z, q(r, w)) + np.einsum("a,c,P->Pac", w, r, q(z, u))))
    np.testing.assert_allclose(O.vvvv_density_full(X, Y, L), expect, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(O.vvvv_density_loops(X, Y, L), expect, rtol=1e-12, atol=1e-14)


def test_identity_vectors_give_matrix_products():
    """L^0_bd = delta_bd: G_ac = sum_b (2 Gamma_abcb - Gamma_abbc) =
    (M + M^T)_ac - (N + N')_ac / 2 with M_ac = sum_b Y_(ab),(mn) X_(mn),(cb),
    N_ac = sum_b Y_(ab),(mn) X_(mn),(bc) and N'_ac = sum_b X_(ab),(mn)
    Y_(mn),(bc) -- plain reshaped matrix products."""
    rng = _rng(33)
    o, v = 3, 4
    X = rng.standard_normal((o, o, v, v))
    Y = rng.standard_normal((o, o, v, v))
    L = np.eye(v)[None]
    M, N, N2 = np.zeros((v, v)), np.zeros((v, v)), np.zeros((v, v))
    for b in range(v):
        ya = Y[:, :, :, b].reshape(o * o, v)      # (mn), a
        xa = X[:, :, :, b].reshape(o * o, v)
        M += ya.T @ X[:, :, :, b].reshape(o * o, v)
        N += ya.T @ X[:, :, b, :].reshape(o * o, v)
        N2 += xa.T @ Y[:, :, b, :].reshape(o * o, v)
    expect = (M + M.T) - 0.5 * (N + N2)
    np.testing.assert_allclose(O.vvvv_density_full(X, Y, L)[0], expect, rtol=1e-12, atol=1e-13)


def test_symmetric_in_the_two_amplitudes():
    """P_+(ab,cd) and the exchange term treat X and Y alike: the result is
    symmetric under X <-> Y."""
    rng = _rng(34)
    o, v, n = 2, 4, 3
    X = rng.standard_normal((o, o, v, v))
    Y = rng.standard_normal((o, o, v, v))
    L = rng.standard_normal((n, v, v))
    np.testing.assert_allclose(O.vvvv_density_full(X, Y, L), O.vvvv_density_full(Y, X, L),
                               rtol=1e-12, atol=1e-13)


def test_symmetric_in_a_c_for_symmetric_vectors():
    """Pair-symmetric amplitudes and L^P_bd = L^P_db give G^P_ac = G^P_ca
    (Gamma~_cdab = Gamma~_abcd for pair-symmetric amplitudes)."""
    rng = _rng(35)
    o, v, n = 3, 4, 2
    X = _pair_sym(rng.standard_normal((o, o, v, v)))
    Y = _pair_sym(rng.standard_normal((o, o, v, v)))
    L = rng.standard_normal((n, v, v))
    L = L + L.transpose(0, 2, 1)
    G = O.vvvv_density_full(X, Y, L)
    np.testing.assert_allclose(G, G.transpose(0, 2, 1), rtol=1e-12, atol=1e-13)


def test_scaling():
    rng = _rng(36)
    o, v, n = 2, 3, 2
    X = rng.standard_normal((o, o, v, v))
    Y = rng.standard_normal((o, o, v, v))
    L = rng.standard_normal((n, v, v))
    G = O.vvvv_density_full(X, Y, L)
    np.testing.assert_allclose(O.vvvv_density_full(2.5 * X, Y, L), 2.5 * G, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(O.vvvv_density_full(X, Y, -3.0 * L), -3.0 * G, rtol=1e-13, atol=1e-14)


# ------------------------------------------------------------------ spin orbitals
def _spin_orbital_amplitudes(T):
    """Antisymmetric spin-orbital doubles from closed-shell spatial ones
    (pair symmetric, T_mn^cd = T_nm^dc), spin-orbital index 2p + s (s = 0
    alpha, 1 beta):
      (a b a b), (b a b a):  T_mn^cd
      (a b b a), (b a a b): -T_mn^dc
      (a a a a), (b b b b):  T_mn^cd - T_mn^dc
    where the spin labels list (m, n, c, d); every other spin case is 0."""
    o, _, v, _ = T.shape
    out = np.zeros((2 * o, 2 * o, 2 * v, 2 * v))
    for sm in (0, 1):
        for sn in (0, 1):
            for sc in (0, 1):
                for sd in (0, 1):
                    if sm == sn == sc == sd:
                        blk = T - T.transpose(0, 1, 3, 2)
                    elif sm != sn and sm == sc and sn == sd:
                        blk = T
                    elif sm != sn and sm == sd and sn == sc:
                        blk = -T.transpose(0, 1, 3, 2)
                    else:
                        continue
                    out[sm::2, sn::2, sc::2, sd::2] = blk
    return out


def _spin_orbital_G(X, Y, L):
    """G^P_ac from the spin-orbital vvvv density:
    V_ABCD = 1/2 sum_MN Y_MN^AB X_MN^CD (each unordered pair MN counted once),
    Gamma_ABCD = 1/2 (V_ABCD + V_CDAB), and the spin-free integrals
    <AB|CD> = (ac|bd) delta(s_A, s_C) delta(s_B, s_D) give
    sum_ABCD Gamma_ABCD <AB|CD> = 2 sum_abcd Gamma~_abcd (ac|bd), i.e.
    G^P_ac = 1/2 sum_{s, s'} sum_bd Gamma_(a s)(b s')(c s)(d s') L^P_bd."""
    Xs, Ys = _spin_orbital_amplitudes(X), _spin_orbital_amplitudes(Y)
    V = 0.5 * np.einsum("MNAB,MNCD->ABCD", Ys, Xs)
    Gam = 0.5 * (V + V.transpose(2, 3, 0, 1))
    nP, v, _ = L.shape
    G = np.zeros((nP, v, v))
    for s in (0, 1):
        for t in (0, 1):
            G += 0.5 * np.einsum("abcd,Pbd->Pac", Gam[s::2, t::2, s::2, t::2], L)
    return G


def test_spin_orbital_amplitudes_are_antisymmetric():
    """The spin-orbital amplitudes built from pair-symmetric spatial ones are
    antisymmetric in (M, N) and in (C, D): the construction above is the
    closed-shell spin adaptation, not an arbitrary choice."""
    rng = _rng(37)
    T = _pair_sym(rng.standard_normal((2, 2, 3, 3)))
    Ts = _spin_orbital_amplitudes(T)
    np.testing.assert_allclose(Ts, -Ts.transpose(1, 0, 2, 3), atol=1e-15)
    np.testing.assert_allclose(Ts, -Ts.transpose(0, 1, 3, 2), atol=1e-15)


@pytest.mark.parametrize("seed", [38, 39])
def test_matches_spin_orbital_density(seed):
    """Every element of G^P_ac (o = 2, v = 3, 2 vectors, non-symmetric L)
    equals the value derived from the spin-orbital amplitudes and density."""
    rng = _rng(seed)
    o, v, n = 2, 3, 2
    X = _pair_sym(rng.standard_normal((o, o, v, v)))
    Y = _pair_sym(rng.standard_normal((o, o, v, v)))
    L = rng.standard_normal((n, v, v))
    expect = _spin_orbital_G(X, Y, L)
    np.testing.assert_allclose(O.vvvv_density_loops(X, Y, L), expect, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(O.vvvv_density_full(X, Y, L), expect, rtol=1e-12, atol=1e-13)


def test_spin_orbital_pin_sees_the_exchange_term():
    """The pin above is not blind to the spin adaptation: the plain
    Gamma_abcd contraction (no exchange term, no factor 2) differs from it."""
    rng = _rng(40)
    o, v, n = 2, 3, 2
    X = _pair_sym(rng.standard_normal((o, o, v, v)))
    Y = _pair_sym(rng.standard_normal((o, o, v, v)))
    L = rng.standard_normal((n, v, v))
    V = np.einsum("mnab,mncd->abcd", Y, X)
    plain = np.einsum("abcd,Pbd->Pac", 0.5 * (V + V.transpose(2, 3, 0, 1)), L)
    assert np.max(np.abs(plain - _spin_orbital_G(X, Y, L))) > 1e-3 * np.max(np.abs(plain))


SYMS = [
    ([3], [5], [4]),
    ([2, 1], [3, 4], [3, 2]),
    ([1, 2, 0, 1], [3, 2, 4, 1], [2, 0, 3, 1]),
    ([1, 1, 1, 0, 1, 0, 1, 1], [2, 3, 1, 2, 0, 2, 1, 3], [2, 1, 0, 2, 1, 1, 0, 2]),
]


@pytest.mark.parametrize("spec", SYMS)
def test_blocks_equal_full_scatter(spec):
    """The symmetry-blocked result equals the definition on the scattered full
    tensors, and symmetry-forbidden entries of the full result are exactly 0."""
    sym = S.sym_custom(*spec)
    prob = S.make_density_problem(sym, seed=13)
    lay = OracleLayout(sym)
    Gb = O.vvvv_density_blocks(sym, prob["X"], prob["Y"], prob["L"])
    Gf = O.vvvv_density_full(lay.full_amp(prob["X"]), lay.full_amp(prob["Y"]), lay.full_B(prob["L"]))
    np.testing.assert_allclose(lay.full_B(Gb), Gf, rtol=1e-12, atol=1e-15)
    # (P, a, c) with irr(a)^irr(c) != irr(P) is forbidden
    h = sym["h"]
    irr_v = np.concatenate([[g] * sym["nvir"][g] for g in range(h)]).astype(int)
    irr_p = np.concatenate([[g] * sym["ncd"][g] for g in range(h)]).astype(int)
    allowed = (irr_p[:, None, None] == (irr_v[None, :, None] ^ irr_v[None, None, :]))
    assert np.all(Gf[~allowed] == 0.0)
