"""Pins of the vvvv two-body-density oracle against things other than
itself: pure-loop brute force, a rank-one closed form, the identity-vector
special case (a plain matrix product), the X <-> Y and a <-> c symmetries the
definition implies, scaling, and the symmetry-blocked form against the full
tensors scattered from the blocks."""
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
    """Y_mn^ab = y_mn u_a u_b, X_mn^cd = x_mn w_c w_d: V_abcd = s u_a u_b w_c w_d
    with s = sum_mn y_mn x_mn, so
    G^P_ac = s/2 [u_a w_c (u . L^P w) + w_a u_c (w . L^P u)]."""
    rng = _rng(32)
    o, v, n = 3, 5, 2
    y, x = rng.standard_normal((o, o)), rng.standard_normal((o, o))
    u, w = rng.standard_normal(v), rng.standard_normal(v)
    L = rng.standard_normal((n, v, v))
    Y = np.einsum("mn,a,b->mnab", y, u, u)
    X = np.einsum("mn,c,d->mncd", x, w, w)
    s = float(np.sum(y * x))
    uLw = np.array([u @ L[P] @ w for P in range(n)])
    wLu = np.array([w @ L[P] @ u for P in range(n)])
    expect = 0.5 * s * (np.einsum("a,c,P->Pac", u, w, uLw) + np.einsum("a,c,P->Pac", w, u, wLu))
    np.testing.assert_allclose(O.vvvv_density_full(X, Y, L), expect, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(O.vvvv_density_loops(X, Y, L), expect, rtol=1e-12, atol=1e-14)


def test_identity_vectors_give_a_matrix_product():
    """L^0_bd = delta_bd: G_ac = (M_ac + M_ca)/2 with M = Y_(ab),(mn) X_(mn),(cb)
    summed over b -- a plain reshaped matrix product."""
    rng = _rng(33)
    o, v = 3, 4
    X = rng.standard_normal((o, o, v, v))
    Y = rng.standard_normal((o, o, v, v))
    L = np.eye(v)[None]
    M = np.zeros((v, v))
    for b in range(v):
        M += Y[:, :, :, b].reshape(o * o, v).T @ X[:, :, :, b].reshape(o * o, v)
    expect = 0.5 * (M + M.T)
    np.testing.assert_allclose(O.vvvv_density_full(X, Y, L)[0], expect, rtol=1e-12, atol=1e-13)


def test_symmetric_in_the_two_amplitudes():
    """P_+(ab,cd) makes the result symmetric under X <-> Y."""
    rng = _rng(34)
    o, v, n = 2, 4, 3
    X = rng.standard_normal((o, o, v, v))
    Y = rng.standard_normal((o, o, v, v))
    L = rng.standard_normal((n, v, v))
    np.testing.assert_allclose(O.vvvv_density_full(X, Y, L), O.vvvv_density_full(Y, X, L),
                               rtol=1e-12, atol=1e-13)


def test_symmetric_in_a_c_for_symmetric_vectors():
    """Pair-symmetric amplitudes and L^P_bd = L^P_db give G^P_ac = G^P_ca."""
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
