"""Pins of the O(O^3 V^3) contraction oracle (M_bi^dc = sum_mn lambda_bi^mn
tau~_mn^dc) against loops, closed forms, special cases and the identity of
the partial symmetric-antisymmetric algorithm."""
import numpy as np
import pytest

import synth as S
from oracle import partial_blocks, partial_full, partial_loops, partial_pm_steps
from oracle.layout import OracleLayout


def _rng(k):
    return np.random.default_rng([77, k])


def _pair_sym(t):
    return 0.5 * (t + t.transpose(1, 0, 3, 2))


def test_loops_equal_definition():
    rng = _rng(1)
    v, o = 3, 2
    lam = rng.standard_normal((v, o, o, o))
    tau = rng.standard_normal((o, o, v, v))
    assert np.allclose(partial_loops(lam, tau), partial_full(lam, tau), rtol=1e-14, atol=1e-14)


def test_rank_one_closed_form():
    """lam = u_b w_i x_m y_n, tau = p_m q_n r_d s_c:
    M_bi^dc = u_b w_i r_d s_c (x . p)(y . q)."""
    rng = _rng(2)
    v, o = 4, 3
    u, r, s_ = (rng.standard_normal(v) for _ in range(3))
    w, x, y, p, q = (rng.standard_normal(o) for _ in range(5))
    lam = np.einsum("b,i,m,n->bimn", u, w, x, y)
    tau = np.einsum("m,n,d,c->mndc", p, q, r, s_)
    ref = np.einsum("b,i,d,c->bidc", u, w, r, s_) * (x @ p) * (y @ q)
    assert np.allclose(partial_loops(lam, tau), ref, rtol=1e-13, atol=1e-15)
    assert np.allclose(partial_full(lam, tau), ref, rtol=1e-13, atol=1e-15)


def test_single_occupied_is_an_outer_product():
    rng = _rng(3)
    v = 5
    lam = rng.standard_normal((v, 1, 1, 1))
    tau = rng.standard_normal((1, 1, v, v))
    ref = lam[:, 0, 0, 0][:, None, None, None] * tau[0, 0][None, None, :, :]
    assert np.array_equal(partial_loops(lam, tau), ref)


def test_one_nonzero_mn_selects_a_slice():
    """tau nonzero only at (m, n) = (2, 0): M_bi^dc = lam_bi^20 tau_20^dc."""
    rng = _rng(4)
    v, o = 3, 3
    lam = rng.standard_normal((v, o, o, o))
    tau = np.zeros((o, o, v, v))
    tau[2, 0] = rng.standard_normal((v, v))
    ref = np.einsum("bi,dc->bidc", lam[:, :, 2, 0], tau[2, 0])
    assert np.allclose(partial_full(lam, tau), ref, rtol=1e-15, atol=0)


def test_linear_in_each_operand():
    rng = _rng(5)
    v, o = 3, 2
    l1, l2 = rng.standard_normal((2, v, o, o, o))
    t1, t2 = rng.standard_normal((2, o, o, v, v))
    f = partial_full
    assert np.allclose(f(2.5 * l1 - l2, t1), 2.5 * f(l1, t1) - f(l2, t1), rtol=1e-13, atol=1e-14)
    assert np.allclose(f(l1, t1 + 3 * t2), f(l1, t1) + 3 * f(l1, t2), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("o,v", [(1, 3), (3, 4), (4, 2)])
def test_partial_pm_identity_for_pair_symmetric_tau(o, v):
    """The +/- algorithm (only d >= c columns of S and A, m >= n terms)
    reproduces the definition when tau~_mn^dc = tau~_nm^cd."""
    rng = _rng(6)
    lam = rng.standard_normal((v, o, o, o))
    tau = _pair_sym(rng.standard_normal((o, o, v, v)))
    assert np.allclose(partial_pm_steps(lam, tau), partial_full(lam, tau), rtol=1e-13, atol=1e-14)


def test_partial_pm_needs_pair_symmetry():
    """Without the pair symmetry of tau the +/- shortcut is wrong: the
    identity is a property of the input, not of the algebra alone."""
    rng = _rng(7)
    v, o = 3, 3
    lam = rng.standard_normal((v, o, o, o))
    tau = rng.standard_normal((o, o, v, v))
    assert not np.allclose(partial_pm_steps(lam, tau), partial_full(lam, tau))


SPECS = [
    ([2], [3], [1]),
    ([2, 1], [3, 4], [1, 1]),
    ([1, 2, 0, 1], [3, 2, 4, 1], [1, 1, 1, 1]),
    ([1, 1, 1, 0, 1, 0, 1, 1], [2, 3, 1, 2, 0, 2, 1, 3], [1] * 8),
]


@pytest.mark.parametrize("spec", SPECS)
def test_blocks_equal_full_scatter(spec):
    """The symmetry-blocked result equals the definition on the scattered
    full tensors, and symmetry-forbidden entries of the full result are 0."""
    sym = S.sym_custom(*spec)
    prob = S.make_partial_problem(sym, seed=11)
    lay = OracleLayout(sym)
    got = partial_blocks(sym, prob["lam"], prob["tau"])
    lam_full = lay.full_vo(prob["lam"], "oo")
    tau_full = lay.full_amp(prob["tau"])
    ref_full = partial_full(lam_full, tau_full)
    got_full = lay.full_vo(got, "vv")
    assert np.allclose(got_full, ref_full, rtol=1e-13, atol=1e-18)
    iv = np.concatenate([[g] * n for g, n in enumerate(sym["nvir"])]).astype(int)
    io = np.concatenate([[g] * n for g, n in enumerate(sym["nocc"])]).astype(int)
    allowed = (iv[:, None, None, None] ^ io[None, :, None, None] ^ iv[None, None, :, None]
               ^ iv[None, None, None, :]) == 0
    assert np.all(ref_full[~allowed] == 0.0)


@pytest.mark.parametrize("spec", SPECS)
def test_vo_layout_round_trip(spec):
    sym = S.sym_custom(*spec)
    prob = S.make_partial_problem(sym, seed=12)
    lay = OracleLayout(sym)
    flat = lay.pack_vo(prob["lam"], "oo")
    assert flat.size == lay.lvo_size == sum(lay.n_vo[G] * lay.n_oo[G] for G in range(lay.h))
    back = lay.unpack_vo(flat, "oo")
    for k, blk in prob["lam"].items():
        assert np.array_equal(back[k], blk)
    # the synthetic tau is pair symmetric (the +/- algorithm relies on it)
    full = lay.full_amp(prob["tau"])
    assert np.array_equal(full, full.transpose(1, 0, 3, 2))
