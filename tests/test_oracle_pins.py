"""Pins of the CPU oracle against things other than itself: pure-loop brute
force, closed forms, invariants, the spin-orbital derivation of the pair
energy, and special cases."""
import itertools

import numpy as np
import pytest

import oracle as O
from oracle.layout import OracleLayout
import synth as S


def _rng(*k):
    return np.random.default_rng(list(k))


def _sym_tau(rng, o, v, sym=True):
    t = rng.standard_normal((o, o, v, v))
    if sym:
        t = 0.5 * (t + t.transpose(1, 0, 3, 2))
    return t


# ----------------------------------------------------------------- T2 ladder
@pytest.mark.parametrize("symB", [True, False])
def test_loops_equal_einsum_brute_force(symB):
    rng = _rng(1, symB)
    o, v, n = 2, 3, 2
    B = rng.standard_normal((n, v, v))
    if symB:
        B = B + B.transpose(0, 2, 1)
    tau = _sym_tau(rng, o, v, sym=False)
    np.testing.assert_allclose(O.t2_ladder_full(B, tau), O.t2_ladder_loops(B, tau), rtol=1e-13, atol=1e-13)


def test_rank_one_closed_form():
    """B^0_ac = u_a w_c  =>  R_ij^ab = u_a u_b sum_cd tau_ij^cd w_c w_d."""
    rng = _rng(2)
    o, v = 3, 5
    u, w = rng.standard_normal(v), rng.standard_normal(v)
    B = np.einsum("a,c->ac", u, w)[None]
    tau = rng.standard_normal((o, o, v, v))
    expect = np.einsum("a,b,ijcd,c,d->ijab", u, u, tau, w, w)
    np.testing.assert_allclose(O.t2_ladder_full(B, tau), expect, rtol=1e-13, atol=1e-14)
    Rb = O.t2_ladder_loops(B, tau)
    np.testing.assert_allclose(Rb, expect, rtol=1e-13, atol=1e-14)


def test_unit_amplitude_picks_one_integral():
    """tau_ij^cd = delta(c,c0) delta(d,d0)  =>  R_ij^ab = (a c0 | b d0)."""
    rng = _rng(3)
    o, v, n = 2, 4, 3
    B = rng.standard_normal((n, v, v))
    c0, d0 = 2, 1
    tau = np.zeros((o, o, v, v))
    tau[:, :, c0, d0] = 1.0
    R = O.t2_ladder_full(B, tau)
    for a, b in itertools.product(range(v), range(v)):
        ref = sum(B[P, a, c0] * B[P, b, d0] for P in range(n))
        assert abs(R[0, 1, a, b] - ref) < 1e-14


def test_pair_symmetry_any_B():
    """R_ij^ab = R_ji^ba for pair-symmetric tau, with non-symmetric B."""
    rng = _rng(4)
    o, v, n = 3, 5, 4
    B = rng.standard_normal((n, v, v))
    tau = _sym_tau(rng, o, v)
    R = O.t2_ladder_full(B, tau)
    np.testing.assert_allclose(R, R.transpose(1, 0, 3, 2), rtol=1e-13, atol=1e-14)


def test_scaling_and_linearity():
    rng = _rng(5)
    o, v, n = 2, 4, 3
    B = rng.standard_normal((n, v, v))
    t1, t2 = _sym_tau(rng, o, v), _sym_tau(rng, o, v)
    R = O.t2_ladder_full(B, t1)
    np.testing.assert_allclose(O.t2_ladder_full(3.0 * B, t1), 9.0 * R, rtol=1e-13)
    np.testing.assert_allclose(O.t2_ladder_full(B, 2 * t1 - t2), 2 * R - O.t2_ladder_full(B, t2), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("restricted", [False, True])
def test_symmetric_antisymmetric_algebra(restricted):
    """Z = S + A equals the plain contraction; S is symmetric and A
    antisymmetric under a<->b and under i<->j."""
    rng = _rng(6, restricted)
    o, v, n = 3, 5, 4
    B = rng.standard_normal((n, v, v))
    tau = _sym_tau(rng, o, v)
    R, Sm, Am = O.t2_ladder_symantisym_full(B, tau, restricted=restricted)
    np.testing.assert_allclose(R, O.t2_ladder_full(B, tau), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(Sm, Sm.transpose(0, 1, 3, 2), atol=1e-13)
    np.testing.assert_allclose(Sm, Sm.transpose(1, 0, 2, 3), atol=1e-13)
    np.testing.assert_allclose(Am, -Am.transpose(0, 1, 3, 2), atol=1e-13)
    np.testing.assert_allclose(Am, -Am.transpose(1, 0, 2, 3), atol=1e-13)


SYMS = [
    ([3], [5], [4]),
    ([2, 1], [3, 4], [3, 2]),
    ([1, 2, 0, 1], [3, 2, 4, 1], [2, 0, 3, 1]),
    ([1, 1, 1, 0, 1, 0, 1, 1], [2, 3, 1, 2, 0, 2, 1, 3], [2, 1, 0, 2, 1, 1, 0, 2]),
]


@pytest.mark.parametrize("spec", SYMS)
@pytest.mark.parametrize("symB", [True, False])
def test_blocks_equal_full_scatter(spec, symB):
    """The symmetry-blocked result equals the brute-force result on the
    scattered full tensors, and symmetry-forbidden full entries are exactly 0."""
    sym = S.sym_custom(*spec)
    prob = S.make_problem(sym, seed=11, kind="t2", symmetric_B=symB)
    lay = OracleLayout(sym)
    Rb = O.t2_ladder_blocks(sym, prob["B"], prob["X"])
    Bf, tf = lay.full_B(prob["B"]), lay.full_amp(prob["X"])
    Rf = O.t2_ladder_full(Bf, tf)
    np.testing.assert_allclose(lay.full_amp(Rb), Rf, rtol=1e-12, atol=1e-15)
    assert np.all(Rf[~lay.allowed_mask()] == 0.0)
    # the generator's tau is exactly pair-symmetric, so R is too
    np.testing.assert_allclose(Rf, Rf.transpose(1, 0, 3, 2), rtol=1e-12, atol=1e-16)


# ------------------------------------------------------------- Lambda ladder
def test_lambda_w_loops():
    """Appendix-A W written as explicit loops on a microscopic system."""
    rng = _rng(7)
    o, v, n = 2, 3, 2
    B = rng.standard_normal((n, v, v))
    Bvo = rng.standard_normal((n, v, o))
    t1 = rng.standard_normal((o, v))
    W = O.lambda_w_full(B, Bvo, t1)
    for e, f, a, b in itertools.product(range(v), repeat=4):
        s = 0.0
        for P in range(n):
            tea = sum(t1[m, e] * Bvo[P, a, m] for m in range(o))
            s += (B[P, e, a] - tea) * B[P, f, b]
            for m in range(o):
                s -= t1[m, f] * B[P, e, a] * Bvo[P, b, m]
        assert abs(W[e, f, a, b] - s) < 1e-13


def test_lambda_w_dressed_difference_form():
    """(B - t)(B - t) - t t is the same W (the signed stack the GPU uses)."""
    rng = _rng(8)
    o, v, n = 3, 5, 4
    B = rng.standard_normal((n, v, v))
    Bvo = rng.standard_normal((n, v, o))
    t1 = rng.standard_normal((o, v))
    tP = np.einsum("ma,Pbm->Pab", t1, Bvo)
    Bt = B - tP
    W2 = np.einsum("Pea,Pfb->efab", Bt, Bt) - np.einsum("Pea,Pfb->efab", tP, tP)
    np.testing.assert_allclose(O.lambda_w_full(B, Bvo, t1), W2, rtol=1e-12, atol=1e-13)


def test_lambda_t1_zero_reduces_to_t2_for_symmetric_B():
    rng = _rng(9)
    o, v, n = 3, 4, 3
    B = rng.standard_normal((n, v, v))
    B = B + B.transpose(0, 2, 1)
    Bvo = rng.standard_normal((n, v, o))
    lam = _sym_tau(rng, o, v)
    Z = O.lambda_ladder_full(B, Bvo, np.zeros((o, v)), lam)
    np.testing.assert_allclose(Z, O.t2_ladder_full(B, lam), rtol=1e-12, atol=1e-13)


def test_lambda_pair_symmetry():
    rng = _rng(10)
    o, v, n = 3, 4, 3
    B = rng.standard_normal((n, v, v))            # no vv symmetry needed
    Bvo = rng.standard_normal((n, v, o))
    t1 = rng.standard_normal((o, v))
    Z = O.lambda_ladder_full(B, Bvo, t1, _sym_tau(rng, o, v))
    np.testing.assert_allclose(Z, Z.transpose(1, 0, 3, 2), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("spec", SYMS)
def test_lambda_blocks_equal_full(spec):
    sym = S.sym_custom(*spec)
    prob = S.make_problem(sym, seed=12, kind="lambda", symmetric_B=False)
    lay = OracleLayout(sym)
    Zb = O.lambda_ladder_blocks(sym, prob["B"], prob["Bvo"], prob["t1"], prob["X"])
    Zf = O.lambda_ladder_full(lay.full_B(prob["B"]), lay.full_Bvo(prob["Bvo"]),
                              lay.full_t1(prob["t1"]), lay.full_amp(prob["X"]))
    np.testing.assert_allclose(lay.full_amp(Zb), Zf, rtol=1e-12, atol=1e-16)
    assert np.all(Zf[~lay.allowed_mask()] == 0.0)


# ------------------------------------------------------------- pair energies
def test_pair_energy_matches_spin_orbital_ladder_energy():
    """For closed-shell amplitudes, sum_ab (2t-t^T) R reproduces the
    spin-orbital particle-particle ladder functional
    (1/8) sum T_IJ^AB <AB||CD> T_IJ^CD pair by pair (the textbook MP3 ladder
    energy when t are first-order amplitudes)."""
    rng = _rng(13)
    o, v, n = 2, 3, 3
    B = rng.standard_normal((n, v, v))
    B = B + B.transpose(0, 2, 1)           # real orbitals: (ac|bd) has 8-fold symmetry
    t = _sym_tau(rng, o, v)
    R = O.t2_ladder_full(B, t)
    e = O.pair_energies_full(t, R)
    eri = np.einsum("Pac,Pbd->acbd", B, B)  # (ac|bd)
    so = lambda n_: [(p, s) for s in (0, 1) for p in range(n_)]
    occ, vir = so(o), so(v)
    no2, nv2 = len(occ), len(vir)
    T = np.zeros((no2, no2, nv2, nv2))
    for (I, (i, si)), (J, (j, sj)), (A, (a, sa)), (Bb, (b, sb)) in itertools.product(
            enumerate(occ), enumerate(occ), enumerate(vir), enumerate(vir)):
        T[I, J, A, Bb] = t[i, j, a, b] * (si == sa) * (sj == sb) - t[i, j, b, a] * (si == sb) * (sj == sa)
    V = np.zeros((nv2,) * 4)  # <AB|CD> = (AC|BD) with spin deltas
    for (A, (a, sa)), (Bb, (b, sb)), (C, (c, sc)), (D, (d, sd)) in itertools.product(*(list(enumerate(vir)),) * 4):
        V[A, Bb, C, D] = eri[a, c, b, d] * (sa == sc) * (sb == sd)
    Vas = V - V.transpose(0, 1, 3, 2)
    F = np.einsum("IJAB,ABCD,IJCD->IJ", T, Vas, T)
    for i, j in itertools.product(range(o), range(o)):
        f_ij = sum(F[I, J] for I, (ii, _) in enumerate(occ) if ii == i for J, (jj, _) in enumerate(occ) if jj == j)
        assert abs(e[i, j] - f_ij / 8.0) < 1e-12 * max(1.0, abs(e[i, j]))
    assert abs(e.sum() - F.sum() / 8.0) < 1e-11


def test_denominator_update_definition():
    rng = _rng(14)
    o, v = 2, 3
    eo, ev = rng.uniform(-2, -0.5, o), rng.uniform(0.2, 3, v)
    R = rng.standard_normal((o, o, v, v))
    d = O.denominator_update_full(R, eo, ev)
    for i, j, a, b in itertools.product(range(o), range(o), range(v), range(v)):
        D = eo[i] + eo[j] - ev[a] - ev[b]
        assert D < 0
        assert abs(d[i, j, a, b] * D - R[i, j, a, b]) < 1e-14


@pytest.mark.parametrize("spec", SYMS)
def test_blockwise_epilogue_equals_full(spec):
    """Pair energies and R/D computed on the symmetry blocks equal the
    definitions on the scattered full tensors (non-pair-symmetric X, so the
    exchange partner's block is exercised); R/D on forbidden entries stays 0."""
    sym = S.sym_custom(*spec)
    lay = OracleLayout(sym)
    rng = _rng(17)
    X = {k: rng.standard_normal(v.shape) for k, v in S.make_problem(sym, seed=12, kind="t2")["X"].items()}
    R = {k: rng.standard_normal(v.shape) for k, v in X.items()}
    e = O.pair_energies_blocks(sym, X, R)
    np.testing.assert_allclose(e, O.pair_energies_full(lay.full_amp(X), lay.full_amp(R)), rtol=1e-13, atol=1e-13)
    eo = [rng.uniform(-2, -0.5, n) for n in sym["nocc"]]
    ev = [rng.uniform(0.2, 3, n) for n in sym["nvir"]]
    d = O.denominator_update_blocks(sym, R, eo, ev)
    df = O.denominator_update_full(lay.full_amp(R), np.concatenate(eo), np.concatenate(ev)) * lay.allowed_mask()
    np.testing.assert_allclose(lay.full_amp(d), df, rtol=1e-14, atol=1e-14)


# ------------------------------------------------------------ single elements
def test_elements_match_blocks():
    sym = S.sym_custom([1, 2, 1, 1], [3, 2, 4, 2], [2, 3, 1, 2])
    lay = OracleLayout(sym)
    pt = S.make_problem(sym, seed=15, kind="t2", symmetric_B=False)
    pl = S.make_problem(sym, seed=15, kind="lambda", symmetric_B=False)
    Rf = lay.full_amp(O.t2_ladder_blocks(sym, pt["B"], pt["X"]))
    Zf = lay.full_amp(O.lambda_ladder_blocks(sym, pl["B"], pl["Bvo"], pl["t1"], pl["X"]))
    rng = _rng(16)
    for _ in range(40):
        i, j = rng.integers(0, lay.nocc_tot, 2)
        a, b = rng.integers(0, lay.nvir_tot, 2)
        assert abs(O.element_t2(sym, pt["B"], pt["X"], i, j, a, b) - Rf[i, j, a, b]) < 1e-14
        assert abs(O.element_lambda(sym, pl["B"], pl["Bvo"], pl["t1"], pl["X"], i, j, a, b) - Zf[i, j, a, b]) < 1e-14


def test_rel_errors():
    ref = {0: np.array([1.0, -4.0]), 1: np.array([2.0])}
    got = {0: np.array([1.0, -4.5]), 1: np.array([2.0])}
    mx, fro = O.rel_errors(got, ref)
    assert mx == pytest.approx(0.5 / 4.0)
    assert fro == pytest.approx(0.5 / np.sqrt(21.0))
