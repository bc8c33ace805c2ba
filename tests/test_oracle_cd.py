"""Pins of the two-step Cholesky decomposition oracle: a hand-worked
five-pair matrix whose pivot order under Q_max = 2 differs both from greedy
pivoting and from the variant with tau_mic = tau (written out literally), the
decomposition error bound, exact reproduction of the pivot rows, reduction to
textbook greedy pivoted Cholesky for Q_max = 1, full and exact-low-rank
cases, invariance under reordering of the pairs, irrep blocks kept apart."""
import numpy as np
import pytest

import oracle.cholesky as OC
import synth as S
from oracle import cd_basis, cd_vectors


def _greedy_pivoted_cholesky(v, tau):
    """Textbook full-pivoting Cholesky (written out here, independently of
    the oracle): pick the largest residual diagonal while it is >= tau."""
    n = v.shape[0]
    R = v.copy()
    piv = []
    while True:
        d = np.diag(R).copy()
        d[piv] = -np.inf
        q = int(np.argmax(d)) if n else 0
        if n == 0 or d[q] < tau:
            break
        col = R[:, q] / np.sqrt(R[q, q])
        R = R - np.outer(col, col)
        piv.append(q)
    return piv


@pytest.mark.parametrize("tau", [1e-4, 1e-7])
def test_error_bound_and_pivot_rows(tau):
    V = S.make_cd_matrices([150, 90, 0, 60], seed=1, kappa=20.0)
    piv, _ = cd_basis(V, tau, sigma=1e-2, qmax=40)
    L = cd_vectors(V, piv)
    for v, p, l in zip(V, piv, L):
        if v.shape[0] == 0:
            assert p.size == 0 and l.shape == (0, 0)
            continue
        res = v - l @ l.T
        assert np.abs(res).max() < tau                       # every residual diagonal < tau bounds all
        assert np.abs(res[p, :]).max() <= 1e-12 * np.abs(v).max()  # pivot rows reproduced
        assert len(set(p.tolist())) == p.size                 # no pivot twice


def test_qmax_one_is_greedy_pivoted_cholesky():
    V = S.make_cd_matrices([80, 50], seed=2, kappa=15.0)
    tau = 1e-6
    piv, _ = cd_basis(V, tau, sigma=1e-2, qmax=1)
    for v, p in zip(V, piv):
        assert p.tolist() == _greedy_pivoted_cholesky(v, tau)


def test_full_rank_tiny_threshold_takes_every_pair():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((30, 30))
    v = a @ a.T + 30 * np.eye(30)
    piv, _ = cd_basis([v], 1e-13, sigma=1e-2, qmax=7)
    assert sorted(piv[0].tolist()) == list(range(30))
    L = cd_vectors([v], piv)[0]
    assert np.abs(v - L @ L.T).max() < 1e-11 * np.abs(v).max()


def test_exact_low_rank():
    rng = np.random.default_rng(4)
    g = rng.standard_normal((60, 9))
    v = g @ g.T
    piv, _ = cd_basis([v], 1e-8, sigma=1e-2, qmax=1000)
    assert piv[0].size == 9
    L = cd_vectors([v], piv)[0]
    assert np.abs(v - L @ L.T).max() < 1e-8


def test_invariant_under_reordering_of_pairs():
    V = S.make_cd_matrices([70], seed=5, kappa=12.0)
    perm = np.random.default_rng(6).permutation(70)
    Vp = [V[0][np.ix_(perm, perm)]]
    piv, _ = cd_basis(V, 1e-6, sigma=1e-2, qmax=10)
    pivp, _ = cd_basis(Vp, 1e-6, sigma=1e-2, qmax=10)
    assert perm[pivp[0]].tolist() == piv[0].tolist()


def test_irrep_blocks_stay_apart():
    """Vectors of one irrep only span that irrep's pairs, and the per-irrep
    decomposition equals the one of the block-diagonal matrix with every
    pair of the other irreps screened out."""
    V = S.make_cd_matrices([40, 25], seed=7, kappa=10.0)
    piv, _ = cd_basis(V, 1e-5, sigma=1e-2, qmax=1)
    full = np.zeros((65, 65))
    full[:40, :40], full[40:, 40:] = V[0], V[1]
    pf, _ = cd_basis([full], 1e-5, sigma=1e-2, qmax=1)
    merged = sorted(piv[0].tolist() + [40 + x for x in piv[1].tolist()])
    assert sorted(pf[0].tolist()) == merged


def test_screening_drops_small_diagonals():
    v = np.diag([1.0, 1e-9, 0.5, 1e-12])
    piv, _ = cd_basis([v], 1e-6)
    assert sorted(piv[0].tolist()) == [0, 2]
    L = cd_vectors([v], piv)[0]
    assert np.abs(v - L @ L.T).max() <= 1e-9


# Hand-worked case (sigma = 1/2, Q_max = 2, tau = 1/2).  Pairs 0..4:
HAND_V = np.array([[25.0, 10.0, 0.0, 0.0, 0.0],
                   [10.0, 20.0, 0.0, 0.0, 4.0],
                   [0.0, 0.0, 18.0, 9.0, 0.0],
                   [0.0, 0.0, 9.0, 12.0, 0.0],
                   [0.0, 4.0, 0.0, 0.0, 9.5]])
# Round 1: D_max = 25; qualified (>= 12.5): 0 (25), 1 (20), 2 (18); the two
#   largest are candidates [0, 1]; tau_mic = 12.5.
#   pivot 0: l = (5, 2, 0, 0, 0); diagonals (0, 16, 18, 12, 9.5).
#   pivot 1 (16 >= 12.5; greedy would take pair 2 with 18 here):
#     residual column of 1 = (0, 16, 0, 0, 4), l = (0, 4, 0, 0, 1);
#     diagonals (0, 0, 18, 12, 8.5).  No candidate left above 12.5.
#   Pairs 0 and 1 (diagonal 0) become inactive.
# Round 2: D_max = 18; qualified (>= 9): 2 (18), 3 (12); pair 4 (8.5) is
#   not; candidates [2, 3]; tau_mic = 9.
#   pivot 2: l = (0, 0, sqrt 18, 9 / sqrt 18, 0); diagonal of 3 becomes
#     12 - 81/18 = 7.5 < 9, so the round ends (with tau_mic = tau = 1/2 it
#     would continue with pair 3).
# Round 3: D_max = 8.5 (pair 4); qualified (>= 4.25): 4 (8.5), 3 (7.5);
#   pivot 4 (its residual column has no entry on 3), then pivot 3.
HAND_ALG1 = [0, 1, 2, 4, 3]
# Greedy pivoting: 0 (25), then 2 (18 > 16), then 1 (16), 4 (8.5), 3 (7.5).
HAND_GREEDY = [0, 2, 1, 4, 3]
# tau_mic = tau: round 2 takes 2 and then 3 (7.5 >= 1/2); round 3 takes 4.
HAND_TAU_MIC_IS_TAU = [0, 1, 2, 3, 4]


def test_hand_worked_pivot_order():
    piv, _ = cd_basis([HAND_V], 0.5, sigma=0.5, qmax=2)
    assert piv[0].tolist() == HAND_ALG1
    assert _greedy_pivoted_cholesky(HAND_V, 0.5) == HAND_GREEDY
    # Q_max large enough to hold every qualified pair: the order of round 1
    # follows the diagonals (0, 2, 1), as greedy pivoting does here
    piv5, _ = cd_basis([HAND_V], 0.5, sigma=0.5, qmax=5)
    assert piv5[0].tolist() == HAND_GREEDY
    L = cd_vectors([HAND_V], piv)[0]
    np.testing.assert_allclose(L @ L.T, HAND_V, atol=1e-13)


def test_hand_worked_tau_mic_matters(monkeypatch):
    """The round threshold decides the order: with tau_mic = tau the same
    matrix gives a different (hand-worked) pivot list."""
    monkeypatch.setattr(OC, "cd_tau_mic", lambda tau, sigma, dmax: tau)
    piv, _ = OC.cd_basis([HAND_V], 0.5, sigma=0.5, qmax=2)
    assert piv[0].tolist() == HAND_TAU_MIC_IS_TAU


def test_hand_worked_two_irreps():
    """The same matrix is block diagonal in {0, 1, 4} and {2, 3}: as two
    irreps the candidates of round 1 are (irrep 0: 0, 1) over (irrep 1: 0),
    and each irrep's list keeps the hand-worked order."""
    v0 = HAND_V[np.ix_([0, 1, 4], [0, 1, 4])]
    v1 = HAND_V[np.ix_([2, 3], [2, 3])]
    piv, _ = cd_basis([v0, v1], 0.5, sigma=0.5, qmax=2)
    assert piv[0].tolist() == [0, 1, 2]
    assert piv[1].tolist() == [0, 1]
