"""Pins of the two-step Cholesky decomposition oracle: the decomposition
error bound, exact reproduction of the pivot rows, reduction to textbook
greedy pivoted Cholesky for Q_max = 1, full and exact-low-rank cases,
invariance under reordering of the pairs, irrep blocks kept apart."""
import numpy as np
import pytest

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
