"""Input generators: pinned splits, determinism, selection rules, recipe."""
import numpy as np

import synth as S
from oracle.layout import OracleLayout


def test_large_split_pinned():
    # exact rational largest remainder, ties to the lowest irrep
    assert S.largest_remainder_split(40, S.SPLIT_D2H) == [8, 5, 6, 4, 6, 4, 4, 3]
    assert S.largest_remainder_split(400, S.SPLIT_D2H) == [80, 44, 60, 40, 64, 36, 44, 32]
    assert S.largest_remainder_split(30, S.SPLIT_D2H) == [6, 3, 5, 3, 5, 3, 3, 2]
    assert S.largest_remainder_split(300, S.SPLIT_D2H) == [60, 33, 45, 30, 48, 27, 33, 24]
    assert S.largest_remainder_split(3000, [1] * 8) == [375] * 8
    assert S.largest_remainder_split(7, [1, 1, 1]) == [3, 2, 2]


def test_pair_counts_of_the_configs():
    lay2 = OracleLayout(S.sym_d2h_medium())
    assert lay2.n_oo == [54, 48, 52, 48, 52, 48, 50, 48]
    assert lay2.n_vv == [5472, 4816, 5264, 4736, 5312, 4688, 5104, 4608]
    lay3 = OracleLayout(S.sym_d2h_large())
    assert lay3.n_oo == [218, 200, 208, 192, 208, 192, 198, 184]
    assert lay3.n_vv == [21888, 19264, 21056, 18944, 21248, 18752, 20416, 18432]


def test_determinism_and_recipe():
    sym = S.sym_custom([2, 1], [3, 2], [5, 4])
    p1 = S.make_problem(sym, seed=3, kind="t2")
    p2 = S.make_problem(sym, seed=3, kind="t2")
    for k in p1["B"]:
        assert np.array_equal(p1["B"][k], p2["B"][k])
    for k in p1["X"]:
        assert np.array_equal(p1["X"][k], p2["X"][k])
    # symmetric B: B^P_ac = B^P_ca across blocks
    for (gP, ga), blk in p1["B"].items():
        gc = ga ^ gP
        assert np.array_equal(blk, p1["B"][(gP, gc)].transpose(1, 0, 2))
    # exact pair symmetry of tau
    lay = OracleLayout(sym)
    tf = lay.full_amp(p1["X"])
    assert np.array_equal(tf, tf.transpose(1, 0, 3, 2))
    assert np.all(tf[~lay.allowed_mask()] == 0)
    eo, ev = p1["eps_occ"], p1["eps_vir"]
    assert all(np.all((x >= -2) & (x <= -0.5)) for x in eo)
    assert all(np.all((x >= 0.2) & (x <= 3)) for x in ev)


def test_batch_shapes():
    syms = S.batch_syms(64, seed=0)
    assert len(syms) == 64
    for s in syms:
        o, v = sum(s["nocc"]), sum(s["nvir"])
        assert 5 <= o <= 20 and 40 <= v <= 160
        assert sum(s["ncd"]) == (15 * (o + v) + 1) // 2
        assert s["h"] in (1, 2, 4, 8)
    assert S.batch_syms(4, seed=0) == syms[:4]


def test_oracle_layout_roundtrip():
    sym = S.sym_custom([1, 2, 0, 1], [3, 2, 4, 1], [2, 0, 3, 1])
    lay = OracleLayout(sym)
    p = S.make_problem(sym, seed=1)
    flat = lay.pack_amp(p["X"])
    assert flat.size == lay.amp_size == sum(a * b for a, b in zip(lay.n_oo, lay.n_vv))
    back = lay.unpack_amp(flat)
    for k in p["X"]:
        assert np.array_equal(back[k], p["X"][k])
    assert lay.pack_B(p["B"]).size == lay.b_size
