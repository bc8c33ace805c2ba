"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle."""
import numpy as np
import pytest

import oracle as O
import synth as S
from oracle.layout import OracleLayout
from tests.gpu_support import blocks, device_problem, oracle_result, problem, run

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12      # normwise relative, max and Frobenius

SMALL = [
    ("c1_tiny", ([2], [5], [3])),
    ("c2_ragged", ([3, 1], [7, 5], [9, 4])),
    ("c2v_empty_irreps", ([2, 0, 1, 1], [6, 3, 0, 5], [5, 0, 4, 2])),
    ("d2h_uneven", ([1, 2, 1, 0, 1, 1, 0, 2], [5, 3, 4, 2, 6, 0, 3, 2], [4, 3, 0, 2, 5, 1, 3, 0])),
    ("d2h_cd_only_sym", ([2, 1, 1, 1, 1, 1, 1, 1], [9, 4, 6, 3, 7, 2, 4, 3], [40, 0, 0, 0, 0, 0, 0, 0])),
    ("c1_tiles_ragged", ([5], [37], [70])),
]


def _check(got, ref, tol, what):
    mx, fro = O.rel_errors(got, ref)
    assert np.isfinite(mx) and mx <= tol and fro <= tol, f"{what}: max {mx:.3e} fro {fro:.3e}"
    return mx, fro


@pytest.mark.parametrize("name,spec", SMALL)
@pytest.mark.parametrize("symB", [True, False])
def test_t2_small_fp64(gpu_lib, name, spec, symB):
    prob = problem(S.sym_custom(*spec), seed=7, symmetric_B=symB)
    d = device_problem(gpu_lib, prob)
    run(gpu_lib, d)
    _check(blocks(d), oracle_result(prob), FP64_TOL, name)


@pytest.mark.parametrize("name,spec", SMALL)
@pytest.mark.parametrize("dressed", [True, False])
def test_lambda_small_fp64(gpu_lib, name, spec, dressed):
    prob = problem(S.sym_custom(*spec), seed=8, kind="lambda", symmetric_B=False, dressed=dressed)
    d = device_problem(gpu_lib, prob)
    run(gpu_lib, d, kind="lambda")
    _check(blocks(d), oracle_result(prob), FP64_TOL, name)


def test_t2_c1_small_fp64_with_epilogue(gpu_lib):
    """o=8, v=40, 300 vectors: result, R/D and pair energies."""
    prob = problem(S.sym_c1_small(), seed=0)
    d = device_problem(gpu_lib, prob, want_delta=True, want_energy=True)
    run(gpu_lib, d)
    ref = oracle_result(prob)
    _check(blocks(d), ref, FP64_TOL, "R")
    lay = OracleLayout(prob["sym"])
    Rf = lay.full_amp(ref)
    eo, ev = np.concatenate(prob["eps_occ"]), np.concatenate(prob["eps_vir"])
    dref = lay.blocks_from_full(O.denominator_update_full(Rf, eo, ev) * lay.allowed_mask())
    _check(blocks(d, "delta"), dref, FP64_TOL, "delta")
    e_ref = O.pair_energies_full(lay.full_amp(prob["X"]), Rf)
    e_got = d["pair_energy"].cpu().numpy().reshape(e_ref.shape)
    assert np.max(np.abs(e_got - e_ref)) <= 1e-12 * max(1.0, np.max(np.abs(e_ref)))


@pytest.mark.parametrize("reading", ["A", "B"])
def test_t2_d2h_medium_fp64(gpu_lib, reading):
    """8 irreps, o=20, v=200, 1500 vectors (all in the totally symmetric irrep,
    or split evenly), with R/D and pair energies."""
    _check_epilogue(gpu_lib, problem(S.sym_d2h_medium(reading), seed=0), "t2", "fp64")


def _check_epilogue(cdcc, prob, kind, precision):
    """Result, R/D and pair energies of one call against the oracle (blocks:
    no full tensors)."""
    d = device_problem(cdcc, prob, want_delta=True, want_energy=True)
    run(cdcc, d, kind=kind, precision=precision)
    sym = prob["sym"]
    ref = oracle_result(prob)
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    mx, fro = _check(blocks(d), ref, tol, f"{kind} {precision} R")
    _check(blocks(d, "delta"), O.denominator_update_blocks(sym, ref, prob["eps_occ"], prob["eps_vir"]), tol,
           f"{kind} {precision} R/D")
    e_ref = O.pair_energies_blocks(sym, prob["X"], ref)
    err_e = float(np.max(np.abs(d["pair_energy"].cpu().numpy().reshape(e_ref.shape) - e_ref)))
    if precision == "fp64":
        assert err_e <= 1e-12 * max(1.0, float(np.max(np.abs(e_ref))))
    else:
        assert err_e <= PAIR_TOL, err_e
    return mx, fro, err_e, d


@pytest.mark.parametrize("reading", ["A", "B"])
def test_lambda_d2h_medium_fp64(gpu_lib, reading):
    """The T1-dressed Lambda ladder on the o=20/v=200 workload: Z, Z/D and
    pair energies."""
    _check_epilogue(gpu_lib, problem(S.sym_d2h_medium(reading), seed=0, kind="lambda"), "lambda", "fp64")


def test_batch_bytes_and_tile_classes_agree(gpu_lib):
    """A tiny batch cap (many bounded batches) and every tile class give the
    same result as the default plan, bitwise."""
    prob = problem(S.sym_custom([3, 2], [21, 14], [50, 31]), seed=3)
    d0 = device_problem(gpu_lib, prob)
    run(gpu_lib, d0)
    r0 = d0["R"].cpu().numpy()
    for kw in ({"batch_bytes": 1 << 16}, {"tile_policy": 1}, {"tile_policy": 2}, {"tile_policy": 3}):
        d = device_problem(gpu_lib, prob)
        run(gpu_lib, d, **kw)
        assert np.array_equal(d["R"].cpu().numpy(), r0), kw


def test_batched_systems_equal_alone(gpu_lib):
    """Several systems of different shapes in one call: each result equals the
    result of the same system alone (bitwise) and the oracle."""
    syms = S.batch_syms(6, seed=1)
    probs = [problem(s, seed=k) for k, s in enumerate(syms)]
    ds = [device_problem(gpu_lib, p) for p in probs]
    run(gpu_lib, ds)
    for p, d in zip(probs, ds):
        alone = device_problem(gpu_lib, p)
        run(gpu_lib, alone)
        assert np.array_equal(alone["R"].cpu().numpy(), d["R"].cpu().numpy())
        _check(blocks(d), oracle_result(p), FP64_TOL, str(p["sym"]))


def test_repeatable_bitwise(gpu_lib):
    prob = problem(S.sym_d2h_medium("B"), seed=4)
    d = device_problem(gpu_lib, prob)
    run(gpu_lib, d)
    r1 = d["R"].cpu().numpy()
    run(gpu_lib, d)
    assert np.array_equal(r1, d["R"].cpu().numpy())


def _pair_symmetric_blocks(sym, Rb):
    """R_ij^ab = R_ji^ba bitwise, block by block (block (G, gi, ga) against
    block (G, gj, gb) with both pairs swapped): no full tensor is formed."""
    h = sym["h"]
    for G in range(h):
        for gi in range(h):
            for ga in range(h):
                a, b = Rb[(G, gi, ga)], Rb[(G, gi ^ G, ga ^ G)]
                if a.size and not np.array_equal(a, b.transpose(1, 0, 3, 2)):
                    return False
    return True


_LARGE = {}


def _d2h_large_reference():
    """The o=40/v=400/N=3000 T2 problem and its oracle result, pair energies
    and R/D, computed once per session (about half a minute of host BLAS)."""
    if not _LARGE:
        prob = problem(S.sym_d2h_large(), seed=0)
        sym = prob["sym"]
        ref = O.t2_ladder_blocks(sym, prob["B"], prob["X"])
        _LARGE.update(prob=prob, ref=ref, e=O.pair_energies_blocks(sym, prob["X"], ref),
                      delta=O.denominator_update_blocks(sym, ref, prob["eps_occ"], prob["eps_vir"]))
    return _LARGE


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_i8"])
def test_t2_d2h_large_full(gpu_lib, precision):
    """o=40, v=400, 3000 vectors (8 irreps) at full size, every element
    against the oracle: R and R/D normwise (1e-12 FP64, 1e-7 split paths),
    pair energies (1e-12 relative FP64, 1e-8 Eh split paths: the tightest
    gate at this size, where |e_ij| is largest), R_ij^ab = R_ji^ba bitwise
    over the whole tensor."""
    L = _d2h_large_reference()
    prob, ref = L["prob"], L["ref"]
    d = device_problem(gpu_lib, prob, want_delta=True, want_energy=True)
    run(gpu_lib, d, precision=precision)
    tol = FP64_TOL if precision == "fp64" else 1e-7
    got = blocks(d)
    mx, fro = _check(got, ref, tol, f"R {precision}")
    _check(blocks(d, "delta"), L["delta"], tol, f"R/D {precision}")
    assert _pair_symmetric_blocks(prob["sym"], got)
    e_got = d["pair_energy"].cpu().numpy().reshape(L["e"].shape)
    err_e = float(np.max(np.abs(e_got - L["e"])))
    print(f"d2h_large {precision}: max {mx:.2e} fro {fro:.2e} pair-energy {err_e:.2e} Eh "
          f"(max |e_ij| {np.max(np.abs(L['e'])):.3f})")
    if precision == "fp64":
        assert err_e <= 1e-12 * max(1.0, float(np.max(np.abs(L["e"]))))
    else:
        assert err_e <= 1e-8


_LARGE_LAMBDA = {}


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_i8"])
def test_lambda_d2h_large_full(gpu_lib, precision):
    """The T1-dressed Lambda ladder at o=40, v=400, 3000 vectors (8 irreps;
    a stack of 750 per irrep with its subtracted half), every element
    against the oracle (computed once per session, about half a minute of
    host BLAS): Z and Z/D normwise (1e-12 FP64, 1e-7 split paths), pair
    energies (1e-12 relative FP64, 1e-8 Eh split paths), Z_ij^ab = Z_ji^ba
    bitwise."""
    if not _LARGE_LAMBDA:
        prob = problem(S.sym_d2h_large(), seed=0, kind="lambda")
        sym = prob["sym"]
        ref = oracle_result(prob)
        _LARGE_LAMBDA.update(prob=prob, ref=ref, e=O.pair_energies_blocks(sym, prob["X"], ref),
                             delta=O.denominator_update_blocks(sym, ref, prob["eps_occ"], prob["eps_vir"]))
    L = _LARGE_LAMBDA
    prob, ref = L["prob"], L["ref"]
    d = device_problem(gpu_lib, prob, want_delta=True, want_energy=True)
    run(gpu_lib, d, kind="lambda", precision=precision)
    tol = FP64_TOL if precision == "fp64" else 1e-7
    got = blocks(d)
    mx, fro = _check(got, ref, tol, f"Z {precision}")
    _check(blocks(d, "delta"), L["delta"], tol, f"Z/D {precision}")
    assert _pair_symmetric_blocks(prob["sym"], got)
    e_got = d["pair_energy"].cpu().numpy().reshape(L["e"].shape)
    err_e = float(np.max(np.abs(e_got - L["e"])))
    print(f"d2h_large lambda {precision}: max {mx:.2e} fro {fro:.2e} pair-energy {err_e:.2e} Eh "
          f"(max |e_ij| {np.max(np.abs(L['e'])):.3f})")
    if precision == "fp64":
        assert err_e <= 1e-12 * max(1.0, float(np.max(np.abs(L["e"]))))
    else:
        assert err_e <= 1e-8


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_t2_d2h_large_one_batch_equals_four(gpu_lib, precision):
    """The o=40/v=400 intermediate (about 14 GB) runs as one batch under the
    default cap and as four under a 4 GiB cap; R and the pair energies are
    bitwise the same."""
    prob = _LARGE["prob"] if _LARGE else problem(S.sym_d2h_large(), seed=0)
    out = []
    for kw in ({}, {"batch_bytes": 4 << 30}):
        d = device_problem(gpu_lib, prob, want_energy=True)
        run(gpu_lib, d, precision=precision, **kw)
        out.append((d["R"].cpu().numpy(), d["pair_energy"].cpu().numpy()))
        del d
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def _workspace_bytes(sym, precision, batch_bytes=0):
    """Device bytes of a T2 call on this system.  The size query reads the
    layout and the options only, so the data pointers are placeholders."""
    import ctypes
    from paper_2512_21909_amd import Layout, _lib
    lay = Layout(sym)
    P = _lib.Problem()
    P.lay = ctypes.pointer(lay.c)
    P.B = P.X = P.R = ctypes.c_void_p(1 << 12)
    o = _lib.Opts()
    o.precision = {"fp64": _lib.FP64, "mixed": _lib.MIXED, "mixed_i8": _lib.MIXED_I8}[precision]
    o.batch_bytes = batch_bytes
    out = ctypes.c_int64(0)
    _lib.check(_lib.load().cdcc_workspace_bytes(1, ctypes.byref(P), ctypes.byref(o), 0, ctypes.byref(out)),
               "cdcc_workspace_bytes")
    return out.value


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_i8"])
def test_default_batch_rule(gpu_lib, precision):
    """Default batch cap: one batch when the whole (ac|bd) intermediate fits
    16 GiB (o=40/v=400: about 14 GB, so the workspace exceeds that of a 4 GiB
    cap by most of it), else batches of at most 4 GiB (o=135/v=543: the
    default plan takes exactly the workspace of an explicit 4 GiB cap)."""
    big = _workspace_bytes(S.sym_d2h_large(), precision)
    capped = _workspace_bytes(S.sym_d2h_large(), precision, 4 << 30)
    assert big - capped > 8e9 and big < capped + (16 << 30)
    hbc = S.sym_hbc_shape()
    assert _workspace_bytes(hbc, precision) == _workspace_bytes(hbc, precision, 4 << 30)


# ---------------------------------------------------------------- mixed path
MIXED_TOL = 1e-7      # normwise relative
PAIR_TOL = 1e-8       # Eh, absolute


def _pair_energy_err(d, prob, ref):
    lay = OracleLayout(prob["sym"])
    e_ref = O.pair_energies_full(lay.full_amp(prob["X"]), lay.full_amp(ref))
    e_got = d["pair_energy"].cpu().numpy().reshape(e_ref.shape)
    return float(np.max(np.abs(e_got - e_ref)))


SPLIT = ["mixed", "mixed_i8"]   # split-BF16 slices; 8-bit digits with int32 accumulation


def _assert_pair_symmetric(sym, got):
    """R_ij^ab = R_ji^ba bitwise over the whole tensor: one (S, A) pair gives
    both elements, and A is exactly zero on the a = b columns."""
    full = OracleLayout(sym).full_amp(got)
    assert np.array_equal(full, full.transpose(1, 0, 3, 2))


@pytest.mark.parametrize("name,spec", SMALL)
@pytest.mark.parametrize("kind", ["t2", "lambda"])
@pytest.mark.parametrize("precision", SPLIT)
def test_mixed_small(gpu_lib, name, spec, kind, precision):
    prob = problem(S.sym_custom(*spec), seed=9, kind=kind, symmetric_B=False)
    d = device_problem(gpu_lib, prob, want_energy=True)
    run(gpu_lib, d, kind=kind, precision=precision)
    ref = oracle_result(prob)
    got = blocks(d)
    _check(got, ref, MIXED_TOL, name)
    _assert_pair_symmetric(prob["sym"], got)
    assert _pair_energy_err(d, prob, ref) <= PAIR_TOL


@pytest.mark.parametrize("wl", ["c1_small", "d2h_medium_A", "d2h_medium_B"])
@pytest.mark.parametrize("kind", ["t2", "lambda"])
@pytest.mark.parametrize("precision", SPLIT)
def test_mixed_named_workloads(gpu_lib, wl, kind, precision):
    sym = {"c1_small": S.sym_c1_small(), "d2h_medium_A": S.sym_d2h_medium("A"),
           "d2h_medium_B": S.sym_d2h_medium("B")}[wl]
    prob = problem(sym, seed=0, kind=kind)
    mx, fro, err_e, d = _check_epilogue(gpu_lib, prob, kind, precision)
    _assert_pair_symmetric(sym, blocks(d))
    print(f"{wl} {kind} {precision}: max {mx:.2e} fro {fro:.2e} pair-energy {err_e:.2e} Eh")


@pytest.mark.parametrize("precision", SPLIT)
def test_mixed_batched_equal_alone(gpu_lib, precision):
    syms = S.batch_syms(5, seed=2)
    probs = [problem(s, seed=k) for k, s in enumerate(syms)]
    ds = [device_problem(gpu_lib, p) for p in probs]
    run(gpu_lib, ds, precision=precision)
    for p, d in zip(probs, ds):
        alone = device_problem(gpu_lib, p)
        run(gpu_lib, alone, precision=precision)
        assert np.array_equal(alone["R"].cpu().numpy(), d["R"].cpu().numpy())
        _check(blocks(d), oracle_result(p), MIXED_TOL, str(p["sym"]))


@pytest.mark.parametrize("precision", SPLIT)
@pytest.mark.parametrize("kind", ["t2", "lambda"])
def test_mixed_tile_classes_agree(gpu_lib, precision, kind):
    """Every assembly tile class of a split path gives bitwise the same result
    (classes change the tile decomposition, never an element's arithmetic)."""
    prob = problem(S.sym_custom([3, 2], [21, 14], [50, 31]), seed=3, kind=kind)
    d0 = device_problem(gpu_lib, prob)
    run(gpu_lib, d0, kind=kind, precision=precision)
    r0 = d0["R"].cpu().numpy()
    _check(blocks(d0), oracle_result(prob), MIXED_TOL, precision)
    for cls in (1, 2, 3, 4):
        d = device_problem(gpu_lib, prob)
        run(gpu_lib, d, kind=kind, precision=precision, tile_policy=cls)
        assert np.array_equal(d["R"].cpu().numpy(), r0), cls


@pytest.mark.parametrize("precision", SPLIT)
@pytest.mark.parametrize("kind", ["t2", "lambda"])
def test_mixed_long_cholesky_index(gpu_lib, precision, kind):
    """More than 32736 stacked Cholesky vectors (T2: N = 33000; Lambda: the
    dressed stack of 2 x 16500): the 8-bit path runs its K in segments (the
    int32 accumulators are exact for 32736 K at a time), the BF16 path
    flushes every 256 K."""
    n = 33000 if kind == "t2" else 16500
    prob = problem(S.sym_custom([2], [6], [n]), seed=5, kind=kind)
    d = device_problem(gpu_lib, prob, want_energy=True)
    run(gpu_lib, d, kind=kind, precision=precision)
    ref = oracle_result(prob)
    _check(blocks(d), ref, MIXED_TOL, f"{kind} N={n}")
    assert _pair_energy_err(d, prob, ref) <= PAIR_TOL


@pytest.mark.parametrize("spec", [([17], [24], [60]), ([23], [80], [40])])
@pytest.mark.parametrize("kind", ["t2", "lambda"])
@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_i8"])
def test_many_contraction_row_tiles(gpu_lib, spec, kind, precision):
    """More than 128 packed occupied pairs in C1 (o=17: 153 rows in three
    64-row contraction tiles per column block, listed together so that they
    share X; o=23, v=80: 276 rows in six 48-row tiles and the K table of
    3240 entries split in two segments, listed in blocks of 3 row tiles x 4
    column blocks of one segment, ragged at both edges).  Every element
    against the oracle."""
    prob = problem(S.sym_custom(*spec), seed=13, kind=kind)
    d = device_problem(gpu_lib, prob, want_energy=True)
    run(gpu_lib, d, kind=kind, precision=precision)
    ref = oracle_result(prob)
    _check(blocks(d), ref, FP64_TOL if precision == "fp64" else MIXED_TOL, f"{spec} {kind}")
    if precision != "fp64":
        assert _pair_energy_err(d, prob, ref) <= PAIR_TOL


@pytest.mark.parametrize("precision", SPLIT)
@pytest.mark.parametrize("kind", ["t2", "lambda"])
def test_split_paths_rows_of_subnormal_magnitude(gpu_lib, precision, kind):
    """Operand rows whose largest entry is subnormal (the row scale 2^e is
    then below 2^-1022): the slicing scales by ldexp, so the result stays
    finite and within the tolerance of the FP64 oracle."""
    sym = S.sym_custom([3, 2], [13, 9], [40, 23])
    prob = problem(sym, seed=14, kind=kind, dressed=False)
    B = {k: v.copy() for k, v in prob["B"].items()}
    for blk in B.values():
        if blk.shape[0] and blk.shape[1]:
            blk[0, :, :] *= 2.0 ** -1060      # every entry of these rows subnormal
    prob["B"] = B
    d = device_problem(gpu_lib, prob)
    run(gpu_lib, d, kind=kind, precision=precision)
    got = d["R"].cpu().numpy()
    assert np.all(np.isfinite(got))
    _check(blocks(d), oracle_result(prob), MIXED_TOL, kind)


def _digit_edge_B(sym, seed):
    """Cholesky vectors whose entries sit on the rounding edges of the 8-bit
    digit expansion (x in units of 1/128 of the row scale): exact halves
    (a tie, the next digit becomes -128), fractions that round the second
    digit up to +128 (a carry into the first), and one entry per row just
    below a power of two (the row scale moves up one binade)."""
    rng = np.random.default_rng([seed, 4242])
    out = {}
    for (gP, ga), blk in S.make_B(sym, seed, True).items():
        m0 = rng.integers(0, 127, size=blk.shape).astype(np.float64)
        kind = rng.integers(0, 3, size=blk.shape)
        frac = np.where(kind == 0, 0.5, np.where(kind == 1, 0.4990234375 + 2.0 ** -30, rng.random(blk.shape)))
        x = (m0 + frac) / 128.0 * np.where(rng.random(blk.shape) < 0.5, -1.0, 1.0)
        x = np.clip(x, -0.99, 0.99)
        if x.shape[-1]:
            x[..., 0] = 0.995 * np.sign(x[..., 0] + 0.5)
        out[(gP, ga)] = x * 2.0 ** int(rng.integers(-3, 4))
    return out


@pytest.mark.parametrize("kind", ["t2", "lambda"])
def test_mixed_i8_digit_edges(gpu_lib, kind):
    """Rounding ties, digit carries and row maxima just below a power of two
    in the operand: the 8-bit path stays within the mixed tolerance (its
    expansion is exact to 2^-32 of the row scale)."""
    sym = S.sym_custom([3, 2], [13, 9], [40, 23])
    prob = problem(sym, seed=6, kind=kind, dressed=False)
    prob["B"] = _digit_edge_B(sym, 6)
    d = device_problem(gpu_lib, prob)
    run(gpu_lib, d, kind=kind, precision="mixed_i8")
    mx, fro = _check(blocks(d), oracle_result(prob), MIXED_TOL, kind)
    assert mx <= 1e-8, mx


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_i8"])
def test_graph_replay_with_new_pointers(gpu_lib, precision):
    """The captured launch sequence is replayed for new buffers of the same
    shape: alternating calls on two inputs give each input's own result, and
    the graph path equals the direct launches bitwise."""
    import os
    import torch
    sym = S.sym_custom([2, 1, 1, 1], [9, 5, 7, 4], [30, 11, 6, 7])
    probs = [problem(sym, seed=s) for s in (21, 22)]
    ds = [device_problem(gpu_lib, p, want_energy=True) for p in probs]
    refs = [oracle_result(p) for p in probs]
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    first = []
    for rep in range(3):
        for d, ref in zip(ds, refs):
            d["R"].fill_(float("nan"))
            run(gpu_lib, d, precision=precision)
            _check(blocks(d), ref, tol, f"replay {rep}")
            if rep == 0:
                first.append(d["R"].cpu().numpy().copy())
            else:
                assert np.array_equal(d["R"].cpu().numpy(), first[ds.index(d)])
    os.environ["CDCC_GRAPH"] = "0"
    try:
        for d, f in zip(ds, first):
            d["R"].fill_(float("nan"))
            run(gpu_lib, d, precision=precision)
            assert np.array_equal(d["R"].cpu().numpy(), f)
    finally:
        del os.environ["CDCC_GRAPH"]
    torch.cuda.synchronize()


_B64 = {}
# systems whose plain oracle cost is below this are checked element by
# element (about two thirds of the 64; ~15 s of host BLAS in all)
B64_FULL_FLOPS = 2e10


def _plain_flops(sym):
    lay = OracleLayout(sym)
    return sum(2.0 * lay.n_oo[G] * lay.n_vv[G] ** 2 for G in range(lay.h))


def _batch64_reference():
    if not _B64:
        syms = S.batch_syms(64, seed=0)
        probs = [problem(s, seed=k) for k, s in enumerate(syms)]
        refs = {}
        for k, p in enumerate(probs):
            if _plain_flops(p["sym"]) <= B64_FULL_FLOPS:
                r = O.t2_ladder_blocks(p["sym"], p["B"], p["X"])
                refs[k] = (r, O.pair_energies_blocks(p["sym"], p["X"], r))
        _B64.update(probs=probs, refs=refs)
    return _B64


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_i8"])
def test_uneven_batch_of_64_systems(gpu_lib, precision):
    """64 systems (o in [5,20], v in [40,160], N = 7.5(o+v), 1/2/4/8 irreps
    with Dirichlet splits) in one batched call.  Systems the oracle affords in
    full (plain cost <= 2e10 flops): every element and the pair energies
    (1e-8 Eh on the split paths).  The others: 40 sampled elements each, and
    on the split paths pair energies within 1e-8 Eh of the FP64 path's.
    Every eighth system also equals its standalone result bitwise."""
    B = _batch64_reference()
    probs, refs = B["probs"], B["refs"]
    assert len(refs) >= 32
    ds = [device_problem(gpu_lib, p, want_energy=True) for p in probs]
    run(gpu_lib, ds, precision=precision)
    e64 = None
    if precision != "fp64":
        d64 = [device_problem(gpu_lib, p, want_energy=True) for p in probs]
        run(gpu_lib, d64, precision="fp64")
        e64 = [d["pair_energy"].cpu().numpy() for d in d64]
        del d64
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    rng = np.random.default_rng(77)
    for k, (p, d) in enumerate(zip(probs, ds)):
        R = d["R"].cpu().numpy()
        assert np.all(np.isfinite(R)), k
        if k % 8 == 0:
            alone = device_problem(gpu_lib, p)
            run(gpu_lib, alone, precision=precision)
            assert np.array_equal(alone["R"].cpu().numpy(), R), k
        lay, sym = d["layout"], p["sym"]
        Rb = lay.unpack_amp(R)
        e_got = d["pair_energy"].cpu().numpy()
        if k in refs:
            ref, e_ref = refs[k]
            _check(Rb, ref, tol, f"system {k}")
            err_e = float(np.max(np.abs(e_got.reshape(e_ref.shape) - e_ref))) if e_ref.size else 0.0
            assert err_e <= (1e-12 * max(1.0, float(np.max(np.abs(e_ref)))) if precision == "fp64" else PAIR_TOL), k
            continue
        if e64 is not None:
            assert float(np.max(np.abs(e_got - e64[k]))) <= PAIR_TOL, k
        scale = max(float(np.max(np.abs(b))) for b in Rb.values() if b.size)
        h, no, nv = sym["h"], sym["nocc"], sym["nvir"]
        for _ in range(40):
            G, gi, ga = (int(x) for x in rng.integers(0, h, 3))
            gj, gb = gi ^ G, ga ^ G
            if not (no[gi] and no[gj] and nv[ga] and nv[gb]):
                continue
            i, j = int(rng.integers(no[gi])), int(rng.integers(no[gj]))
            a, b = int(rng.integers(nv[ga])), int(rng.integers(nv[gb]))
            ref = O.element_t2(sym, p["B"], p["X"], lay.occ_off[gi] + i, lay.occ_off[gj] + j,
                               lay.vir_off[ga] + a, lay.vir_off[gb] + b)
            assert abs(Rb[(G, gi, ga)][i, j, a, b] - ref) <= tol * scale, (k, G, gi, ga)


# ------------------------------------------------------------ dressing once
def _oracle_stack(sym, prob):
    """U of cdcc_lambda_dress from the oracle's t^P_ea (Appendix A): per
    (GP, Ga) block, rows (a, e), [B^P_ea - t^P_ea | t^P_ea], flattened like
    the library's layout."""
    import oracle as O
    lay = OracleLayout(sym)
    Bf, Bvof, t1f = lay.full_B(prob["B"]), lay.full_Bvo(prob["Bvo"]), lay.full_t1(prob["t1"])
    tP = O.t1_dressing_full(Bvof, t1f)                 # [P, e, a] = sum_m t_m^e L^P_am
    h, nv, nc = sym["h"], sym["nvir"], sym["ncd"]
    vo = np.concatenate([[0], np.cumsum(nv)]).astype(int)
    po = np.concatenate([[0], np.cumsum(nc)]).astype(int)
    out = []
    for gP in range(h):
        for ga in range(h):
            ge = ga ^ gP
            a_sl, e_sl, p_sl = slice(vo[ga], vo[ga + 1]), slice(vo[ge], vo[ge + 1]), slice(po[gP], po[gP + 1])
            b = Bf[p_sl, e_sl, a_sl].transpose(2, 1, 0)    # [a, e, P] = B^P_ea
            t = tP[p_sl, e_sl, a_sl].transpose(2, 1, 0)    # [a, e, P] = t^P_ea
            out.append(np.concatenate([b - t, t], axis=2).ravel())
    return np.concatenate(out)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_i8"])
def test_lambda_with_stack_built_once(gpu_lib, precision):
    """cdcc_lambda_dress builds the dressed stack once (checked element by
    element against the oracle's t^P_ea); Lambda calls that pass it match the
    oracle and, in FP64, the call that dresses from Bvo and t1 bitwise; two
    systems in one batched call."""
    import torch
    cdcc = gpu_lib
    specs = [([2, 1, 1, 1], [9, 5, 7, 4], [30, 11, 6, 7]), ([3, 2], [21, 14], [50, 31])]
    probs = [problem(S.sym_custom(*sp), seed=60 + k, kind="lambda", symmetric_B=False) for k, sp in enumerate(specs)]
    ds, with_u = [], []
    for p in probs:
        d = device_problem(cdcc, p, want_energy=True)
        lay = d["layout"]
        u = torch.full((2 * lay.b_size,), float("nan"), dtype=torch.float64, device="cuda")
        cdcc.lambda_dress({"layout": lay, "B": d["B"], "Bvo": d["Bvo"], "t1": d["t1"], "U": u})
        torch.cuda.synchronize()
        ref_u = _oracle_stack(p["sym"], p)
        got_u = u.cpu().numpy()
        mask = np.isfinite(got_u)
        assert mask.sum() == ref_u.size or np.all(ref_u[~mask] == 0)  # only empty blocks stay unwritten
        np.testing.assert_allclose(got_u[mask], ref_u[mask], rtol=0, atol=1e-14 * np.abs(ref_u).max())
        e = device_problem(cdcc, p, want_energy=True)
        e_u = dict(e)
        e_u.pop("Bvo"), e_u.pop("t1")
        e_u["U"] = u
        ds.append(d)
        with_u.append(e_u)
    run(cdcc, ds, kind="lambda", precision=precision)           # dressed from Bvo and t1
    run(cdcc, with_u, kind="lambda", precision=precision)       # the prebuilt stack
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    for p, d, e in zip(probs, ds, with_u):
        ref = oracle_result(p)
        _check(blocks(e), ref, tol, "stack")
        if precision == "fp64":
            assert np.array_equal(e["R"].cpu().numpy(), d["R"].cpu().numpy())
        else:
            assert _pair_energy_err(e, p, ref) <= PAIR_TOL


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kind", ["t2", "lambda"])
def test_pair_energy_from_other_amplitudes(gpu_lib, kind, precision):
    """energy_amps: the pair energies weight R with a caller-given
    pair-symmetric tensor T (here the amplitudes of another seed) in place of
    X; R itself is bitwise unchanged by the option, and without it X is used."""
    from tests.gpu_support import to_dev
    prob = problem(S.sym_custom([3, 2], [21, 14], [50, 31]), seed=8, kind=kind)
    other = problem(prob["sym"], seed=9)["X"]
    d0 = device_problem(gpu_lib, prob, want_energy=True)
    run(gpu_lib, d0, kind=kind, precision=precision)
    d = device_problem(gpu_lib, prob, want_energy=True)
    d["energy_amps"] = to_dev(d["layout"].pack_amp(other))
    run(gpu_lib, d, kind=kind, precision=precision)
    assert np.array_equal(d["R"].cpu().numpy(), d0["R"].cpu().numpy())
    ref = oracle_result(prob)
    lay = OracleLayout(prob["sym"])
    Rf = lay.full_amp(ref)
    for dd, amps in ((d, other), (d0, prob["X"])):
        e_ref = O.pair_energies_full(lay.full_amp(amps), Rf)
        e_got = dd["pair_energy"].cpu().numpy().reshape(e_ref.shape)
        tol = 1e-12 * max(1.0, np.max(np.abs(e_ref))) if precision == "fp64" else PAIR_TOL
        assert np.max(np.abs(e_got - e_ref)) <= tol


def test_pair_energy_after_a_call_without(gpu_lib):
    """A call of the same shape without pair energies first: its cached plan
    holds no pair-energy work, and the next call, which asks for them, must
    not reuse it (regression test: the energies were left unwritten)."""
    prob = problem(S.sym_custom([2, 2], [9, 7], [23, 19]), seed=4)
    run(gpu_lib, device_problem(gpu_lib, prob))
    d = device_problem(gpu_lib, prob, want_energy=True)
    run(gpu_lib, d)
    assert _pair_energy_err(d, prob, oracle_result(prob)) <= 1e-12


@pytest.mark.parametrize("precision", SPLIT)
@pytest.mark.parametrize("kind", ["t2", "lambda"])
@pytest.mark.parametrize("spec", [([2, 1], [9, 7], [5, 17]), ([1], [5], [16500])])
def test_split_tile_classes_short_and_long_k(gpu_lib, spec, kind, precision):
    """Every split tile class, forced, on K of one to three 16-wide blocks
    (5 and 17 vectors: the K loops' tails) and on K far beyond the 256-wide
    flush interval (16500 vectors; 33000 stacked for Lambda): bitwise equal
    across classes and within the mixed tolerance of the oracle."""
    prob = problem(S.sym_custom(*spec), seed=21, kind=kind)
    ref = oracle_result(prob)
    r0 = None
    for cls in (1, 2, 3, 4):
        d = device_problem(gpu_lib, prob)
        run(gpu_lib, d, kind=kind, precision=precision, tile_policy=cls)
        r = d["R"].cpu().numpy()
        if r0 is None:
            r0 = r
            _check(blocks(d), ref, MIXED_TOL, f"{spec} {kind} class {cls}")
        else:
            assert np.array_equal(r, r0), cls
