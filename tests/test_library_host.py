"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol the header declares, its layout matches the oracle's independent
layout, its flop count matches brute enumeration, and bad arguments are
rejected before any device work."""
import ctypes
import itertools
import os
import re

import numpy as np
import pytest

import synth as S
from oracle.layout import OracleLayout

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2512_21909_amd import _lib
    return _lib


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "cdcc.h")).read()
    declared = set(re.findall(r"^\s*(?:int|const char \*)\s*(cdcc_\w+)\s*\(", hdr, re.M))
    assert declared == set(lib.EXPORTS)
    L = lib.load()
    for name in declared:
        assert hasattr(L, name), name


def test_struct_sizes_match_header(lib):
    # 4 + 3*8*4 = 100 -> padded to 104 by the following int64 arrays
    assert ctypes.sizeof(lib.Sym) == 100
    assert ctypes.sizeof(lib.LayoutC) == 104 + 8 * (5 * 8 + 4 * 64 + 4 * 8 + 7)
    assert ctypes.sizeof(lib.Problem) == 12 * 8
    assert ctypes.sizeof(lib.DressProblem) == 5 * 8
    assert ctypes.sizeof(lib.Opts) == 24


SPECS = [
    ([8], [40], [300]),
    ([2, 1], [3, 4], [3, 2]),
    ([1, 2, 0, 1], [3, 2, 4, 1], [2, 0, 3, 1]),
    ([4, 2, 3, 2, 3, 2, 2, 2], [40, 22, 30, 20, 32, 18, 22, 16], [1500, 0, 0, 0, 0, 0, 0, 0]),
    ([0, 1, 1, 0, 2, 0, 1, 1], [2, 0, 1, 2, 0, 2, 1, 3], [0, 1, 0, 2, 1, 1, 0, 2]),
]


@pytest.mark.parametrize("spec", SPECS)
def test_layout_matches_oracle_layout(spec):
    from paper_2512_21909_amd import Layout
    sym = S.sym_custom(*spec)
    L, O = Layout(sym), OracleLayout(sym)
    assert L.n_oo == O.n_oo and L.n_vv == O.n_vv
    assert L.amp_off == O.amp_off and L.oo_off == O.oo_off and L.vv_off == O.vv_off
    assert L.b_off == O.b_off and L.bvo_off == O.bvo_off and L.t1_off == O.t1_off
    assert [L.amp_size, L.b_size, L.bvo_size, L.t1_size] == [O.amp_size, O.b_size, O.bvo_size, O.t1_size]
    assert L.occ_off == O.occ_off and L.vir_off == O.vir_off and L.cd_off == O.cd_off
    # packed pair counts by enumeration of x>=y in orbital order
    io = np.concatenate([[g] * n for g, n in enumerate(sym["nocc"])]).astype(int)
    iv = np.concatenate([[g] * n for g, n in enumerate(sym["nvir"])]).astype(int)
    for G in range(sym["h"]):
        assert L.n_oo_pk[G] == sum(1 for x in range(len(io)) for y in range(x + 1) if io[x] ^ io[y] == G)
        assert L.n_vv_pk[G] == sum(1 for x in range(len(iv)) for y in range(x + 1) if iv[x] ^ iv[y] == G)
    # round trip through the library's packing equals the oracle's packing
    p = S.make_problem(sym, seed=2)
    assert np.array_equal(L.pack_amp(p["X"]), O.pack_amp(p["X"]))
    assert np.array_equal(L.pack_B(p["B"]), O.pack_B(p["B"]))


def _brute_flops(sym, kind):
    """Enumerate every multiply-add of the stored-half algorithm."""
    h, no, nv, nc = sym["h"], sym["nocc"], sym["nvir"], sym["ncd"]
    io = [g for g in range(h) for _ in range(no[g])]
    iv = [g for g in range(h) for _ in range(nv[g])]
    kap = 1 if kind == 0 else 2
    fw = fc = fd = 0
    V = len(iv)
    for a in range(V):
        for b in range(a + 1):
            for c in range(V):
                for d in range(V):
                    if iv[a] ^ iv[b] ^ iv[c] ^ iv[d]:
                        continue
                    fw += 2 * kap * nc[iv[a] ^ iv[c]]
    for i in range(len(io)):
        for j in range(i + 1):
            for a in range(V):
                for b in range(a + 1):
                    for c in range(V):
                        for d in range(c + 1):
                            if io[i] ^ io[j] ^ iv[a] ^ iv[b] or iv[c] ^ iv[d] ^ iv[a] ^ iv[b]:
                                continue
                            ga, gc, gd = iv[a], iv[c], iv[d]
                            # the irrep-ordered pair (c>=d by irrep) decides which W block
                            if nc[ga ^ gc] == 0 and nc[ga ^ gd] == 0:
                                continue
                            fc += 2
                            if i != j and a != b and c != d:
                                fc += 2
    if kind == 2:
        for gP in range(h):
            for ga in range(h):
                ge = ga ^ gP
                fd += 2 * no[ge] * nv[ge] * nv[ga] * nc[gP]
    return fw, fc, fd


@pytest.mark.parametrize("spec", SPECS[1:3] + SPECS[4:])
@pytest.mark.parametrize("kind", [0, 1, 2])
def test_flops_match_enumeration(spec, kind):
    from paper_2512_21909_amd import Layout
    sym = S.sym_custom(*spec)
    got = Layout(sym).flops(kind)
    assert tuple(int(round(x)) for x in got) == _brute_flops(sym, kind)


def test_flops_of_the_named_workloads():
    from paper_2512_21909_amd import Layout
    f = lambda s, k: sum(Layout(s).flops(k))
    assert f(S.sym_c1_small(), 0) == pytest.approx(8.70e8, rel=2e-3)
    assert f(S.sym_c1_small(), 2) == pytest.approx(1.67e9, rel=5e-3)  # table rounds 1.6646e9 up
    assert f(S.sym_d2h_medium(), 0) == pytest.approx(4.65e10, rel=2e-3)
    assert f(S.sym_d2h_medium(), 2) == pytest.approx(9.17e10, rel=2e-3)
    assert f(S.sym_d2h_large(), 0) == pytest.approx(1.53e12, rel=2e-3)
    assert f(S.sym_serving_large(), 0) == pytest.approx(3.77e11, rel=2e-3)


def test_error_codes_before_device_work(lib):
    L = lib.load()
    s = lib.Sym()
    out = lib.LayoutC()
    s.nirrep = 3
    assert L.cdcc_irrep_layout(ctypes.byref(s), ctypes.byref(out)) == lib.EUNSUPPORTED
    s.nirrep = 2
    s.nocc[0] = -1
    assert L.cdcc_irrep_layout(ctypes.byref(s), ctypes.byref(out)) == lib.EINVAL
    assert L.cdcc_irrep_layout(None, ctypes.byref(out)) == lib.EINVAL
    assert L.cdcc_ladder_t2(0, None, None, None) == lib.EINVAL
    assert L.cdcc_ladder_lambda(-1, None, None, None) == lib.EINVAL
    # a problem with a missing required pointer
    s.nocc[0] = 1
    assert L.cdcc_irrep_layout(ctypes.byref(s), ctypes.byref(out)) == lib.OK
    arr = (lib.Problem * 1)()
    arr[0].lay = ctypes.pointer(out)
    assert L.cdcc_ladder_t2(1, arr, None, None) == lib.EINVAL
    arr[0].B = arr[0].X = arr[0].R = ctypes.c_void_p(0x1000)
    arr[0].delta = ctypes.c_void_p(0x2000)  # delta without orbital energies
    assert L.cdcc_ladder_t2(1, arr, None, None) == lib.EINVAL
    arr[0].delta = None
    arr[0].t1 = ctypes.c_void_p(0x3000)     # t1 without Bvo
    assert L.cdcc_ladder_lambda(1, arr, None, None) == lib.EINVAL
    o = lib.Opts()
    o.precision = 7
    assert L.cdcc_ladder_t2(1, arr, ctypes.byref(o), None) == lib.EINVAL
    o.precision, o.tile_policy = lib.FP64, 4      # class 4 exists only on the split paths
    assert L.cdcc_ladder_t2(1, arr, ctypes.byref(o), None) == lib.EINVAL
    o.tile_policy = 5
    for prec in (lib.MIXED, lib.MIXED_I8):
        o.precision = prec
        assert L.cdcc_ladder_t2(1, arr, ctypes.byref(o), None) == lib.EINVAL
    assert L.cdcc_status_string(lib.ENOMEM).decode().startswith("device workspace")


# ---------------------------------------------------------------- vvvv density
def _brute_density_flops(sym):
    h, no, nv, nc = sym["h"], sym["nocc"], sym["nvir"], sym["ncd"]
    irr_v = [g for g in range(h) for _ in range(nv[g])]
    irr_o = [g for g in range(h) for _ in range(no[g])]
    irr_p = [g for g in range(h) for _ in range(nc[g])]
    n_oo = [sum(1 for m in irr_o for n in irr_o if m ^ n == G) for G in range(h)]
    fv = fl = 0
    for a in irr_v:
        for c in irr_v:
            gP = a ^ c
            if nc[gP] == 0:
                continue
            for b in irr_v:
                for d in irr_v:
                    if b ^ d != gP:
                        continue
                    fv += 4 * n_oo[a ^ b]
                    fl += 2 * sum(1 for p in irr_p if p == gP)
    return fv, fl


@pytest.mark.parametrize("spec", [SPECS[1], SPECS[2], SPECS[4], ([1, 0], [3, 2], [2, 2])])
def test_density_flops_match_enumeration(spec):
    from paper_2512_21909_amd import Layout
    sym = S.sym_custom(*spec)
    got = Layout(sym).density_flops()
    assert tuple(int(round(x)) for x in got) == _brute_density_flops(sym)


def test_density_error_codes_before_device_work(lib):
    L = lib.load()
    s = lib.Sym()
    out = lib.LayoutC()
    s.nirrep = 2
    s.nocc[0] = s.nvir[0] = s.ncd[0] = 1
    assert L.cdcc_irrep_layout(ctypes.byref(s), ctypes.byref(out)) == lib.OK
    arr = (lib.DensityProblem * 1)()
    arr[0].lay = ctypes.pointer(out)
    assert L.cdcc_vvvv_density(1, arr, None, None) == lib.EINVAL      # no pointers
    assert L.cdcc_vvvv_density(-1, None, None, None) == lib.EINVAL
    assert L.cdcc_vvvv_density(0, None, None, None) == lib.OK         # nothing to do
    o = lib.Opts()
    arr[0].L = arr[0].X = arr[0].Y = arr[0].G = ctypes.c_void_p(0x1000)
    for prec in (lib.MIXED, lib.MIXED_I8):
        o.precision = prec
        assert L.cdcc_vvvv_density(1, arr, ctypes.byref(o), None) == lib.EUNSUPPORTED
    assert L.cdcc_density_flops(None, None) == lib.EINVAL


# ------------------------------------------- partial symmetric-antisymmetric
@pytest.mark.parametrize("spec", SPECS)
def test_vo_layout_matches_oracle_layout(spec):
    from paper_2512_21909_amd import Layout
    sym = S.sym_custom(*spec)
    L, O = Layout(sym), OracleLayout(sym)
    assert L.n_vo == O.n_vo and L.vo_off == O.vo_off
    assert L.lvo_off == O.lvo_off and L.mvo_off == O.mvo_off
    assert (L.lvo_size, L.mvo_size) == (O.lvo_size, O.mvo_size)
    p = S.make_partial_problem(sym, seed=4)
    assert np.array_equal(L.pack_vo(p["lam"], "oo"), O.pack_vo(p["lam"], "oo"))


def _brute_partial_flops(sym):
    h, no, nv = sym["h"], sym["nocc"], sym["nvir"]
    io = [g for g in range(h) for _ in range(no[g])]
    iv = [g for g in range(h) for _ in range(nv[g])]
    fs = fa = 0
    for G in range(h):
        nvo = sum(1 for b in iv for i in io if b ^ i == G)
        kp = sum(1 for m in range(len(io)) for n in range(m + 1) if io[m] ^ io[n] == G)
        km = sum(1 for m in range(len(io)) for n in range(m) if io[m] ^ io[n] == G)
        cp = sum(1 for d in range(len(iv)) for c in range(d + 1) if iv[d] ^ iv[c] == G)
        cm = sum(1 for d in range(len(iv)) for c in range(d) if iv[d] ^ iv[c] == G)
        fs += 2 * nvo * kp * cp
        fa += 2 * nvo * km * cm
    return fs, fa


@pytest.mark.parametrize("spec", SPECS[:3] + SPECS[4:])
def test_partial_flops_match_enumeration(spec):
    from paper_2512_21909_amd import Layout
    sym = S.sym_custom(*spec)
    got = Layout(sym).partial_flops()
    assert tuple(int(round(x)) for x in got) == _brute_partial_flops(sym)


def test_partial_flops_halve_the_plain_contraction():
    """S + A is about half of the plain 2 n_vo n_oo n_vv (exactly half up to
    the diagonal m = n and d = c terms)."""
    from paper_2512_21909_amd import Layout
    sym = S.sym_d2h_medium()
    L = Layout(sym)
    plain = sum(2.0 * L.n_vo[G] * L.n_oo[G] * L.n_vv[G] for G in range(L.h))
    fs, fa = L.partial_flops()
    assert 0.45 < (fs + fa) / plain < 0.56


def test_partial_error_codes_before_device_work(lib):
    L = lib.load()
    s = lib.Sym()
    out = lib.LayoutC()
    s.nirrep = 2
    s.nocc[0] = s.nvir[0] = s.ncd[0] = 1
    assert L.cdcc_irrep_layout(ctypes.byref(s), ctypes.byref(out)) == lib.OK
    arr = (lib.PartialProblem * 1)()
    arr[0].lay = ctypes.pointer(out)
    assert L.cdcc_partial_contract(1, arr, None, None) == lib.EINVAL      # no pointers
    assert L.cdcc_partial_contract(-1, None, None, None) == lib.EINVAL
    assert L.cdcc_partial_contract(0, None, None, None) == lib.OK         # nothing to do
    o = lib.Opts()
    arr[0].lam = arr[0].tau = arr[0].M = ctypes.c_void_p(0x1000)
    for prec in (lib.MIXED, lib.MIXED_I8):
        o.precision = prec
        assert L.cdcc_partial_contract(1, arr, ctypes.byref(o), None) == lib.EUNSUPPORTED
    assert L.cdcc_partial_flops(None, None) == lib.EINVAL
    assert L.cdcc_vo_layout(None, None) == lib.EINVAL


# ------------------------------------------------------ two-step Cholesky
def test_cd_argument_errors_before_device_work(lib):
    L = lib.load()
    m = lib.CdMatrix()
    prm = lib.CdParams()
    prm.tau, prm.sigma, prm.qmax = 1e-6, 1e-2, 100
    piv = (ctypes.POINTER(lib._i64) * 8)()
    npiv = (lib._i64 * 8)()
    assert L.cdcc_cd_basis(None, ctypes.byref(prm), piv, npiv, None) == lib.EINVAL
    m.nirrep = 3
    assert L.cdcc_cd_basis(ctypes.byref(m), ctypes.byref(prm), piv, npiv, None) == lib.EUNSUPPORTED
    m.nirrep = 1
    m.n[0] = 4
    assert L.cdcc_cd_basis(ctypes.byref(m), ctypes.byref(prm), piv, npiv, None) == lib.EINVAL  # V NULL
    m.V[0] = 0x1000
    for tau, sigma, qmax in [(0.0, 1e-2, 10), (1e-6, 0.0, 10), (1e-6, 1.5, 10), (1e-6, 1e-2, 0), (1e-6, 1e-2, 4096)]:
        prm.tau, prm.sigma, prm.qmax = tau, sigma, qmax
        assert L.cdcc_cd_basis(ctypes.byref(m), ctypes.byref(prm), piv, npiv, None) == lib.EINVAL
    prm.tau, prm.sigma, prm.qmax = 1e-6, 1e-2, 10
    assert L.cdcc_cd_basis(ctypes.byref(m), ctypes.byref(prm), piv, npiv, None) == lib.EINVAL  # piv[0] NULL
    # second step: pivot out of range, more pivots than pairs
    p0 = (lib._i64 * 2)(0, 7)
    pp = (ctypes.POINTER(lib._i64) * 8)(ctypes.cast(p0, ctypes.POINTER(lib._i64)))
    npv = (lib._i64 * 8)(2)
    outs = (ctypes.c_void_p * 8)(0x2000)
    assert L.cdcc_cd_vectors(ctypes.byref(m), pp, npv, outs, None) == lib.EINVAL
    npv[0] = 5
    assert L.cdcc_cd_vectors(ctypes.byref(m), pp, npv, outs, None) == lib.EINVAL


def test_tile_size_class_keys():
    """The tile table's size-class key: a function of the shape's size (the
    same for a permutation of irreps that keeps every count), different for a
    shape of another size, and per precision and kind."""
    import paper_2512_21909_amd as cdcc
    import synth as S
    k = cdcc.ladder.tile_key
    a = S.sym_custom([3, 2], [21, 14], [50, 31])
    assert k(a, "mixed", "t2").startswith("mixed t2 b2 ")
    assert k(a, "mixed", "t2") != k(a, "fp64", "t2") and k(a, "mixed", "t2") != k(a, "mixed", "lambda")
    assert k(S.sym_custom([3, 2], [21, 14], [50, 32]), "mixed", "t2") == k(a, "mixed", "t2")   # same bucket
    assert k(S.sym_d2h_large(), "mixed", "t2") != k(S.sym_d2h_medium("B"), "mixed", "t2")
    parts = k(S.sym_d2h_large(), "fp64", "t2").split()
    assert parts[2] == "b8" and all(p.lstrip("-").isdigit() for p in parts[3:])


def test_tile_table_reader_round_trip(tmp_path):
    """The autotuner's table writer and reader agree (exact and size-class
    keys, class with and without a contraction segment)."""
    from paper_2512_21909_amd import autotune
    t = {"fp64 t2 1 8 40 300": "1", "mixed t2 b8 37 17 14": "2:2048"}
    path = str(tmp_path / "tile_table.txt")
    autotune.write_table(t, path)
    assert autotune.load_table(path) == t
