"""Python entry points over the C ABI.  Device buffers are torch tensors
(memory and streams only); every step of the computation runs in the HIP
library.  There is no CPU fallback: a missing library or GPU raises."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _lib
from .layout import Layout

_PREC = {"fp64": _lib.FP64, "mixed": _lib.MIXED, "mixed_i8": _lib.MIXED_I8}


def _torch():
    import torch
    return torch


def require_gpu() -> None:
    """Raise unless the HIP library is built and a GPU is visible."""
    _lib.load()
    torch = _torch()
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the ladder library runs only on the GPU")


def _ptr(t, n, name, optional=False):
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, layout needs {n}")
    return ctypes.c_void_p(t.data_ptr())


def make_problems(problems: list[dict], lambda_: bool):
    """Marshal a list of problem dicts into a ctypes array of cdcc_problem_t.
    Keys: layout (Layout), B, X, R; optional eps_occ, eps_vir, delta,
    pair_energy, energy_amps (the T of the pair energies, default X);
    Lambda: Bvo, t1, or U (the stack of lambda_dress)."""
    arr = (_lib.Problem * len(problems))()
    keep = []
    for k, p in enumerate(problems):
        lay: Layout = p["layout"]
        keep.append(lay)
        q = arr[k]
        q.lay = ctypes.pointer(lay.c)
        q.B = _ptr(p["B"], lay.b_size, "B")
        q.X = _ptr(p["X"], lay.amp_size, "X")
        q.R = _ptr(p["R"], lay.amp_size, "R")
        q.eps_occ = _ptr(p.get("eps_occ"), lay.nocc_tot, "eps_occ", True)
        q.eps_vir = _ptr(p.get("eps_vir"), lay.nvir_tot, "eps_vir", True)
        q.delta = _ptr(p.get("delta"), lay.amp_size, "delta", True)
        q.pair_energy = _ptr(p.get("pair_energy"), lay.nocc_tot * lay.nocc_tot, "pair_energy", True)
        q.energy_amps = _ptr(p.get("energy_amps"), lay.amp_size, "energy_amps", True)
        if lambda_:
            q.Bvo = _ptr(p.get("Bvo"), lay.bvo_size, "Bvo", True)
            q.t1 = _ptr(p.get("t1"), lay.t1_size, "t1", True)
            q.U = _ptr(p.get("U"), 2 * lay.b_size, "U", True)
    return arr, keep


def lambda_dress(problems, stream=None) -> None:
    """Build the T1-dressed Lambda stack U (2 * b_size doubles, caller-owned)
    from B, Bvo and t1, once per Lambda solve; pass it as the problem's "U"
    to ladder_lambda.  Keys: layout, B, Bvo, t1, U (out)."""
    if isinstance(problems, dict):
        problems = [problems]
    arr = (_lib.DressProblem * len(problems))()
    keep = []
    for k, p in enumerate(problems):
        lay: Layout = p["layout"]
        keep.append(lay)
        q = arr[k]
        q.lay = ctypes.pointer(lay.c)
        q.B = _ptr(p["B"], lay.b_size, "B")
        q.Bvo = _ptr(p["Bvo"], lay.bvo_size, "Bvo")
        q.t1 = _ptr(p["t1"], lay.t1_size, "t1")
        q.U = _ptr(p["U"], 2 * lay.b_size, "U")
    st = _lib.load().cdcc_lambda_dress(len(problems), arr, _stream(stream))
    _lib.check(st, "cdcc_lambda_dress")


def _opts(precision, tile_policy, batch_bytes, contract_kseg=0):
    o = _lib.Opts()
    o.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
    o.tile_policy = int(tile_policy)
    o.batch_bytes = int(batch_bytes)
    o.contract_kseg = int(contract_kseg)
    return o


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _maybe_tune(problems, kind, precision, tile_policy):
    """With CDCC_AUTOTUNE=1, shapes whose size class has no tile-table entry
    are tuned first (autotune.ensure); a forced tile class needs no table."""
    if tile_policy or os.environ.get("CDCC_AUTOTUNE") != "1":
        return
    from .autotune import ensure
    prec = precision if isinstance(precision, str) else {v: k for k, v in _PREC.items()}[int(precision)]
    ensure([p["layout"].sym for p in problems], kind, prec)


def ladder_t2(problems, precision="fp64", stream=None, tile_policy=0, batch_bytes=0, contract_kseg=0) -> None:
    """T2 ladder R_ij^ab = sum_cd tau_ij^cd (ac|bd) for one problem dict or a
    list of them (one batched launch sequence).  Asynchronous on ``stream``."""
    if isinstance(problems, dict):
        problems = [problems]
    _maybe_tune(problems, "t2", precision, tile_policy)
    arr, keep = make_problems(problems, False)
    o = _opts(precision, tile_policy, batch_bytes, contract_kseg)
    st = _lib.load().cdcc_ladder_t2(len(problems), arr, ctypes.byref(o), _stream(stream))
    _lib.check(st, "cdcc_ladder_t2")


def ladder_t2_noalloc(problems, precision="fp64", stream=None, tile_policy=0, batch_bytes=0, contract_kseg=0) -> None:
    """The T2 ladder of ``ladder_t2`` without any device allocation: plan
    tables and workspace in the library's static scratch array (calls that
    overlap on one GPU race).  Raises CdccError with status ESCRATCH when the
    problem does not fit it."""
    if isinstance(problems, dict):
        problems = [problems]
    arr, keep = make_problems(problems, False)
    o = _opts(precision, tile_policy, batch_bytes, contract_kseg)
    st = _lib.load().cdcc_ladder_t2_noalloc(len(problems), arr, ctypes.byref(o), _stream(stream))
    _lib.check(st, "cdcc_ladder_t2_noalloc")


def ladder_lambda(problems, precision="fp64", stream=None, tile_policy=0, batch_bytes=0, contract_kseg=0) -> None:
    """Lambda ladder Z_ij^ab = sum_ef lambda_ij^ef W_efab (Appendix-A W)."""
    if isinstance(problems, dict):
        problems = [problems]
    _maybe_tune(problems, "lambda", precision, tile_policy)
    arr, keep = make_problems(problems, True)
    o = _opts(precision, tile_policy, batch_bytes, contract_kseg)
    st = _lib.load().cdcc_ladder_lambda(len(problems), arr, ctypes.byref(o), _stream(stream))
    _lib.check(st, "cdcc_ladder_lambda")


def vvvv_density(problems, stream=None, batch_bytes=0) -> None:
    """vvvv contraction of the spin-adapted two-body density, G^P_ac =
    sum_bd (2 Gamma_abcd - Gamma_abdc) L^P_bd with Gamma_abcd = 1/2 sum_mn
    [Y_mn^ab X_mn^cd + Y_mn^cd X_mn^ab] (FP64), for one problem dict or a
    list of them.  Keys: layout (Layout), L, X (tau~), Y (lambda), G (out;
    Cholesky layout).  Asynchronous on ``stream``."""
    if isinstance(problems, dict):
        problems = [problems]
    arr = (_lib.DensityProblem * len(problems))()
    keep = []
    for k, p in enumerate(problems):
        lay: Layout = p["layout"]
        keep.append(lay)
        q = arr[k]
        q.lay = ctypes.pointer(lay.c)
        q.L = _ptr(p["L"], lay.b_size, "L")
        q.X = _ptr(p["X"], lay.amp_size, "X")
        q.Y = _ptr(p["Y"], lay.amp_size, "Y")
        q.G = _ptr(p["G"], lay.b_size, "G")
    o = _opts("fp64", 0, batch_bytes)
    st = _lib.load().cdcc_vvvv_density(len(problems), arr, ctypes.byref(o), _stream(stream))
    _lib.check(st, "cdcc_vvvv_density")


def partial_contract(problems, stream=None) -> None:
    """M_bi^dc = sum_mn lambda_bi^mn tau_mn^dc (FP64, partial
    symmetric-antisymmetric algorithm) for one problem dict or a list.  Keys:
    layout (Layout), lam (vo layout), tau (amplitude layout, pair symmetric),
    M (out, vo layout).  Asynchronous on ``stream``."""
    if isinstance(problems, dict):
        problems = [problems]
    arr = (_lib.PartialProblem * len(problems))()
    keep = []
    for k, p in enumerate(problems):
        lay: Layout = p["layout"]
        keep.append(lay)
        q = arr[k]
        q.lay = ctypes.pointer(lay.c)
        q.lam = _ptr(p["lam"], lay.lvo_size, "lam")
        q.tau = _ptr(p["tau"], lay.amp_size, "tau")
        q.M = _ptr(p["M"], lay.mvo_size, "M")
    o = _opts("fp64", 0, 0)
    st = _lib.load().cdcc_partial_contract(len(problems), arr, ctypes.byref(o), _stream(stream))
    _lib.check(st, "cdcc_partial_contract")


def _cd_matrix(V):
    m = _lib.CdMatrix()
    if len(V) not in (1, 2, 4, 8):
        raise ValueError("one matrix per irrep: 1, 2, 4 or 8 of them")
    m.nirrep = len(V)
    for g, v in enumerate(V):
        n = int(v.shape[0]) if v is not None else 0
        m.n[g] = n
        m.V[g] = _ptr(v, n * n, f"V[{g}]").value if n else None
    return m


def cd_basis(V, tau: float, sigma: float = 1e-2, qmax: int = 1000, stream=None):
    """First step of the two-step Cholesky decomposition (Algorithm 1):
    V = list of dense symmetric (n_g, n_g) float64 device tensors, one per
    irrep.  Returns the pivots of each irrep (int64 numpy arrays, in the
    order chosen).  Synchronous."""
    m = _cd_matrix(V)
    prm = _lib.CdParams()
    prm.tau, prm.sigma, prm.qmax = float(tau), float(sigma), int(qmax)
    bufs = [np.zeros(max(int(m.n[g]), 1), dtype=np.int64) for g in range(_lib.MAX_IRREP)]
    ptrs = (ctypes.POINTER(_lib._i64) * _lib.MAX_IRREP)(
        *[b.ctypes.data_as(ctypes.POINTER(_lib._i64)) for b in bufs])
    npiv = (_lib._i64 * _lib.MAX_IRREP)()
    st = _lib.load().cdcc_cd_basis(ctypes.byref(m), ctypes.byref(prm), ptrs, npiv, _stream(stream))
    _lib.check(st, "cdcc_cd_basis")
    return [bufs[g][:int(npiv[g])].copy() for g in range(len(V))]


def cd_vectors(V, piv, L, stream=None) -> None:
    """Second step: L[g] (device, float64, n_g x npiv_g, [r][P]) receives the
    Cholesky vectors K^-1 V[piv, :] of irrep g.  Waits for the stream."""
    m = _cd_matrix(V)
    pv = [np.ascontiguousarray(np.asarray(p, dtype=np.int64)) for p in piv]
    if len(pv) != len(V) or len(L) != len(V):
        raise ValueError("one pivot list and one output per irrep")
    keep = [x if x.size else np.zeros(1, dtype=np.int64) for x in pv]
    ptrs = (ctypes.POINTER(_lib._i64) * _lib.MAX_IRREP)(
        *[k.ctypes.data_as(ctypes.POINTER(_lib._i64)) for k in keep])
    npiv = (_lib._i64 * _lib.MAX_IRREP)(*[int(x.size) for x in pv])
    outs = (ctypes.c_void_p * _lib.MAX_IRREP)()
    for g, x in enumerate(pv):
        n = int(m.n[g])
        outs[g] = _ptr(L[g], n * x.size, f"L[{g}]").value if x.size else None
    st = _lib.load().cdcc_cd_vectors(ctypes.byref(m), ptrs, npiv, outs, _stream(stream))
    _lib.check(st, "cdcc_cd_vectors")


def workspace_bytes(problems, lambda_=False, precision="fp64", tile_policy=0, batch_bytes=0, contract_kseg=0) -> int:
    if isinstance(problems, dict):
        problems = [problems]
    arr, keep = make_problems(problems, lambda_)
    o = _opts(precision, tile_policy, batch_bytes, contract_kseg)
    out = ctypes.c_int64(0)
    _lib.check(_lib.load().cdcc_workspace_bytes(len(problems), arr, ctypes.byref(o), int(bool(lambda_)),
                                                ctypes.byref(out)), "cdcc_workspace_bytes")
    return int(out.value)


def tile_key(sym: dict, precision="fp64", kind="t2") -> str:
    """The size-class key of the tile table for a shape (cdcc_tile_key)."""
    buf = ctypes.create_string_buffer(256)
    c = Layout(sym).c.sym
    st = _lib.load().cdcc_tile_key(ctypes.byref(c), _PREC[precision], int(kind == "lambda"), buf, 256)
    _lib.check(st, "cdcc_tile_key")
    return buf.value.decode()


def tile_table_reload(path=None) -> None:
    """Plans built from now on read the tile table again (from ``path``, or
    the default location)."""
    st = _lib.load().cdcc_tile_table_reload(path.encode() if path else None)
    _lib.check(st, "cdcc_tile_table_reload")


def release() -> None:
    _lib.check(_lib.load().cdcc_release(), "cdcc_release")


KERNEL_CLASSES = ("dress", "pack", "assemble", "contract", "energy", "slice", "density_w", "density_g",
                  "density_r", "partial_pack", "partial_gemm", "cd_residual", "cd_micro", "cd_vectors")


def timing_enable(on: bool = True) -> None:
    """Record HIP event pairs around each kernel class of every call."""
    _lib.check(_lib.load().cdcc_timing_enable(int(bool(on))), "cdcc_timing_enable")


def timing_read() -> dict:
    """{class: (total_ms, launches)} since the last read (waits for the events)."""
    nk = len(KERNEL_CLASSES)
    ms = (ctypes.c_double * nk)()
    n = (_lib._i64 * nk)()
    _lib.check(_lib.load().cdcc_timing_read(ms, n), "cdcc_timing_read")
    return {KERNEL_CLASSES[k]: (float(ms[k]), int(n[k])) for k in range(nk) if n[k]}
