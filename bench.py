#!/usr/bin/env python3
"""Benchmark of the Cholesky-decomposed CCSD particle-particle ladder on one
MI355X.

Default workload (the largest single-GPU ladder configuration): the T2 ladder
R = sum_cd tau (ac|bd) on 8 irreps, o=40 (8,5,6,4,6,4,4,3), v=400
(80,44,60,40,64,36,44,32), 3000 Cholesky vectors split evenly, with the
symmetric-antisymmetric split, the (ac|bd) batches assembled on the fly and
the FP64 epilogue (R/D and pair energies).  One step = one such evaluation;
inputs are resident in HBM before the timed region.  Every path is gated
against the FP64 oracle on every element (1e-12 FP64, 1e-7 split paths
normwise; pair energies 1e-8 Eh).

value = algorithmic TFLOP/s (symmetry-blocked, stored-halves flop count) of
the fastest of the FP64 and split-BF16 paths that passes its gate.  Beside
it: the 8-bit digit path, the roofline of the dominant kernel of every path,
the 8-irrep o=20/v=200 workload (T2 + T1-dressed Lambda) and the batch of 64
uneven systems as extra workloads with their own gates, rooflines and CPU
baselines, and the serving loop (FP64 and split-BF16) with p50/p99 latency.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CD ladder residual TFLOP/s, FP64 vs split-precision at 1e-7; p50/p99 latency"
PEAK = {"fp64": 78.6, "bf16": 2500.0, "int8": 5000.0}  # MI355X dense MFMA, TFLOP/s (int8: TOP/s)
# Precision forms the headline value is taken from (FP64, and split-BF16 with
# FP32 accumulation and FP64 combination); the 8-bit digit path is measured
# and reported beside them.
HEADLINE_FORMS = ("fp64", "mixed")
# MFMA products issued per algorithmic term: eleven BF16 slice products,
# thirteen 8-bit digit products
NPROD = {"mixed": 11, "mixed_i8": 13}
DTYPE = {"fp64": "f64", "mixed": "bf16x4-split/f32-acc/f64-sum", "mixed_i8": "i8x4-split/i32-acc/f64-sum"}
# MFMA type (peak) of each kernel class per path
KERNEL_PEAK = {"assemble": {"fp64": "fp64", "mixed": "bf16", "mixed_i8": "int8"},
               "contract": {"fp64": "fp64", "mixed": "fp64", "mixed_i8": "fp64"}}
KERNEL_NAME = {"assemble": "(ac|bd) batch assembly", "contract": "S/A contraction + unpack"}
HBM_PEAK = 8000.0  # GB/s
GATE = {"fp64": 1e-12, "mixed": 1e-7, "mixed_i8": 1e-7}
PAIR_GATE = 1e-8   # Eh, split paths (FP64: 1e-12 relative to max |e_ij|)
# Bytes one launch of a kernel class moves between L2 and the memory fabric,
# from rocprofv3 FETCH_SIZE + WRITE_SIZE per dispatch (scaled x2.0 and x1.0 by
# a plain 256 MiB device copy), per (workload, path, kernel), for the kernels
# as committed (profiles/).  A "launch" is what the library times as one: an
# assembly launch (the T2 and the Lambda launch of a step averaged), or one
# batch's contraction with its split-K reduction and unpack (at o=40/v=400 a
# call is one batch and its contraction one K segment, with no reduction).  The vvvv density
# and partial-contraction entries are the launch of their GEMM kernel,
# counted the same way.
TRAFFIC = {("d2h_medium", "mixed", "assemble"): 2.641e9, ("d2h_medium", "fp64", "assemble"): 2.276e9,
           ("d2h_medium", "mixed_i8", "assemble"): 1.396e9,
           ("d2h_large", "fp64", "assemble"): 45.957e9, ("d2h_large", "mixed", "assemble"): 42.393e9,
           ("d2h_large", "mixed_i8", "assemble"): 25.243e9,
           ("d2h_large", "fp64", "contract"): 28.984e9, ("d2h_large", "mixed", "contract"): 28.984e9,
           ("d2h_large", "mixed_i8", "contract"): 28.984e9,
           ("vvvv_d2h_medium", "fp64", "gemm"): 3.800e9,
           ("pm_d2h_medium", "fp64", "gemm"): 0.277e9, ("pm_d2h_large", "fp64", "gemm"): 7.494e9}
# A single system is checked on every element when the plain oracle costs at
# most this many flops; in a batched call, systems up to SYSTEM_FULL_FLOPS
# are checked in full and the others on sampled elements.
FULL_ORACLE_FLOPS = 5e12
SYSTEM_FULL_FLOPS = 2e10


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:  # pragma: no cover
        pass
    import platform
    return platform.processor() or "unknown"


def blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return int(max((d.get("num_threads", 1) for d in threadpool_info()), default=os.cpu_count()))
    except Exception:  # pragma: no cover
        return int(os.cpu_count() or 1)


def workload(name):
    """(description, [(kind, [problem, ...]), ...]): each entry is one library
    call (a list of several problems is one batched call)."""
    import synth as S
    if name == "d2h_medium":
        sym = S.sym_d2h_medium("A")
        return ("d2h_medium: 8 irreps, o=20, v=200, Ncd=1500 (all in the totally symmetric irrep); "
                "T2 + T1-dressed Lambda ladder",
                [("t2", [S.make_problem(sym, 0, "t2")]), ("lambda", [S.make_problem(sym, 0, "lambda")])])
    if name == "c1_small":
        sym = S.sym_c1_small()
        return ("c1_small: 1 irrep, o=8, v=40, Ncd=300; T2 + T1-dressed Lambda ladder",
                [("t2", [S.make_problem(sym, 0, "t2")]), ("lambda", [S.make_problem(sym, 0, "lambda")])])
    if name == "d2h_large":
        sym = S.sym_d2h_large()
        return ("d2h_large: 8 irreps, o=40, v=400, Ncd=3000 (even split); T2 ladder",
                [("t2", [S.make_problem(sym, 0, "t2")])])
    if name == "hbc_shape":
        sym = S.sym_hbc_shape()
        return ("hbc_shape: 8 irreps, o=135, v=543, Ncd=3710 (even split; the size of the paper's largest D2h "
                "molecule); T2 ladder", [("t2", [S.make_problem(sym, 0, "t2")])])
    if name == "c1_large":
        sym = S.sym_custom([40], [400], [3000])
        return ("c1_large: 1 irrep, o=40, v=400, Ncd=3000 (the o=40 system without point-group symmetry); "
                "T2 ladder", [("t2", [S.make_problem(sym, 0, "t2")])])
    if name == "batch64":
        syms = S.batch_syms(64, seed=0)
        return ("batch64: 64 uneven systems (o 5-20, v 40-160, Ncd 7.5(o+v), 1/2/4/8 irreps) in one batched "
                "T2 call", [("t2", [S.make_problem(s, k, "t2") for k, s in enumerate(syms)])])
    raise SystemExit(f"unknown workload {name}")


def build_inputs(cdcc, entries):
    """Device buffers of every call.  The T1-dressed Lambda operand is built
    once here (cdcc_lambda_dress, as once per Lambda solve) and passed to
    every Lambda step; its time is returned separately (ms, or None)."""
    import torch
    from tests.gpu_support import device_problem
    dev, dress_ms = [], None
    for kind, probs in entries:
        ds = [device_problem(cdcc, p, want_delta=True, want_energy=True, nan_fill=False) for p in probs]
        if kind == "lambda":
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            for d in ds:
                d["U"] = torch.empty(2 * d["layout"].b_size, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            a.record()
            cdcc.lambda_dress([{k: d[k] for k in ("layout", "B", "Bvo", "t1", "U")} for d in ds])
            b.record()
            torch.cuda.synchronize()
            dress_ms = (dress_ms or 0.0) + a.elapsed_time(b)
        dev.append((kind, probs, ds))
    return dev, dress_ms


TILE_POLICY = 0


def step(cdcc, dev, precision):
    for kind, _, ds in dev:
        fn = cdcc.ladder_t2 if kind == "t2" else cdcc.ladder_lambda
        fn(ds, precision=precision, tile_policy=TILE_POLICY)


def _plain_flops(p):
    from oracle.layout import OracleLayout
    lay = OracleLayout(p["sym"])
    return sum(2.0 * lay.n_oo[G] * lay.n_vv[G] ** 2 for G in range(lay.h))


def _alg_flops(kind, p):
    from paper_2512_21909_amd import Layout
    return sum(Layout(p["sym"]).flops(0 if kind == "t2" else 2))


def _oracle(kind, p):
    import oracle as O
    if kind == "t2":
        return O.t2_ladder_blocks(p["sym"], p["B"], p["X"])
    return O.lambda_ladder_blocks(p["sym"], p["B"], p["Bvo"], p["t1"], p["X"])


def reference(entries):
    """Oracle results (R, R/D, pair energies) of every problem the oracle
    affords in full (None for the others), and the host time and algorithmic
    flops of those oracle evaluations (a CPU-baseline sample)."""
    import oracle as O
    refs, secs, flops, n = [], 0.0, 0.0, 0
    for kind, probs in entries:
        single = len(probs) == 1
        row = []
        for p in probs:
            if _plain_flops(p) > (FULL_ORACLE_FLOPS if single else SYSTEM_FULL_FLOPS):
                row.append(None)
                continue
            t0 = time.perf_counter()
            r = _oracle(kind, p)
            secs += time.perf_counter() - t0
            flops += _alg_flops(kind, p)
            n += 1
            sym = p["sym"]
            row.append({"R": r, "e": O.pair_energies_blocks(sym, p["X"], r),
                        "delta": O.denominator_update_blocks(sym, r, p["eps_occ"], p["eps_vir"])})
        refs.append(row)
    return refs, {"seconds": secs, "flops": flops, "evaluations": n}


def accuracy(cdcc, dev, refs, precision, e_fp64=None, samples=40):
    """Errors of one evaluation against the oracle.  Problems with a full
    reference: normwise max and Frobenius errors of R and R/D, pair energies.
    The others: ``samples`` elements each computed one by one by the oracle
    (max error relative to max|R|), and, when the FP64 path's pair energies
    are given, the pair energies against them.  Metrics that were not
    computed are None.  Returns (per-kind errors, pair energies per call)."""
    import torch
    import oracle as O
    step(cdcc, dev, precision)
    torch.cuda.synchronize()
    out, energies = {}, []
    rng = np.random.default_rng(2024)
    for ci, (kind, probs, ds) in enumerate(dev):
        acc = {"max_rel": 0.0, "fro_rel": None, "delta_max_rel": None, "pair_energy_abs": None,
               "pair_energy_abs_vs_fp64": None, "pair_energy_ref_max": None, "full_systems": 0,
               "sampled_systems": 0, "sampled_elements": 0}
        e_call = []
        for pi, (p, d) in enumerate(zip(probs, ds)):
            lay = d["layout"]
            got = lay.unpack_amp(d["R"].cpu().numpy())
            e_got = d["pair_energy"].cpu().numpy()
            e_call.append(e_got)
            ref = refs[ci][pi] if refs is not None else None
            if ref is not None:
                mx, fro = O.rel_errors(got, ref["R"])
                dmx, _ = O.rel_errors(lay.unpack_amp(d["delta"].cpu().numpy()), ref["delta"])
                ee = float(np.max(np.abs(e_got.reshape(ref["e"].shape) - ref["e"]))) if ref["e"].size else 0.0
                if precision == "fp64":
                    ee /= max(1.0, float(np.max(np.abs(ref["e"])))) if ref["e"].size else 1.0
                acc["max_rel"] = max(acc["max_rel"], mx)
                acc["fro_rel"] = max(acc["fro_rel"] or 0.0, fro)
                acc["delta_max_rel"] = max(acc["delta_max_rel"] or 0.0, dmx)
                acc["pair_energy_abs"] = max(acc["pair_energy_abs"] or 0.0, ee)
                if ref["e"].size:  # the scale the absolute pair-energy error is against
                    acc["pair_energy_ref_max"] = max(acc["pair_energy_ref_max"] or 0.0, float(np.max(np.abs(ref["e"]))))
                acc["full_systems"] += 1
                continue
            sym, h = p["sym"], p["sym"]["h"]
            no, nv = sym["nocc"], sym["nvir"]
            scale = max(float(np.max(np.abs(b))) for b in got.values() if b.size)
            for _ in range(samples):
                G, gi, ga = (int(x) for x in rng.integers(0, h, 3))
                gj, gb = gi ^ G, ga ^ G
                if not (no[gi] and no[gj] and nv[ga] and nv[gb]):
                    continue
                i, j = int(rng.integers(no[gi])), int(rng.integers(no[gj]))
                a, b = int(rng.integers(nv[ga])), int(rng.integers(nv[gb]))
                args = (lay.occ_off[gi] + i, lay.occ_off[gj] + j, lay.vir_off[ga] + a, lay.vir_off[gb] + b)
                r = (O.element_t2(sym, p["B"], p["X"], *args) if kind == "t2"
                     else O.element_lambda(sym, p["B"], p["Bvo"], p["t1"], p["X"], *args))
                acc["max_rel"] = max(acc["max_rel"], abs(got[(G, gi, ga)][i, j, a, b] - r) / scale)
                acc["sampled_elements"] += 1
            acc["sampled_systems"] += 1
            if e_fp64 is not None:
                ee = float(np.max(np.abs(e_got - e_fp64[ci][pi]))) if e_got.size else 0.0
                acc["pair_energy_abs_vs_fp64"] = max(acc["pair_energy_abs_vs_fp64"] or 0.0, ee)
                if e_got.size:
                    acc["pair_energy_ref_max"] = max(acc["pair_energy_ref_max"] or 0.0,
                                                     float(np.max(np.abs(e_fp64[ci][pi]))))
        out[kind] = acc
        energies.append(e_call)
    return out, energies


def gate_ok(acc, precision):
    """Every metric that was computed is within its gate (None = not
    computed, left out)."""
    if acc is None:
        return True
    g = GATE[precision]
    for a in acc.values():
        if a["max_rel"] > g:
            return False
        for k in ("fro_rel", "delta_max_rel"):
            if a[k] is not None and a[k] > g:
                return False
        pe = 1e-12 if precision == "fp64" else PAIR_GATE
        if a["pair_energy_abs"] is not None and a["pair_energy_abs"] > pe:
            return False
        if a["pair_energy_abs_vs_fp64"] is not None and a["pair_energy_abs_vs_fp64"] > PAIR_GATE:
            return False
    return True


def timed(cdcc, dev, precision, steps, warmup):
    """Mean seconds per step over the timed steps (host clock around the
    whole loop), plus the per-step device times (ms) from events recorded on
    the launch stream between the steps."""
    import torch
    for _ in range(warmup):
        step(cdcc, dev, precision)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        step(cdcc, dev, precision)
        ev[k + 1].record()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    return sec, [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]


def kernel_times(cdcc, dev, precision, steps):
    """Per-class kernel durations from HIP events recorded by the library on
    the stream it launches on."""
    import torch
    torch.cuda.synchronize()
    cdcc.timing_read()
    cdcc.timing_enable(True)
    for _ in range(steps):
        step(cdcc, dev, precision)
    torch.cuda.synchronize()
    cdcc.timing_enable(False)
    return cdcc.timing_read()


def kernel_rooflines(name, precision, kt, flops_cls, steps):
    """Roofline object of the assembly and of the contraction of one path:
    algorithmic flops per launch / average launch time."""
    out = {}
    for cls, fidx in (("assemble", 0), ("contract", 1)):
        ms, n = kt.get(cls, (0.0, 0))
        if not n or not ms:
            continue
        per_launch = flops_cls[fidx] * steps / n
        avg_ms = ms / n
        ach = per_launch / (avg_ms * 1e-3) / 1e12
        pk = KERNEL_PEAK[cls][precision]
        o = {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK[pk],
             "unit": "TOP/s" if pk == "int8" else "TFLOP/s", "frac": round(ach / PEAK[pk], 4),
             "traffic": TRAFFIC.get((name, precision, cls)), "kernel": KERNEL_NAME[cls], "launches": n,
             "avg_launch_ms": avg_ms, "flops_per_launch": per_launch, "ms_per_step": ms / steps}
        if pk != "fp64" and precision in NPROD:
            o["issued_" + ("bf16_tflops" if pk == "bf16" else "int8_tops")] = round(ach * NPROD[precision], 3)
            o["issued_frac"] = round(ach * NPROD[precision] / PEAK[pk], 4)
        out[cls] = o
    return out


def measure_ladder(cdcc, name, args, paths):
    """Every path on one workload: accuracy gate, timing, per-kernel
    rooflines; plus the oracle's own timing from the gate (CPU sample)."""
    desc, entries = workload(name)
    dev, dress_ms = build_inputs(cdcc, entries)
    flops_step, flops_cls, flops_dress = 0.0, [0.0, 0.0, 0.0], 0.0
    for kind, _, ds in dev:
        for d in ds:
            # Lambda steps take the stack built once per solve: no dressing flops
            f = d["layout"].flops(0 if kind == "t2" else 1)
            flops_step += sum(f)
            flops_cls = [a + b for a, b in zip(flops_cls, f)]
            if kind == "lambda":
                flops_dress += d["layout"].flops(2)[2]
    log(f"{desc}; F_alg per step {flops_step:.4e} (assembly {flops_cls[0]:.4e}, contraction {flops_cls[1]:.4e})")
    refs, oracle_t = (None, None)
    if not args.no_check:
        t0 = time.perf_counter()
        refs, oracle_t = reference(entries)
        log(f"{name}: oracle references in {time.perf_counter() - t0:.1f} s "
            f"({oracle_t['evaluations']} full evaluations)")
    results, e_fp64 = {}, None
    for prec in paths:
        try:
            acc = None
            if refs is not None:
                acc, energies = accuracy(cdcc, dev, refs, prec, e_fp64=e_fp64 if prec != "fp64" else None)
                if prec == "fp64":
                    e_fp64 = energies
        except cdcc.CdccError as e:
            log(f"{prec}: unavailable ({e})")
            continue
        sec, per_step = timed(cdcc, dev, prec, args.steps, args.warmup)
        kt = kernel_times(cdcc, dev, prec, args.steps)
        ok = gate_ok(acc, prec)
        roofs = kernel_rooflines(name, prec, kt, flops_cls, args.steps)
        dom = max(roofs, key=lambda c: roofs[c]["ms_per_step"]) if roofs else None
        results[prec] = {"ms_per_step": sec * 1e3, "tflops": flops_step / sec / 1e12, "accuracy": acc,
                         "passes_gate": ok, "step_ms_median": float(np.median(per_step)),
                         "step_ms_min": float(np.min(per_step)), "dominant_kernel": dom, "rooflines": roofs,
                         "kernels_ms": kt}
        log(f"{name} {prec}: {sec * 1e3:.3f} ms/step, {flops_step / sec / 1e12:.2f} TFLOP/s, gate ok={ok}, "
            f"kernels={kt}")
    good = [p for p in results if results[p]["passes_gate"] and (p in HEADLINE_FORMS or len(results) == 1)]
    best = max(good, key=lambda p: results[p]["tflops"]) if good else None
    out = {"workload": desc, "flops_per_step": flops_step, "flops_assembly": flops_cls[0],
           "flops_contraction": flops_cls[1], "paths": results, "best": best,
           **({"lambda_dress_once": {"ms": dress_ms, "flops": flops_dress,
                                     "note": "T1-dressed stack built once per Lambda solve, outside the steps"}}
              if dress_ms is not None else {}),
           "value": round(results[best]["tflops"], 4) if best else None,
           "ms_per_step": round(results[best]["ms_per_step"], 4) if best else None,
           "passes_gate": best is not None}
    if best:
        r = results[best]
        out["roofline"] = r["rooflines"].get(r["dominant_kernel"])
    if "fp64" in results and "mixed" in results:
        out["mixed_speedup_vs_fp64"] = results["mixed"]["tflops"] / results["fp64"]["tflops"]
    if "fp64" in results and "mixed_i8" in results:
        out["mixed_i8_speedup_vs_fp64"] = results["mixed_i8"]["tflops"] / results["fp64"]["tflops"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(entries, oracle_t, budget_1t=args.cpu_budget_1t if name != "d2h_large" else 0)
    return out


def cpu_baseline(entries, oracle_t, budget_s=12.0, budget_1t=0.0):
    """The FP64 oracle (NumPy + host BLAS) on the same workload: the gate's
    own oracle evaluations when there were any (else whole evaluations
    repeated for a bounded time), and optionally a run with the host BLAS
    held to one thread."""
    cores = blas_threads()

    def run_for(budget):
        t0 = time.perf_counter()
        done_flops, items = 0.0, 0
        while items == 0 or time.perf_counter() - t0 < budget:
            for kind, probs in entries:
                for p in probs:
                    _oracle(kind, p)
                    done_flops += _alg_flops(kind, p)
                    items += 1
                    if time.perf_counter() - t0 >= budget:
                        return done_flops, time.perf_counter() - t0, items
        return done_flops, time.perf_counter() - t0, items

    if oracle_t and oracle_t["evaluations"] and oracle_t["seconds"] >= 2.0:
        f, dt, n = oracle_t["flops"], oracle_t["seconds"], oracle_t["evaluations"]
        how = "the accuracy gate's own oracle runs"
    else:
        f, dt, n = run_for(budget_s)
        how = "oracle runs repeated for a bounded time"
    out = {"value": f / dt / 1e12, "unit": "TFLOP/s", "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{n} ladder evaluation(s) of this workload in {dt:.1f} s ({how}; symmetry-blocked plain "
                     f"FP64 contraction, NumPy + host BLAS); rate = their algorithmic flops / time"}
    if budget_1t > 0:
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1):
                f1, d1, n1 = run_for(budget_1t)
            out["value_1_thread"] = f1 / d1 / 1e12
            out["sample_1_thread"] = f"{n1} evaluations in {d1:.1f} s with the host BLAS on one thread"
        except Exception:  # pragma: no cover
            pass
    return out


def serving_pool(seed=5, n_shapes=12):
    """Device-resident inputs of the serving mix: twelve shapes drawn like the
    uneven batch, plus the large request (o=30, v=300, 2500 vectors, 8
    irreps)."""
    import torch
    import synth as S
    from paper_2512_21909_amd import Layout

    def dev(x):
        return torch.from_numpy(np.ascontiguousarray(x)).cuda()

    syms = S.batch_syms(n_shapes, seed=seed) + [S.sym_serving_large()]
    pool = []
    for k, sym in enumerate(syms):
        p = S.make_problem(sym, seed=100 + k, kind="t2")
        lay = Layout(sym)
        pool.append({"layout": lay, "B": dev(lay.pack_B(p["B"])), "X": dev(lay.pack_amp(p["X"])),
                     "flops": sum(lay.flops(0)), "large": k == len(syms) - 1})
    return pool


def compact(m):
    """An extra workload's summary for the bench line."""
    keep = ("workload", "value", "ms_per_step", "passes_gate", "best", "flops_per_step", "roofline",
            "mixed_speedup_vs_fp64", "mixed_i8_speedup_vs_fp64", "cpu_baseline", "lambda_dress_once")
    out = {k: m[k] for k in keep if k in m}
    out["paths"] = {p: {k: v for k, v in r.items() if k != "kernels_ms"} for p, r in m["paths"].items()}
    return out


def ladder_main(args, cdcc):
    paths = ["fp64", "mixed", "mixed_i8"] if args.precision == "all" else [args.precision]
    m = measure_ladder(cdcc, args.workload, args, paths)
    if m["best"] is None:
        log("no path passed its accuracy gate")
        print(json.dumps({"metric": METRIC, "value": None, "error": "no path passed its accuracy gate",
                          "paths": m["paths"]}, default=str), flush=True)
        sys.exit(1)
    best = m["best"]
    line = {
        "metric": METRIC, "value": m["value"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[best], "data": "synthetic",
        # the S/A contraction (and everything after it) is FP64 in every path;
        # the split forms apply to the (ac|bd) assembly
        "dtype_contraction": "f64",
        "config": {"workload": m["workload"], "flops_per_step": m["flops_per_step"], "path": best},
        "roofline": m["roofline"],
        "paths": m["paths"],
    }
    for k in ("mixed_speedup_vs_fp64", "mixed_i8_speedup_vs_fp64"):
        if k in m:
            line[k] = m[k]
    extras = [] if args.extras in ("", "none") else args.extras.split(",")
    if extras:
        line["workloads"] = {}
        for name in extras:
            line["workloads"][name] = compact(measure_ladder(cdcc, name, args, paths))
    if args.serving:
        from paper_2512_21909_amd import serve
        pool = serving_pool()
        line["serving"] = {}
        for prec in args.serving_precisions.split(","):
            line["serving"][prec] = serve.measure(pool, prec, n_requests=args.serving, warmup=args.serving_warmup,
                                                  load=args.serving_load)
            s = line["serving"][prec]
            log(f"serving {prec}: saturation {s['saturation'].get('requests_per_s', 0):.1f} req/s, "
                f"load {args.serving_load}: p50 {s['stream'].get('p50_ms', 0):.2f} ms, "
                f"p99 {s['stream'].get('p99_ms', 0):.2f} ms")
    if "cpu_baseline" in m:
        line["cpu_baseline"] = m["cpu_baseline"]
    line["paper_context"] = PAPER_CONTEXT
    print(json.dumps(line, default=str), flush=True)


# The paper's own timings with their hardware (Section "Analysis of timings"),
# context only: whole CD-CCSD geometry optimisations, not ladder evaluations,
# so no ratio against them is formed (vs_baseline stays null).
PAPER_CONTEXT = {
    "hexabenzocoronene_cc-pVDZ": {
        "size": "o=135, v=543, about 3710 Cholesky vectors, D2h",
        "time": "about 4 d 15 h for 24 geometry-optimisation steps (about 4.6 h per gradient step)",
        "hardware": "AMD EPYC 7282 16-core node, 32 OpenMP threads",
    },
    "coronene_cc-pVTZ": {
        "size": "o=78, v=810, about 4420 Cholesky vectors, D2h",
        "time": "about 2 d for 8 geometry-optimisation steps",
        "hardware": "Intel Xeon Gold 6140M node, 32 OpenMP threads",
    },
    "note": "a gradient step holds every T2 and Lambda iteration, the densities and the derivative contractions",
}


def serving_sweep_main(args, cdcc):
    """Saturation once, then one Poisson stream per load, per precision."""
    from paper_2512_21909_amd import serve
    pool = serving_pool()
    loads = [float(x) for x in args.serving_sweep.split(",")]
    out = {}
    for prec in args.serving_precisions.split(","):
        out[prec] = serve.measure_sweep(pool, prec, n_requests=args.serving, loads=loads,
                                        warmup=args.serving_warmup, log=log)
    print(json.dumps(out), flush=True)


DENSITY_METRIC = "vvvv two-body-density contraction with Cholesky vectors, TFLOP/s (FP64)"


def density_workload(name):
    import synth as S
    syms = {"vvvv_d2h_medium": ("vvvv density: 8 irreps, o=20, v=200, Ncd=1500 (all in the totally symmetric "
                                "irrep)", S.sym_d2h_medium("A")),
            "vvvv_d2h_medium_B": ("vvvv density: 8 irreps, o=20, v=200, Ncd=1500 (even split)",
                                  S.sym_d2h_medium("B")),
            "vvvv_c1_small": ("vvvv density: 1 irrep, o=8, v=40, Ncd=300", S.sym_c1_small()),
            "vvvv_c1_medium": ("vvvv density: 1 irrep, o=20, v=200, Ncd=1500 (the o=20 system without "
                               "point-group symmetry)", S.sym_custom([20], [200], [1500]))}
    if name not in syms:
        raise SystemExit(f"unknown workload {name}")
    desc, sym = syms[name]
    return desc, S.make_density_problem(sym, 0)


def density_main(args, cdcc):
    """One step = one vvvv density contraction; accuracy: every element
    against the oracle (max error relative to max|G|)."""
    import torch
    import oracle as O
    from oracle.layout import OracleLayout
    from tests.gpu_support import to_dev
    desc, prob = density_workload(args.workload)
    sym = prob["sym"]
    lay = cdcc.Layout(sym)
    d = {"layout": lay, "L": to_dev(lay.pack_B(prob["L"])), "X": to_dev(lay.pack_amp(prob["X"])),
         "Y": to_dev(lay.pack_amp(prob["Y"])), "G": torch.zeros(lay.b_size, dtype=torch.float64, device="cuda")}
    fv, fl = lay.density_flops()
    flops = fv + fl
    print(f"[bench] {desc}; F_alg {flops:.4e} ((ab|cd) {fv:.4e}, contraction {fl:.4e})", file=sys.stderr, flush=True)
    cdcc.vvvv_density([d])
    torch.cuda.synchronize()
    acc = None
    if not args.no_check:
        ref = OracleLayout(sym).pack_B(O.vvvv_density_blocks(sym, prob["X"], prob["Y"], prob["L"]))
        err = float(np.max(np.abs(d["G"].cpu().numpy() - ref)))
        acc = {"max_rel": err / float(np.max(np.abs(ref))), "checked": "every element"}
    for _ in range(args.warmup):
        cdcc.vvvv_density([d])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cdcc.vvvv_density([d])
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    cdcc.timing_read()
    cdcc.timing_enable(True)
    for _ in range(args.steps):
        cdcc.vvvv_density([d])
    torch.cuda.synchronize()
    cdcc.timing_enable(False)
    kt = cdcc.timing_read()
    ok = acc is None or acc["max_rel"] <= 1e-12
    print(f"[bench] density: {sec * 1e3:.3f} ms/step, {flops / sec / 1e12:.2f} TFLOP/s, gate ok={ok}, kernels={kt}",
          file=sys.stderr, flush=True)
    g_ms, g_n = kt.get("density_g", (0.0, 0))
    w_ms, w_n = kt.get("density_w", (0.0, 0))
    ach = fl * args.steps / (g_ms * 1e-3) / 1e12 if g_ms else 0.0
    line = {
        "metric": DENSITY_METRIC, "value": round(flops / sec / 1e12, 4), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "flops_per_step": flops, "path": "fp64"},
        "roofline": {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK["fp64"], "unit": "TFLOP/s",
                     "frac": round(ach / PEAK["fp64"], 4),
                     "traffic": TRAFFIC.get((args.workload, "fp64", "gemm")),
                     "kernel": "contraction of the (ab|cd) batch with L", "launches": g_n,
                     "avg_launch_ms": g_ms / max(g_n, 1), "flops_per_launch": fl * args.steps / max(g_n, 1)},
        "stage_ab_cd": {"ms_per_step": w_ms / args.steps, "tflops": fv * args.steps / (w_ms * 1e-3) / 1e12 if w_ms else 0},
        "split_k_reduce_ms_per_step": kt.get("density_r", (0.0, 0))[0] / args.steps,
        "accuracy": acc, "passes_gate": ok, "kernels_ms": kt,
    }
    if not args.no_cpu_baseline:
        try:
            from threadpoolctl import threadpool_info
            cores = max((x.get("num_threads", 1) for x in threadpool_info()), default=os.cpu_count())
        except Exception:  # pragma: no cover
            cores = os.cpu_count()
        reps = 0
        t0 = time.perf_counter()
        while reps < 20 and (reps == 0 or time.perf_counter() - t0 < 10.0):
            O.vvvv_density_blocks(sym, prob["X"], prob["Y"], prob["L"])
            reps += 1
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": flops * reps / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores),
                                "kind": "oracle", "cpu_model": cpu_model(),
                                "sample": f"the whole workload, {reps} oracle runs in {dt:.1f} s"}
    print(json.dumps(line), flush=True)
    if not ok:
        sys.exit(1)


PARTIAL_METRIC = ("O(O^3 V^3) contraction M_bi^dc = sum_mn lambda_bi^mn tau_mn^dc, partial "
                  "symmetric-antisymmetric algorithm, TFLOP/s (FP64)")


def partial_workload(name):
    import synth as S
    syms = {"pm_d2h_medium": ("M_bi^dc contraction: 8 irreps, o=20, v=200", S.sym_d2h_medium("A")),
            "pm_d2h_large": ("M_bi^dc contraction: 8 irreps, o=40, v=400", S.sym_d2h_large()),
            "pm_c1_small": ("M_bi^dc contraction: 1 irrep, o=8, v=40", S.sym_c1_small())}
    if name not in syms:
        raise SystemExit(f"unknown workload {name}")
    desc, sym = syms[name]
    return desc, S.make_partial_problem(sym, 0)


def partial_main(args, cdcc):
    """One step = one M_bi^dc contraction (packing + GEMM); accuracy: every
    element against the oracle's plain definition."""
    import torch
    import oracle as O
    from oracle.layout import OracleLayout
    from tests.gpu_support import to_dev
    desc, prob = partial_workload(args.workload)
    sym = prob["sym"]
    lay = cdcc.Layout(sym)
    d = {"layout": lay, "lam": to_dev(lay.pack_vo(prob["lam"], "oo")), "tau": to_dev(lay.pack_amp(prob["tau"])),
         "M": torch.zeros(lay.mvo_size, dtype=torch.float64, device="cuda")}
    fs, fa = lay.partial_flops()
    flops = fs + fa
    plain = sum(2.0 * lay.n_vo[G] * lay.n_oo[G] * lay.n_vv[G] for G in range(lay.h))
    # algorithmic bytes: lambda and tau read once, M written once
    nbytes = 8.0 * (lay.lvo_size + lay.amp_size + lay.mvo_size)
    print(f"[bench] {desc}; F_alg {flops:.4e} (S {fs:.4e}, A {fa:.4e}; plain {plain:.4e}); "
          f"bytes {nbytes:.4e}", file=sys.stderr, flush=True)
    cdcc.partial_contract([d])
    torch.cuda.synchronize()
    acc = None
    if not args.no_check:
        ref = OracleLayout(sym).pack_vo(O.partial_blocks(sym, prob["lam"], prob["tau"]), "vv")
        err = float(np.max(np.abs(d["M"].cpu().numpy() - ref)))
        acc = {"max_rel": err / float(np.max(np.abs(ref))), "checked": "every element"}
        del ref
    for _ in range(args.warmup):
        cdcc.partial_contract([d])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cdcc.partial_contract([d])
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    cdcc.timing_read()
    cdcc.timing_enable(True)
    for _ in range(args.steps):
        cdcc.partial_contract([d])
    torch.cuda.synchronize()
    cdcc.timing_enable(False)
    kt = cdcc.timing_read()
    ok = acc is None or acc["max_rel"] <= 1e-12
    print(f"[bench] partial: {sec * 1e3:.4f} ms/step, {flops / sec / 1e12:.2f} TFLOP/s, gate ok={ok}, kernels={kt}",
          file=sys.stderr, flush=True)
    g_ms, g_n = kt.get("partial_gemm", (0.0, 0))
    p_ms, _ = kt.get("partial_pack", (0.0, 0))
    g_s = g_ms * 1e-3 / max(g_n, 1)
    # the GEMM kernel reads the packed operands and writes M; its algorithmic
    # bytes are M written once plus lambda+/- and tau+/- read once
    gemm_bytes = 8.0 * lay.mvo_size + 8.0 * (lay.lvo_size + lay.amp_size)
    intensity = flops / gemm_bytes
    if intensity >= PEAK["fp64"] / (HBM_PEAK / 1e3):
        roof = {"bound": "mfma", "achieved": round(flops / g_s / 1e12, 3) if g_ms else 0.0, "peak": PEAK["fp64"],
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": round(gemm_bytes / g_s / 1e9, 1) if g_ms else 0.0, "peak": HBM_PEAK,
                "unit": "GB/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4)
    roof.update({"traffic": TRAFFIC.get((args.workload, "fp64", "gemm")), "kernel": "pm_gemm (S and A, both orders of M)",
                 "launches": g_n, "avg_launch_ms": g_ms / max(g_n, 1), "flops_per_launch": flops,
                 "algorithmic_bytes_per_launch": gemm_bytes, "intensity_flop_per_byte": round(intensity, 2)})
    line = {
        "metric": PARTIAL_METRIC, "value": round(flops / sec / 1e12, 4), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "flops_per_step": flops, "plain_flops": plain, "path": "fp64"},
        "roofline": roof, "pack_ms_per_step": p_ms / args.steps,
        "accuracy": acc, "passes_gate": ok, "kernels_ms": kt,
    }
    if not args.no_cpu_baseline:
        try:
            from threadpoolctl import threadpool_info
            cores = max((x.get("num_threads", 1) for x in threadpool_info()), default=os.cpu_count())
        except Exception:  # pragma: no cover
            cores = os.cpu_count()
        reps = 0
        t0 = time.perf_counter()
        while reps < 20 and (reps == 0 or time.perf_counter() - t0 < 10.0):
            O.partial_blocks(sym, prob["lam"], prob["tau"])
            reps += 1
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": flops * reps / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores),
                                "kind": "oracle", "cpu_model": cpu_model(),
                                "sample": f"the whole workload, {reps} oracle runs (plain definition, "
                                          f"{plain:.3e} flops each) in {dt:.1f} s; rate in the partial "
                                          f"algorithm's flops"}
    print(json.dumps(line), flush=True)
    if not ok:
        sys.exit(1)


CD_METRIC = ("symmetry-adapted two-step Cholesky decomposition (basis + vectors) of a synthetic PSD "
             "integral matrix, wall time")


def cd_workload(name):
    import synth as S
    cfgs = {"cd_d2h": ("two-step CD: 8 irreps x 2000 pairs, tau=1e-6, sigma=1e-2, Q_max=1000",
                       [2000] * 8, 60.0, 1e-6),
            "cd_c1": ("two-step CD: 1 irrep x 4000 pairs, tau=1e-6, sigma=1e-2, Q_max=1000", [4000], 120.0, 1e-6)}
    if name not in cfgs:
        raise SystemExit(f"unknown workload {name}")
    desc, npairs, kappa, tau = cfgs[name]
    return desc, S.make_cd_matrices(npairs, 0, kappa), tau


def cd_main(args, cdcc):
    """One step = cdcc_cd_basis + cdcc_cd_vectors on device-resident
    matrices; the pivots must equal the oracle's and the vectors agree within
    the conditioning-derived tolerance; decomposition error < tau."""
    import torch
    import oracle as O
    from tests.gpu_support import to_dev
    desc, V, tau = cd_workload(args.workload)
    sigma, qmax = 1e-2, 1000
    dV = [to_dev(v) for v in V]
    piv = cdcc.cd_basis(dV, tau, sigma, qmax)
    L = [torch.zeros((v.shape[0], len(p)), dtype=torch.float64, device="cuda") for v, p in zip(V, piv)]
    cdcc.cd_vectors(dV, piv, L)
    torch.cuda.synchronize()
    npiv = int(sum(len(p) for p in piv))
    print(f"[bench] {desc}; {npiv} vectors", file=sys.stderr, flush=True)
    acc = None
    if not args.no_check:
        rpiv, _ = O.cd_basis(V, tau, sigma, qmax)
        same = all(a.tolist() == b.tolist() for a, b in zip(piv, rpiv))
        R = O.cd_vectors(V, rpiv)
        err = rec = 0.0
        ok_v = True
        u = np.finfo(np.float64).eps
        for v, p, l, r in zip(V, piv, L, R):
            if len(p) == 0:
                continue
            ln = l.cpu().numpy()
            kf = np.linalg.cholesky(v[np.ix_(p, p)])
            tol = 64 * np.linalg.cond(kf) * u * np.abs(r).max()
            d = float(np.abs(ln - r).max()) if same else float("inf")
            ok_v &= d <= tol
            err = max(err, d / np.abs(r).max())
            rec = max(rec, float(np.abs(v - ln @ ln.T).max()))
        acc = {"pivots_equal_oracle": same, "vectors_max_rel": err, "vectors_within_tol": bool(ok_v),
               "max_abs_residual": rec, "tau": tau}
    for _ in range(args.warmup):
        p2 = cdcc.cd_basis(dV, tau, sigma, qmax)
        cdcc.cd_vectors(dV, p2, L)
    torch.cuda.synchronize()
    cdcc.timing_read()
    cdcc.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        p2 = cdcc.cd_basis(dV, tau, sigma, qmax)
        cdcc.cd_vectors(dV, p2, L)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    cdcc.timing_enable(False)
    kt = cdcc.timing_read()
    ok = acc is None or (acc["pivots_equal_oracle"] and acc["vectors_within_tol"] and acc["max_abs_residual"] < tau)
    ms = {k: v[0] / args.steps for k, v in kt.items() if k.startswith("cd_")}
    print(f"[bench] cd: {sec * 1e3:.3f} ms/step, per class {ms}, gate ok={ok}", file=sys.stderr, flush=True)
    # dominant phase: the micro iterations, one argmax launch and one column
    # launch per vector (dependent, so latency-bound)
    micro_ms = ms.get("cd_micro", 0.0)
    line = {
        "metric": CD_METRIC, "value": round(sec * 1e3, 4), "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": desc, "vectors": npiv, "path": "fp64"},
        "phases_ms_per_step": ms, "micro_us_per_vector": round(micro_ms * 1e3 / max(npiv, 1), 3),
        "roofline": {"bound": "latency", "achieved": round(micro_ms * 1e3 / max(npiv, 1), 3), "peak": None,
                     "unit": "us per vector (one dependent launch)", "frac": None, "traffic": None,
                     "kernel": "cd_micro_kernel (micro iterations)"},
        "accuracy": acc, "passes_gate": ok, "kernels_ms": kt,
    }
    if not args.no_cpu_baseline:
        try:
            from threadpoolctl import threadpool_info
            cores = max((x.get("num_threads", 1) for x in threadpool_info()), default=os.cpu_count())
        except Exception:  # pragma: no cover
            cores = os.cpu_count()
        reps = 0
        t0 = time.perf_counter()
        while reps < 20 and (reps == 0 or time.perf_counter() - t0 < 10.0):
            rp, _ = O.cd_basis(V, tau, sigma, qmax)
            O.cd_vectors(V, rp)
            reps += 1
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": dt / reps * 1e3, "unit": "ms", "cores": int(cores), "kind": "oracle", "cpu_model": cpu_model(),
                                "sample": f"the whole workload, {reps} oracle runs in {dt:.1f} s"}
    print(json.dumps(line), flush=True)
    if not ok:
        sys.exit(1)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="d2h_large")
    ap.add_argument("--extras", default=None,
                    help="comma-separated extra ladder workloads measured beside the headline one "
                         "(default with d2h_large: d2h_medium,batch64; 'none' to skip)")
    ap.add_argument("--precision", default="all", choices=["all", "fp64", "mixed", "mixed_i8"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-1t", type=float, default=6.0,
                    help="seconds of the one-thread CPU baseline of the extra workloads (0 = skip)")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle accuracy gate")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for HBM byte counters)")
    ap.add_argument("--tile-policy", type=int, default=0, help="0 = tile table, 1..4 force a tile class")
    ap.add_argument("--serving", type=int, default=2000,
                    help="requests of each measured serving run (0 = skip the serving runs)")
    ap.add_argument("--serving-warmup", type=int, default=200, help="warm-up requests before the serving runs")
    ap.add_argument("--serving-load", type=float, default=0.7, help="Poisson rate as a fraction of saturation")
    ap.add_argument("--serving-precisions", default="fp64,mixed")
    ap.add_argument("--serving-sweep", default=None,
                    help="comma-separated loads: only the serving sweep (saturation, one stream per load)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the ladder library runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.extras is None:
        args.extras = "d2h_medium,batch64" if args.workload == "d2h_large" else ""

    import torch
    import paper_2512_21909_amd as cdcc
    cdcc.require_gpu()
    global TILE_POLICY
    TILE_POLICY = args.tile_policy
    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.serving_sweep:
        serving_sweep_main(args, cdcc)
        return
    if args.workload.startswith("vvvv_"):
        density_main(args, cdcc)
        return
    if args.workload.startswith("pm_"):
        partial_main(args, cdcc)
        return
    if args.workload.startswith("cd_"):
        cd_main(args, cdcc)
        return
    ladder_main(args, cdcc)


if __name__ == "__main__":
    main()
