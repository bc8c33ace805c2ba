"""Tile autotuner: times every assembly tile class of the library per system
shape, kind (T2 / Lambda) and precision, and writes the fastest into
tile_table.txt next to libcdcc.so (the library reads it when it builds a plan;
the key is the exact symmetry shape, so a system's tile shape never depends on
what else is in its batch).

Usage (on the GPU): python -m paper_2512_21909_amd.autotune [--workloads ...]
"""
from __future__ import annotations

import argparse
import os
import time

from . import _lib

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile_table.txt")


def shape_key(sym: dict, precision: str, kind: str) -> str:
    h = sym["h"]
    vals = [precision, kind, str(h)] + [str(x) for a in ("nocc", "nvir", "ncd") for x in sym[a][:h]]
    return " ".join(vals)


def load_table(path: str = TABLE) -> dict:
    out = {}
    if os.path.exists(path):
        for line in open(path):
            line = line.strip()
            if line and not line.startswith("#"):
                key, cls = line.rsplit(" ", 1)
                out[key] = int(cls)
    return out


def write_table(table: dict, path: str = TABLE) -> None:
    with open(path, "w") as f:
        f.write("# precision kind h nocc[h] nvir[h] ncd[h] -> assembly tile class "
                "(fp64: 0=64x64 1=128x64 2=128x128; mixed, mixed_i8: 0=64x128 1=128x64 2=128x128/8 waves 3=64x64)\n")
        for k in sorted(table):
            f.write(f"{k} {table[k]}\n")


NCLASS = {"fp64": 3, "mixed": 4, "mixed_i8": 4}


def time_classes(cdcc, dev_problem: dict, kind: str, precision: str, reps: int = 3) -> list[float]:
    """Assembly milliseconds per call for every tile class of the path."""
    import torch
    fn = cdcc.ladder_t2 if kind == "t2" else cdcc.ladder_lambda
    out = []
    for cls in range(NCLASS[precision]):
        fn(dev_problem, precision=precision, tile_policy=cls + 1)   # plan + warm-up
        torch.cuda.synchronize()
        cdcc.timing_read()
        cdcc.timing_enable(True)
        for _ in range(reps):
            fn(dev_problem, precision=precision, tile_policy=cls + 1)
        torch.cuda.synchronize()
        cdcc.timing_enable(False)
        ms, n = cdcc.timing_read().get("assemble", (0.0, 0))
        out.append(ms / max(reps, 1))
    return out


def tune(syms: list[dict], kinds=("t2", "lambda"), precisions=("fp64", "mixed", "mixed_i8"), seed: int = 0,
         table: dict | None = None, log=print) -> dict:
    import synth as S
    import paper_2512_21909_amd as cdcc
    from tests.gpu_support import device_problem
    table = dict(table or {})
    for sym in syms:
        for kind in kinds:
            p = S.make_problem(sym, seed=seed, kind=kind)
            d = device_problem(cdcc, p, nan_fill=False)
            for prec in precisions:
                t = time_classes(cdcc, d, kind, prec)
                best = min(range(len(t)), key=lambda c: t[c])
                table[shape_key(sym, prec, kind)] = best
                log(f"[autotune] {prec} {kind} h={sym['h']} o={sum(sym['nocc'])} v={sum(sym['nvir'])} "
                    f"N={sum(sym['ncd'])}: assembly ms per class {[round(x, 3) for x in t]} -> {best}")
            del d
    return table


def main():
    import synth as S
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workloads", default="c1_small,d2h_medium,d2h_medium_B,serving_large,batch64")
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--precisions", default="fp64,mixed,mixed_i8", help="paths to tune (the others keep their entries)")
    args = ap.parse_args()
    precs = tuple(p for p in args.precisions.split(",") if p)
    syms, kinds = [], {}
    for w in args.workloads.split(","):
        if w == "c1_small":
            syms.append((S.sym_c1_small(), ("t2", "lambda")))
        elif w == "d2h_medium":
            syms.append((S.sym_d2h_medium("A"), ("t2", "lambda")))
        elif w == "d2h_medium_B":
            syms.append((S.sym_d2h_medium("B"), ("t2", "lambda")))
        elif w == "d2h_large":
            syms.append((S.sym_d2h_large(), ("t2", "lambda")))
        elif w == "serving_large":
            syms.append((S.sym_serving_large(), ("t2",)))
        elif w == "batch64":
            syms += [(s, ("t2",)) for s in S.batch_syms(64, seed=0)]
        else:
            raise SystemExit(f"unknown workload {w}")
    t0 = time.time()
    table = load_table(args.out)
    for sym, ks in syms:
        table = tune([sym], kinds=ks, precisions=precs, table=table)
    write_table(table, args.out)
    _lib.load().cdcc_release()
    print(f"[autotune] {len(table)} entries -> {args.out} in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
