"""Tile autotuner: times every assembly tile class of the library per system
shape, kind (T2 / Lambda) and precision, and writes the fastest into
tile_table.txt next to libcdcc.so (the library reads it when it builds a plan;
the key is the exact symmetry shape, so a system's tile shape never depends on
what else is in its batch).

Usage (on the GPU): python -m paper_2512_21909_amd.autotune shapes.json
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


def random_problem(cdcc, sym: dict, kind: str, seed: int = 0) -> dict:
    """Device buffers of one ladder call with random values of a realistic
    scale (timing does not depend on the values; the tile class never changes
    an element's arithmetic)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    lay = cdcc.Layout(sym)

    def rnd(n, scale):
        return torch.randn(max(n, 1), generator=g, dtype=torch.float64, device="cuda")[:n] * scale

    d = {"layout": lay, "B": rnd(lay.b_size, 1.0), "X": rnd(lay.amp_size, 1e-3),
         "R": torch.empty(lay.amp_size, dtype=torch.float64, device="cuda")}
    if kind == "lambda":
        d["Bvo"], d["t1"] = rnd(lay.bvo_size, 1.0), rnd(lay.t1_size, 1e-3)
    return d


def tune(syms: list[dict], kinds=("t2", "lambda"), precisions=("fp64", "mixed", "mixed_i8"), seed: int = 0,
         table: dict | None = None, log=print) -> dict:
    import paper_2512_21909_amd as cdcc
    table = dict(table or {})
    for sym in syms:
        for kind in kinds:
            d = random_problem(cdcc, sym, kind, seed)
            for prec in precisions:
                t = time_classes(cdcc, d, kind, prec)
                best = min(range(len(t)), key=lambda c: t[c])
                table[shape_key(sym, prec, kind)] = best
                log(f"[autotune] {prec} {kind} h={sym['h']} o={sum(sym['nocc'])} v={sum(sym['nvir'])} "
                    f"N={sum(sym['ncd'])}: assembly ms per class {[round(x, 3) for x in t]} -> {best}")
            del d
    return table


def main():
    """Tune the shapes listed in a JSON file: a list of {"nocc": [...],
    "nvir": [...], "ncd": [...], "kinds": ["t2", "lambda"]} objects."""
    import json
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("shapes", help="JSON file with the shapes to tune")
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--precisions", default="fp64,mixed,mixed_i8", help="paths to tune (the others keep their entries)")
    args = ap.parse_args()
    precs = tuple(p for p in args.precisions.split(",") if p)
    t0 = time.time()
    table = load_table(args.out)
    for e in json.load(open(args.shapes)):
        sym = {"h": len(e["nocc"]), "nocc": list(e["nocc"]), "nvir": list(e["nvir"]), "ncd": list(e["ncd"])}
        table = tune([sym], kinds=tuple(e.get("kinds", ("t2",))), precisions=precs, table=table)
    write_table(table, args.out)
    _lib.load().cdcc_release()
    print(f"[autotune] {len(table)} entries -> {args.out} in {time.time() - t0:.1f} s")
