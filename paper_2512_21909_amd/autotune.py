"""Tile autotuner.

For a system shape, kind (T2 / Lambda) and precision it times every
assembly tile class of the library and then, with the fastest class, a set
of contraction K-segment lengths, on random inputs of that shape, and keeps
the fastest pair.  Results are persisted in ``tile_cache.json`` (JSON, one
entry per key with the measured times) and written to ``tile_table.txt``
next to ``libcdcc.so``, which the library reads when it builds a plan.

Two kinds of keys: the exact shape, and the shape's size class
(``cdcc_tile_key``: half-octave buckets of its assembly tile count, mean
Cholesky length and largest contraction row count).  A shape never tuned
itself takes the choice of its size class, so serving requests of unseen
shapes get a tuned choice.  ``ensure`` tunes the size classes of the given
shapes that have no entry yet (tune on a miss) and reloads the library's
table; the binding calls it before each ladder call when CDCC_AUTOTUNE=1.
A tile class never changes an element's arithmetic in the assembly, and the
K-segment length is fixed per shape, so a system's result is the same alone
and in any batch.

Usage (on the GPU): python -m paper_2512_21909_amd.autotune shapes.json
"""
from __future__ import annotations

import argparse
import json
import os
import time

from . import _lib

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile_table.txt")
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile_cache.json")
HEADER = ("# key -> assembly tile class[:contraction K segment] (fp64: 0=64x64 1=128x64 2=128x128; mixed, "
          "mixed_i8: 0=64x128 1=128x64 2=128x128 (4 waves of 64x64; 8-bit Lambda stacks: 8 waves) 3=64x64); keys: "
          "'<precision> <kind> h nocc[h] nvir[h] ncd[h]' (exact shape) or '<precision> <kind> b<h> <T> <K> <M>' "
          "(size class)")
NCLASS = {"fp64": 3, "mixed": 4, "mixed_i8": 4}
KSEGS = (0, 1024, 2048, 4096)


def shape_key(sym: dict, precision: str, kind: str) -> str:
    h = sym["h"]
    vals = [precision, kind, str(h)] + [str(x) for a in ("nocc", "nvir", "ncd") for x in sym[a][:h]]
    return " ".join(vals)


def load_table(path: str = TABLE) -> dict:
    """{key: "class" or "class:kseg"}"""
    out = {}
    if os.path.exists(path):
        for line in open(path):
            line = line.strip()
            if line and not line.startswith("#"):
                key, val = line.rsplit(" ", 1)
                out[key] = val
    return out


def write_table(table: dict, path: str = TABLE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write(HEADER + "\n")
        for k in sorted(table):
            f.write(f"{k} {table[k]}\n")
    os.replace(tmp, path)


def load_cache(path: str = CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {"entries": {}}


def save_cache(cache: dict, path: str = CACHE) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def random_problem(cdcc, sym: dict, kind: str, seed: int = 0) -> dict:
    """Device buffers of one ladder call with random values of a realistic
    scale (timing does not depend on the values)."""
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


def _time(cdcc, d, kind, precision, cls, kseg, which, reps):
    import torch
    fn = cdcc.ladder_t2 if kind == "t2" else cdcc.ladder_lambda
    kw = {"precision": precision, "tile_policy": cls + 1, "contract_kseg": kseg}
    fn(d, **kw)                                  # plan + warm-up
    torch.cuda.synchronize()
    cdcc.timing_read()
    cdcc.timing_enable(True)
    for _ in range(reps):
        fn(d, **kw)
    torch.cuda.synchronize()
    cdcc.timing_enable(False)
    return cdcc.timing_read().get(which, (0.0, 0))[0] / max(reps, 1)


def tune_shape(cdcc, sym: dict, kind: str, precision: str, reps: int = 3, seed: int = 0) -> dict:
    """Fastest assembly class, then fastest contraction K segment with it."""
    d = random_problem(cdcc, sym, kind, seed)
    asm = [_time(cdcc, d, kind, precision, c, 0, "assemble", reps) for c in range(NCLASS[precision])]
    best = min(range(len(asm)), key=lambda c: asm[c])
    con = {k: _time(cdcc, d, kind, precision, best, k, "contract", reps) for k in KSEGS}
    kbest = min(KSEGS, key=lambda k: con[k])
    return {"class": best, "kseg": kbest, "assembly_ms": [round(x, 4) for x in asm],
            "contract_ms": {str(k): round(v, 4) for k, v in con.items()},
            "shape": {k: sym[k] for k in ("h", "nocc", "nvir", "ncd")}, "precision": precision, "kind": kind}


def _table_value(entry: dict) -> str:
    return f"{entry['class']}:{entry['kseg']}" if entry.get("kseg") else str(entry["class"])


def ensure(syms: list, kind: str, precision: str, cache_path: str = CACHE, table_path: str = TABLE,
           reps: int = 3, log=None) -> list:
    """Tune on a miss: every shape whose exact key and size class are both
    absent from the table gets its size class tuned (persisted in the JSON
    cache and the table); the library then rereads the table.  Returns the
    size-class keys of the shapes."""
    import paper_2512_21909_amd as cdcc
    from .ladder import tile_key, tile_table_reload
    table = load_table(table_path)
    cache = load_cache(cache_path)
    keys, changed = [], False
    for sym in syms:
        key = tile_key(sym, precision, kind)
        keys.append(key)
        if key in table or shape_key(sym, precision, kind) in table:
            continue
        if key not in cache["entries"]:
            t0 = time.time()
            cache["entries"][key] = tune_shape(cdcc, sym, kind, precision, reps)
            if log:
                log(f"[autotune] {key}: {cache['entries'][key]} in {time.time() - t0:.1f} s")
        table[key] = _table_value(cache["entries"][key])
        changed = True
    if changed:
        save_cache(cache, cache_path)
        write_table(table, table_path)
        tile_table_reload(table_path if table_path != TABLE else None)
    return keys


def main():
    """Tune the shapes listed in a JSON file: a list of {"nocc": [...],
    "nvir": [...], "ncd": [...], "kinds": ["t2", "lambda"]} objects; each
    gets an exact entry and, if absent, a size-class entry."""
    import paper_2512_21909_amd as cdcc
    from .ladder import tile_key
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("shapes", help="JSON file with the shapes to tune")
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--cache", default=CACHE)
    ap.add_argument("--precisions", default="fp64,mixed,mixed_i8", help="paths to tune (the others keep their entries)")
    args = ap.parse_args()
    precs = tuple(p for p in args.precisions.split(",") if p)
    t0 = time.time()
    table, cache = load_table(args.out), load_cache(args.cache)
    for e in json.load(open(args.shapes)):
        sym = {"h": len(e["nocc"]), "nocc": list(e["nocc"]), "nvir": list(e["nvir"]), "ncd": list(e["ncd"])}
        for kind in e.get("kinds", ("t2",)):
            for prec in precs:
                ent = tune_shape(cdcc, sym, kind, prec)
                table[shape_key(sym, prec, kind)] = _table_value(ent)
                bkey = tile_key(sym, prec, kind)
                cache["entries"].setdefault(bkey, ent)
                table.setdefault(bkey, _table_value(cache["entries"][bkey]))
                print(f"[autotune] {shape_key(sym, prec, kind)}: {ent['class']}:{ent['kseg']}", flush=True)
    save_cache(cache, args.cache)
    write_table(table, args.out)
    _lib.load().cdcc_release()
    print(f"[autotune] {len(table)} entries -> {args.out} in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
