"""Autotuner: a shape in no table gets its size class tuned on a miss, the
choice is persisted (JSON cache and tile table) and used by the library, and
results are bitwise the same for every assembly tile class at the tuned
contraction segment."""
import json

import numpy as np
import pytest

import synth as S
from tests.gpu_support import device_problem, problem, run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_unseen_shape_gets_a_tuned_class(gpu_lib, tmp_path, precision):
    from paper_2512_21909_amd import autotune
    cdcc = gpu_lib
    sym = S.sym_custom([3, 2, 2, 1], [23, 17, 19, 11], [61, 29, 40, 33])
    table, cache = str(tmp_path / "tile_table.txt"), str(tmp_path / "tile_cache.json")
    try:
        (key,) = autotune.ensure([sym], "t2", precision, cache_path=cache, table_path=table, reps=1)
        entry = json.load(open(cache))["entries"][key]
        assert 0 <= entry["class"] < autotune.NCLASS[precision] and entry["kseg"] in autotune.KSEGS
        assert autotune.load_table(table)[key] == autotune._table_value(entry)
        # a second call finds it (no retuning)
        assert autotune.ensure([sym], "t2", precision, cache_path=cache, table_path=table) == [key]
        prob = problem(sym, seed=70)
        d0 = device_problem(cdcc, prob)
        run(cdcc, d0, precision=precision)                      # the library's choice from the table
        r0 = d0["R"].cpu().numpy()
        for cls in range(autotune.NCLASS[precision]):
            d = device_problem(cdcc, prob)
            run(cdcc, d, precision=precision, tile_policy=cls + 1, contract_kseg=entry["kseg"])
            assert np.array_equal(d["R"].cpu().numpy(), r0), cls
    finally:
        cdcc.ladder.tile_table_reload(None)
