"""The allocation-free T2 entry point (cdcc_ladder_t2_noalloc, through the C
ABI) against the allocating one: two calls in a row on the shared static
scratch, the second with a smaller system, each equal to cdcc_ladder_t2's
result (bitwise: the batch cap only changes which columns share a batch,
never an element's arithmetic) and within the oracle tolerance; FP64 and
split-BF16; a problem beyond the scratch is refused with CDCC_ESCRATCH
before anything runs."""
import numpy as np
import pytest

import synth as S
from tests.gpu_support import blocks, device_problem, oracle_result, problem, run

pytestmark = pytest.mark.gpu


def _rel(got, ref):
    import oracle as O
    return O.rel_errors(got, ref)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_allocating_entry_point(gpu_lib, precision):
    import torch
    cdcc = gpu_lib
    big = problem(S.sym_d2h_medium("B"), seed=31)                           # 8 irreps, o=20, v=200
    small = problem(S.sym_custom([3, 2, 1, 2], [17, 11, 9, 13], [40, 22, 0, 31]), seed=32)
    tol = 1e-12 if precision == "fp64" else 1e-7
    for prob in (big, small):                      # second call: a smaller input on the same scratch
        d_ref = device_problem(cdcc, prob, want_delta=True, want_energy=True)
        run(cdcc, d_ref, precision=precision)
        d = device_problem(cdcc, prob, want_delta=True, want_energy=True)
        cdcc.ladder_t2_noalloc(d, precision=precision)
        torch.cuda.synchronize()
        for key in ("R", "delta", "pair_energy"):
            a, b = d[key].cpu().numpy(), d_ref[key].cpu().numpy()
            assert np.all(np.isfinite(a)), key
            assert np.array_equal(a, b), key
        mx, fro = _rel(blocks(d), oracle_result(prob))
        assert mx <= tol and fro <= tol, (mx, fro)


def test_noalloc_rejects_problems_beyond_the_scratch(gpu_lib):
    """o=256, v=48 (C1): the packed +/- amplitudes alone (2 x 32896 x 1176
    doubles, 619 MB) exceed the 256 MiB scratch; the call is refused before
    anything is enqueued (the buffers are never read)."""
    import torch
    from paper_2512_21909_amd._lib import CdccError, ESCRATCH
    cdcc = gpu_lib
    lay = cdcc.Layout(S.sym_custom([256], [48], [8]))
    d = {"layout": lay, "B": torch.empty(lay.b_size, dtype=torch.float64, device="cuda"),
         "X": torch.empty(lay.amp_size, dtype=torch.float64, device="cuda"),
         "R": torch.empty(lay.amp_size, dtype=torch.float64, device="cuda")}
    with pytest.raises(CdccError) as e:
        cdcc.ladder_t2_noalloc(d)
    assert e.value.status == ESCRATCH
