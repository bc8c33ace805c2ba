"""Serving loop: results identical alone and in the mix, admission by HBM
footprint, and clean failure of one request without failing the others."""
import os

import numpy as np
import pytest

import synth as S
from tests.gpu_support import to_dev

pytestmark = pytest.mark.gpu


def _pool(cdcc, syms, seed=0):
    pool = []
    for k, sym in enumerate(syms):
        p = S.make_problem(sym, seed=seed + k, kind="t2")
        lay = cdcc.Layout(sym)
        pool.append({"layout": lay, "B": to_dev(lay.pack_B(p["B"])), "X": to_dev(lay.pack_amp(p["X"])),
                     "flops": sum(lay.flops(0)), "large": False})
    return pool


def _requests(serve, pool, n, seed=1):
    return serve.make_stream(pool, n, 0.0, seed=seed, p_large=0.0)


def _alone(cdcc, req, precision):
    import torch
    R = torch.empty(req.layout.amp_size, dtype=torch.float64, device="cuda")
    E = torch.empty(req.layout.nocc_tot ** 2, dtype=torch.float64, device="cuda")
    cdcc.ladder_t2({"layout": req.layout, "B": req.B, "X": req.X, "R": R, "pair_energy": E}, precision=precision)
    torch.cuda.synchronize()
    return R.cpu().numpy(), E.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_i8"])
def test_results_identical_alone_and_in_the_mix(gpu_lib, precision):
    import torch
    from paper_2512_21909_amd import serve
    pool = _pool(gpu_lib, S.batch_syms(6, seed=3))
    reqs = _requests(serve, pool, 24)
    srv = serve.LadderServer(int(torch.cuda.mem_get_info()[0] * 0.5), n_streams=3, precision=precision, max_batch=5)
    done = srv.serve(reqs)
    assert sorted(r.rid for r in done) == list(range(24))
    assert all(r.status == "done" for r in done)
    assert max(len(b) for b in [[r for r in done if r.t_launch == t] for t in {r.t_launch for r in done}]) > 1
    for r in done:
        Ra, Ea = _alone(gpu_lib, r, precision)
        assert np.array_equal(r.R.cpu().numpy(), Ra), r.rid
        assert np.array_equal(r.pair_energy.cpu().numpy(), Ea), r.rid


def test_admission_rejects_oversize_and_serves_the_rest(gpu_lib):
    from paper_2512_21909_amd import serve
    pool = _pool(gpu_lib, [S.sym_custom([2, 1], [6, 5], [20, 9]), S.sym_c1_small()])
    small, big = pool
    need_big = big["layout"].amp_size * 8 + gpu_lib.workspace_bytes(
        {"layout": big["layout"], "B": big["B"], "X": big["X"], "R": big["X"]})
    reqs = [serve.Request(rid=k, arrival=0.0, layout=p["layout"], B=p["B"], X=p["X"], flops=p["flops"])
            for k, p in enumerate([small, big, small, small])]
    srv = serve.LadderServer(need_big - 1, n_streams=2)
    done = {r.rid: r for r in srv.serve(reqs)}
    assert done[1].status == "rejected"
    assert all(done[k].status == "done" for k in (0, 2, 3))


def test_allocation_failure_fails_one_request_only(gpu_lib):
    from paper_2512_21909_amd import serve
    gpu_lib.release()
    pool = _pool(gpu_lib, [S.sym_custom([2, 1], [6, 5], [20, 9]), S.sym_custom([1, 2], [5, 7], [11, 16]),
                           S.sym_c1_small()])
    ws = [gpu_lib.workspace_bytes({"layout": p["layout"], "B": p["B"], "X": p["X"], "R": p["X"]}) for p in pool]
    small_max = max(ws[:2])
    assert ws[2] > 2 * small_max
    reqs = [serve.Request(rid=k, arrival=0.0, layout=pool[k % 3]["layout"], B=pool[k % 3]["B"],
                          X=pool[k % 3]["X"], flops=pool[k % 3]["flops"]) for k in range(9)]
    os.environ["CDCC_FAIL_ALLOC_ABOVE"] = str(small_max + 1)   # any batch of two, and the big one, fail
    try:
        srv = serve.LadderServer(1 << 34, n_streams=1, max_batch=9)
        done = {r.rid: r for r in srv.serve(reqs)}
    finally:
        del os.environ["CDCC_FAIL_ALLOC_ABOVE"]
        gpu_lib.release()
    for k, r in done.items():
        if k % 3 == 2:
            assert r.status == "failed" and "status -2" in r.error
        else:
            assert r.status == "done", (k, r.status, r.error)
            Ra, _ = _alone(gpu_lib, r, "fp64")
            assert np.array_equal(r.R.cpu().numpy(), Ra)


def test_load_sweep_reports_every_load(gpu_lib):
    """The sweep measures saturation once and one Poisson stream per load;
    every request of every run completes."""
    from paper_2512_21909_amd import serve
    out = serve.measure_sweep("mixed", n_requests=24, loads=(0.3, 0.9), warmup=4, max_batch=4)
    assert out["saturation"]["done"] == 24 and out["saturation"]["requests_per_s"] > 0
    assert [s["load"] for s in out["streams"]] == [0.3, 0.9]
    for s in out["streams"]:
        assert s["done"] == 24 and s["rejected"] == 0 and s["failed"] == 0
        assert s["rate_hz"] == pytest.approx(s["load"] * out["saturation"]["requests_per_s"])
        assert 0 < s["p50_ms"] <= s["p99_ms"]
