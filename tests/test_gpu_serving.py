"""Serving loop: results identical alone and in the mix (the large
o=30/v=300 request included) and equal to the oracle, admission by HBM
footprint, and clean failure of one request without failing the others."""
import os

import numpy as np
import pytest

import synth as S
from tests.gpu_support import to_dev

pytestmark = pytest.mark.gpu


def _pool(cdcc, syms, seed=0, large=None, keep=False):
    """Device-resident request inputs; ``large`` marks the last shape as the
    large request; ``keep`` also returns the generator problems."""
    pool = []
    for k, sym in enumerate(syms):
        p = S.make_problem(sym, seed=seed + k, kind="t2")
        lay = cdcc.Layout(sym)
        pool.append({"layout": lay, "B": to_dev(lay.pack_B(p["B"])), "X": to_dev(lay.pack_amp(p["X"])),
                     "flops": sum(lay.flops(0)), "large": bool(large) and k == len(syms) - 1})
        if keep:
            pool[-1]["prob"] = p
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


def test_large_requests_run_alone(gpu_lib):
    """Under the default policy a request of at least ``solo_flops`` is a
    batch of its own, the small requests are still batched together, and
    every result equals its standalone one bitwise."""
    import torch
    from paper_2512_21909_amd import serve
    pool = _pool(gpu_lib, S.batch_syms(4, seed=3) + [S.sym_custom([10, 8], [90, 80], [700, 600])])
    reqs = [serve.Request(rid=k, arrival=0.0, layout=pool[k % 5]["layout"], B=pool[k % 5]["B"],
                          X=pool[k % 5]["X"], flops=pool[k % 5]["flops"], want_energy=True) for k in range(20)]
    solo = sorted({r.flops for r in reqs})[-1]
    assert solo > 4 * sorted({r.flops for r in reqs})[-2]
    srv = serve.LadderServer(int(torch.cuda.mem_get_info()[0] * 0.5), n_streams=3, max_batch=8, solo_flops=solo)
    done = srv.serve(reqs)
    assert sorted(r.rid for r in done) == list(range(20)) and all(r.status == "done" for r in done)
    batches = [[r for r in done if r.t_launch == t] for t in {r.t_launch for r in done}]
    for b in batches:
        if any(r.flops >= solo for r in b):
            assert len(b) == 1
    assert max(len(b) for b in batches) > 1
    for r in done:
        Ra, Ea = _alone(gpu_lib, r, "fp64")
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
    pool = _pool(gpu_lib, S.batch_syms(4, seed=9))
    out = serve.measure_sweep(pool, "mixed", n_requests=24, loads=(0.3, 0.9), warmup=4, max_batch=4)
    assert out["saturation"]["done"] == 24 and out["saturation"]["requests_per_s"] > 0
    assert [s["load"] for s in out["streams"]] == [0.3, 0.9]
    for s in out["streams"]:
        assert s["done"] == 24 and s["rejected"] == 0 and s["failed"] == 0
        assert s["rate_hz"] == pytest.approx(s["load"] * out["saturation"]["requests_per_s"])
        assert 0 < s["p50_ms"] <= s["p99_ms"]


_MIX_REF = {}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mix_with_the_large_request_matches_alone_and_oracle(gpu_lib, precision):
    """The serving mix with the large request (o=30, v=300, 2500 vectors, 8
    irreps, drawn with probability 0.3 here and batched like the small ones,
    so that it lands in batches with them): every request completes, equals
    its standalone result bitwise, and every distinct shape matches the
    oracle (R normwise, pair energies) within the path's tolerance."""
    import torch
    import oracle as O
    from paper_2512_21909_amd import serve
    pool = _pool(gpu_lib, S.batch_syms(5, seed=11) + [S.sym_serving_large()], seed=40, large=True, keep=True)
    reqs = serve.make_stream(pool, 30, 0.0, seed=3, p_large=0.3)
    assert 3 <= sum(r.layout is pool[-1]["layout"] for r in reqs) < 30
    srv = serve.LadderServer(int(torch.cuda.mem_get_info()[0] * 0.5), n_streams=3, precision=precision, max_batch=6,
                             solo_flops=None)
    done = srv.serve(reqs)
    assert sorted(r.rid for r in done) == list(range(30)) and all(r.status == "done" for r in done)
    tol = 1e-12 if precision == "fp64" else 1e-7
    checked = set()
    for r in done:
        Ra, Ea = _alone(gpu_lib, r, precision)
        assert np.array_equal(r.R.cpu().numpy(), Ra), r.rid
        assert np.array_equal(r.pair_energy.cpu().numpy(), Ea), r.rid
        k = next(i for i, p in enumerate(pool) if p["layout"] is r.layout)
        if k in checked:
            continue
        checked.add(k)
        p = pool[k]["prob"]
        if k not in _MIX_REF:
            ref = O.t2_ladder_blocks(p["sym"], p["B"], p["X"])
            _MIX_REF[k] = (ref, O.pair_energies_blocks(p["sym"], p["X"], ref))
        ref, e_ref = _MIX_REF[k]
        mx, fro = O.rel_errors(r.layout.unpack_amp(Ra), ref)
        assert mx <= tol and fro <= tol, (k, mx, fro)
        err_e = float(np.max(np.abs(Ea.reshape(e_ref.shape) - e_ref)))
        assert err_e <= (1e-12 * max(1.0, float(np.max(np.abs(e_ref)))) if precision == "fp64" else 1e-8), (k, err_e)
    assert len(pool) - 1 in checked
