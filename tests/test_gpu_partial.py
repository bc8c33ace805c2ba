"""GPU parity of the O(O^3 V^3) contraction M_bi^dc = sum_mn lambda_bi^mn
tau~_mn^dc with the partial symmetric-antisymmetric algorithm (through the C
ABI) against the oracle's plain definition: ragged and empty irreps, irreps
without occupied orbitals (K = 0 blocks), virtual irreps smaller than and not
a multiple of the 8-wide squares, C1 and 8-irrep shapes, several systems in
one call (bitwise equal alone), repeatability."""
import numpy as np
import pytest

import synth as S

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _dev(cdcc, prob):
    import torch
    from gpu_support import to_dev
    lay = cdcc.Layout(prob["sym"])
    return {"layout": lay, "lam": to_dev(lay.pack_vo(prob["lam"], "oo")), "tau": to_dev(lay.pack_amp(prob["tau"])),
            "M": torch.full((lay.mvo_size,), float("nan"), dtype=torch.float64, device="cuda")}


def _run(cdcc, ds):
    import torch
    cdcc.partial_contract(ds)
    torch.cuda.synchronize()


def _ref(prob):
    import oracle as O
    from oracle.layout import OracleLayout
    lay = OracleLayout(prob["sym"])
    return lay.pack_vo(O.partial_blocks(prob["sym"], prob["lam"], prob["tau"]), "vv")


def _rel(got, ref):
    d = np.abs(got - ref)
    return float(d.max() / max(np.abs(ref).max(), 1e-300))


SYMS = [
    ([3], [5], [1]),
    ([2, 1], [3, 4], [1, 1]),
    ([1, 2, 0, 1], [3, 2, 4, 1], [1, 1, 1, 1]),
    ([1, 1, 1, 0, 1, 0, 1, 1], [2, 3, 1, 2, 0, 2, 1, 3], [1] * 8),
    ([0, 2], [5, 3], [1, 1]),                    # an irrep without occupied orbitals
    ([2, 3, 1, 2], [9, 0, 7, 17], [1] * 4),      # an empty virtual irrep, squares with 1 and 9 columns
    ([1], [1], [1]),                             # one orbital of each kind
]


@pytest.mark.parametrize("spec", SYMS)
def test_small_systems(gpu_lib, spec):
    cdcc = gpu_lib
    prob = S.make_partial_problem(S.sym_custom(*spec), seed=3)
    d = _dev(cdcc, prob)
    _run(cdcc, [d])
    got = d["M"].cpu().numpy()
    assert np.all(np.isfinite(got))
    assert _rel(got, _ref(prob)) <= TOL


@pytest.mark.parametrize("sym", [S.sym_c1_small(), S.sym_custom([4, 2, 3, 2], [20, 11, 15, 10], [1] * 4),
                                 S.sym_custom([4, 2, 3, 2, 3, 2, 2, 2], [40, 22, 30, 20, 32, 18, 22, 16], [1] * 8)],
                         ids=["c1", "c2v_like", "d2h_o20_v200"])
def test_named_shapes(gpu_lib, sym):
    cdcc = gpu_lib
    prob = S.make_partial_problem(sym, seed=5)
    d = _dev(cdcc, prob)
    _run(cdcc, [d])
    got = d["M"].cpu().numpy()
    assert np.all(np.isfinite(got))
    assert _rel(got, _ref(prob)) <= TOL


def test_batched_systems_equal_alone(gpu_lib):
    cdcc = gpu_lib
    probs = [S.make_partial_problem(S.sym_custom(*spec), seed=10 + k) for k, spec in enumerate(SYMS)]
    alone = []
    for p in probs:
        d = _dev(cdcc, p)
        _run(cdcc, [d])
        alone.append(d["M"].cpu().numpy())
    ds = [_dev(cdcc, p) for p in probs]
    _run(cdcc, ds)
    for k, d in enumerate(ds):
        assert np.array_equal(d["M"].cpu().numpy(), alone[k])


def test_repeatable(gpu_lib):
    cdcc = gpu_lib
    prob = S.make_partial_problem(S.sym_custom([3, 2], [11, 9], [1, 1]), seed=8)
    d = _dev(cdcc, prob)
    _run(cdcc, [d])
    first = d["M"].cpu().numpy()
    for _ in range(3):
        d["M"].fill_(float("nan"))
        _run(cdcc, [d])
        assert np.array_equal(d["M"].cpu().numpy(), first)
