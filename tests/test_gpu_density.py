"""GPU parity of the vvvv two-body-density contraction (through the C ABI)
against the oracle: small and ragged systems (empty irreps, irreps without
occupied orbitals), a C1 and an 8-irrep system, several systems in one call
(bitwise equal alone), a tiny batch cap (bitwise equal), repeatability."""
import numpy as np
import pytest

import synth as S

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _dev(cdcc, prob):
    import torch
    from gpu_support import to_dev
    lay = cdcc.Layout(prob["sym"])
    return {"layout": lay, "L": to_dev(lay.pack_B(prob["L"])), "X": to_dev(lay.pack_amp(prob["X"])),
            "Y": to_dev(lay.pack_amp(prob["Y"])),
            "G": torch.full((lay.b_size,), float("nan"), dtype=torch.float64, device="cuda")}


def _run(cdcc, ds, **kw):
    import torch
    cdcc.vvvv_density(ds, **kw)
    torch.cuda.synchronize()


def _ref(prob):
    import oracle as O
    from oracle.layout import OracleLayout
    lay = OracleLayout(prob["sym"])
    return lay.pack_B(O.vvvv_density_blocks(prob["sym"], prob["X"], prob["Y"], prob["L"]))


def _rel(got, ref):
    d = np.abs(got - ref)
    return float(d.max() / max(np.abs(ref).max(), 1e-300))


SYMS = [
    ([3], [5], [4]),
    ([2, 1], [3, 4], [3, 2]),
    ([1, 2, 0, 1], [3, 2, 4, 1], [2, 0, 3, 1]),
    ([1, 1, 1, 0, 1, 0, 1, 1], [2, 3, 1, 2, 0, 2, 1, 3], [2, 1, 0, 2, 1, 1, 0, 2]),
    ([0, 2], [5, 3], [3, 4]),                    # an irrep without occupied orbitals
    ([2, 3, 1, 2], [9, 0, 7, 5], [0, 11, 6, 9]),  # an empty virtual irrep, no totally symmetric vectors
]


@pytest.mark.parametrize("spec", SYMS)
def test_small_systems(gpu_lib, spec):
    cdcc = gpu_lib
    prob = S.make_density_problem(S.sym_custom(*spec), seed=3)
    d = _dev(cdcc, prob)
    _run(cdcc, [d])
    got = d["G"].cpu().numpy()
    assert np.all(np.isfinite(got))
    assert _rel(got, _ref(prob)) <= TOL


@pytest.mark.parametrize("sym", [S.sym_c1_small(), S.sym_custom([4, 2, 3, 2], [20, 11, 15, 10], [80, 70, 75, 75])],
                         ids=["c1", "c2v_like"])
def test_named_shapes(gpu_lib, sym):
    cdcc = gpu_lib
    prob = S.make_density_problem(sym, seed=5)
    d = _dev(cdcc, prob)
    _run(cdcc, [d])
    got = d["G"].cpu().numpy()
    assert _rel(got, _ref(prob)) <= TOL


def test_batched_systems_equal_alone_and_small_cap(gpu_lib):
    cdcc = gpu_lib
    probs = [S.make_density_problem(S.sym_custom(*spec), seed=10 + k) for k, spec in enumerate(SYMS)]
    alone = []
    for p in probs:
        d = _dev(cdcc, p)
        _run(cdcc, [d])
        alone.append(d["G"].cpu().numpy())
    ds = [_dev(cdcc, p) for p in probs]
    _run(cdcc, ds)
    for k, d in enumerate(ds):
        assert np.array_equal(d["G"].cpu().numpy(), alone[k])
    ds = [_dev(cdcc, p) for p in probs]
    _run(cdcc, ds, batch_bytes=4096)  # one a per region, many batches
    for k, d in enumerate(ds):
        assert np.array_equal(d["G"].cpu().numpy(), alone[k])


def test_repeatable(gpu_lib):
    cdcc = gpu_lib
    prob = S.make_density_problem(S.sym_custom([2, 1], [6, 5], [7, 3]), seed=8)
    d = _dev(cdcc, prob)
    _run(cdcc, [d])
    first = d["G"].cpu().numpy()
    for _ in range(3):
        d["G"].fill_(float("nan"))
        _run(cdcc, [d])
        assert np.array_equal(d["G"].cpu().numpy(), first)


# K = n_vv(GP) above one GEMM K segment (2048): partial tiles and the
# segment-order reduction; ragged last segments, K not a multiple of 4 (padded
# W rows) or of the 16-wide K block, several segments per output tile.
SPLIT_SYMS = [
    ([2], [47], [9]),                  # K = 2209: segments 2048 + 161
    ([1, 1], [40, 30], [5, 6]),        # K = 2500 (GP = 0), 2400 (GP = 1)
    ([1], [68], [3]),                  # K = 4624: three segments, the last 528 = 33 blocks exactly
]


@pytest.mark.parametrize("spec", SPLIT_SYMS)
def test_split_k_segments(gpu_lib, spec):
    cdcc = gpu_lib
    prob = S.make_density_problem(S.sym_custom(*spec), seed=21)
    d = _dev(cdcc, prob)
    _run(cdcc, [d])
    got = d["G"].cpu().numpy()
    assert np.all(np.isfinite(got))
    assert _rel(got, _ref(prob)) <= TOL


def test_split_k_batched_and_small_cap_bitwise(gpu_lib):
    cdcc = gpu_lib
    probs = [S.make_density_problem(S.sym_custom(*spec), seed=30 + k) for k, spec in enumerate(SPLIT_SYMS[:2])]
    alone = []
    for p in probs:
        d = _dev(cdcc, p)
        _run(cdcc, [d])
        alone.append(d["G"].cpu().numpy())
    ds = [_dev(cdcc, p) for p in probs]
    _run(cdcc, ds)
    for k, d in enumerate(ds):
        assert np.array_equal(d["G"].cpu().numpy(), alone[k])
    ds = [_dev(cdcc, p) for p in probs]
    _run(cdcc, ds, batch_bytes=1 << 20)  # a few a per region, several batches
    for k, d in enumerate(ds):
        assert np.array_equal(d["G"].cpu().numpy(), alone[k])
