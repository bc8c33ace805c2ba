"""Helpers shared by the GPU tests: marshal generator blocks to the device,
run the library, bring results back as blocks."""
import numpy as np

import synth as S


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def device_problem(cdcc, prob, want_delta=False, want_energy=False, nan_fill=True):
    """Device buffers for one generator problem; R/delta pre-filled with NaN so
    that an element the library fails to write shows up."""
    import torch
    sym = prob["sym"]
    lay = cdcc.Layout(sym)
    d = {"layout": lay,
         "B": to_dev(lay.pack_B(prob["B"])),
         "X": to_dev(lay.pack_amp(prob["X"])),
         "R": torch.full((lay.amp_size,), float("nan") if nan_fill else 0.0, dtype=torch.float64, device="cuda")}
    if prob["kind"] == "lambda" and prob.get("Bvo") is not None and prob.get("dressed", True):
        d["Bvo"] = to_dev(lay.pack_Bvo(prob["Bvo"]))
        d["t1"] = to_dev(lay.pack_t1(prob["t1"]))
    if want_delta:
        d["eps_occ"] = to_dev(lay.pack_eps(prob["eps_occ"]))
        d["eps_vir"] = to_dev(lay.pack_eps(prob["eps_vir"]))
        d["delta"] = torch.full((lay.amp_size,), float("nan"), dtype=torch.float64, device="cuda")
    if want_energy:
        d["pair_energy"] = torch.full((lay.nocc_tot ** 2,), float("nan"), dtype=torch.float64, device="cuda")
    return d


def run(cdcc, probs, kind="t2", precision="fp64", **kw):
    import torch
    if kind == "t2":
        cdcc.ladder_t2(probs, precision=precision, **kw)
    else:
        cdcc.ladder_lambda(probs, precision=precision, **kw)
    torch.cuda.synchronize()


def blocks(d, key="R"):
    return d["layout"].unpack_amp(d[key].cpu().numpy())


def oracle_result(prob):
    import oracle as O
    sym = prob["sym"]
    if prob["kind"] == "t2":
        return O.t2_ladder_blocks(sym, prob["B"], prob["X"])
    if prob.get("dressed", True):
        return O.lambda_ladder_blocks(sym, prob["B"], prob["Bvo"], prob["t1"], prob["X"])
    zero = [np.zeros_like(x) for x in prob["t1"]]
    return O.lambda_ladder_blocks(sym, prob["B"], prob["Bvo"], zero, prob["X"])


def problem(sym, seed=0, kind="t2", symmetric_B=True, dressed=True):
    p = S.make_problem(sym, seed=seed, kind=kind, symmetric_B=symmetric_B)
    p["dressed"] = dressed
    return p
