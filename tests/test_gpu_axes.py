"""GPU parity with one periodic axis (the 1-D Ewald top level) and with two
periodic axes in the orientations other than x, y: every stage is written
per axis, so these run the same kernels with other wrap/crop choices."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05961_amd import msm
from paper_2510_05961_amd import workloads as WL

from helpers import TOL, assert_parity, cast, gpu_forward, mask_of, rel_rms

pytestmark = pytest.mark.gpu

CASES = [
    # box, periodic, p, h, a, L, fp64, n
    ((13.0, 11.0, 9.0), (0, 0, 1), 4, 0.75, 3.5, 3, True, 500),
    ((13.0, 11.0, 9.0), (0, 0, 1), 6, 1.0, 3.5, 3, False, 501),
    ((9.0, 12.0, 11.0), (1, 0, 0), 6, 1.0, 4.0, 3, True, 433),
    ((9.0, 12.0, 11.0), (1, 0, 0), 8, 1.0, 4.0, 2, False, 433),
    ((12.0, 8.0, 11.0), (0, 1, 0), 4, 1.0, 3.5, 4, True, 380),
    ((12.0, 8.0, 11.0), (0, 1, 0), 4, 0.75, 3.5, 3, False, 381),
    ((12.0, 10.0, 13.0), (1, 0, 1), 6, 1.0, 4.0, 3, True, 450),
    ((12.0, 10.0, 13.0), (1, 0, 1), 4, 0.75, 4.0, 3, False, 450),
    ((10.0, 12.0, 12.0), (0, 1, 1), 4, 1.0, 4.0, 3, True, 420),
    ((10.0, 12.0, 12.0), (0, 1, 1), 8, 1.25, 4.0, 2, False, 421),
]


def _check(g, ref, fp64, what=""):
    tol = TOL["fp64" if fp64 else "fp32"]
    eE = abs(g["E"] - ref["E"]) / abs(ref["E"])
    print(f"  {what}relE={eE:.2e} relF={rel_rms(g['F'], ref['F']):.2e} "
          f"relPhi={rel_rms(g['phi'], ref['phi']):.2e}", flush=True)
    assert eE <= tol["E"]
    assert_parity(g["F"], ref["F"], tol["F"], "F")
    assert_parity(g["phi"], ref["phi"], tol["phi"], "phi")


@pytest.mark.parametrize("case", CASES)
def test_periodic_axes(case):
    box, per, p, h, a, L, fp64, n = case
    pos, q = WL.gaussian_charges(n, box, 0.5, seed=n + 3)
    pos, q = cast(pos, q, fp64)
    print(f"case n={n} box={box} per={per} p={p} h={h} L={L} {'fp64' if fp64 else 'fp32'}",
          flush=True)
    plan = msm.Plan(box, mask_of(per), p, h, a, L, msm.MSM_FP64 if fp64 else msm.MSM_FP32, n)
    g = gpu_forward(plan, pos, q)
    assert plan.status() == 0
    _check(g, O.OracleMSM(box, per, p, h, a, L).compute(pos, q), fp64)


@pytest.mark.parametrize("per", [(0, 0, 1), (1, 0, 1)])
def test_periodic_axes_grid_tiles(per):
    """The tiled level-1 anterpolation (MSM_ANTERP_TILES=1, the path of
    large grids) with free and periodic axes mixed."""
    box, p, h, a, L, n = (22.0, 18.0, 16.0), 4, 0.75, 4.0, 3, 2000
    pos, q = WL.gaussian_charges(n, box, 0.5, seed=43)
    plan = msm.Plan(box, mask_of(per), p, h, a, L, msm.MSM_FP64, n)
    res = {}
    for tiles in ("0", "1"):
        print(f"case per={per} MSM_ANTERP_TILES={tiles}", flush=True)
        os.environ["MSM_ANTERP_TILES"] = tiles
        try:
            res[tiles] = gpu_forward(plan, pos, q)
        finally:
            del os.environ["MSM_ANTERP_TILES"]
        assert plan.status() == 0
    assert abs(res["1"]["E"] - res["0"]["E"]) <= 1e-12 * abs(res["0"]["E"])
    assert rel_rms(res["1"]["F"], res["0"]["F"]) <= 1e-12
    _check(res["1"], O.OracleMSM(box, per, p, h, a, L).compute(pos, q), True, "tiles: ")


@pytest.mark.parametrize("per,fp64", [((0, 1, 0), True), ((0, 0, 1), False), ((1, 0, 1), True)])
def test_periodic_axes_backward(per, fp64):
    import torch
    box, p, h, a, L, n = (12.0, 11.0, 10.0), 4, 1.0, 3.5, 3, 300
    pos, q = WL.gaussian_charges(n, box, 0.5, seed=47)
    pos, q = cast(pos, q, fp64)
    v = WL.force_cotangent(n, seed=48)
    if not fp64:
        v = v.astype(np.float32).astype(np.float64)
    print(f"case backward per={per} {'fp64' if fp64 else 'fp32'}", flush=True)
    plan = msm.Plan(box, mask_of(per), p, h, a, L, msm.MSM_FP64 if fp64 else msm.MSM_FP32, n)
    dt = plan.dtype
    P = torch.tensor(pos, dtype=dt, device="cuda")
    Q = torch.tensor(q, dtype=dt, device="cuda")
    ws = torch.empty(plan.workspace_bytes(n), dtype=torch.uint8, device="cuda")
    plan.energy_forces(P, Q, ws=ws)
    gE = torch.tensor([0.7], dtype=torch.float64, device="cuda")
    gpos, gq = plan.backward(P, Q, ws, gE=gE, gF=torch.tensor(v, dtype=dt, device="cuda"))
    torch.cuda.synchronize()
    assert plan.status() == 0
    rq, rpos = O.OracleMSM(box, per, p, h, a, L).backward(pos, q, 0.7, v)
    tol = TOL["fp64" if fp64 else "fp32"]["F"]
    gpos, gq = gpos.double().cpu().numpy(), gq.double().cpu().numpy()
    print(f"  grad_pos rel={rel_rms(gpos, rpos):.2e} grad_q rel={rel_rms(gq, rq):.2e}", flush=True)
    assert_parity(gpos, rpos, tol, "grad_pos")
    assert_parity(gq, rq, tol, "grad_q")
