"""GPU cell derivative dE/dH of triclinic plans
(msm_energy_forces_cell_gradient) against the oracle's central differences
of the energy in the cell (grid counts held), which Euler's relation pins on
the CPU."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05961_amd import msm
from paper_2510_05961_amd import workloads as WL

from helpers import cast

pytestmark = pytest.mark.gpu

CELL = np.array([[9.0, 0.0, 0.0], [2.1, 8.5, 0.0], [-1.3, 1.7, 9.4]])


def _charges(cell, n, seed):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3)) @ cell
    q = rng.normal(0.0, 0.5, n)
    q -= q.mean()
    return pos, q


def _gpu(plan, pos, q):
    import torch
    P = torch.tensor(pos, dtype=plan.dtype, device="cuda")
    Q = torch.tensor(q, dtype=plan.dtype, device="cuda")
    E, F, dq, G = plan.energy_forces_cell_gradient(P, Q)
    torch.cuda.synchronize()
    assert plan.status() == 0
    return E.item(), F.double().cpu().numpy(), G.cpu().numpy()


CASES = [
    # p, h, a, L, fp64, n
    (4, 1.0, 3.5, 2, True, 300),
    (6, 0.9, 3.5, 3, True, 300),
    (4, 1.0, 3.5, 2, False, 400),
    (6, 0.9, 3.0, 3, False, 400),
]


@pytest.mark.parametrize("case", CASES)
def test_cell_gradient_matches_oracle(case):
    p, h, a, L, fp64, n = case
    pos, q = _charges(CELL, n, seed=n + p + L)
    pos, q = cast(pos, q, fp64)
    print(f"case cell gradient p={p} h={h} a={a} L={L} {'fp64' if fp64 else 'fp32'}", flush=True)
    plan = msm.Plan(None, 7, p, h, a, L, msm.MSM_FP64 if fp64 else msm.MSM_FP32, n, cell=CELL)
    _, _, G = _gpu(plan, pos, q)
    o = O.OracleMSM(None, None, p, h, a, L, cell=CELL)
    ref = o.cell_gradient(pos, q)
    err = np.linalg.norm(G - ref) / np.linalg.norm(ref)
    print(f"  rel |dE/dH - FD| = {err:.2e}", flush=True)
    assert err < (1e-6 if fp64 else 2e-5)


_R6_REF = {}


@pytest.mark.parametrize("fp64", [True, False])
def test_r6_cell_gradient_matches_oracle(fp64):
    """The r^-6 kernel (msm_plan_create_cell_kernel): its own virial,
    derivative stencils and top table in every term.  Spaced positions (no
    pair closer than about 0.8: at 0.1 the stiff r^-6 pair terms of the
    fixed-fractional derivative and of sum_i F_i s_i^T are 10^3 times the
    result and cancel, beyond FP32); the inputs are FP32 values, so that
    both precisions share one oracle derivative."""
    n, p, h, a, L = 300, 4, 0.5, 4.0, 2
    s, _ = WL.spaced_charges(n, 1.0, True, seed=71)
    pos = s @ CELL
    c = np.random.default_rng(72).uniform(0.5, 1.5, n)
    pos, c = cast(pos, c, False)
    print(f"case r6 cell gradient {'fp64' if fp64 else 'fp32'}", flush=True)
    plan = msm.Plan(None, 7, p, h, a, L, msm.MSM_FP64 if fp64 else msm.MSM_FP32, n, cell=CELL,
                    kernel=6)
    _, _, G = _gpu(plan, pos, c)
    if "G" not in _R6_REF:
        _R6_REF["G"] = O.OracleMSM(None, None, p, h, a, L, cell=CELL, nu=6).cell_gradient(pos, c)
    ref = _R6_REF["G"]
    err = np.linalg.norm(G - ref) / np.linalg.norm(ref)
    print(f"  rel |dE/dH - FD| = {err:.2e}", flush=True)
    assert err < (1e-6 if fp64 else 1e-4)


def test_cell_gradient_after_set_cell():
    n = 300
    cell2 = CELL @ np.array([[1.02, 0.01, 0.0], [0.0, 0.99, -0.02], [0.01, 0.0, 1.01]])
    pos, q = _charges(cell2, n, seed=61)
    print("case cell gradient after set_cell", flush=True)
    plan = msm.Plan(None, 7, 4, 1.0, 3.5, 2, msm.MSM_FP64, n, cell=CELL)
    _gpu(plan, pos, q)  # (derivative stencils of the first cell)
    plan.set_cell(cell2)
    _, _, G = _gpu(plan, pos, q)
    ntop = plan.describe()["levels_info"][-1]["n"]
    ref = O.OracleMSM(None, None, 4, 1.0, 3.5, 2, cell=cell2, ntop=ntop).cell_gradient(pos, q)
    err = np.linalg.norm(G - ref) / np.linalg.norm(ref)
    print(f"  rel |dE/dH - FD| = {err:.2e}", flush=True)
    assert err < 1e-6


def test_cell_gradient_refuses_orthorhombic_plans():
    plan = msm.Plan((10.0, 10.0, 10.0), 7, 4, 1.0, 3.0, 2, msm.MSM_FP64, 10)
    import torch
    P = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    Q = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(msm.MSMError):
        plan.energy_forces_cell_gradient(P, Q)
