"""GPU test of msm_energy_forces_noalloc (through the C ABI): its outputs
against msm_energy_forces on the same plan and inputs, at the parity bars,
on two calls in a row, the second with fewer particles; and its capacity
error for a call whose working memory exceeds the library's static array.
"""
import numpy as np
import pytest

from paper_2510_05961_amd import msm
from paper_2510_05961_amd import workloads as WL

from helpers import TOL, assert_parity, cast, config_case, mask_of

pytestmark = pytest.mark.gpu


def _outs(torch, n, dt):
    return (torch.empty(1, dtype=torch.float64, device="cuda"),
            torch.empty((n, 3), dtype=dt, device="cuda"),
            torch.empty(n, dtype=dt, device="cuda"))


CASES = [
    # (label, pos, q, box, periodic, p, h, a, L, fp64)
    ("water, 3,000 charges, FP32", *config_case(2, 0.03)),
    ("slab, 14,000 charges, p=6, FP32", *config_case(3, 0.014)),
    ("free ions, 1,000 charges, FP64", *config_case(1, 1.0)),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_energy_forces(case):
    import torch
    label, pos, q, box, per, p, h, a, L, fp64 = case
    pos, q = cast(pos, q, fp64)
    n = len(q)
    plan = msm.Plan(box, mask_of(per), p, h, a, L, msm.MSM_FP64 if fp64 else msm.MSM_FP32, n)
    dt = plan.dtype
    tol = TOL["fp64" if fp64 else "fp32"]
    # two calls in a row, the second with the first 60% of the particles
    for m in (n, (3 * n) // 5):
        print(f"case {label}: n={m}", flush=True)
        P = torch.tensor(pos[:m], dtype=dt, device="cuda").contiguous()
        Q = torch.tensor(q[:m], dtype=dt, device="cuda").contiguous()
        ref = plan.energy_forces(P, Q)
        out = _outs(torch, m, dt)
        plan.energy_forces_noalloc(P, Q, out)
        torch.cuda.synchronize()
        assert plan.status() == 0
        E0, E1 = ref[0].item(), out[0].item()
        F0, F1 = ref[1].double().cpu().numpy(), out[1].double().cpu().numpy()
        d0, d1 = ref[2].double().cpu().numpy(), out[2].double().cpu().numpy()
        eE = abs(E1 - E0) / abs(E0)
        eF = assert_parity(F1, F0, tol["F"], "F")
        eP = assert_parity(d1, d0, tol["phi"], "dE/dq")
        print(f"  relE={eE:.2e} relF={eF[0]:.2e} relPhi={eP[0]:.2e}", flush=True)
        assert eE <= tol["E"]


def test_noalloc_capacity_error():
    """A call whose working memory would exceed the static array is refused
    on the host (no kernel runs)."""
    import torch
    box = (40.0, 40.0, 40.0)
    plan = msm.Plan(box, 7, 4, 1.0, 8.0, 3, msm.MSM_FP32, 1)
    n = 2_000_000
    P = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    Q = torch.zeros(n, dtype=torch.float32, device="cuda")
    with pytest.raises(msm.MSMError) as e:
        plan.energy_forces_noalloc(P, Q, _outs(torch, n, torch.float32))
    assert e.value.code == 7  # MSM_ERR_CAPACITY
