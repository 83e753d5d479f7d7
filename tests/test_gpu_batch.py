"""Batched path (many free-space systems, one launch sequence, hipGraph)
against the oracle per system and against single-system plans."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05961_amd import msm
from paper_2510_05961_amd import workloads as WL

from helpers import TOL, assert_parity, rel_rms

pytestmark = pytest.mark.gpu


def _small_batch(n_sys, seed):
    off, boxes, pos, q = WL.clusters(n_sys, 2, 70, 6.0, 14.0, 0.5, seed)
    levels = np.where(boxes <= 10.0, 2, 3).astype(np.int32)
    return off, boxes, pos, q, levels


def _run_batch(bp, off, pos, q):
    import torch
    dt = bp.dtype
    O_ = torch.tensor(off, dtype=torch.int32, device="cuda")
    P = torch.tensor(pos, dtype=dt, device="cuda")
    Q = torch.tensor(q, dtype=dt, device="cuda")
    E, F, dq = bp.energy_forces(O_, P, Q)
    torch.cuda.synchronize()
    return E.cpu().numpy(), F.double().cpu().numpy(), dq.double().cpu().numpy()


_ORACLE_CACHE = {}  # (fp64, system) -> oracle result of the fixed small batch


@pytest.mark.parametrize("form", ["auto", "direct", "factored"])
@pytest.mark.parametrize("tile", [None, "0", "1", "2", "3"])
@pytest.mark.parametrize("fp64", [True, False])
def test_batch_matches_oracle_per_system(fp64, tile, form):
    """Every convolution tile shape (MSM_BATCH_TILE pins one; None lets the
    autotuner choose) and both forms of the intermediate levels
    (MSM_FACTORED) against the oracle, system by system."""
    off, boxes, pos, q, levels = _small_batch(40, seed=11)
    dt = np.float64 if fp64 else np.float32
    pos, q = pos.astype(dt).astype(np.float64), q.astype(dt).astype(np.float64)
    env = {}
    if tile is not None:
        env["MSM_BATCH_TILE"] = tile
    if form != "auto":
        env["MSM_FACTORED"] = "1" if form == "factored" else "0"
    print(f"case batch oracle {'fp64' if fp64 else 'fp32'} tile={tile} form={form}", flush=True)
    os.environ.update(env)
    try:
        bp = msm.BatchPlan(boxes, levels, 4, 1.0, 3.0, msm.MSM_FP64 if fp64 else msm.MSM_FP32,
                           int(off[-1]))
    finally:
        for k in env:
            del os.environ[k]
    convs = bp.describe()["convs"]
    if tile is not None:
        assert all(c["tile_cfg"] == int(tile) for c in convs), convs
    if form != "auto":
        inter = [c for c in convs if not c["top"]]
        assert all(c["factored"] == (form == "factored") for c in inter), convs
    E, F, dq = _run_batch(bp, off, pos, q)
    assert bp.status() == 0
    tol = TOL["fp64" if fp64 else "fp32"]
    for s in range(len(boxes)):
        a, b = off[s], off[s + 1]
        key = (fp64, s)
        if key not in _ORACLE_CACHE:
            b3 = (boxes[s],) * 3
            _ORACLE_CACHE[key] = O.OracleMSM(b3, (0, 0, 0), 4, 1.0, 3.0, int(levels[s])).compute(
                pos[a:b], q[a:b])
        ref = _ORACLE_CACHE[key]
        if b - a >= 2:
            assert_parity(F[a:b], ref["F"], tol["F"], f"F of system {s}")
        assert abs(E[s] - ref["E"]) <= tol["E"] * max(abs(ref["E"]), 1e-3), s
        if b > a:
            assert_parity(dq[a:b], ref["phi"], tol["phi"], f"phi of system {s}")


def test_batch_equals_single_system_plans():
    import torch
    off, boxes, pos, q, levels = _small_batch(12, seed=12)
    bp = msm.BatchPlan(boxes, levels, 4, 1.0, 3.0, msm.MSM_FP64, int(off[-1]))
    E, F, dq = _run_batch(bp, off, pos, q)
    for s in range(len(boxes)):
        a, b = off[s], off[s + 1]
        pl = msm.Plan((boxes[s],) * 3, 0, 4, 1.0, 3.0, int(levels[s]), msm.MSM_FP64, max(b - a, 1))
        Es, Fs, dqs = pl.energy_forces(torch.tensor(pos[a:b], device="cuda"),
                                       torch.tensor(q[a:b], device="cuda"))
        assert E[s] == pytest.approx(Es.item(), rel=1e-11, abs=1e-12)
        if b > a:
            np.testing.assert_allclose(F[a:b], Fs.cpu().numpy(), rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("fp64", [True, False])
def test_batch_factored_levels_match_direct(fp64):
    """Intermediate levels in the factored form (three omega' passes onto
    grids extended by M, then the ball of k-samples; forced with
    MSM_FACTORED=1) against the direct stencil (MSM_FACTORED=0) on the same
    batch, and the oracle per system.  By default the autotuner keeps the
    faster form per level."""
    off, boxes, pos, q = WL.clusters(10, 20, 120, 12.0, 26.0, 0.5, seed=14)
    levels = np.where(boxes <= 20.0, 2, 3).astype(np.int32)
    dt = np.float64 if fp64 else np.float32
    pos, q = pos.astype(dt).astype(np.float64), q.astype(dt).astype(np.float64)
    prec = msm.MSM_FP64 if fp64 else msm.MSM_FP32
    print(f"case batch factored vs direct {'fp64' if fp64 else 'fp32'}", flush=True)
    os.environ["MSM_FACTORED"] = "1"
    try:
        bp = msm.BatchPlan(boxes, levels, 4, 1.0, 6.0, prec, int(off[-1]))
    finally:
        del os.environ["MSM_FACTORED"]
    convs = bp.describe()["convs"]
    assert sum(c["factored"] for c in convs) == 2, convs  # levels 1 and 2
    E, F, dq = _run_batch(bp, off, pos, q)
    assert bp.status() == 0
    os.environ["MSM_FACTORED"] = "0"
    try:
        bd = msm.BatchPlan(boxes, levels, 4, 1.0, 6.0, prec, int(off[-1]))
    finally:
        del os.environ["MSM_FACTORED"]
    assert not any(c["factored"] for c in bd.describe()["convs"])
    Ed, Fd, dqd = _run_batch(bd, off, pos, q)
    tol = 1e-12 if fp64 else 1e-6
    print(f"  relE {np.max(np.abs(E - Ed) / np.abs(Ed)):.1e} relF {rel_rms(F, Fd):.1e}", flush=True)
    assert np.all(np.abs(E - Ed) <= tol * np.abs(Ed))
    assert rel_rms(F, Fd) <= tol and rel_rms(dq, dqd) <= tol
    bars = TOL["fp64" if fp64 else "fp32"]
    for s in (0, 4, 9):
        a, b = off[s], off[s + 1]
        ref = O.OracleMSM((boxes[s],) * 3, (0, 0, 0), 4, 1.0, 6.0, int(levels[s])).compute(
            pos[a:b], q[a:b])
        assert_parity(F[a:b], ref["F"], bars["F"], f"F of system {s}")
        assert abs(E[s] - ref["E"]) <= bars["E"] * abs(ref["E"]), s


def test_batch_graph_replays_match_eager():
    import torch
    off, boxes, pos, q, levels = _small_batch(30, seed=13)
    bp = msm.BatchPlan(boxes, levels, 4, 1.0, 3.0, msm.MSM_FP32, int(off[-1]))
    O_ = torch.tensor(off, dtype=torch.int32, device="cuda")
    P = torch.tensor(pos, dtype=torch.float32, device="cuda")
    Q = torch.tensor(q, dtype=torch.float32, device="cuda")
    os.environ["MSM_BATCH_GRAPH"] = "0"
    try:
        E0, F0, d0 = bp.energy_forces(O_, P, Q)
        torch.cuda.synchronize()
        E0, F0 = E0.clone(), F0.clone()
    finally:
        os.environ.pop("MSM_BATCH_GRAPH")
    out = (torch.empty_like(E0), torch.empty_like(F0), torch.empty_like(d0))
    for rep in range(4):
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        bp.energy_forces(O_, P, Q, out=out)
        torch.cuda.synchronize()
        assert torch.allclose(out[0], E0, rtol=1e-5, atol=1e-6), rep
        assert torch.allclose(out[1], F0, rtol=1e-4, atol=1e-5), rep
        del junk


def test_batch_malformed_offsets_flagged():
    import torch
    off, boxes, pos, q, levels = _small_batch(5, seed=14)
    bp = msm.BatchPlan(boxes, levels, 4, 1.0, 3.0, msm.MSM_FP32, int(off[-1]))
    bad = off.copy()
    bad[2], bad[3] = bad[3], bad[2]  # decreasing range
    _run_batch(bp, bad, pos, q)
    assert bp.status() == 1
    assert bp.status() == 0


def test_batch_full_size_sampled():
    """The full batched workload (4,096 clusters of 8-256 charges in 10-30 A
    boxes, p = 4, h = 1, a = 6, FP32; two or three levels by box size) in the
    launch configuration the benchmark times; a sample of systems (the
    largest and smallest box, the most charges, five at random) against the
    oracle, and every system's E = 1/2 sum q phi."""
    off, boxes, pos, q, levels = WL.make_batch(4096, seed=5)
    pos32, q32 = pos.astype(np.float32), q.astype(np.float32)
    bp = msm.BatchPlan(boxes, levels, 4, 1.0, 6.0, msm.MSM_FP32, int(off[-1]))
    E, F, dq = _run_batch(bp, off, pos32, q32)
    assert bp.status() == 0
    qd = q32.astype(np.float64)
    for s in range(len(boxes)):
        a, b = off[s], off[s + 1]
        half = 0.5 * float(np.dot(qd[a:b], dq[a:b]))
        scale = 0.5 * float(np.sum(np.abs(qd[a:b] * dq[a:b])))
        assert abs(E[s] - half) <= 1e-6 * max(scale, 1e-6), s
    counts = np.diff(off)
    pick = {int(np.argmax(boxes)), int(np.argmin(boxes)), int(np.argmax(counts))}
    pick |= set(np.random.default_rng(3).choice(len(boxes), 5, replace=False).tolist())
    tol = TOL["fp32"]
    for s in sorted(pick):
        a, b = off[s], off[s + 1]
        print(f"system {s}: n={b - a} box={boxes[s]:.2f} L={levels[s]}", flush=True)
        ref = O.OracleMSM((boxes[s],) * 3, (0, 0, 0), 4, 1.0, 6.0, int(levels[s])).compute(
            pos32[a:b].astype(np.float64), qd[a:b])
        assert_parity(F[a:b], ref["F"], tol["F"], f"F of system {s}")
        assert abs(E[s] - ref["E"]) <= tol["E"] * max(abs(ref["E"]), 1e-3), s
        assert_parity(dq[a:b], ref["phi"], tol["phi"], f"phi of system {s}")


_R6_CACHE = {}  # (fp64, system) -> oracle result of the r^-6 batch


@pytest.mark.parametrize("form", ["direct", "factored"])
@pytest.mark.parametrize("fp64", [True, False])
def test_batch_r6_matches_oracle_per_system(fp64, form):
    """The dispersion kernel r^-6 in the batch (msm_batch_plan_create_kernel):
    positive coefficients c_i, both forms of the intermediate levels, against
    the oracle's r^-6 MSM system by system.  A system with no pair inside the
    cutoff has only the grid's small, smooth r^-6 forces; FP32 meets them to
    1.45e-5 here (5 charges 4.3 apart in a 12 box), the single-system FP32
    plan to the same 1.45e-5, so such systems take a 5e-5 bar in FP32."""
    off, boxes, pos, _ = WL.clusters(24, 2, 60, 6.0, 12.0, 0.5, 31)
    levels = np.where(boxes <= 9.0, 2, 3).astype(np.int32)
    c = np.random.default_rng(32).uniform(0.5, 1.5, len(pos))
    dt = np.float64 if fp64 else np.float32
    pos, c = pos.astype(dt).astype(np.float64), c.astype(dt).astype(np.float64)
    print(f"case batch r6 {'fp64' if fp64 else 'fp32'} form={form}", flush=True)
    os.environ["MSM_FACTORED"] = "1" if form == "factored" else "0"
    try:
        bp = msm.BatchPlan(boxes, levels, 4, 0.5, 3.0, msm.MSM_FP64 if fp64 else msm.MSM_FP32,
                           int(off[-1]), kernel=6)
    finally:
        del os.environ["MSM_FACTORED"]
    assert bp.describe()["kernel_power"] == 6
    E, F, _ = _run_batch(bp, off, pos, c)
    assert bp.status() == 0
    tol = TOL["fp64" if fp64 else "fp32"]
    worst = 0.0
    for s in range(len(boxes)):
        a, b = off[s], off[s + 1]
        key = (fp64, s)
        if key not in _R6_CACHE:
            _R6_CACHE[key] = O.OracleMSM((boxes[s],) * 3, (0, 0, 0), 4, 0.5, 3.0, int(levels[s]),
                                         nu=6).compute(pos[a:b], c[a:b])
        ref = _R6_CACHE[key]
        if b - a >= 2:
            p = pos[a:b]
            d2 = ((p[:, None] - p[None]) ** 2).sum(-1) + np.eye(b - a) * 1e9
            bar = tol["F"] if (fp64 or d2.min() < 3.0 ** 2) else 5e-5
            e = assert_parity(F[a:b], ref["F"], bar, f"F of system {s}")
            worst = max(worst, e[0])
        assert abs(E[s] - ref["E"]) <= tol["E"] * max(abs(ref["E"]), 1e-3), s
    print(f"  worst relF {worst:.1e}", flush=True)
