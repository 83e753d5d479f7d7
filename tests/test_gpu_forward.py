"""GPU forward parity: the HIP path (through the C ABI) against the oracle.

Element by element on the same seeded inputs (the oracle gets the inputs
rounded to the run's precision), at sizes the oracle finishes in seconds;
sampled outputs at the full workload sizes.
"""
import hashlib
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05961_amd import msm
from paper_2510_05961_amd import workloads as WL

from helpers import TOL, assert_parity, cast, config_case, gpu_forward, mask_of, periodic_of, rel_rms

pytestmark = pytest.mark.gpu


def _run(pos, q, box, periodic, p, h, a, L, fp64, M=None, check_phi=True):
    pos, q = cast(pos, q, fp64)
    prec = msm.MSM_FP64 if fp64 else msm.MSM_FP32
    print(f"case n={len(q)} box={box} per={periodic} p={p} h={h} a={a} L={L} "
          f"{'fp64' if fp64 else 'fp32'}", flush=True)
    plan = msm.Plan(box, mask_of(periodic), p, h, a, L, prec, max(len(q), 1),
                    -1 if M is None else M)
    g = gpu_forward(plan, pos, q)
    assert plan.status() == 0
    ref = O.OracleMSM(box, periodic, p, h, a, L, M).compute(pos, q)
    tol = TOL["fp64" if fp64 else "fp32"]
    eF = rel_rms(g["F"], ref["F"])
    eE = abs(g["E"] - ref["E"]) / max(abs(ref["E"]), 1e-300)
    ePhi = rel_rms(g["phi"], ref["phi"])
    print(f"  E gpu={g['E']:.12g} ref={ref['E']:.12g} relE={eE:.2e} relF={eF:.2e} "
          f"relPhi={ePhi:.2e}", flush=True)
    assert_parity(g["F"], ref["F"], tol["F"], "F")
    assert eE <= tol["E"]
    if check_phi:
        assert_parity(g["phi"], ref["phi"], tol["phi"], "phi")
    return plan, g, ref


# --- the workloads at reduced size (same recipe, same density) --------------
@pytest.mark.parametrize("cfg,scale", [(1, 1.0), (2, 0.03), (3, 0.014), (4, 0.04)])
def test_config_reduced(cfg, scale):
    _run(*config_case(cfg, scale))


# --- small cases spanning several tiles and ragged tails ---------------------
SMALL = [
    # box, periodic, p, h, a, L, fp64, n
    ((13.0, 11.0, 12.0), (0, 0, 0), 4, 1.0, 3.0, 3, True, 777),
    ((13.0, 11.0, 12.0), (0, 0, 0), 6, 1.0, 3.0, 2, False, 777),
    ((12.0, 12.0, 12.0), (1, 1, 1), 4, 0.75, 4.0, 4, True, 500),
    ((12.0, 12.0, 12.0), (1, 1, 1), 6, 1.0, 4.0, 3, False, 513),
    ((14.0, 13.0, 9.0), (1, 1, 0), 4, 1.0, 4.0, 3, True, 400),
    ((14.0, 13.0, 9.0), (1, 1, 0), 8, 1.0, 4.0, 2, False, 401),
    ((10.0, 10.0, 10.0), (1, 1, 1), 8, 1.25, 3.0, 3, True, 300),
    # a single level (the top level is level 1)
    ((11.0, 10.0, 12.0), (0, 0, 0), 4, 1.0, 3.0, 1, True, 200),
    ((12.0, 12.0, 12.0), (1, 1, 1), 4, 1.0, 4.0, 1, False, 256),
]


@pytest.mark.parametrize("case", SMALL)
def test_small_cases(case):
    box, per, p, h, a, L, fp64, n = case
    pos, q = WL.gaussian_charges(n, box, 0.5, seed=n)
    _run(pos, q, box, per, p, h, a, L, fp64)


@pytest.mark.parametrize("fp64", [True, False])
def test_degenerate_sizes(fp64):
    box = (9.0, 9.0, 9.0)
    for n in (0, 1, 2):
        pos, q = WL.random_ions(max(n, 1), box, seed=3)
        pos, q = pos[:n], q[:n]
        if n == 1:
            q = np.array([0.7])
        pos, q = cast(pos, q, fp64)
        for per in ((0, 0, 0), (1, 1, 1)):
            plan = msm.Plan(box, mask_of(per), 4, 1.0, 3.0, 2,
                            msm.MSM_FP64 if fp64 else msm.MSM_FP32, 4)
            g = gpu_forward(plan, pos, q)
            o = O.OracleMSM(box, per, 4, 1.0, 3.0, 2)
            ref = o.compute(pos, q)
            # for n <= 2 the energy is a small residual of the grid self-energy
            # 1/2 sum q^2 sum_l k_l(0); FP32 is held to 1e-6 of that scale
            scale = 0.5 * float(np.sum(q * q)) * o.self_constant()
            assert abs(g["E"] - ref["E"]) <= (1e-11 if fp64 else 1e-6) * max(scale, 1e-30)
            if n:
                np.testing.assert_allclose(g["F"], ref["F"], rtol=1e-4, atol=1e-7)


@pytest.mark.parametrize("stream", ["0", "1"])
@pytest.mark.parametrize("geom", [((12.0, 12.0, 9.0), (1, 1, 0), 4),
                                  ((10.0, 11.0, 9.0), (0, 0, 0), 6),
                                  ((12.0, 12.0, 12.0), (1, 1, 1), 8)])
def test_stage_grids_match_oracle(stream, geom):
    """Per-stage parity: q~^l after restriction vs direct anterpolation, and
    e^{l+} after prolongation vs the nested sum of the oracle's level
    potentials (prolongation written out from its formula).  stream = 1
    forces the streaming restriction and prolongation of large grids
    (MSM_GRID_STREAM), 0 the tiled ones."""
    import os
    from test_oracle_pins import _prolong_axis
    box, per, p = geom
    h, a, L = 0.75, 3.0, 3
    pos, q = WL.gaussian_charges(600, box, 0.5, seed=9)
    pos, q = cast(pos, q, True)
    plan = msm.Plan(box, mask_of(per), p, h, a, L, msm.MSM_FP64, 600)
    print(f"case per={per} p={p} MSM_GRID_STREAM={stream}", flush=True)
    os.environ["MSM_GRID_STREAM"] = stream
    try:
        gpu_forward(plan, pos, q)
    finally:
        del os.environ["MSM_GRID_STREAM"]
    assert plan.status() == 0
    o = O.OracleMSM(box, per, p, h, a, L)
    J = {n: 2.0 ** (1 - p) * math.comb(p, n + p // 2) for n in range(-p // 2, p // 2 + 1)}
    elev = []
    for l in range(1, L + 1):
        qg = o.grid_charge(l, pos, q)
        np.testing.assert_allclose(plan.grid(l, 0).cpu().numpy(), qg, rtol=0,
                                   atol=1e-12 * np.abs(qg).max())
        elev.append(o.level_potential(l, qg))
    nested = elev[L - 1]
    assert np.allclose(plan.grid(L, 1).cpu().numpy(), nested, rtol=0,
                       atol=1e-12 * np.abs(nested).max())
    for l in range(L - 1, 0, -1):
        n_f, lo_f, _ = o.levels[l - 1]
        n_c, lo_c, _ = o.levels[l]
        up = nested
        for ax3, arr_ax in ((0, 2), (1, 1), (2, 0)):
            up = _prolong_axis(up, arr_ax, J, lo_f[ax3], lo_c[ax3], n_f[ax3], per[ax3])
        nested = elev[l - 1] + up
        got = plan.grid(l, 1).cpu().numpy()
        # FP64 rounding of the nested sums (9 taps per axis at p = 8 on a
        # periodic grid) reaches a few 1e-12 of the largest value
        dev = float(np.abs(got - nested).max() / np.abs(nested).max())
        print(f"  level {l} nested e: max deviation {dev:.2e} of the largest value", flush=True)
        np.testing.assert_allclose(got, nested, rtol=0, atol=1e-11 * np.abs(nested).max())


def test_error_flags():
    import torch
    box = (10.0, 10.0, 10.0)
    plan = msm.Plan(box, 0, 4, 1.0, 3.0, 2, msm.MSM_FP32, 10)
    pos = torch.rand(10, 3, device="cuda") * 10
    q = torch.ones(10, device="cuda")
    plan.energy_forces(pos, q)
    assert plan.status() == 0
    bad = pos.clone()
    bad[3, 1] = 10.5  # outside the free box
    plan.energy_forces(bad, q)
    assert plan.status() == 5
    assert plan.status() == 0  # cleared
    nanq = q.clone()
    nanq[2] = float("nan")
    plan.energy_forces(pos, nanq)
    assert plan.status() == 6
    with pytest.raises(msm.MSMError):
        plan.energy_forces(torch.rand(11, 3, device="cuda"), torch.ones(11, device="cuda"))


# --- full workload sizes: sampled outputs + properties -----------------------
@pytest.mark.parametrize("cfg", [2, 3, 4])
def test_full_size_sampled(cfg):
    pos, q, box, per, p, h, a, L, fp64 = config_case(cfg, 1.0)
    pos, q = cast(pos, q, fp64)
    print(f"full workload {cfg}: n={len(q)}", flush=True)
    plan = msm.Plan(box, mask_of(per), p, h, a, L, msm.MSM_FP32, len(q))
    g = gpu_forward(plan, pos, q)
    assert plan.status() == 0
    # E = 1/2 sum q_i phi_i (FP64 sum of the GPU's own outputs)
    e_half = 0.5 * float(np.dot(q, g["phi"]))
    scale = 0.5 * float(np.sum(np.abs(q * g["phi"])))
    assert abs(g["E"] - e_half) <= 1e-6 * scale
    # the oracle's full-size FP64 energy of these FP32 inputs (tests/golden)
    rec = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "full_size_energies.json")))[str(cfg)]
    digest = hashlib.sha256(np.ascontiguousarray(pos, dtype=np.float32).tobytes() +
                            np.ascontiguousarray(q, dtype=np.float32).tobytes()).hexdigest()[:16]
    assert digest == rec["input_sha256_16"]
    eE = abs(g["E"] - rec["E"]) / abs(rec["E"])
    print(f"  relE vs full-size oracle energy {eE:.2e}", flush=True)
    assert eE <= TOL["fp32"]["E"]
    sel = np.random.default_rng(cfg).choice(len(q), 16 if cfg == 3 else 32, replace=False)
    phi_r, F_r = O.OracleMSM(box, per, p, h, a, L).sampled(pos, q, sel)
    eF = rel_rms(g["F"][sel], F_r)
    eP = rel_rms(g["phi"][sel], phi_r)
    print(f"  sampled relF={eF:.2e} relPhi={eP:.2e}", flush=True)
    assert_parity(g["F"][sel], F_r, TOL["fp32"]["F"], "F")
    assert_parity(g["phi"][sel], phi_r, TOL["fp32"]["phi"], "phi")


@pytest.mark.parametrize("n", [100_000, 600_000])
def test_large_grid_sampled(n):
    """A 128^3 periodic level-1 grid (h = 1, a = 3, p = 4, L = 5, FP32) with
    charges +-1 at uniform random positions: the sizes at which the library
    picks its large-grid passes by itself (streaming restriction and
    prolongation; tiled anterpolation at 0.05 charges per grid point,
    super-cell bricks at 0.29).  Sampled outputs against the oracle, and
    E = 1/2 sum q phi over all charges."""
    rng = np.random.default_rng(n)
    box = (128.0, 128.0, 128.0)
    pos = rng.random((n, 3)) * 128.0
    q = np.where(rng.permutation(n) < n // 2, 1.0, -1.0)
    pos, q = cast(pos, q, False)
    print(f"large grid: n={n}", flush=True)
    plan = msm.Plan(box, 7, 4, 1.0, 3.0, 5, msm.MSM_FP32, n)
    assert plan.grid_dims(1) == (128, 128, 128)
    g = gpu_forward(plan, pos, q)
    assert plan.status() == 0
    e_half = 0.5 * float(np.dot(q, g["phi"]))
    assert abs(g["E"] - e_half) <= 1e-6 * 0.5 * float(np.sum(np.abs(q * g["phi"])))
    sel = rng.choice(n, 32, replace=False)
    phi_r, F_r = O.OracleMSM(box, (1, 1, 1), 4, 1.0, 3.0, 5).sampled(pos, q, sel)
    eF, eP = rel_rms(g["F"][sel], F_r), rel_rms(g["phi"][sel], phi_r)
    print(f"  sampled relF={eF:.2e} relPhi={eP:.2e}", flush=True)
    assert_parity(g["F"][sel], F_r, TOL["fp32"]["F"], "F")
    assert_parity(g["phi"][sel], phi_r, TOL["fp32"]["phi"], "phi")


@pytest.mark.parametrize("fp64", [True, False])
def test_streams_match_single_stream(fp64):
    """The four-stream forward (pair sum and coarse levels beside level 1)
    against everything on the caller's stream: equal up to the order of the
    atomic additions."""
    import os
    box, per, p, h, a, L = (24.0, 24.0, 24.0), (1, 1, 1), 4, 0.75, 4.0, 4
    pos, q = WL.gaussian_charges(3000, box, 0.5, seed=21)
    pos, q = cast(pos, q, fp64)
    plan = msm.Plan(box, mask_of(per), p, h, a, L, msm.MSM_FP64 if fp64 else msm.MSM_FP32, 3000)
    out = {}
    for mode in ("0", "1"):
        os.environ["MSM_STREAMS"] = mode
        try:
            out[mode] = gpu_forward(plan, pos, q)
        finally:
            del os.environ["MSM_STREAMS"]
    tol = 1e-12 if fp64 else 1e-6
    assert abs(out["0"]["E"] - out["1"]["E"]) <= tol * abs(out["0"]["E"])
    assert rel_rms(out["1"]["F"], out["0"]["F"]) <= tol
    assert rel_rms(out["1"]["phi"], out["0"]["phi"]) <= tol


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("geom", ["periodic", "slab", "free"])
def test_folded_matches_unfolded(fp64, geom):
    """Mirrored stencil z-planes summed before one pass over their shared
    coefficients, against the plain walk over every plane (MSM_FOLD=0).  The
    periodic case has even top-level grids (their residue tables are split
    at n/2), the slab a free z axis, the free case direct stencils only."""
    import os
    if geom == "periodic":
        box, per, L = (24.0, 24.0, 24.0), (1, 1, 1), 4
    elif geom == "slab":
        box, per, L = (20.0, 20.0, 14.0), (1, 1, 0), 3
    else:
        box, per, L = (14.0, 14.0, 14.0), (0, 0, 0), 3
    p, h, a = 4, 0.75, 4.0
    pos, q = WL.gaussian_charges(2000, box, 0.5, seed=23)
    pos, q = cast(pos, q, fp64)
    prec = msm.MSM_FP64 if fp64 else msm.MSM_FP32
    os.environ["MSM_FOLD"] = "0"
    try:
        plain = msm.Plan(box, mask_of(per), p, h, a, L, prec, 2000)
    finally:
        del os.environ["MSM_FOLD"]
    folded = msm.Plan(box, mask_of(per), p, h, a, L, prec, 2000)
    g0, g1 = gpu_forward(plain, pos, q), gpu_forward(folded, pos, q)
    # FP64: the mirrored coefficients are averaged (changes of 1e-12 of the
    # largest at most); FP32: one more rounding of the summed input planes
    tol = 1e-10 if fp64 else 1e-6
    assert abs(g0["E"] - g1["E"]) <= tol * abs(g0["E"])
    assert rel_rms(g1["F"], g0["F"]) <= tol
    assert rel_rms(g1["phi"], g0["phi"]) <= tol


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("geom", ["periodic", "slab", "free"])
def test_super_cell_bricks(fp64, geom):
    """Anterpolation bricks that gather kc^3 cells of the cell list (forced
    with MSM_BRICK_CELLS; kc = 4 leaves ragged super-cells at the far faces)
    against one brick per cell and against the oracle.  The bricks only
    change the fixed-point scale (per brick) and which adds meet in LDS."""
    import os
    # h = 1.5 with cells of about 4: bricks of up to 4^3 (p = 4), 3^3 (p = 6,
    # 8) cells fit in LDS, so the forced sizes below take effect, and 6, 5, 3
    # or 4 cells per axis leave ragged super-cells
    if geom == "periodic":
        box, per, L, p = (24.0, 24.0, 24.0), (1, 1, 1), 3, 4
    elif geom == "slab":
        box, per, L, p = (24.0, 20.0, 14.0), (1, 1, 0), 3, 6
    else:
        box, per, L, p = (18.0, 18.0, 18.0), (0, 0, 0), 3, 8
    h, a = 1.5, 4.0
    pos, q = WL.gaussian_charges(2000, box, 0.5, seed=29)
    pos, q = cast(pos, q, fp64)
    prec = msm.MSM_FP64 if fp64 else msm.MSM_FP32
    plan = msm.Plan(box, mask_of(per), p, h, a, L, prec, 2000)
    res = {}
    for kc in (1, 2, 3, 4):
        print(f"case {geom} p={p} {'fp64' if fp64 else 'fp32'} bricks of up to {kc}^3 cells",
              flush=True)
        os.environ["MSM_BRICK_CELLS"] = str(kc)
        try:
            res[kc] = gpu_forward(plan, pos, q)
            res[kc]["q1"] = plan.grid(1, 0).double().cpu().numpy()
        finally:
            del os.environ["MSM_BRICK_CELLS"]
        assert plan.status() == 0
    tol = 1e-12 if fp64 else 1e-6
    for kc in (2, 3, 4):
        assert rel_rms(res[kc]["q1"], res[1]["q1"]) <= tol
        assert abs(res[kc]["E"] - res[1]["E"]) <= tol * abs(res[1]["E"])
        assert rel_rms(res[kc]["F"], res[1]["F"]) <= tol
        assert rel_rms(res[kc]["phi"], res[1]["phi"]) <= tol
    ref = O.OracleMSM(box, per, p, h, a, L).compute(pos, q)
    t = TOL["fp64" if fp64 else "fp32"]
    assert abs(res[4]["E"] - ref["E"]) <= t["E"] * abs(ref["E"])
    assert_parity(res[4]["F"], ref["F"], t["F"], "F")
    assert_parity(res[4]["phi"], ref["phi"], t["phi"], "phi")


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("geom", ["periodic", "slab", "free", "tiny"])
def test_anterp_tiles(fp64, geom):
    """Level-1 charges summed in grid tiles that gather the charges of the
    cells around them (the path of large grids, forced with
    MSM_ANTERP_TILES=1; the tiles write every grid value, so the grid is not
    cleared first) against the per-cell bricks and the oracle.  "tiny" is a
    periodic grid smaller than one tile, whose tiles gather several images
    of each cell."""
    import os
    if geom == "periodic":
        box, per, L, n, p = (24.0, 24.0, 24.0), (1, 1, 1), 4, 2000, 4
    elif geom == "slab":
        box, per, L, n, p = (24.0, 20.0, 14.0), (1, 1, 0), 3, 2000, 6
    elif geom == "free":
        box, per, L, n, p = (18.0, 18.0, 18.0), (0, 0, 0), 3, 2000, 4
    else:
        box, per, L, n, p = (9.0, 9.0, 9.0), (1, 1, 1), 2, 300, 8
    h, a = 0.75, 4.0
    pos, q = WL.gaussian_charges(n, box, 0.5, seed=37)
    pos, q = cast(pos, q, fp64)
    prec = msm.MSM_FP64 if fp64 else msm.MSM_FP32
    plan = msm.Plan(box, mask_of(per), p, h, a, L, prec, n)
    res = {}
    for tiles in ("0", "1"):
        print(f"case {geom} {'fp64' if fp64 else 'fp32'} MSM_ANTERP_TILES={tiles}", flush=True)
        os.environ["MSM_ANTERP_TILES"] = tiles
        try:
            # twice: the second call must not see the first one's grid
            gpu_forward(plan, pos, q)
            res[tiles] = gpu_forward(plan, pos, q)
            res[tiles]["q1"] = plan.grid(1, 0).double().cpu().numpy()
        finally:
            del os.environ["MSM_ANTERP_TILES"]
        assert plan.status() == 0
    tol = 1e-12 if fp64 else 1e-6
    assert rel_rms(res["1"]["q1"], res["0"]["q1"]) <= tol
    assert abs(res["1"]["E"] - res["0"]["E"]) <= tol * abs(res["0"]["E"])
    assert rel_rms(res["1"]["F"], res["0"]["F"]) <= tol
    ref = O.OracleMSM(box, per, p, h, a, L).compute(pos, q)
    t = TOL["fp64" if fp64 else "fp32"]
    assert abs(res["1"]["E"] - ref["E"]) <= t["E"] * abs(ref["E"])
    assert_parity(res["1"]["F"], ref["F"], t["F"], "F")
    assert_parity(res["1"]["phi"], ref["phi"], t["phi"], "phi")


@pytest.mark.parametrize("fp64", [True, False])
@pytest.mark.parametrize("scale", [1e-12, 1e12])
def test_charge_scale_homogeneity(fp64, scale):
    """E and F are quadratic in the charges, phi = dE/dq linear: scaling every
    charge by s scales them by s^2 and s.  The level-1 charges are summed in
    LDS as 64-bit fixed point with a power-of-two scale chosen per cell from
    its total |q|, so tiny and huge charges keep full relative precision."""
    box = (18.0, 18.0, 18.0)
    pos, q = WL.gaussian_charges(1500, box, 0.5, seed=31)
    pos, q = cast(pos, q, fp64)
    plan = msm.Plan(box, 7, 4, 0.75, 4.0, 3, msm.MSM_FP64 if fp64 else msm.MSM_FP32, 1500)
    g1 = gpu_forward(plan, pos, q)
    gs = gpu_forward(plan, pos, (q * scale).astype(q.dtype))
    assert plan.status() == 0
    tol = 1e-12 if fp64 else 1e-6
    assert abs(gs["E"] / scale**2 - g1["E"]) <= tol * abs(g1["E"])
    assert rel_rms(gs["F"] / scale**2, g1["F"]) <= tol
    assert rel_rms(gs["phi"] / scale, g1["phi"]) <= tol


def test_profile_stage_filter():
    import torch
    box = (16.0, 16.0, 16.0)
    pos, q = WL.gaussian_charges(500, box, 0.5, seed=4)
    plan = msm.Plan(box, 7, 4, 1.0, 4.0, 3, msm.MSM_FP32, 500)
    P = torch.tensor(pos, dtype=torch.float32, device="cuda")
    Q = torch.tensor(q, dtype=torch.float32, device="cuda")
    plan.set_profile_stages(["pair", "interp"])
    plan.set_profiling(True)
    plan.energy_forces(P, Q)
    plan.energy_forces(P, Q)
    plan.set_profiling(False)
    prof = plan.profile(reset=True)
    assert set(prof) == {"pair", "interp"}
    assert all(v["launches"] == 2 and v["ms"] > 0 for v in prof.values())
    plan.set_profile_stages(None)
    plan.set_profiling(True)
    plan.energy_forces(P, Q)
    plan.set_profiling(False)
    prof = plan.profile(reset=True)
    assert {"bin", "pair", "anterp", "conv_l1", "interp"} <= set(prof)
    # timeline offsets after the call's first stage: the call starts with
    # binning, which precedes anterpolation; interpolation comes last
    assert prof["bin"]["start_ms"] == 0.0
    assert all(0.0 <= v["start_ms"] <= v["end_ms"] for v in prof.values())
    assert prof["bin"]["end_ms"] <= prof["anterp"]["start_ms"]
    assert prof["interp"]["start_ms"] >= max(prof["pair"]["end_ms"], prof["conv_l1"]["end_ms"])
