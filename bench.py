#!/usr/bin/env python3
"""MSM energy+forces throughput on one MI355X (libmsm, HIP kernels).

Headline workload: the mixed-periodicity slab -- 10^6 point charges +-1
(neutral) uniform in a 100 x 100 x 60 A box, periodic in x and y, free in z,
FP32, quintic B-splines (p = 6), h = 1.25 A, cutoff a = 12 A, L = 5 grid
levels: the largest configuration that fits one GPU.  Inputs are synthetic
(seeded) and resident in HBM before the timed region.  One step = one
msm_energy_forces call (all stages: binning and cluster layout, pair sum,
anterpolation, restriction, stencil convolution per level, top level,
prolongation, interpolation, FP64 energy), timed with profiling off.

The roofline of the dominant kernel comes from per-stage HIP events with
every stage on one stream (no overlap), so each duration is the kernel's
own; algorithmic work: 28 + 4p flops per unique pair within the cutoff for
the pair sum, 2 flops per (output, in-grid input) pair with a non-zero
coefficient for a convolution.

Extras (each with its error against the FP64 oracle): the periodic water box,
the learnable-charge box forward vs forward + backward (and through
torch.autograd), the 4,096-cluster batch vs one plan per system, the
free-space FP64 ion cloud, the charged Lennard-Jonesium MD loop (steps/s
and its NVE energy measure), and the grid-pass HBM sweep.

Prints ONE JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MSM energy+forces particles/s at fixed force error; batched/autograd vs plain"

# MI355X published peaks
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def _pos_key(pos32):
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(pos32, dtype=np.float32).tobytes()).hexdigest()[:16]


def _pair_count(cfg, pos32):
    """Unique pairs within the cutoff of workload cfg's FP32 input, from
    tests/golden/pair_counts.json (exact k-d tree counts written by
    tests/golden/make_pair_counts.py), or None if the input differs."""
    try:
        rec = json.load(open(os.path.join(ROOT, "tests", "golden", "pair_counts.json")))[str(cfg)]
    except (OSError, KeyError, ValueError):
        return None
    return int(rec["pairs"]) if rec.get("positions_sha256_16") == _pos_key(pos32) else None


def _golden_energy(cfg, pos32, q32):
    """FP64 oracle energy of the full-size workload (tests/golden), or None."""
    import numpy as np
    try:
        rec = json.load(open(os.path.join(ROOT, "tests", "golden",
                                          "full_size_energies.json")))[str(cfg)]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(pos32, dtype=np.float32).tobytes())
    h.update(np.ascontiguousarray(q32, dtype=np.float32).tobytes())
    return float(rec["E"]) if rec.get("input_sha256_16") == h.hexdigest()[:16] else None


def _measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the FETCH_SIZE /
    WRITE_SIZE counter runs in profiles/traffic_<workload>.md, or None when
    that kernel's source has changed since (first 16 hex digits of the
    file's SHA-256 differ)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    try:
        line = next(l for l in open(path) if l.startswith("traffic-json: "))
        rec = json.loads(line[len("traffic-json: "):])[kernel]
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, StopIteration, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    return int(rec["bytes"])


def _time(fn, torch, reps):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _rel(a, b):
    import numpy as np
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _worst(a, b):
    """Worst particle's error over the RMS reference magnitude."""
    import numpy as np
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        a, b = a[:, None], b[:, None]
    return float(np.linalg.norm(a - b, axis=1).max() / np.sqrt(np.mean(np.sum(b * b, axis=1))))


class Workload:
    """One single-system workload on the GPU: seeded inputs, plan, outputs."""

    def __init__(self, cfg, torch, msm, WL, np):
        self.cfg = cfg
        self.c = c = WL.WORKLOADS[cfg]
        pos64, q64, self.box = WL.make_config(cfg, 1.0)
        dt = np.float64 if c["fp64"] else np.float32
        self.pos_t, self.q_t = pos64.astype(dt), q64.astype(dt)
        self.pos64, self.q64 = self.pos_t.astype(np.float64), self.q_t.astype(np.float64)
        self.n = n = len(q64)
        tdt = torch.float64 if c["fp64"] else torch.float32
        dev = torch.device("cuda:0")
        self.P = torch.from_numpy(self.pos_t).to(dev).contiguous()
        self.Q = torch.from_numpy(self.q_t).to(dev).contiguous()
        self.plan = msm.Plan(self.box, c["periodic"], c["p"], c["h"], c["a"], c["L"],
                             msm.MSM_FP64 if c["fp64"] else msm.MSM_FP32, n)
        self.E = torch.empty(1, dtype=torch.float64, device=dev)
        self.F = torch.empty((n, 3), dtype=tdt, device=dev)
        self.dq = torch.empty(n, dtype=tdt, device=dev)
        self.torch = torch

    def step(self):
        self.plan.energy_forces(self.P, self.Q, out=(self.E, self.F, self.dq))

    def timed(self, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        if self.plan.status() != 0:
            raise RuntimeError(f"device error flag set in workload {self.cfg}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def stages(self, steps, names=None, one_stream=True):
        """Per-stage ms per call from the plan's HIP events (one stream: each
        stage's own duration)."""
        torch = self.torch
        if one_stream:
            os.environ["MSM_STREAMS"] = "0"
        try:
            self.plan.set_profile_stages(names)
            self.plan.profile(reset=True)
            self.plan.set_profiling(True)
            for _ in range(steps):
                self.step()
            torch.cuda.synchronize()
            self.plan.set_profiling(False)
            prof = self.plan.profile(reset=True)
        finally:
            if one_stream:
                del os.environ["MSM_STREAMS"]
        return prof

    def oracle(self, O):
        c = self.c
        per = [bool((c["periodic"] >> k) & 1) for k in range(3)]
        return O.OracleMSM(self.box, per, c["p"], c["h"], c["a"], c["L"])


def _rooflines(w, stages, npairs):
    """Kernel rooflines from the one-stream stage times: the pair sum
    against FP32 peak, the level-1 convolution against FP64 peak (it
    accumulates in FP64)."""
    desc = w.plan.describe()
    l1 = desc["levels_info"][0]
    G1 = l1["n"][0] * l1["n"][1] * l1["n"][2]
    if l1.get("factored"):
        conv_flops = 2.0 * l1["ext"][0] * l1["ext"][1] * l1["ext"][2] * l1["samples_nnz"]
    else:
        conv_flops = 2.0 * G1 * l1["stencil_nnz"]
    per = {k: v["ms"] / max(v["launches"], 1) for k, v in stages.items()}
    out = {}
    if npairs is not None and "pair" in per:
        fl = (28 + 4 * w.c["p"]) * npairs
        a = fl / (per["pair"] * 1e-3) / 1e12
        out["pair"] = {"bound": "alu", "kernel": f"k_pair_pc<{'double' if w.c['fp64'] else 'float'}, "
                                                 f"{w.c['p']}>",
                       "achieved": round(a, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(a / PEAK_FP32_VECTOR_TFLOPS, 4),
                       "algorithmic_per_launch": fl, "unique_pairs_in_cutoff": npairs,
                       "flops_per_pair": 28 + 4 * w.c["p"], "avg_launch_ms": round(per["pair"], 5)}
    if "conv_l1" in per:
        a = conv_flops / (per["conv_l1"] * 1e-3) / 1e12
        out["conv_l1"] = {"bound": "alu", "kernel": "k_conv (level 1)", "achieved": round(a, 3),
                          "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                          "frac": round(a / PEAK_FP64_TFLOPS, 4),
                          "algorithmic_per_launch": conv_flops,
                          "avg_launch_ms": round(per["conv_l1"], 5)}
    return out


def _oracle_sampled_error(w, O, np, nsel, seed):
    sel = np.sort(np.random.default_rng(seed).choice(w.n, nsel, replace=False))
    o = w.oracle(O)
    phi_r, F_r = o.sampled(w.pos64, w.q64, sel)
    Fg = w.F.double().cpu().numpy()[sel]
    pg = w.dq.double().cpu().numpy()[sel]
    return {"sampled_particles": nsel, "force_rel_rms": _rel(Fg, F_r),
            "force_worst_particle": _worst(Fg, F_r), "phi_rel_rms": _rel(pg, phi_r)}


def _cpu_baseline(w, O, np, S, threads):
    """The oracle (FP64, unchanged) on a linear 1/k share of every part of
    one full evaluation of the workload: the short-range sums of S random
    target charges (cell list, all partners), the anterpolation of those S
    charges onto every level, the level potentials at a random S/N share of
    every level's grid points, and the interpolation at the S targets.  Each
    part's work is its full-size work times S/N, so S / time is the full
    evaluation's particles/s extrapolated linearly."""
    o = w.oracle(O)
    L = w.c["L"]
    for l in range(1, L + 1):
        o.stencil(l)  # plan-time work, not timed (as on the GPU)
    rng = np.random.default_rng(1234 + S)
    sel = np.sort(rng.choice(w.n, S, replace=False))
    ps, qs = np.ascontiguousarray(w.pos64[sel]), np.ascontiguousarray(w.q64[sel])
    pts = []
    for l in range(1, L + 1):
        G = int(np.prod(o.grid_shape(l)))
        pts.append(np.sort(rng.choice(G, max(1, round(G * S / w.n)), replace=False)))
    old = O.num_threads()
    O.set_num_threads(threads)
    try:
        t0 = time.perf_counter()
        o.short_range(w.pos64, w.q64, sel=sel, cells=True)
        phi = np.zeros(S)
        F = np.zeros((S, 3))
        for l in range(1, L + 1):
            qg = o.grid_charge(l, ps, qs)
            eg = o.level_potential(l, qg, points=pts[l - 1])
            O.lib().orc_interpolate(o._gp, l, S, O._ptr(ps), O._ptr(qs), O._ptr(eg),
                                    O._ptr(phi), O._ptr(F))
        dt = time.perf_counter() - t0
    finally:
        O.set_num_threads(old)
    return S / dt, dt


def _water(torch, msm, WL, np, O, steps, check):
    """The periodic water box: 33,333 rigid 3-site molecules (99,999
    charges), 100 A cube, p = 4, h = 1.5625, a = 10, L = 5, FP32."""
    w = Workload(2, torch, msm, WL, np)
    t = w.timed(steps, 5)
    st = w.stages(min(steps, 20))
    out = {"workload": "periodic water box, 33,333 rigid 3-site molecules (99,999 charges), "
                       "100 A cube, p=4, h=1.5625, a=10, L=5, FP32", "n": w.n,
           "particles_per_s": round(w.n / t, 1), "ms_per_step": round(t * 1e3, 4),
           "stages_ms_one_stream": {k: round(v["ms"] / v["launches"], 5) for k, v in st.items()},
           "rooflines": {k: dict(v, traffic=_measured_traffic("water100k_fp32", k))
                         for k, v in _rooflines(w, st, _pair_count(2, w.pos_t)).items()}}
    if check:
        ref = w.oracle(O).compute(w.pos64, w.q64)
        out["energy_rel_err_vs_fp64_oracle"] = abs(w.E.item() - ref["E"]) / abs(ref["E"])
        out["force_rel_err_vs_fp64_oracle"] = _rel(w.F.double().cpu().numpy(), ref["F"])
        out["force_worst_particle_vs_fp64_oracle"] = _worst(w.F.double().cpu().numpy(), ref["F"])
    return out


def _free_ions(torch, msm, WL, np, O, check):
    """The free-space ion cloud: 1,000 charges +-1 in a 20 A cube, FP64, p = 4,
    h = 2, a = 8, L = 3."""
    w = Workload(1, torch, msm, WL, np)
    t = w.timed(50, 5)
    out = {"workload": "free-space ion cloud, 1,000 charges +-1, 20 A cube, p=4, h=2, a=8, L=3, "
                       "FP64", "n": w.n, "particles_per_s": round(w.n / t, 1),
           "ms_per_step": round(t * 1e3, 4)}
    if check:
        ref = w.oracle(O).compute(w.pos64, w.q64)
        out["energy_rel_err_vs_fp64_oracle"] = abs(w.E.item() - ref["E"]) / abs(ref["E"])
        out["force_rel_err_vs_fp64_oracle"] = _rel(w.F.double().cpu().numpy(), ref["F"])
        # the MSM's own error: against the exact all-pairs Coulomb sum
        _, F_exact = O.direct_coulomb(w.pos64, w.q64)
        out["msm_force_rel_err_vs_exact_coulomb"] = _rel(w.F.double().cpu().numpy(), F_exact)
    return out


def _autograd_vs_plain(torch, msm, WL, np, O, check):
    """Learnable-charge workload (200,000 Gaussian charges, 60 A periodic
    cube, p=4, h=1.5, a=10, L=4, FP32): plain forward vs forward + backward
    of L = E + sum v.F (v ~ N(0,1)), and the same through torch.autograd."""
    w = Workload(4, torch, msm, WL, np)
    n, dev = w.n, torch.device("cuda:0")
    v64 = WL.force_cotangent(n, seed=40)
    v = torch.tensor(v64, dtype=torch.float32, device=dev)
    ws = torch.empty(w.plan.workspace_bytes(n), dtype=torch.uint8, device=dev)
    gE = torch.ones(1, dtype=torch.float64, device=dev)
    t_fwd = _time(w.step, torch, 20)
    grads = {}

    def fwd_bwd():
        w.plan.energy_forces(w.P, w.Q, ws=ws, out=(w.E, w.F, w.dq))
        grads["pos"], grads["q"] = w.plan.backward(w.P, w.Q, ws, gE=gE, gF=v)
    t_fb = _time(fwd_bwd, torch, 20)
    Pg = w.P.clone().requires_grad_(True)
    Qg = w.Q.clone().requires_grad_(True)

    def autograd_step():
        Pg.grad = None
        Qg.grad = None
        e, f, _ = msm.energy_forces(Pg, Qg, w.plan)
        (e.sum() + (f * v).sum()).backward()
    t_ag = _time(autograd_step, torch, 10)
    out = {"workload": "200,000 Gaussian charges, 60 A periodic cube, p=4, h=1.5, a=10, L=4, "
                       "FP32", "n": n,
           "forward_particles_per_s": round(n / t_fwd, 1),
           "forward_backward_particles_per_s": round(n / t_fb, 1),
           "torch_autograd_particles_per_s": round(n / t_ag, 1),
           "forward_backward_over_forward_time": round(t_fb / t_fwd, 3)}
    if check:
        sel = np.sort(np.random.default_rng(41).choice(n, 16, replace=False))
        o = w.oracle(O)
        v_t = v64.astype(np.float32).astype(np.float64)
        rq, rpos = o.sampled_backward(w.pos64, w.q64, 1.0, v_t, sel)
        gq = grads["q"].double().cpu().numpy()[sel]
        gp = grads["pos"].double().cpu().numpy()[sel]
        out["grad_q_rel_err_vs_fp64_oracle_sampled"] = _rel(gq, rq)
        out["grad_pos_rel_err_vs_fp64_oracle_sampled"] = _rel(gp, rpos)
        out["sampled_particles"] = len(sel)
        Eg = _golden_energy(4, w.pos_t, w.q_t)
        if Eg is not None:
            out["energy_rel_err_vs_fp64_oracle"] = abs(w.E.item() - Eg) / abs(Eg)
    return out


def _batched_vs_plain(torch, msm, WL, np, O, check):
    """4,096 free-space clusters of 8-256 charges in 10-30 A boxes (p=4, h=1,
    a=6, FP32): one batched launch sequence vs one plan per system run one
    after another (timed on the first 256 systems, per particle)."""
    off, boxes, pos, q, levels = WL.make_batch(4096, seed=5)
    dev = torch.device("cuda:0")
    O_ = torch.tensor(off, dtype=torch.int32, device=dev)
    P = torch.tensor(pos, dtype=torch.float32, device=dev)
    Q = torch.tensor(q, dtype=torch.float32, device=dev)
    ntot = int(off[-1])
    bp = msm.BatchPlan(boxes, levels, 4, 1.0, 6.0, msm.MSM_FP32, ntot)
    E = torch.empty(len(boxes), dtype=torch.float64, device=dev)
    F = torch.empty((ntot, 3), dtype=torch.float32, device=dev)
    dq = torch.empty(ntot, dtype=torch.float32, device=dev)
    t_b = _time(lambda: bp.energy_forces(O_, P, Q, out=(E, F, dq)), torch, 10)
    ns = 256
    plans, args_ = [], []
    for s in range(ns):
        a, b = int(off[s]), int(off[s + 1])
        pl = msm.Plan((float(boxes[s]),) * 3, 0, 4, 1.0, 6.0, int(levels[s]), msm.MSM_FP32,
                      max(b - a, 1))
        plans.append(pl)
        args_.append((P[a:b], Q[a:b], (torch.empty(1, dtype=torch.float64, device=dev),
                                       torch.empty((b - a, 3), dtype=torch.float32, device=dev),
                                       torch.empty(b - a, dtype=torch.float32, device=dev))))

    def plain():
        for pl, (pp, qq, o) in zip(plans, args_):
            pl.energy_forces(pp, qq, out=o)
    t_p = _time(plain, torch, 3)
    n_sub = int(off[ns])
    out = {"workload": "4,096 free-space clusters, 8-256 charges, 10-30 A boxes, p=4, h=1, "
                       "a=6, FP32", "n_systems": len(boxes), "n": ntot,
           "batched_particles_per_s": round(ntot / t_b, 1),
           "plain_particles_per_s": round(n_sub / t_p, 1),
           "plain_sample_systems": ns,
           "batched_over_plain": round((ntot / t_b) / (n_sub / t_p), 2)}
    if check:
        bp.energy_forces(O_, P, Q, out=(E, F, dq))
        torch.cuda.synchronize()
        Eg, Fg = E.cpu().numpy(), F.double().cpu().numpy()
        sys_sel = np.random.default_rng(6).choice(len(boxes), 8, replace=False)
        eE, eF = [], []
        for s in sys_sel:
            a, b = int(off[s]), int(off[s + 1])
            p32 = pos[a:b].astype(np.float32).astype(np.float64)
            q32 = q[a:b].astype(np.float32).astype(np.float64)
            o = O.OracleMSM((float(boxes[s]),) * 3, [False] * 3, 4, 1.0, 6.0, int(levels[s]))
            r = o.compute(p32, q32)
            eE.append(abs(Eg[s] - r["E"]) / abs(r["E"]))
            eF.append(_rel(Fg[a:b], r["F"]))
        out["sampled_systems"] = len(sys_sel)
        out["energy_rel_err_vs_fp64_oracle_max"] = float(max(eE))
        out["force_rel_err_vs_fp64_oracle_max"] = float(max(eF))
    return out


def _grid_pass_sweep(torch, msm, steps):
    """HBM rate of the grid passes (anterpolation, restriction, prolongation,
    interpolation) on level-1 grids of 128^3 to 512^3 points and 1e7 to 6e7
    charges: periodic cube of edge n1 h (h = 1), uniform random positions,
    charges +-1 in equal numbers, FP32, p = 4, a = 3, levels down to an 8^3
    top grid.  Every stage runs on one stream (no overlap), timed by the
    plan's stage events; algorithmic bytes per pass count 4-byte grid values
    and 16 bytes (position + charge) per charge read or (force + potential)
    written:
      anterpolation  16 N + 4 G1
      restriction    sum_l 4 (G_l + G_l+1)
      prolongation   sum_l 4 (G_l+1 + 2 G_l)
      interpolation  16 N + 4 G1 + 16 N
    (6e7 is near the largest count an FP32 plan accepts: its cluster buffers
    use 32-bit byte offsets.)"""
    cases = [(128, 10_000_000), (256, 10_000_000), (512, 10_000_000), (512, 60_000_000)]
    dev = torch.device("cuda:0")
    out = []
    os.environ["MSM_STREAMS"] = "0"
    try:
        for n1, n in cases:
            g = torch.Generator(device=dev)
            g.manual_seed(1000 + n1 + n // 1_000_000)
            box = float(n1)
            L = (n1 // 8).bit_length()  # top grid 8^3
            P = torch.rand((n, 3), generator=g, device=dev, dtype=torch.float32) * box
            Q = torch.ones(n, dtype=torch.float32, device=dev)
            Q[torch.randperm(n, generator=g, device=dev)[: n // 2]] = -1.0
            plan = msm.Plan((box,) * 3, 7, 4, 1.0, 3.0, L, msm.MSM_FP32, n)
            lev = plan.describe()["levels_info"]
            G = [li["n"][0] * li["n"][1] * li["n"][2] for li in lev]
            E = torch.empty(1, dtype=torch.float64, device=dev)
            F = torch.empty((n, 3), dtype=torch.float32, device=dev)
            dq = torch.empty(n, dtype=torch.float32, device=dev)
            plan.energy_forces(P, Q, out=(E, F, dq))
            torch.cuda.synchronize()
            if plan.status() != 0:
                raise RuntimeError("device error flag set in the grid-pass sweep")
            names = ["anterp", "restrict", "prolong", "interp"]
            plan.set_profile_stages(names + ["bin", "cluster", "pair"])
            plan.profile(reset=True)
            plan.set_profiling(True)
            for _ in range(steps):
                plan.energy_forces(P, Q, out=(E, F, dq))
            torch.cuda.synchronize()
            plan.set_profiling(False)
            prof = plan.profile(reset=True)
            alg = {"anterp": 16 * n + 4 * G[0],
                   "restrict": sum(4 * (G[l] + G[l + 1]) for l in range(L - 1)),
                   "prolong": sum(4 * (G[l + 1] + 2 * G[l]) for l in range(L - 1)),
                   "interp": 32 * n + 4 * G[0]}
            # the cell-list build and the pair sum, for scale (not grid passes)
            rec = {"grid1": [n1] * 3, "n": n, "levels": L,
                   "other_ms": {k: round(prof[k]["ms"] / steps, 4)
                                for k in ("bin", "cluster", "pair") if k in prof}}
            for k in names:
                ms = prof[k]["ms"] / steps
                gbs = alg[k] / (ms * 1e-3) / 1e9
                rec[k] = {"ms": round(ms, 4), "bytes": alg[k], "GBps": round(gbs, 1),
                          "frac_hbm": round(gbs / PEAK_HBM_GBS, 4)}
            out.append(rec)
            del plan, P, Q, E, F, dq
            torch.cuda.empty_cache()
    finally:
        del os.environ["MSM_STREAMS"]
    return out


def _md(torch, msm, np, steps=2000):
    """Charged Lennard-Jonesium (Sec. MD simulation of charged
    Lennard-Jonesium) in reduced units: 1,000 particles at density 0.85,
    |q| = sqrt(50), rock-salt start, velocities at 2 x 3.15; LJ cutoff 4,
    switch from 3.5; MSM p = 6, h = 0.5, a = 4, L = 3, skin 0.3; dt = 5e-4.
    Velocity-Verlet steps per second replayed from a graph and launched
    eagerly, the Verlet-skin rebuilds, and the NVE stability measure."""
    n_side = 10
    n = n_side ** 3
    L = (n / 0.85) ** (1.0 / 3.0)
    rng = np.random.default_rng(31)
    g = (np.arange(n_side) + 0.5) * (L / n_side)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos += rng.normal(scale=0.02, size=pos.shape)
    q = np.where(np.indices((n_side,) * 3).sum(0).ravel() % 2 == 0, 1.0, -1.0) * np.sqrt(50.0)
    vel = np.random.default_rng(32).normal(scale=np.sqrt(2 * 3.15), size=pos.shape)
    vel -= vel.mean(axis=0)
    out = {"workload": "charged Lennard-Jonesium, 1,000 particles, density 0.85, |q| = sqrt(50), "
                       "reduced units, dt = 5e-4, LJ cutoff 4 (switch from 3.5), MSM p=6 h=0.5 "
                       "a=4 L=3, skin 0.3"}
    for name, prec, dt_ in (("fp32", msm.MSM_FP32, torch.float32),
                            ("fp64", msm.MSM_FP64, torch.float64)):
        rec = {}
        for graph in (True, False):
            plan = msm.Plan((L, L, L), 7, 6, 0.5, 4.0, 3, prec, n)
            plan.set_skin(0.3)
            md = msm.MD(plan, n, 5e-4, 1.0, 1.0, 4.0, 3.5, log_steps=steps)
            T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=dt_, device="cuda")  # noqa
            md.set_state(T(pos), T(vel), T(q), T(np.ones(n)))
            md.run(1, graph=graph)  # (the capture, when graph)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            md.run(steps - 1, graph=graph)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / (steps - 1)
            if plan.status() != 0:
                raise RuntimeError("device error flag set in the MD run")
            key = "graph" if graph else "eager"
            rec[f"{key}_ms_per_step"] = round(t * 1e3, 4)
            rec[f"{key}_steps_per_s"] = round(1.0 / t, 1)
            if graph:
                log = md.energies()
                tot = log.sum(axis=1)
                half = len(tot) // 2
                calls, rebuilds = plan.skin_stats()
                rec.update({"steps": int(len(log)), "cell_list_rebuilds": rebuilds,
                            "msm_calls": calls,
                            "std_total_over_std_kinetic": float(tot.std() / log[:, 0].std()),
                            "mean_total_change_over_std_kinetic":
                                float(abs(tot[half:].mean() - tot[:half].mean()) / log[:, 0].std())})
            md.close()
            plan.close()
        out[name] = rec
    return out


def _accuracy_sweep(torch, msm, WL, np, O, reps):
    """Cost against accuracy over the method's parameters (Sec.
    Accuracy-performance tradeoff): 10^4 charges no two closer than 0.6 d
    (d = (V/N)^(1/3) = 2 A), uniform charges in [-1, 1] minus their mean, in a
    free cube and in a periodic one; h = d; interpolation order p = 4, 6, 8,
    cutoff a = 3..10 d, FP32 and FP64; then the degree M of omega' at a = 6 d
    in FP64.  The exact reference is the all-pairs Coulomb sum (free) or the
    Ewald sum (periodic), both from the FP64 oracle.  Error: force RMSE over
    the reference forces' standard deviation (the paper's metric), with the
    relative RMS of F and phi beside it; time: one msm_energy_forces call
    (cell-list build included) replayed from a graph, the median of five
    means over `reps` replays."""
    n, dbar = 10_000, 2.0
    L = dbar * n ** (1.0 / 3.0)
    dev = torch.device("cuda:0")
    out = {"workload": f"{n} charges, minimum distance 0.6 d, d = {dbar} A, cube of {L:.2f} A, "
                       "charges U[-1, 1] minus the mean; h = d; levels 3",
           "systems": {}}
    for periodic in (False, True):
        pos, q = WL.spaced_charges(n, L, periodic, seed=900 + int(periodic))
        t0 = time.perf_counter()
        if periodic:
            phi_r, F_r = O.ewald3d_system((L, L, L), pos, q)
        else:
            phi_r, F_r = O.direct_coulomb(pos, q)
        ref_s = time.perf_counter() - t0
        std = float(np.std(F_r))
        points = []

        def run(p, a, fp64, M=-1):
            dt = np.float64 if fp64 else np.float32
            P = torch.from_numpy(pos.astype(dt)).to(dev)
            Q = torch.from_numpy(q.astype(dt)).to(dev)
            plan = msm.Plan((L, L, L), 7 if periodic else 0, p, dbar, a * dbar, 3,
                            msm.MSM_FP64 if fp64 else msm.MSM_FP32, n, quasi_degree=M)
            E, F, dq = plan.energy_forces(P, Q)
            torch.cuda.synchronize()
            # one call captured in a graph and replayed: the GPU's time per
            # call, without the host's launch cost of ~30 small kernels
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                plan.energy_forces(P, Q, out=(E, F, dq), stream=torch.cuda.current_stream())
            ts = sorted(_time(g.replay, torch, reps) for _ in range(5))
            t = ts[2]
            if plan.status() != 0:
                raise RuntimeError("device error flag set in the accuracy sweep")
            Fg, pg = F.double().cpu().numpy(), dq.double().cpu().numpy()
            rec = {"p": p, "a_over_d": a, "precision": "fp64" if fp64 else "fp32",
                   "M": plan.describe()["M"], "ms": round(t * 1e3, 4),
                   "force_rmse_over_std": float(np.sqrt(np.mean((Fg - F_r) ** 2)) / std),
                   "force_rel_rms": _rel(Fg, F_r), "phi_rel_rms": _rel(pg, phi_r)}
            plan.close()
            return rec

        for fp64 in (False, True):
            for p in (4, 6, 8):
                for a in range(3, 11):
                    points.append(run(p, a, fp64))
        msweep = []
        for p in (4, 6, 8):
            for M in (p // 2 - 1, p // 2, p, 2 * p):
                msweep.append(run(p, 6, True, M))
        print(f"accuracy sweep: {'periodic' if periodic else 'free'} system done",
              file=sys.stderr, flush=True)
        out["systems"]["periodic" if periodic else "free"] = {
            "reference": "Ewald sum (structure factors)" if periodic else "all-pairs Coulomb",
            "reference_seconds": round(ref_s, 2), "force_std": std,
            "points": points, "quasi_degree_sweep": msweep}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error-check", action="store_true")
    ap.add_argument("--extras", default="water,autograd,batched,free_ions,md",
                    help="comma-separated extra workloads to run beside the headline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the water, autograd, batched, free-ion and MD workloads")
    ap.add_argument("--no-grid-sweep", action="store_true",
                    help="skip the grid-pass timing on 128^3-512^3 level-1 grids with 1e7-6e7 "
                         "charges (HBM fraction of anterpolation, restriction, prolongation, "
                         "interpolation)")
    ap.add_argument("--accuracy-sweep", action="store_true",
                    help="add the cost-vs-accuracy sweep (p = 4/6/8, cutoff 3-10 mean spacings, "
                         "FP32/FP64, degree of omega') on 10^4 spaced charges, free and periodic")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after the timed region, one device-to-device copy of this many MiB "
                         "(reference kernel for the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: libmsm runs on exactly one GPU (got --gpus {args.gpus}); "
              "sharding across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2510_05961_amd import msm
    from paper_2510_05961_amd import workloads as WL

    w = Workload(3, torch, msm, WL, np)
    # timed region: the production forward (pair sum and coarse levels on
    # their own streams), no profiling events
    t_step = w.timed(args.steps, args.warmup)
    value = w.n / t_step
    # each stage on its own (one stream, HIP events around every stage)
    st = w.stages(min(args.steps, 10))
    stage_ms = {k: v["ms"] / max(v["launches"], 1) for k, v in st.items()}
    npairs = _pair_count(3, w.pos_t)
    roofs = _rooflines(w, st, npairs)
    dom = max(stage_ms, key=stage_ms.get)
    roofline = dict(roofs.get(dom, {}))
    if roofline:
        roofline["stage"] = dom
        roofline["traffic"] = _measured_traffic("slab1m_fp32", dom)
    # the cell-list build (binning, cluster layout) opens every call on the
    # caller's stream; the paper's timings leave the neighbour list out
    nl_ms = stage_ms.get("bin", 0.0) + stage_ms.get("cluster", 0.0)
    desc = w.plan.describe()
    result = {
        "metric": METRIC, "value": round(value, 1), "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_step * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "slab, 10^6 charges +-1, 100 x 100 x 60 A, periodic x and y, "
                               "free z, p=6, h=1.25, a=12, L=5, FP32",
                   "n": w.n, "box": list(w.box), "periodic": "xy", "order": w.c["p"],
                   "h": desc["levels_info"][0]["h"][0], "cutoff": w.c["a"],
                   "levels": w.c["L"], "precision": "fp32"},
        "roofline": roofline,
        "kernels": roofs,
        "stages_ms_one_stream": {k: round(v, 5) for k, v in stage_ms.items()},
        "neighbour_list_ms_one_stream": round(nl_ms, 4),
    }

    if args.calib_copy_mb > 0:
        nb = args.calib_copy_mb * (1 << 20)
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        result["calib_copy_bytes"] = nb
        del src, dst

    check = not args.no_error_check
    if check or not args.no_cpu_baseline or not args.no_extras:
        from oracle import oracle as O
    if check:
        w.step()
        torch.cuda.synchronize()
        err = _oracle_sampled_error(w, O, np, 32, seed=0)
        Eg = _golden_energy(3, w.pos_t, w.q_t)
        if Eg is not None:
            err["energy_rel_err_vs_fp64_oracle"] = abs(w.E.item() - Eg) / abs(Eg)
        phi = w.dq.double().cpu().numpy()
        e2 = 0.5 * float(np.dot(w.q64, phi))
        err["energy_vs_half_sum_q_phi"] = abs(w.E.item() - e2) / abs(e2)
        result["error_vs_fp64_oracle"] = err

    if not args.no_cpu_baseline:
        runs = [_cpu_baseline(w, O, np, 20000, O.num_threads()) for _ in range(3)]
        one = _cpu_baseline(w, O, np, 2000, 1)
        vals = sorted(r[0] for r in runs)
        result["cpu_baseline"] = {
            "value": round(vals[1], 1), "unit": "particles/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": "the FP64 oracle on a linear 20,000/10^6 share of every part of one full "
                      "evaluation of the same slab input (short-range sums of 20,000 random "
                      "targets over all partners by cell list, anterpolation of those charges on "
                      "all 5 levels, level potentials at the same share of every level's grid "
                      "points, interpolation at the targets); value = targets / seconds, median "
                      "of 3 runs",
            "runs_seconds": [round(r[1], 3) for r in runs],
            "one_thread": {"value": round(one[0], 1), "cores": 1, "targets": 2000,
                           "seconds": round(one[1], 3)}}

    if not args.no_extras:
        want = set(args.extras.split(","))
        Oc = O if check else None
        if "water" in want:
            result["water"] = _water(torch, msm, WL, np, Oc, args.steps, check)
        if "autograd" in want:
            result["autograd"] = _autograd_vs_plain(torch, msm, WL, np, Oc, check)
        if "batched" in want:
            result["batched"] = _batched_vs_plain(torch, msm, WL, np, Oc, check)
        if "free_ions" in want:
            result["free_ions_fp64"] = _free_ions(torch, msm, WL, np, Oc, check)
        if "md" in want:
            result["md"] = _md(torch, msm, np)

    if not args.no_grid_sweep:
        try:
            result["grid_pass_sweep"] = _grid_pass_sweep(torch, msm, max(args.steps // 10, 3))
        except RuntimeError as e:  # (MSMError and out-of-memory included) keep the headline line
            result["grid_pass_sweep"] = {"error": str(e)}

    if args.accuracy_sweep:
        from oracle import oracle as O
        result["accuracy_sweep"] = _accuracy_sweep(torch, msm, WL, np, O, 20)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
