"""Shared helpers of the GPU parity tests (marshalling and error metrics)."""
import math

import numpy as np

from paper_2510_05961_amd import workloads as WL

# Parity bars: FP32 path force RMS relative error <= 1e-5 and energy <= 1e-6;
# FP64 path <= 1e-10 for both.
TOL = {"fp32": {"F": 1e-5, "E": 1e-6, "phi": 1e-5}, "fp64": {"F": 1e-10, "E": 1e-10, "phi": 1e-10}}


def mask_of(periodic):
    return sum(1 << k for k in range(3) if periodic[k])


def periodic_of(mask):
    return tuple(bool((mask >> k) & 1) for k in range(3))


def cast(pos, q, fp64):
    """Inputs rounded to the run's precision, returned as FP64 for the oracle."""
    dt = np.float64 if fp64 else np.float32
    return pos.astype(dt).astype(np.float64), q.astype(dt).astype(np.float64)


def rel_rms(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a - b))


def per_particle_ratio(a, b):
    """max_i |a_i - b_i| / rms_i |b_i| (rows of [n,3] arrays, elements of
    [n] arrays): the worst particle against the typical magnitude."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        a, b = a[:, None], b[:, None]
    if len(b) == 0:
        return 0.0
    err = np.linalg.norm(a - b, axis=1)
    rms = math.sqrt(float(np.mean(np.sum(b * b, axis=1))))
    return float(err.max() / rms) if rms > 0 else float(err.max())


def assert_parity(a, b, bar, what=""):
    """The parity bar on relative RMS error, and a per-particle bound: no
    particle may be off by more than 10 x bar x the RMS magnitude (so a few
    wrong particles cannot hide under a global RMS)."""
    e, m = rel_rms(a, b), per_particle_ratio(a, b)
    assert e <= bar and m <= 10 * bar, f"{what}: rel RMS {e:.3e}, worst particle {m:.3e} (bar {bar:g})"
    return e, m


def gpu_forward(plan, pos, q, ws=False):
    import torch
    dt = plan.dtype
    P = torch.tensor(pos, dtype=dt, device="cuda").contiguous()
    Q = torch.tensor(q, dtype=dt, device="cuda").contiguous()
    W = None
    if ws:
        W = torch.empty(plan.workspace_bytes(len(q)), dtype=torch.uint8, device="cuda")
    E, F, dq = plan.energy_forces(P, Q, ws=W)
    torch.cuda.synchronize()
    out = {"E": float(E.item()), "F": F.double().cpu().numpy(), "phi": dq.double().cpu().numpy()}
    if ws:
        out["ws"] = W
        out["P"], out["Q"] = P, Q
    return out


def config_case(cfg, scale):
    """(pos, q, box, periodic, p, h, a, L, fp64) of workload cfg at a scale."""
    c = WL.WORKLOADS[cfg]
    pos, q, box = WL.make_config(cfg, scale)
    return pos, q, box, periodic_of(c["periodic"]), c["p"], c["h"], c["a"], c["L"], c["fp64"]
