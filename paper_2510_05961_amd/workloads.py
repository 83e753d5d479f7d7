"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers (numpy PCG64, ``default_rng(seed)``);
it holds none of the method's arithmetic, so the oracle and the HIP path can
both be fed from it.  Every generator returns FP64 arrays; FP32 runs cast
them once and give the oracle the cast values.

The paper's own inputs (PACKMOL boxes, Sec. "Benchmarks") are not
available, so these stand in for them:

* ``random_ions``: N point charges uniform in a box, exactly half +1 and half
  -1 (neutral), randomly permuted.
* ``water_box``: rigid 3-site water-like molecules (O -0.834, H +0.417,
  O-H 0.9572, H-O-H 104.52 degrees), oxygen uniform in a periodic box,
  uniformly random orientation (unit quaternion from four normals), all sites
  wrapped into the box; overlaps allowed.
* ``gaussian_charges``: N sites uniform in a box, charges N(0, sigma) with the
  mean removed (zero net charge).
* ``clusters``: many small non-periodic systems with uniformly random sizes
  and box edges, Gaussian neutral charges, concatenated in CSR form.
* ``spaced_charges``: N sites in a cubic box no two closer than 0.6 d, with
  d = (V/N)^(1/3) the mean spacing (minimum image when periodic), charges
  uniform in [-1, 1] minus their mean: the recipe of the paper's benchmark
  inputs (Sec. Benchmarks), drawn here by random sequential addition instead
  of PACKMOL and a relaxation.
"""
from __future__ import annotations

import numpy as np


def random_ions(n, box, seed):
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    pos = rng.random((n, 3)) * box
    q = np.concatenate([np.ones(n // 2), -np.ones(n - n // 2)])
    rng.shuffle(q)
    return pos, q


def water_box(n_molecules, box_len, seed):
    rng = np.random.default_rng(seed)
    box = float(box_len)
    O = rng.random((n_molecules, 3)) * box
    quat = rng.standard_normal((n_molecules, 4))
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    w, x, y, z = quat.T
    R = np.empty((n_molecules, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    bond, half = 0.9572, np.deg2rad(104.52) / 2
    local = np.array([[np.sin(half), 0.0, np.cos(half)], [-np.sin(half), 0.0, np.cos(half)]]) * bond
    H1 = O + np.einsum("nij,j->ni", R, local[0])
    H2 = O + np.einsum("nij,j->ni", R, local[1])
    pos = np.stack([O, H1, H2], axis=1).reshape(-1, 3)
    pos = pos - box * np.floor(pos / box)
    pos[pos >= box] = 0.0
    q = np.tile(np.array([-0.834, 0.417, 0.417]), n_molecules)
    return pos, q


def gaussian_charges(n, box, sigma, seed):
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    pos = rng.random((n, 3)) * box
    q = rng.normal(0.0, sigma, n)
    q -= q.mean()
    return pos, q


def clusters(n_sys, nmin, nmax, box_min, box_max, sigma, seed):
    """Returns (offsets[n_sys+1], boxes[n_sys], pos[N,3], q[N])."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, n_sys)
    boxes = rng.uniform(box_min, box_max, n_sys)
    offsets = np.zeros(n_sys + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    pos = np.empty((offsets[-1], 3))
    q = np.empty(offsets[-1])
    for s in range(n_sys):
        a, b = offsets[s], offsets[s + 1]
        pos[a:b] = rng.random((b - a, 3)) * boxes[s]
        qs = rng.normal(0.0, sigma, b - a)
        q[a:b] = qs - qs.mean()
    return offsets, boxes, pos, q


def force_cotangent(n, seed=40):
    """Random FP64 cotangent on the forces, N(0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 3))


def spaced_charges(n, box_len, periodic, seed, min_frac=0.6):
    """Random sequential addition: candidates uniform in the cube are kept if
    no kept site lies within min_frac * (V/n)^(1/3) (minimum image when
    periodic).  Returns positions [n, 3] in [0, box_len)^3 and charges."""
    rng = np.random.default_rng(seed)
    L = float(box_len)
    dmin = min_frac * L / n ** (1.0 / 3.0)
    nc = max(1, int(L // dmin))
    cs = L / nc
    grid = {}
    pos = np.empty((n, 3))
    k = 0
    while k < n:
        c = rng.random(3) * L
        ic = np.minimum((c // cs).astype(int), nc - 1)
        ok = True
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    jc = ic + (dx, dy, dz)
                    if periodic:
                        jc %= nc
                    elif (jc < 0).any() or (jc >= nc).any():
                        continue
                    for j in grid.get(tuple(jc), ()):
                        d = c - pos[j]
                        if periodic:
                            d -= L * np.round(d / L)
                        if d @ d < dmin * dmin:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            pos[k] = c
            grid.setdefault(tuple(ic), []).append(k)
            k += 1
    q = rng.uniform(-1.0, 1.0, n)
    q -= q.mean()
    return pos, q


# --- the five workloads -----------------------------------------------------
# Parameters: box, periodic mask (bit k = axis k), order p, spacing h, cutoff
# a, levels L, precision.
WORKLOADS = {
    1: dict(name="C1 non-periodic 1k ions, FP64", box=(20.0, 20.0, 20.0), periodic=0,
            p=4, h=2.0, a=8.0, L=3, fp64=True),
    2: dict(name="C2 periodic water 33,333 molecules (99,999 sites), 100 A box, FP32",
            box=(100.0, 100.0, 100.0), periodic=7, p=4, h=1.5, a=10.0, L=5, fp64=False),
    3: dict(name="C3 slab 1e6 ions 100x100x60 A, FP32", box=(100.0, 100.0, 60.0), periodic=3,
            p=6, h=1.25, a=12.0, L=5, fp64=False),
    4: dict(name="C4 periodic 2e5 Gaussian charges 60 A, FP32", box=(60.0, 60.0, 60.0),
            periodic=7, p=4, h=1.5, a=10.0, L=4, fp64=False),
    5: dict(name="C5 4096 clusters 8-256 atoms, FP32", box=None, periodic=0, p=4, h=1.0,
            a=6.0, L=None, fp64=False),
}


def make_config(cfg, scale=1.0):
    """Inputs of workload ``cfg`` (1..4); ``scale`` < 1 shrinks N and the box
    at fixed density for the small parity cases."""
    c = WORKLOADS[cfg]
    if cfg == 1:
        n = max(2, int(round(1000 * scale)))
        L = 20.0 * scale ** (1.0 / 3.0)
        pos, q = random_ions(n, (L, L, L), seed=1)
        return pos, q, (L, L, L)
    if cfg == 2:
        nm = max(1, int(round(33333 * scale)))
        L = 100.0 * scale ** (1.0 / 3.0)
        pos, q = water_box(nm, L, seed=2)
        return pos, q, (L, L, L)
    if cfg == 3:
        n = max(2, int(round(1_000_000 * scale)))
        s = scale ** (1.0 / 3.0)
        box = (100.0 * s, 100.0 * s, 60.0 * s)
        pos, q = random_ions(n, box, seed=3)
        return pos, q, box
    if cfg == 4:
        n = max(2, int(round(200_000 * scale)))
        L = 60.0 * scale ** (1.0 / 3.0)
        pos, q = gaussian_charges(n, (L, L, L), 0.5, seed=4)
        return pos, q, (L, L, L)
    raise ValueError(cfg)


def make_batch(n_sys=4096, seed=5):
    """Workload C5: clusters of 8-256 atoms in cubic boxes of 10-30 A."""
    offsets, boxes, pos, q = clusters(n_sys, 8, 256, 10.0, 30.0, 0.5, seed)
    levels = np.where(boxes <= 20.0, 2, 3).astype(np.int32)
    return offsets, boxes, pos, q, levels
