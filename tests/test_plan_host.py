"""Host-side plan of libmsm vs the oracle (no GPU needed).

The plan is built with msm_plan_create_host, which runs the same FP64 host
code as a device plan but allocates nothing on a GPU.  Its constants and
stencils must agree with the oracle's independent derivations.
"""
import ctypes
import math
import re

import numpy as np
import pytest

from oracle import constants as C
from oracle import oracle as O
from paper_2510_05961_amd import msm


def _mask(periodic):
    return sum(1 << k for k in range(3) if periodic[k])


def _fold(off, K, periodic, n):
    """Stencil box -> dict keyed by offset (free axes) / residue (periodic)."""
    out = {}
    lz, ly, lx = K.shape
    for z in range(lz):
        for y in range(ly):
            for x in range(lx):
                v = K[z, y, x]
                if v == 0.0:
                    continue
                d = [off[0] + x, off[1] + y, off[2] + z]
                key = tuple(d[k] % n[k] if periodic[k] else d[k] for k in range(3))
                out[key] = out.get(key, 0.0) + v
    return out


def _oracle_stencil_folded(o, level):
    W, K = o.stencil(level)
    n = o.levels[level - 1][0]
    return _fold([-W[0], -W[1], -W[2]], K, o.periodic, n)


CASES = [
    ((20.0, 20.0, 20.0), (0, 0, 0), 4, 2.0, 8.0, 3),   # C1 parameters
    ((16.0, 16.0, 16.0), (1, 1, 1), 4, 1.0, 4.0, 4),
    ((12.0, 12.0, 9.0), (1, 1, 0), 6, 0.75, 3.0, 3),
    ((10.0, 11.0, 12.0), (0, 0, 0), 6, 1.0, 3.0, 2),
    # one periodic axis (1-D Ewald top level), each axis in turn
    ((9.0, 10.0, 7.5), (0, 0, 1), 6, 0.75, 3.0, 3),
    ((7.5, 9.0, 10.0), (1, 0, 0), 4, 0.75, 3.0, 3),
    ((9.0, 7.0, 8.0), (0, 1, 0), 4, 1.0, 3.0, 2),
    # two periodic axes with the free one along x or y
    ((12.0, 9.0, 12.0), (1, 0, 1), 6, 0.75, 3.0, 3),
    ((9.0, 12.0, 12.0), (0, 1, 1), 4, 1.0, 3.0, 3),
]


def test_library_exports_every_header_symbol():
    lib = msm.lib()
    hdr = open(msm.HERE + "/../include/msm.h").read()
    declared = set(re.findall(r"\b(msm_[a-z_]+)\s*\(", hdr))
    assert declared == set(msm.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("p,M", [(4, 4), (6, 6), (8, 8), (4, 1)])
def test_constants_match_oracle(p, M):
    pl = msm.Plan((10.0, 10.0, 10.0), 0, p, 1.0, 3.0, 2, msm.MSM_FP64, 1, M, device=False)
    d = pl.describe()
    om = [float(w) for w in C.omega_prime(p, M)]
    np.testing.assert_allclose(d["omega"], om, rtol=1e-14, atol=1e-15)
    J = [2.0 ** (1 - p) * math.comb(p, k) for k in range(p + 1)]
    assert d["J"] == J
    # softening polynomial in t against the oracle's gamma
    for rho in np.linspace(0, 0.999, 17):
        t = rho * rho
        g = sum(c * t ** k for k, c in enumerate(d["gamma_t_coeffs"]))
        assert g == pytest.approx(O.gamma(p, rho), rel=1e-14, abs=1e-15)
    assert d["self_const"] == pytest.approx(O.gamma(p, 0.0) / 3.0, rel=1e-15)


@pytest.mark.parametrize("case", CASES)
def test_geometry_matches_oracle(case):
    box, per, p, h, a, L = case
    pl = msm.Plan(box, _mask(per), p, h, a, L, msm.MSM_FP64, 1, device=False)
    o = O.OracleMSM(box, per, p, h, a, L)
    d = pl.describe()
    for l in range(1, L + 1):
        info = d["levels_info"][l - 1]
        n, lo, hl = o.levels[l - 1]
        assert info["n"] == n and info["lo"] == lo
        np.testing.assert_allclose(info["h"], hl, rtol=1e-15)
        assert pl.grid_dims(l) == tuple(n)


@pytest.mark.parametrize("case", CASES)
def test_stencils_match_oracle(case):
    box, per, p, h, a, L = case
    pl = msm.Plan(box, _mask(per), p, h, a, L, msm.MSM_FP64, 1, device=False)
    o = O.OracleMSM(box, per, p, h, a, L)
    for l in range(1, L + 1):
        ln, off, K = pl.stencil(l)
        n = o.levels[l - 1][0]
        mine = _fold(off, K, o.periodic, n)
        ref = _oracle_stencil_folded(o, l)
        # free axes: the plan crops to |d| < n, the oracle to |d| <= n-1 as well
        scale = max(abs(v) for v in ref.values())
        keys = set(mine) | set(ref)
        err = max(abs(mine.get(k, 0.0) - ref.get(k, 0.0)) for k in keys)
        assert err <= 1e-12 * scale, (l, err, scale)


def test_parameter_errors():
    lib = msm.lib()
    h = ctypes.c_void_p()
    box = (ctypes.c_double * 3)(10, 10, 10)
    def create(**kw):
        args = dict(mask=0, p=4, h=1.0, a=3.0, L=2, prec=0, max_n=10, M=-1)
        args.update(kw)
        return lib.msm_plan_create_host(ctypes.byref(h), box, args["mask"], args["p"], args["h"],
                                        args["a"], args["L"], args["prec"], args["max_n"],
                                        args["M"])
    assert create() == 0
    lib.msm_plan_destroy(h)
    assert create(p=5) == 2            # odd order
    assert create(mask=8) == 1         # no such axis
    assert create(mask=7, a=6.0) == 3  # a > L/2
    assert create(h=-1.0) == 1
    assert create(L=0) == 1
    assert create(prec=3) == 1
    # host-only plans refuse compute calls
    assert create() == 0
    E = (ctypes.c_double * 1)()
    rc = lib.msm_energy_forces(h, 0, None, None, None, ctypes.cast(E, ctypes.c_void_p), None,
                               None, None)
    assert rc == 10
    assert lib.msm_plan_destroy(h) == 0


def test_workspace_and_batch_boundary_errors():
    """Host-side argument checks of the workspace query and the batched
    entry points (no GPU is touched: they fail before any device call)."""
    lib = msm.lib()
    h = ctypes.c_void_p()
    box = (ctypes.c_double * 3)(10, 10, 10)
    assert lib.msm_plan_create_host(ctypes.byref(h), box, 0, 4, 1.0, 3.0, 2, 0, 100, -1) == 0
    assert lib.msm_workspace_bytes(h, 100, 0) > 0
    assert lib.msm_workspace_bytes(h, 100, 1) == 0   # reserved flags
    assert lib.msm_workspace_bytes(h, -1, 0) == 0
    assert lib.msm_workspace_bytes(None, 100, 0) == 0
    lib.msm_plan_destroy(h)
    boxes = (ctypes.c_double * 6)(10, 10, 10, 12, 12, 12)
    levels = (ctypes.c_int * 2)(2, 2)
    args = (4, 1.0, 3.0, 0, 100, -1)
    assert lib.msm_batch_plan_create(ctypes.byref(h), 2, boxes, levels, 7, *args) == 2
    assert lib.msm_batch_plan_create(ctypes.byref(h), 2, boxes, levels, 3, *args) == 2
    oblong = (ctypes.c_double * 6)(10, 10, 10, 12, 12, 13)
    assert lib.msm_batch_plan_create(ctypes.byref(h), 2, oblong, levels, 0, *args) == 2
    bad = (ctypes.c_double * 6)(10, 10, 10, -1, -1, -1)
    assert lib.msm_batch_plan_create(ctypes.byref(h), 2, bad, levels, 0, *args) == 1
    assert lib.msm_batch_plan_create(ctypes.byref(h), 0, boxes, levels, 0, *args) == 1


def test_skin_cell_geometry():
    """msm_plan_set_skin on a host plan: cells of edge >= a + skin, never more
    cells per axis than before; argument errors."""
    plan = msm.Plan((30.0, 24.0, 17.0), 7, 4, 1.0, 4.0, 2, msm.MSM_FP32, 100, device=False)
    assert plan.describe()["cells"] == [7, 6, 4]
    plan.set_skin(1.0)
    d = plan.describe()
    assert d["skin"] == 1.0 and d["cells"] == [6, 4, 3]
    for k, L in enumerate((30.0, 24.0, 17.0)):
        assert L / d["cells"][k] >= 5.0
    plan.set_skin(0.0)
    assert plan.describe()["cells"] == [7, 6, 4]
    lib = msm.lib()
    assert lib.msm_plan_set_skin(plan._h, -0.5) == 1
    assert lib.msm_plan_set_skin(plan._h, float("nan")) == 1
    assert lib.msm_plan_set_skin(None, 1.0) == 1
