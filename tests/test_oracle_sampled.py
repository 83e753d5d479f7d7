"""Pins of the oracle's sampled paths, which the full-size parity tests use.

OracleMSM.sampled() evaluates phi_i and F_i only for listed particles: the
short range by a selection branch, the level potentials only at the grid
points the listed particles touch (support_points() plus the point-list
branch of the stencil convolution).  sampled_backward() does the same for
the adjoint.  Each must equal the full evaluation at the listed rows; the
listed particles include ones within h of every periodic face, ones given
outside a periodic box (wrapped), and ones exactly on the faces of a free
axis, so an index that fails to wrap, or a swapped selection index, fails
here.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05961_amd import workloads as WL

BOX = (11.0, 10.0, 12.0)
GEOMS = {"free": (0, 0, 0), "periodic": (1, 1, 1), "slab": (1, 1, 0)}


def _case(periodic, seed):
    pos, q = WL.gaussian_charges(300, BOX, 0.5, seed=seed)
    h = 0.8
    special = [
        (0, 0, 0.05), (1, 0, BOX[0] - 0.03), (2, 1, 0.1), (3, 1, BOX[1] - 0.2),
        (4, 2, 0.0), (5, 2, BOX[2]), (6, 0, 0.0), (7, 1, BOX[1]),
    ]
    for i, k, x in special:
        pos[i, k] = x
    pos[8] = (0.02, BOX[1] - 0.01, 0.03)          # a corner
    pos[9] = (BOX[0] - 0.5 * h, 0.5 * h, BOX[2] - 0.5 * h)
    if periodic[0]:
        pos[10, 0] = -0.3                          # outside a periodic box
        pos[11, 1] = BOX[1] + 0.4
    sel = np.array([0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 57, 123, 299])
    return pos, q, sel, h


def _close(a, b, rel=1e-13):
    a, b = np.asarray(a), np.asarray(b)
    scale = max(np.abs(b).max(), 1e-300)
    assert np.abs(a - b).max() <= rel * scale, (np.abs(a - b).max(), scale)


@pytest.mark.parametrize("p", [4, 6, 8])
@pytest.mark.parametrize("geom", list(GEOMS))
def test_sampled_equals_full_evaluation(geom, p):
    per = GEOMS[geom]
    pos, q, sel, h = _case(per, seed=60 + p)
    o = O.OracleMSM(BOX, per, p, h, 4.5, 3)
    full = o.compute(pos, q)
    phi, F = o.sampled(pos, q, sel)
    _close(phi, full["phi"][sel])
    _close(F, full["F"][sel])
    # the support points are exactly the grid points with a non-zero basis
    # value at the particle (brute force over the whole grid)
    for l in range(1, o.L + 1):
        for i in (0, 1, 5, 8, 10):
            pts = set(o.support_points(l, pos[i:i + 1]).tolist())
            g = o.grid_charge(l, pos[i:i + 1], np.ones(1))
            nz = set(np.flatnonzero(np.abs(g) > 0).tolist())
            assert nz <= pts, (l, i)
            assert len(pts) <= p ** 3


@pytest.mark.parametrize("p", [4, 6])
@pytest.mark.parametrize("geom", list(GEOMS))
def test_sampled_backward_equals_full_backward(geom, p):
    per = GEOMS[geom]
    pos, q, sel, h = _case(per, seed=70 + p)
    o = O.OracleMSM(BOX, per, p, h, 4.5, 3)
    v = WL.force_cotangent(len(q), seed=71)
    gq, gr = o.backward(pos, q, 0.7, v)
    sq, sr = o.sampled_backward(pos, q, 0.7, v, sel)
    _close(sq, gq[sel])
    _close(sr, gr[sel])


@pytest.mark.parametrize("periodic", [(0, 0, 0), (1, 1, 1), (1, 1, 0)])
def test_short_range_vjp_cell_list_equals_brute_force(periodic):
    box = (21.0, 19.0, 23.0)
    o = O.OracleMSM(box, periodic, 4, 1.0, 6.5, 2)
    pos, q = WL.random_ions(1500, box, seed=11)
    v = WL.force_cotangent(1500, seed=3)
    a_q, a_r = o.short_range_vjp(pos, q, v, cells=False)
    b_q, b_r = o.short_range_vjp(pos, q, v, cells=True)
    _close(b_q, a_q, 1e-12)
    _close(b_r, a_r, 1e-12)
    sel = np.array([0, 3, 700, 1499])
    c_q, c_r = o.short_range_vjp(pos, q, v, sel=sel)
    _close(c_q, a_q[sel], 1e-13)
    _close(c_r, a_r[sel], 1e-13)


@pytest.mark.parametrize("periodic", [(0, 0, 0), (1, 1, 1), (1, 1, 0)])
def test_short_range_selected_cell_list_equals_brute_force(periodic):
    """The cell-list short range for listed particles (as the sampled
    parity and the CPU baseline use it) against the brute-force pair loop,
    with particles near every face of the box among the listed ones."""
    box = (21.0, 19.0, 23.0)
    o = O.OracleMSM(box, periodic, 4, 1.0, 6.5, 2)
    pos, q = WL.random_ions(1500, box, seed=12)
    near = np.flatnonzero(np.any((pos < 0.7) | (pos > np.array(box) - 0.7), axis=1))[:20]
    sel = np.concatenate([near, [0, 3, 700, 1499]]).astype(np.int64)
    a_phi, a_F = o.short_range(pos, q, cells=False)
    b_phi, b_F = o.short_range(pos, q, sel=sel, cells=True)
    c_phi, c_F = o.short_range(pos, q, sel=sel, cells=False)
    _close(b_phi, a_phi[sel], 1e-12)
    _close(b_F, a_F[sel], 1e-12)
    _close(c_phi, a_phi[sel], 1e-13)
    _close(c_F, a_F[sel], 1e-13)
