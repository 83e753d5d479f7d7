"""CPU pins of the oracle's adjoint through the charge gradient dE/dq = phi
(a cotangent w on phi, as in charge-equilibration losses; Sec. Fundamentals:
phi is one of the method's outputs).  The oracle takes the bilinear form
w^T G q apart by polarisation; these tests check the symmetry that rests on
and the cotangents against central differences of the full loss
L = gE E + sum v.F + sum w.phi.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05961_amd import workloads as WL

BOX = (9.0, 10.0, 8.5)
GEOMS = {"free": (0, 0, 0), "periodic": (1, 1, 1), "slab": (1, 1, 0)}
CELL = np.array([[9.0, 0.0, 0.0], [2.1, 8.5, 0.0], [-1.3, 1.7, 9.4]])


def _oracle(geom, p=4):
    if geom == "triclinic":
        return O.OracleMSM(None, None, p, 0.9, 3.5, 2, cell=CELL)
    return O.OracleMSM(BOX, GEOMS[geom], p, 0.9, 3.5, 2)


def _inputs(geom, n, seed):
    if geom == "triclinic":
        rng = np.random.default_rng(seed)
        pos = rng.random((n, 3)) @ CELL
        q = rng.normal(0.0, 0.5, n)
        q -= q.mean()
    else:
        pos, q = WL.gaussian_charges(n, BOX, 0.5, seed=seed)
    w = np.random.default_rng(seed + 1).normal(size=n)
    v = WL.force_cotangent(n, seed=seed + 2)
    return pos, q, w, v


@pytest.mark.parametrize("geom", list(GEOMS) + ["triclinic"])
def test_potential_matrix_is_symmetric(geom):
    """w . phi(q) = q . phi(w): the MSM potentials come from one symmetric
    matrix (stencils even in the offset, the same basis functions for
    anterpolation and interpolation, a constant self term)."""
    o = _oracle(geom, 6)
    pos, q, w, _ = _inputs(geom, 60, 5)
    a = float(np.dot(w, o.compute(pos, q)["phi"]))
    b = float(np.dot(q, o.compute(pos, w)["phi"]))
    assert a == pytest.approx(b, rel=1e-12)


@pytest.mark.parametrize("geom", list(GEOMS) + ["triclinic"])
def test_charge_cotangent_matches_finite_differences(geom):
    o = _oracle(geom)
    pos, q, w, v = _inputs(geom, 30, 7)
    gE = 0.4
    gq, gr = o.backward(pos, q, gE, v, w=w)

    def L(pp, qq):
        r = o.compute(pp, qq)
        return gE * r["E"] + float(np.sum(v * r["F"])) + float(np.dot(w, r["phi"]))

    eps = 1e-5
    for i in (0, 11, 29):
        qp, qm = q.copy(), q.copy()
        qp[i] += eps
        qm[i] -= eps
        assert (L(pos, qp) - L(pos, qm)) / (2 * eps) == pytest.approx(gq[i], rel=1e-6, abs=1e-8)
        for k in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, k] += eps
            pm[i, k] -= eps
            assert (L(pp, q) - L(pm, q)) / (2 * eps) == pytest.approx(gr[i, k], rel=1e-6,
                                                                      abs=1e-8)


@pytest.mark.parametrize("geom", list(GEOMS))
def test_sampled_charge_cotangent_equals_full(geom):
    o = O.OracleMSM(BOX, GEOMS[geom], 4, 0.9, 3.5, 2)
    pos, q, w, v = _inputs(geom, 200, 9)
    sel = np.array([0, 3, 77, 150, 199])
    gq, gr = o.backward(pos, q, 0.3, v, w=w)
    sq, sr = o.sampled_backward(pos, q, 0.3, v, sel, w=w)
    np.testing.assert_allclose(sq, gq[sel], rtol=0, atol=1e-12 * np.abs(gq).max())
    np.testing.assert_allclose(sr, gr[sel], rtol=0, atol=1e-12 * np.abs(gr).max())
