"""CPU pins of the oracle's triclinic cells (unit-cube transform, Sec. MSM core
algorithm, long-range part): each compares the oracle with something it does
not compute itself -- the tabulated rock-salt Madelung constant, lattice
identities of the Ewald sum, the orthorhombic path, finite differences, and
Euler's relation for a homogeneous energy.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05961_amd import workloads as WL

# a moderately skewed cell (rows a, b, c) and a unimodular change of basis
CELL = np.array([[9.0, 0.0, 0.0], [2.1, 8.5, 0.0], [-1.3, 1.7, 9.4]])
U = np.array([[1, 0, 0], [1, 1, 0], [0, -1, 1]])


def _madelung_ref():
    with open(__file__.replace("test_oracle_triclinic.py", "golden/nacl_madelung.txt")) as f:
        return float([l for l in f if not l.startswith("#")][0])


def _random_in_cell(cell, n, seed):
    rng = np.random.default_rng(seed)
    s = rng.random((n, 3))
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    rng.shuffle(q)
    return s @ np.asarray(cell), q


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


def test_ewald_cell_matches_box_for_a_diagonal_cell():
    box = (7.0, 8.0, 9.0)
    for x in ([1.1, -2.3, 0.7], [0.0, 0.0, 0.0], [3.4, 3.9, -4.4]):
        reg = not any(x)
        assert O.ewald_psi_cell(np.diag(box), x, reg=reg) == pytest.approx(
            O.ewald_psi(box, x, reg=reg), rel=1e-13, abs=1e-14)


def test_ewald_cell_alpha_and_basis_independence():
    """The lattice sum depends on the lattice only: the splitting parameter and
    the choice of basis vectors (H U, U unimodular) change nothing."""
    x = [1.1, -2.3, 0.7]
    ref = O.ewald_psi_cell(CELL, x)
    assert O.ewald_psi_cell(CELL, x, alpha=0.35) == pytest.approx(ref, rel=1e-12)
    assert O.ewald_psi_cell(CELL, x, alpha=0.95) == pytest.approx(ref, rel=1e-12)
    assert O.ewald_psi_cell(U @ CELL, x) == pytest.approx(ref, rel=1e-12)
    # a lattice vector added to x changes nothing either
    x2 = np.asarray(x) + CELL[1] - 2 * CELL[2]
    assert O.ewald_psi_cell(CELL, x2) == pytest.approx(ref, rel=1e-12)


def test_ewald_cell_nacl_primitive_madelung():
    """Rock salt in its 2-ion primitive (face-centred, triclinic) cell: the
    energy per ion pair is -M q^2 / d_min (Sec. Madelung constants)."""
    prim = np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])  # d_min = 1
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    q = np.array([1.0, -1.0])
    E = 0.5 * float(np.dot(q, O.ewald_potentials_cell(prim, pos, q)))
    assert -E == pytest.approx(_madelung_ref(), abs=5e-7)


def test_msm_diagonal_cell_equals_box():
    box = (12.0, 11.0, 13.0)
    pos, q = WL.random_ions(300, box, seed=21)
    a = O.OracleMSM(box, (1, 1, 1), 4, 1.0, 4.0, 2).compute(pos, q)
    b = O.OracleMSM(None, None, 4, 1.0, 4.0, 2, cell=np.diag(box)).compute(pos, q)
    assert b["E"] == pytest.approx(a["E"], rel=1e-12)
    assert _rel(b["F"], a["F"]) < 1e-12
    assert _rel(b["phi"], a["phi"]) < 1e-12


def _min_width(cell):
    return 1.0 / np.linalg.norm(np.linalg.inv(np.asarray(cell, dtype=float).T), axis=1).max()


@pytest.mark.parametrize("cell,bar", [(CELL, 3e-5), (U @ CELL, 3e-4)], ids=["H", "HU"])
def test_msm_cell_converges_to_ewald(cell, bar):
    """Both bases of the lattice (the second more skewed, so its cutoff, half
    its smallest width, is smaller): the MSM error against the exact
    triclinic Ewald result falls with p and with h."""
    pos, q = _random_in_cell(CELL, 60, seed=22)
    phie = O.ewald_potentials_cell(CELL, pos, q)
    a = min(3.5, _min_width(cell) / 2)
    e = []
    for p, h in ((4, 0.6), (6, 0.6), (6, 0.45)):
        r = O.OracleMSM(None, None, p, h, a, 2, cell=cell).compute(pos, q)
        e.append(_rel(r["phi"], phie))
    assert e[0] < 2e-3
    assert e[1] < e[0] and e[2] < e[1] and e[2] < bar


def test_msm_cell_nacl_primitive_supercell():
    """Rock salt in a 4 x 4 x 4 supercell of the primitive cell (cutoff half its
    smallest width): the MSM Madelung constant approaches the tabulated value
    as the grid refines."""
    prim = np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    k = 4
    pos, q = [], []
    for i in range(k):
        for j in range(k):
            for m in range(k):
                o = i * prim[0] + j * prim[1] + m * prim[2]
                pos += [o, o + np.array([1.0, 0.0, 0.0])]
                q += [1.0, -1.0]
    pos, q = np.array(pos) + 0.05, np.array(q)
    cell = k * prim
    errs = []
    for h in (0.5, 0.35):
        E = O.OracleMSM(None, None, 6, h, _min_width(cell) / 2, 2, cell=cell).compute(pos, q)["E"]
        errs.append(abs(-E / k ** 3 - _madelung_ref()))
    assert errs[1] < errs[0] and errs[1] < 5e-4


def test_cell_short_range_cell_list_equals_brute_force():
    pos, q = _random_in_cell(CELL, 900, seed=23)
    o = O.OracleMSM(None, None, 4, 1.0, 4.0, 2, cell=CELL)
    p1, F1 = o.short_range(pos, q, cells=False)
    p2, F2 = o.short_range(pos, q, cells=True)
    np.testing.assert_allclose(p2, p1, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(F2, F1, rtol=1e-12, atol=1e-12)
    # positions moved by lattice vectors are the same system
    p3, F3 = o.short_range(pos + 2 * CELL[0] - CELL[2], q, cells=False)
    np.testing.assert_allclose(p3, p1, rtol=1e-10, atol=1e-10)


def test_cell_forces_and_potentials_are_gradients():
    pos, q = _random_in_cell(CELL, 40, seed=24)
    o = O.OracleMSM(None, None, 4, 0.8, 3.5, 2, cell=CELL)
    r = o.compute(pos, q)
    eps = 1e-5
    for i in (0, 17, 39):
        for k in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, k] += eps
            pm[i, k] -= eps
            fd = -(o.compute(pp, q)["E"] - o.compute(pm, q)["E"]) / (2 * eps)
            assert fd == pytest.approx(r["F"][i, k], rel=1e-6, abs=1e-8)
        qp, qm = q.copy(), q.copy()
        qp[i] += eps
        qm[i] -= eps
        fd = (o.compute(pos, qp)["E"] - o.compute(pos, qm)["E"]) / (2 * eps)
        assert fd == pytest.approx(r["phi"][i], rel=1e-6, abs=1e-8)


def test_cell_adjoint_matches_finite_differences():
    pos, q = _random_in_cell(CELL, 30, seed=25)
    v = WL.force_cotangent(30, seed=26)
    o = O.OracleMSM(None, None, 4, 0.8, 3.5, 2, cell=CELL)
    gq, gr = o.backward(pos, q, 0.7, v)

    def L(pp, qq):
        r = o.compute(pp, qq)
        return 0.7 * r["E"] + float(np.sum(v * r["F"]))
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


def test_cell_gradient_satisfies_euler_relation():
    """The Coulomb energy is homogeneous of degree -1 under r -> lambda r,
    H -> lambda H.  With fractional coordinates s fixed, dE/dH|_s =
    dE/dH|_r - sum_i F_i s_i^T, so sum_ab H_ab dE/dH_ab|_s = -E for the exact
    (Ewald) energy and, within the MSM error, for the MSM one."""
    pos, q = _random_in_cell(CELL, 40, seed=27)
    o = O.OracleMSM(None, None, 4, 0.5, 3.5, 2, cell=CELL)
    r = o.compute(pos, q)
    dEdH = o.cell_gradient(pos, q)
    s = (np.linalg.inv(o.H) @ pos.T).T
    dEdH_s = dEdH - np.einsum("ia,ib->ab", r["F"], s)
    euler = float(np.sum(o.H * dEdH_s))
    assert euler == pytest.approx(-r["E"], rel=5e-4)
