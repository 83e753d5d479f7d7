"""Pins of the oracle's Ewald sums with one periodic axis (and with two
periodic axes in any orientation), and of its MSM with those top levels.

The 1-D sum (one periodic axis of length L, two free axes) is pinned by:
  * alpha-independence (the split parameter cancels, for any charges);
  * the alpha -> infinity form, a library Bessel-function series away from
    the axis: psi = -(2/L) ln(rho/L) + (4/L) sum_m cos(k_m z) K0(k_m rho),
    which also fixes the constant kept for non-neutral lines;
  * brute-force image sums with the logarithm of the line taken out:
    sum_{|n|<=N} 1/|x + n L e| - (2/L)(ln 2N + 1/(2N)) -> psi(x) as N grows,
    at points on and near the axis where the Bessel series does not reach;
  * the regular part at a lattice point, (2/L)(gamma_E - ln 2).
The MSM with one periodic axis converges to these potentials as p and h
are refined, and relabelling the axes of a system relabels its result.
"""
import math

import numpy as np
import pytest
from scipy.special import k0

from oracle import oracle as O
from paper_2510_05961_amd import workloads as WL

L = 3.7
BOX = (10.0, 11.0, L)
LINE_Z = (False, False, True)


def _bessel_series(x):
    rho, z = math.hypot(x[0], x[1]), x[2]
    s = -2.0 / L * math.log(rho / L)
    m = 1
    while 2 * math.pi * m / L * rho < 700.0:
        k = 2 * math.pi * m / L
        s += 4.0 / L * math.cos(k * z) * k0(k * rho)
        m += 1
    return s


def _brute(x, N):
    n = np.arange(-N, N + 1, dtype=np.float64)
    r = np.sqrt(x[0] ** 2 + x[1] ** 2 + (x[2] + n * L) ** 2)
    r = r[r > 0]
    return float(np.sum(1.0 / r)) - 2.0 / L * (math.log(2 * N) + 1.0 / (2 * N))


POINTS = [(1.5, 0.7, 0.4), (3.0, -2.0, 0.3), (-4.0, 6.5, 2.9), (0.2, 0.1, 1.9),
          (0.0, 0.0, 1.2), (1e-3, 0.0, -0.5)]


@pytest.mark.parametrize("x", POINTS)
def test_line_sum_alpha_independent(x):
    vals = [O.ewald_psi(BOX, x, alpha=s / L, periodic=LINE_Z) for s in (0.6, 1.0, 1.7, 2.8)]
    assert max(vals) - min(vals) <= 2e-15 * max(1.0, abs(vals[0]))


@pytest.mark.parametrize("x", [p for p in POINTS if math.hypot(p[0], p[1]) > L / 4])
def test_line_sum_equals_bessel_series(x):
    assert O.ewald_psi(BOX, x, periodic=LINE_Z) == pytest.approx(_bessel_series(x), abs=2e-15)


@pytest.mark.parametrize("x", POINTS)
def test_line_sum_equals_brute_force_images(x):
    # the residual of the truncated sum falls as 1/N^2: Richardson on N, 2N
    b1, b2 = _brute(x, 100_000), _brute(x, 200_000)
    assert O.ewald_psi(BOX, x, periodic=LINE_Z) == pytest.approx((4 * b2 - b1) / 3, abs=1e-13)


def test_line_sum_regular_part_at_lattice_point():
    reg = O.ewald_psi(BOX, (0.0, 0.0, 0.0), periodic=LINE_Z, reg=True)
    assert reg == pytest.approx(2.0 / L * (np.euler_gamma - math.log(2.0)), abs=1e-15)
    assert O.ewald_psi(BOX, (0.0, 0.0, 2 * L), periodic=LINE_Z, reg=True) == pytest.approx(reg, abs=1e-15)


def test_line_and_slab_sums_follow_the_axes():
    x = np.array([0.9, -1.3, 0.4])
    box = np.array([6.0, 7.0, 8.0])
    for perm in ((2, 0, 1), (1, 2, 0), (0, 2, 1)):
        perm = list(perm)
        for per in ((0, 0, 1), (1, 1, 0)):
            a = O.ewald_psi(box, x, periodic=per)
            pper = [per[k] for k in perm]
            b = O.ewald_psi(box[perm], x[perm], periodic=pper)
            assert a == pytest.approx(b, abs=1e-15), (perm, per)


def test_neutral_line_energy_independent_of_convention():
    # the constant kept in the logarithm refers to the period; a neutral
    # system does not see it, so a period of 2L holding two copies has twice
    # the energy of one copy with period L
    pos, q = WL.random_ions(24, BOX, seed=31)
    E1 = 0.5 * np.dot(q, O.ewald_potentials(BOX, pos, q, periodic=LINE_Z))
    box2 = (BOX[0], BOX[1], 2 * L)
    pos2 = np.concatenate([pos, pos + np.array([0.0, 0.0, L])])
    q2 = np.concatenate([q, q])
    E2 = 0.5 * np.dot(q2, O.ewald_potentials(box2, pos2, q2, periodic=LINE_Z))
    assert E2 == pytest.approx(2 * E1, rel=1e-12)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("per", [(0, 0, 1), (0, 1, 1)])
def test_msm_converges_to_line_and_slab_ewald(per):
    box = (8.0, 8.0, 7.2)
    pos, q = WL.random_ions(50, box, seed=16)
    phie = O.ewald_potentials(box, pos, q, periodic=per)
    e = []
    for p, h in ((4, 0.5), (6, 0.5), (6, 0.25)):
        r = O.OracleMSM(box, per, p, h, 3.5, 3).compute(pos, q)
        e.append(_rel(r["phi"], phie))
    assert e[0] < 1e-3 and e[1] < e[0] and e[2] < e[1] and e[2] < 2e-6


@pytest.mark.parametrize("per,perm", [((1, 0, 0), (2, 0, 1)), ((1, 0, 1), (0, 2, 1))])
def test_msm_relabelled_axes(per, perm):
    # the system with its axes permuted, periodic flags permuted alike
    box = np.array([7.5, 8.0, 9.0])
    pos, q = WL.random_ions(40, box, seed=32)
    perm = list(perm)
    r1 = O.OracleMSM(tuple(box), per, 4, 0.6, 3.0, 3).compute(pos, q)
    r2 = O.OracleMSM(tuple(box[perm]), [per[k] for k in perm], 4, 0.6, 3.0, 3).compute(
        np.ascontiguousarray(pos[:, perm]), q)
    assert r2["E"] == pytest.approx(r1["E"], rel=1e-12)
    np.testing.assert_allclose(r2["F"], r1["F"][:, perm], rtol=0, atol=1e-11 * np.abs(r1["F"]).max())
