"""CPU pins of the oracle's MSM for the dispersion kernel k(r) = r^-6, the
paper's splitting applied to another power (Sec. Splitting for Coulomb
kernels; the package's core is meant to take other kernels): the softener's
contact with r^-6, the telescoping split, the MSM against the exact
all-pairs sum (free space); the Ewald sums of r^-6 over three, two or one
periodic axes against brute-force lattice sums, and the periodic MSM
against them."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2510_05961_amd import workloads as WL

NU = 6


@pytest.mark.parametrize("p", [4, 6, 8])
def test_softener_meets_r6_smoothly(p):
    for rho in (1.0, 1.3, 2.0):
        assert O.gamma_nu(NU, p, rho) == pytest.approx(rho ** -NU, rel=1e-14)
    # gamma and its first two derivatives are continuous at rho = 1
    e = 1e-7
    for d in range(3):
        assert O.gamma_nu(NU, p, 1 - e, d) == pytest.approx(O.gamma_nu(NU, p, 1 + e, d),
                                                            rel=1e-5, abs=1e-5)
    # and the Taylor polynomial of s^-3 reproduces its first p derivatives in s
    # at s = 1: the value at rho^2 = 1 - t differs by O(t^p)
    for t in (0.02, 0.01):
        s = 1.0 - t
        err = abs(O.gamma_nu(NU, p, np.sqrt(s)) - s ** -3)
        assert err < 40.0 ** p * t ** p


@pytest.mark.parametrize("p", [4, 6])
def test_split_telescopes_to_r6(p):
    a, L = 2.5, 4
    for r in (0.3, 1.0, 2.4, 2.6, 7.0, 19.0, 45.0):
        total = sum(O.kernel(l, L, a, p, r, NU) for l in range(L + 1))
        assert total == pytest.approx(r ** -NU, rel=1e-12)
        for l in range(1, L):
            if r >= 2 ** l * a:
                assert O.kernel(l, L, a, p, r, NU) == 0.0


def _system(n, L, seed):
    pos, _ = WL.spaced_charges(n, L, False, seed=seed)
    c = np.random.default_rng(seed + 1).uniform(0.5, 1.5, n)  # dispersion coefficients
    return pos, c


def test_msm_r6_converges_to_the_direct_sum():
    """The error falls with h and with p.  The softened r^-6 is stiffer than the
    softened 1/r (the Taylor coefficients of s^-3 grow fast), so the orders
    only pay once a/h is about 8 or more."""
    pos, c = _system(200, 10.0, 3)
    phi_x, F_x = O.direct_sum(pos, c, NU)
    errs = []
    for p, h in ((4, 0.5), (4, 0.35), (6, 0.35), (8, 0.35)):
        r = O.OracleMSM((10.0,) * 3, (0, 0, 0), p, h, 3.0, 3, nu=NU).compute(pos, c)
        errs.append(np.linalg.norm(r["F"] - F_x) / np.linalg.norm(F_x))
        ephi = np.linalg.norm(r["phi"] - phi_x) / np.linalg.norm(phi_x)
        assert ephi < errs[-1]
    assert errs[0] > errs[1] > errs[2] > errs[3] and errs[0] < 2e-4 and errs[3] < 1e-5, errs


def test_msm_r6_derivatives():
    pos, c = _system(40, 9.0, 5)
    o = O.OracleMSM((9.0,) * 3, (0, 0, 0), 4, 0.7, 2.5, 2, nu=NU)
    r = o.compute(pos, c)
    eps = 1e-6
    for i, k in ((0, 0), (13, 1), (39, 2)):
        pp, pm = pos.copy(), pos.copy()
        pp[i, k] += eps
        pm[i, k] -= eps
        fd = -(o.compute(pp, c)["E"] - o.compute(pm, c)["E"]) / (2 * eps)
        assert r["F"][i, k] == pytest.approx(fd, rel=1e-6, abs=1e-9)
        cp, cm = c.copy(), c.copy()
        cp[i] += eps
        cm[i] -= eps
        fdq = (o.compute(pos, cp)["E"] - o.compute(pos, cm)["E"]) / (2 * eps)
        assert r["phi"][i] == pytest.approx(fdq, rel=1e-7, abs=1e-10)
    v = WL.force_cotangent(len(c), seed=6)
    gq, gr = o.backward(pos, c, 0.5, v)

    def Lf(pp, cc):
        rr = o.compute(pp, cc)
        return 0.5 * rr["E"] + float(np.sum(v * rr["F"]))
    for i in (3, 20):
        pp, pm = pos.copy(), pos.copy()
        pp[i, 1] += eps
        pm[i, 1] -= eps
        assert gr[i, 1] == pytest.approx((Lf(pp, c) - Lf(pm, c)) / (2 * eps), rel=1e-5,
                                         abs=1e-8)
        cp, cm = c.copy(), c.copy()
        cp[i] += eps
        cm[i] -= eps
        assert gq[i] == pytest.approx((Lf(pos, cp) - Lf(pos, cm)) / (2 * eps), rel=1e-5,
                                      abs=1e-8)


def test_msm_r6_sampled_equals_full():
    pos, c = _system(200, 10.0, 7)
    o = O.OracleMSM((10.0,) * 3, (0, 0, 0), 6, 0.8, 2.5, 3, nu=NU)
    full = o.compute(pos, c)
    sel = np.array([0, 5, 77, 199])
    phi, F = o.sampled(pos, c, sel)
    np.testing.assert_allclose(phi, full["phi"][sel], rtol=1e-12)
    np.testing.assert_allclose(F, full["F"][sel], rtol=1e-12, atol=1e-14)


CELL = np.array([[8.0, 0.0, 0.0], [1.5, 8.2, 0.0], [-1.0, 0.8, 8.4]])  # rows a, b, c


def _cell_brute(cell, x, Ns=(16, 32, 64)):
    """sum over |n_k| <= N of |x + H n|^-6, extrapolated in M = N + 1/2 as for
    the orthorhombic blocks (a parallelepiped block is centrally symmetric)."""
    H = np.asarray(cell, dtype=np.float64).T
    T = []
    for N in Ns:
        r = np.arange(-N, N + 1, dtype=np.float64)
        n = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
        d = n @ H.T + np.asarray(x, dtype=np.float64)
        r2 = np.einsum("ij,ij->i", d, d)
        T.append(float(np.sum(r2 ** -3)))
    A = np.array([[1.0, (N + 0.5) ** -3, (N + 0.5) ** -5] for N in Ns])
    return float(np.linalg.solve(A, T)[0])


def test_r6_cell_lattice_sum():
    x = (0.3, -0.7, 1.1)
    # a diagonal cell is the orthorhombic box
    box = (3.0, 3.5, 4.0)
    assert O.ewald_psi_cell_r6(np.diag(box), x) == pytest.approx(O.ewald_psi_r6(box, x),
                                                                   rel=1e-13)
    vals = [O.ewald_psi_cell_r6(CELL, x, alpha=a) for a in (0.3, 0.5, 0.8)]
    assert max(vals) - min(vals) <= 1e-13 * abs(vals[0])
    # another basis of the same lattice, and the brute-force sum
    cell2 = CELL.copy()
    cell2[1] = CELL[1] + CELL[0]
    cell2[2] = CELL[2] - CELL[1]
    assert O.ewald_psi_cell_r6(cell2, x) == pytest.approx(vals[0], rel=1e-13)
    assert vals[0] == pytest.approx(_cell_brute(CELL, x), rel=1e-10)


def test_msm_r6_triclinic_converges_to_ewald():
    pos, _ = WL.spaced_charges(60, 1.0, True, seed=23)
    pos = pos @ CELL  # spaced fractional positions into the cell
    c = np.random.default_rng(24).uniform(0.5, 1.5, 60)
    phie = O.ewald_potentials_cell_r6(CELL, pos, c)
    errs = []
    for p, h in ((4, 0.5), (6, 0.5), (6, 0.4)):
        r = O.OracleMSM(None, (1, 1, 1), p, h, 3.5, 3, cell=CELL, nu=NU).compute(pos, c)
        errs.append(np.linalg.norm(r["phi"] - phie) / np.linalg.norm(phie))
    assert errs[0] < 5e-5 and errs[0] > errs[1] > errs[2], errs


def test_msm_r6_cell_gradient():
    """dE/dH of the r^-6 MSM energy (central differences in H, grid counts
    held): the energy is homogeneous of degree -6 under r -> lambda r,
    H -> lambda H, so sum_ab H_ab dE/dH_ab at fixed fractional coordinates
    is -6 E for the exact lattice sum and, within the MSM error, for the MSM
    one; and the whole 3x3 derivative approaches that of the exact sum
    (the Ewald energy differentiated in H) as the order rises."""
    n = 40
    pos, _ = WL.spaced_charges(n, 1.0, True, seed=23)
    pos = pos @ CELL
    c = np.random.default_rng(24).uniform(0.5, 1.5, n)

    def exact_energy(H):
        return 0.5 * float(c @ O.ewald_potentials_cell_r6(H.T, pos, c))

    errs = []
    for p in (4, 6):
        o = O.OracleMSM(None, (1, 1, 1), p, 0.5, 3.5, 3, cell=CELL, nu=NU)
        r = o.compute(pos, c)
        G = o.cell_gradient(pos, c)
        s = (np.linalg.inv(o.H) @ pos.T).T
        G_s = G - np.einsum("ia,ib->ab", r["F"], s)
        assert float(np.sum(o.H * G_s)) == pytest.approx(-NU * r["E"], rel=1e-4)
        if p == 4:
            eps = 1e-5 * float(np.abs(o.H).max())
            Gx = np.zeros((3, 3))
            for a in range(3):
                for b in range(3):
                    Hp, Hm = o.H.copy(), o.H.copy()
                    Hp[a, b] += eps
                    Hm[a, b] -= eps
                    Gx[a, b] = (exact_energy(Hp) - exact_energy(Hm)) / (2 * eps)
        errs.append(np.linalg.norm(G - Gx) / np.linalg.norm(Gx))
    assert errs[0] < 5e-4 and errs[1] < errs[0], errs


# --------------------------------------------------------------------------
# periodic r^-6: the 3-D Ewald sum of the dispersion kernel and the MSM on it
# --------------------------------------------------------------------------
def _lattice_brute(box, x, reg, periodic=(1, 1, 1), Ns=None):
    """sum over |n_k| <= N (periodic axes k) of |x + n o box|^-6 at three N,
    extrapolated in the half-width M = N + 1/2 of the summed block: with d
    periodic axes the missing tail is c/M^(6-d) + c'/M^(8-d) + ... (the sum
    over a block's complement against its integral, symmetric in the shift x)."""
    box = np.asarray(box, dtype=np.float64)
    axes = [k for k in range(3) if periodic[k]]
    d = len(axes)
    if Ns is None:
        Ns = {3: (16, 32, 64), 2: (200, 400, 800), 1: (2000, 4000, 8000)}[d]
    T = []
    for N in Ns:
        r = np.arange(-N, N + 1, dtype=np.float64)
        grids = np.meshgrid(*[r * box[k] for k in axes], indexing="ij")
        comp = [np.full(grids[0].shape, float(x[k])) for k in range(3)]
        for g, k in zip(grids, axes):
            comp[k] = comp[k] + g
        r2 = comp[0] ** 2 + comp[1] ** 2 + comp[2] ** 2
        if reg:
            r2 = r2[r2 > 0]
        T.append(float(np.sum(r2 ** -3)))
    A = np.array([[1.0, (N + 0.5) ** -(6 - d), (N + 0.5) ** -(8 - d)] for N in Ns])
    return float(np.linalg.solve(A, T)[0])


R6_POINTS = [((3.0, 3.5, 4.0), (0.3, -0.7, 1.1), False), ((3.0, 3.5, 4.0), (1.4, 1.6, 1.9), False),
             ((4.0, 4.0, 5.0), (0.0, 0.0, 0.0), True), ((1.0, 1.0, 1.0), (0.0, 0.0, 0.0), True)]


@pytest.mark.parametrize("box,x,reg", R6_POINTS)
def test_r6_lattice_sum_alpha_independent(box, x, reg):
    # (a large alpha makes the sum a difference of terms of order alpha^6 / 6
    # and alpha^3 / V: the bound allows that rounding)
    vals = [O.ewald_psi_r6(box, x, alpha=a, reg=reg) for a in (0.2, 0.3, 0.5, 0.8)]
    assert max(vals) - min(vals) <= 1e-12 * abs(vals[0])


@pytest.mark.parametrize("box,x,reg", R6_POINTS)
def test_r6_lattice_sum_equals_brute_force(box, x, reg):
    # absolutely convergent: the Ewald value is the plain lattice sum (for the
    # unit cube at 0, the simple cubic lattice's sum of |n|^-6 over n != 0)
    assert O.ewald_psi_r6(box, x, reg=reg) == pytest.approx(_lattice_brute(box, x, reg),
                                                              rel=1e-10)


R6_AXES = [((1, 1, 0), (0.3, -0.7, 1.1), False), ((1, 1, 0), (0.0, 0.0, 0.0), True),
           ((1, 0, 1), (1.4, 1.6, 1.9), False), ((0, 0, 1), (0.3, -0.7, 1.1), False),
           ((0, 0, 1), (0.0, 0.0, 0.0), True), ((0, 1, 0), (0.2, 0.1, 0.0), False)]


@pytest.mark.parametrize("per,x,reg", R6_AXES)
def test_r6_slab_and_line_sums(per, x, reg):
    """Two periodic axes or one: alpha-independence and brute-force lattice
    sums, as for three."""
    box = (3.0, 3.5, 4.0)
    vals = [O.ewald_psi_r6(box, x, alpha=a, reg=reg, periodic=per) for a in (0.3, 0.5, 0.8)]
    assert max(vals) - min(vals) <= 1e-12 * abs(vals[0])
    assert vals[0] == pytest.approx(_lattice_brute(box, x, reg, per), rel=1e-12)


def test_r6_lattice_sum_sublattices():
    # the lattice of box is the union of the 8 shifted lattices of 2 box
    box = np.array([3.0, 3.5, 4.0])
    x = np.array([0.3, -0.7, 1.1])
    whole = O.ewald_psi_r6(box, x)
    parts = sum(O.ewald_psi_r6(2 * box, x + box * np.array(s))
                for s in np.ndindex(2, 2, 2))
    assert parts == pytest.approx(whole, rel=1e-13)


def _periodic_system(n, L, seed):
    pos, _ = WL.spaced_charges(n, L, True, seed=seed)
    c = np.random.default_rng(seed + 1).uniform(0.5, 1.5, n)
    return pos, c


@pytest.mark.parametrize("per", [(1, 1, 1), (1, 1, 0), (0, 0, 1)])
def test_msm_r6_periodic_converges_to_ewald(per):
    box = (8.0, 8.0, 8.0)
    pos, c = _periodic_system(60, 8.0, 5)
    phie = O.ewald_potentials_r6(box, pos, c, periodic=per)
    errs = []
    for p, h in ((4, 0.5), (6, 0.5), (6, 0.4)):
        r = O.OracleMSM(box, per, p, h, 4.0, 3, nu=NU).compute(pos, c)
        errs.append(np.linalg.norm(r["phi"] - phie) / np.linalg.norm(phie))
        assert abs(r["E"] - 0.5 * c @ phie) <= 3 * errs[-1] * abs(0.5 * c @ phie)
    assert errs[0] < 2e-5 and errs[0] > errs[1] > errs[2] and errs[2] < 2e-6, errs


def test_msm_r6_periodic_derivatives():
    box = (7.0, 7.0, 7.0)
    pos, c = _periodic_system(30, 7.0, 9)
    o = O.OracleMSM(box, (1, 1, 1), 4, 0.45, 3.5, 2, nu=NU)
    r = o.compute(pos, c)
    eps = 1e-5
    for i in (0, 13, 29):
        for k in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, k] += eps
            pm[i, k] -= eps
            dE = (o.compute(pp, c)["E"] - o.compute(pm, c)["E"]) / (2 * eps)
            assert -dE == pytest.approx(r["F"][i, k], rel=1e-5, abs=1e-7)
        cp, cm = c.copy(), c.copy()
        cp[i] += eps
        cm[i] -= eps
        dq = (o.compute(pos, cp)["E"] - o.compute(pos, cm)["E"]) / (2 * eps)
        assert dq == pytest.approx(r["phi"][i], rel=1e-6)
