"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each checks it against an
independent fact (a closed form, an identity, a second derivation, brute
force, a textbook method, or an invariance), chosen so that a dropped term, a
wrong sign or index, or a transposed operand fails one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import constants as C
from oracle import oracle as O
from paper_2510_05961_amd import workloads as WL


# --------------------------------------------------------------------------
# softening function (Sec. "Splitting for Coulomb kernels")
# --------------------------------------------------------------------------
@pytest.mark.parametrize("p", [4, 6, 8])
def test_gamma_value_at_zero_closed_form(p):
    # gamma(0) = sum_{k<p} C(2k,k)/4^k = 2p C(2p,p) / 4^p (partial sums of the
    # central binomial series), e.g. 35/16 for p = 4.
    expect = 2 * p * math.comb(2 * p, p) / 4 ** p
    assert O.gamma(p, 0.0) == pytest.approx(expect, rel=1e-15)
    if p == 4:
        assert O.gamma(4, 0.0) == pytest.approx(35 / 16, rel=1e-15)


@pytest.mark.parametrize("p", [4, 6, 8])
def test_gamma_matches_inverse_to_order_p(p):
    # gamma = 1/rho for rho >= 1, and the Taylor construction makes
    # gamma(1-eps) - 1/(1-eps) = O(eps^p): halving eps divides by ~2^p.
    for rho in (1.0, 1.5, 3.0):
        assert O.gamma(p, rho) == pytest.approx(1 / rho, rel=1e-15)
    d = [abs(O.gamma(p, 1 - e) - 1 / (1 - e)) for e in (2e-2, 1e-2)]
    assert d[0] / d[1] == pytest.approx(2 ** p, rel=0.1)
    # and not of order p+1 or p-1 (the degree is exactly p-1 in s)
    assert not (d[0] / d[1] == pytest.approx(2 ** (p + 1), rel=0.1))


def test_kernel_splitting_sums_to_coulomb():
    # eq. (kernel_splitting): sum_{l=0..L} k_l(r) = 1/r, each k_l (l < L) has
    # range 2^l a, and k_1..k_L are finite at 0 with sum gamma(0)/a.
    a, p, L = 1.7, 6, 4
    for r in (0.3, 1.0, 2.9, 7.0, 30.0):
        s = sum(O.kernel(l, L, a, p, r) for l in range(L + 1))
        assert s == pytest.approx(1 / r, rel=1e-13)
    for l in range(L):
        assert O.kernel(l, L, a, p, 2 ** l * a * 1.0000001) == pytest.approx(0.0, abs=1e-12)
    s0 = sum(O.kernel(l, L, a, p, 0.0) for l in range(1, L + 1))
    assert s0 == pytest.approx(O.gamma(p, 0.0) / a, rel=1e-14)


# --------------------------------------------------------------------------
# B-splines (Sec. "B-spline interpolation")
# --------------------------------------------------------------------------
def _cubic_textbook(t):
    t = abs(t)
    if t < 1:
        return 2 / 3 - t * t + t ** 3 / 2
    if t < 2:
        return (2 - t) ** 3 / 6
    return 0.0


def test_cubic_bspline_textbook_form():
    for t in np.linspace(-2.5, 2.5, 101):
        assert O.bspline(4, t) == pytest.approx(_cubic_textbook(t), abs=1e-15)


@pytest.mark.parametrize("p", [4, 6, 8])
def test_bspline_partition_of_unity_symmetry_derivatives(p):
    rng = np.random.default_rng(0)
    for x in rng.uniform(-3, 3, 20):
        s = sum(O.bspline(p, x - m) for m in range(-p - 4, p + 5))
        assert s == pytest.approx(1.0, abs=1e-14)
        # derivative of the partition of unity vanishes
        sd = sum(O.bspline(p, x - m, 1) for m in range(-p - 4, p + 5))
        assert sd == pytest.approx(0.0, abs=1e-13)
        assert O.bspline(p, x) == pytest.approx(O.bspline(p, -x), abs=1e-15)
        e = 1e-6
        fd1 = (O.bspline(p, x + e) - O.bspline(p, x - e)) / (2 * e)
        assert O.bspline(p, x, 1) == pytest.approx(fd1, abs=1e-8)
        fd2 = (O.bspline(p, x + e, 1) - O.bspline(p, x - e, 1)) / (2 * e)
        assert O.bspline(p, x, 2) == pytest.approx(fd2, abs=1e-7)
    # unit integral, support (-p/2, p/2)
    t = np.linspace(-p / 2, p / 2, 20001)
    v = np.array([O.bspline(p, x) for x in t])
    assert np.trapezoid(v, t) == pytest.approx(1.0, abs=1e-8)
    assert O.bspline(p, p / 2) == 0.0 and O.bspline(p, -p / 2) == 0.0


@pytest.mark.parametrize("p", [4, 6, 8])
def test_two_scale_relation(p):
    # Phi(x/2) = sum_n J_n Phi(x - n) with J_n = 2^(1-p) C(p, n + p/2) (the
    # restriction taps of eq. restriction_prolongation_explicit_formulas).
    J = {n: 2.0 ** (1 - p) * math.comb(p, n + p // 2) for n in range(-p // 2, p // 2 + 1)}
    assert sum(J.values()) == pytest.approx(2.0, abs=1e-15)
    for x in np.random.default_rng(1).uniform(-p, p, 25):
        rhs = sum(J[n] * O.bspline(p, x - n) for n in J)
        assert O.bspline(p, x / 2) == pytest.approx(rhs, abs=2e-16 * 8)


# --------------------------------------------------------------------------
# omega' (eq. kernel_stencil_by_conv_with_universal_coeff)
# --------------------------------------------------------------------------
def _omega_by_z_taylor(p, M):
    """Second derivation: Bhat(theta) as a polynomial in z = sin^2(theta/2)
    (cos(n theta) = T_n(1 - 2z)), power-series inverse of Bhat^2 to degree M,
    then z^k = 4^-k sum_j (-1)^j C(2k, k+j) e^{ij theta}."""
    b = C.bspline_integer_values(p)
    # polynomials in z as lists of Fractions
    def mul(u, v):
        out = [Fraction(0)] * (len(u) + len(v) - 1)
        for i, x in enumerate(u):
            for j, y in enumerate(v):
                out[i + j] += x * y
        return out
    x = [Fraction(1), Fraction(-2)]  # 1 - 2z
    T = [[Fraction(1)], x]
    for n in range(2, p):
        t2 = mul([Fraction(2) * c for c in x], T[-1])
        prev = T[-2] + [Fraction(0)] * (len(t2) - len(T[-2]))
        T.append([u - v for u, v in zip(t2, prev)])
    B = [Fraction(0)] * p
    for n, v in b.items():
        for i, c in enumerate(T[abs(n)]):
            B[i] += v * c
    B2 = mul(B, B) + [Fraction(0)] * (M + 2)
    inv = [Fraction(0)] * (M + 1)
    inv[0] = 1 / B2[0]
    for k in range(1, M + 1):
        inv[k] = -sum(B2[j] * inv[k - j] for j in range(1, k + 1)) / B2[0]
    return [sum(inv[k] * Fraction(1, 4 ** k) * (-1) ** j * math.comb(2 * k, k + j)
                for k in range(j, M + 1)) for j in range(M + 1)]


@pytest.mark.parametrize("p,M", [(4, 1), (4, 4), (6, 2), (6, 6), (8, 8)])
def test_omega_two_derivations_agree(p, M):
    assert C.omega_prime(p, M) == _omega_by_z_taylor(p, M)


def test_omega_known_values():
    # minimal order-4 quasi-interpolant and unit sum
    assert C.omega_prime(4, 1) == [Fraction(5, 3), Fraction(-1, 3)]
    for p, M in ((4, 4), (6, 6), (8, 8)):
        w = C.omega_prime(p, M)
        assert w[0] + 2 * sum(w[1:]) == 1


@pytest.mark.parametrize("p,M", [(4, 4), (6, 6)])
def test_double_interpolation_reproduces_polynomials(p, M):
    # sum_m sum_n Phi(x-m) [omega' * f](m-n) Phi(x'-n) = f(x-x') for
    # polynomials f of degree < p (interpolation in both arguments).
    om = [float(w) for w in C.omega_prime(p, M)]
    rng = np.random.default_rng(2)
    for deg in range(p):
        f = lambda d: d ** deg
        def K(j):
            return sum(om[abs(k)] * f(j - k) for k in range(-M, M + 1))
        for _ in range(3):
            x, xp = rng.uniform(-2, 2, 2)
            g = 0.0
            for m in range(math.floor(x) - p, math.floor(x) + p + 1):
                wm = O.bspline(p, x - m)
                if wm == 0:
                    continue
                for n in range(math.floor(xp) - p, math.floor(xp) + p + 1):
                    g += wm * K(m - n) * O.bspline(p, xp - n)
            assert g == pytest.approx(f(x - xp), abs=1e-9 * (1 + abs(f(x - xp))))


# --------------------------------------------------------------------------
# stencils and grid operators
# --------------------------------------------------------------------------
def test_stencil_level_scaling_and_symmetry():
    # Sec. "Splitting for Coulomb kernels": K^l = K^1 / 2^(l-1), l < L.
    o = O.OracleMSM((64.0, 64.0, 64.0), (1, 1, 1), 4, 1.0, 2.0, 4)
    W1, K1 = o.stencil(1)
    for l in (2, 3):
        Wl, Kl = o.stencil(l)
        assert Wl == W1
        np.testing.assert_allclose(Kl, K1 / 2 ** (l - 1), rtol=0, atol=1e-14 * np.abs(K1).max())
    tol = 1e-14 * np.abs(K1).max()
    np.testing.assert_allclose(K1, K1[::-1, ::-1, ::-1], rtol=0, atol=tol)
    np.testing.assert_allclose(K1, np.transpose(K1, (2, 1, 0)), rtol=0, atol=tol)


def _restrict_axis(x, axis, J, lo_f, lo_c, n_c, periodic):
    """(I q)_m = sum_n J_{n-2m} q_n along one axis (absolute grid indices)."""
    x = np.moveaxis(x, axis, -1)
    n_f = x.shape[-1]
    out = np.zeros(x.shape[:-1] + (n_c,))
    for mi in range(n_c):
        m = mi + lo_c
        for k, jv in J.items():
            nabs = 2 * m + k
            ni = nabs % n_f if periodic else nabs - lo_f
            if 0 <= ni < n_f:
                out[..., mi] += jv * x[..., ni]
    return np.moveaxis(out, -1, axis)


def _prolong_axis(e, axis, J, lo_f, lo_c, n_f, periodic):
    """(I e)_m = sum_n J_{m-2n} e_n along one axis (paper's corrected form)."""
    e = np.moveaxis(e, axis, -1)
    n_c = e.shape[-1]
    out = np.zeros(e.shape[:-1] + (n_f,))
    for ni in range(n_c):
        nabs = ni + lo_c
        for k, jv in J.items():
            mabs = 2 * nabs + k
            mi = mabs % n_f if periodic else mabs - lo_f
            if 0 <= mi < n_f:
                out[..., mi] += jv * e[..., ni]
    return np.moveaxis(out, -1, axis)


@pytest.mark.parametrize("periodic", [(0, 0, 0), (1, 1, 1), (1, 1, 0)])
def test_nested_restriction_equals_direct_anterpolation(periodic):
    p = 4
    J = {n: 2.0 ** (1 - p) * math.comb(p, n + p // 2) for n in range(-p // 2, p // 2 + 1)}
    box = (9.0, 8.0, 7.0)
    o = O.OracleMSM(box, periodic, p, 0.5, 2.0, 3)
    pos, q = WL.random_ions(50, box, seed=7)
    q = q * np.linspace(0.5, 1.5, 50)
    q1 = o.grid_charge(1, pos, q)
    for l in (1, 2):
        n_f, lo_f, _ = o.levels[l - 1]
        n_c, lo_c, _ = o.levels[l]
        r = q1 if l == 1 else r
        for ax3, arr_ax in ((0, 2), (1, 1), (2, 0)):
            r = _restrict_axis(r, arr_ax, J, lo_f[ax3], lo_c[ax3], n_c[ax3], periodic[ax3])
        direct = o.grid_charge(l + 1, pos, q)
        np.testing.assert_allclose(r, direct, atol=1e-13)
        assert direct.sum() == pytest.approx(q.sum(), abs=1e-12)
    # prolongation (paper's corrected index form) is the transpose of restriction
    rng = np.random.default_rng(3)
    n_f, lo_f, _ = o.levels[0]
    n_c, lo_c, _ = o.levels[1]
    x = rng.standard_normal(o.grid_shape(1))
    y = rng.standard_normal(o.grid_shape(2))
    Rx, Py = x, y
    for ax3, arr_ax in ((0, 2), (1, 1), (2, 0)):
        Rx = _restrict_axis(Rx, arr_ax, J, lo_f[ax3], lo_c[ax3], n_c[ax3], periodic[ax3])
        Py = _prolong_axis(Py, arr_ax, J, lo_f[ax3], lo_c[ax3], n_f[ax3], periodic[ax3])
    assert np.sum(Rx * y) == pytest.approx(np.sum(x * Py), rel=1e-13)


# --------------------------------------------------------------------------
# short range
# --------------------------------------------------------------------------
@pytest.mark.parametrize("periodic", [(0, 0, 0), (1, 1, 1), (1, 1, 0)])
def test_short_range_cell_list_equals_brute_force(periodic):
    box = (21.0, 19.0, 23.0)
    o = O.OracleMSM(box, periodic, 4, 1.0, 6.5, 2)
    pos, q = WL.random_ions(1500, box, seed=11)
    p1, F1 = o.short_range(pos, q, cells=False)
    p2, F2 = o.short_range(pos, q, cells=True)
    np.testing.assert_allclose(p1, p2, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(F1, F2, rtol=1e-12, atol=1e-12)
    # minimum image: translating everything by a box vector changes nothing
    if periodic == (1, 1, 1):
        p3, F3 = o.short_range(pos + np.array(box) * np.array([1, -2, 3]), q, cells=False)
        np.testing.assert_allclose(p3, p1, rtol=1e-10, atol=1e-10)


# --------------------------------------------------------------------------
# whole MSM vs exact sums
# --------------------------------------------------------------------------
def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


def test_msm_nonperiodic_converges_to_direct_sum():
    # Sec. "Accuracy-performance tradeoff": the non-periodic reference is the
    # exact all-pairs sum.  The MSM error must fall with h and with p.
    box = (10.0, 10.0, 10.0)
    pos, q = WL.random_ions(200, box, seed=12)
    phid, Fd = O.direct_coulomb(pos, q)
    Ed = 0.5 * np.dot(q, phid)
    errs = {}
    for p, h in ((4, 1.0), (4, 0.5), (6, 0.5)):
        r = O.OracleMSM(box, (0, 0, 0), p, h, 3.5, 3).compute(pos, q)
        errs[(p, h)] = (_rel(r["F"], Fd), abs(r["E"] - Ed) / abs(Ed), _rel(r["phi"], phid))
    assert errs[(4, 1.0)][0] < 2e-2
    assert errs[(4, 0.5)][0] < errs[(4, 1.0)][0] / 4
    assert errs[(6, 0.5)][0] < errs[(4, 0.5)][0]
    assert errs[(6, 0.5)][1] < 1e-4 and errs[(6, 0.5)][2] < 1e-4


def test_two_charges_and_single_charge():
    # single charge: E is only the MSM self-energy error (~0); two charges:
    # E ~ q1 q2 / r within the MSM error.
    box = (12.0, 12.0, 12.0)
    o = O.OracleMSM(box, (0, 0, 0), 6, 0.5, 3.0, 3)
    r = o.compute(np.array([[5.1, 6.3, 4.7]]), np.array([1.0]))
    assert abs(r["E"]) < 1e-4
    pos = np.array([[3.1, 4.2, 5.3], [8.3, 7.1, 6.2]])
    r = o.compute(pos, np.array([1.0, -2.0]))
    d = np.linalg.norm(pos[0] - pos[1])
    assert r["E"] == pytest.approx(-2.0 / d, rel=1e-4)
    Fex = -2.0 * (pos[0] - pos[1]) / d ** 3
    tol = 5e-3 * np.linalg.norm(Fex)
    np.testing.assert_allclose(r["F"][0], -r["F"][1], rtol=0, atol=tol)
    np.testing.assert_allclose(r["F"][0], Fex, rtol=0, atol=tol)


def _nacl_supercell(k):
    a0 = 2.0
    na = np.array([[0, 0, 0], [1, 1, 0], [1, 0, 1], [0, 1, 1]], float)
    cl = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1]], float)
    pos, q = [], []
    for i in range(k):
        for j in range(k):
            for l in range(k):
                off = np.array([i, j, l]) * a0
                pos += [b + off for b in na] + [b + off for b in cl]
                q += [1.0] * 4 + [-1.0] * 4
    return np.array(pos), np.array(q), (a0 * k,) * 3


def _madelung_ref():
    with open(__file__.replace("test_oracle_pins.py", "golden/nacl_madelung.txt")) as f:
        return float([l for l in f if not l.startswith("#")][0])


def test_ewald3d_nacl_madelung_and_alpha_independence():
    pos, q, box = _nacl_supercell(1)
    for alpha in (0.8, 1.3, 2.0):
        E = 0.5 * np.dot(q, O.ewald_potentials(box, pos, q, alpha=alpha))
        assert -E / 4.0 == pytest.approx(_madelung_ref(), abs=5e-7)
    pos, q = WL.random_ions(16, (5.0, 6.0, 7.0), seed=13)
    E1 = 0.5 * np.dot(q, O.ewald_potentials((5.0, 6.0, 7.0), pos, q, alpha=0.6))
    E2 = 0.5 * np.dot(q, O.ewald_potentials((5.0, 6.0, 7.0), pos, q, alpha=1.1))
    assert E1 == pytest.approx(E2, rel=1e-12)


def test_msm_nacl_madelung():
    # Sec. "Madelung constants": p = 6 reaches the tabulated value; here a
    # 4x4x4 supercell (cutoff a <= L/2) with p = 6, h = d_min/4, a = 4 d_min.
    pos, q, box = _nacl_supercell(4)
    o = O.OracleMSM(box, (1, 1, 1), 6, 0.25, 4.0, 4)
    E = o.compute(pos + 0.123, q)["E"]
    Mad = -E / (4 * 4 ** 3)
    assert abs(Mad - _madelung_ref()) <= 1e-6


def test_msm_periodic_converges_to_ewald():
    box = (8.0, 8.0, 8.0)
    pos, q = WL.random_ions(60, box, seed=14)
    phie = O.ewald_potentials(box, pos, q)
    Ee = 0.5 * np.dot(q, phie)
    e = []
    for p, h in ((4, 0.5), (6, 0.5), (6, 0.25)):
        r = O.OracleMSM(box, (1, 1, 1), p, h, 3.5, 3).compute(pos, q)
        e.append((abs(r["E"] - Ee) / abs(Ee), _rel(r["phi"], phie)))
    assert e[0][1] < 1e-3
    assert e[1][1] < e[0][1] and e[2][1] < e[1][1] and e[2][1] < 2e-5


def test_ewald2d_against_padded_3d():
    # 2-D Ewald (Parry) vs 3-D Ewald of the slab padded with vacuum plus the
    # dipole correction 2 pi M_z^2 / V (Yeh-Berkowitz); the gap error decays.
    box2 = (6.0, 7.0, 5.0)
    pos, q = WL.random_ions(12, box2, seed=15)
    E2a = 0.5 * np.dot(q, O.ewald_potentials(box2, pos, q, slab=True, alpha=0.5))
    E2b = 0.5 * np.dot(q, O.ewald_potentials(box2, pos, q, slab=True, alpha=0.9))
    assert E2a == pytest.approx(E2b, rel=1e-11)
    errs = []
    for Lz in (40.0, 80.0):
        b3 = (6.0, 7.0, Lz)
        V = b3[0] * b3[1] * b3[2]
        E3 = 0.5 * np.dot(q, O.ewald_potentials(b3, pos, q))
        Mz = np.dot(q, pos[:, 2])
        errs.append(abs(E3 + 2 * np.pi * Mz ** 2 / V - E2a) / abs(E2a))
    assert errs[1] < 2e-4 and errs[1] < errs[0]


def test_msm_slab_converges_to_ewald2d():
    box = (8.0, 8.0, 6.0)
    pos, q = WL.random_ions(50, box, seed=16)
    phie = O.ewald_potentials(box, pos, q, slab=True)
    e = []
    for p, h in ((4, 0.5), (6, 0.5)):
        r = O.OracleMSM(box, (1, 1, 0), p, h, 3.5, 3).compute(pos, q)
        e.append(_rel(r["phi"], phie))
    assert e[0] < 1e-3 and e[1] < e[0]


# --------------------------------------------------------------------------
# invariants and derivatives
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_periodic():
    box = (7.0, 7.0, 7.0)
    o = O.OracleMSM(box, (1, 1, 1), 4, 0.5, 3.0, 3)
    pos, q = WL.gaussian_charges(40, box, 0.5, seed=17)
    return o, pos, q


@pytest.fixture(scope="module")
def small_free():
    box = (7.0, 7.0, 7.0)
    o = O.OracleMSM(box, (0, 0, 0), 4, 0.7, 2.5, 3)
    pos, q = WL.gaussian_charges(40, box, 0.5, seed=18)
    pos = 0.5 + pos * (6.0 / 7.0)
    return o, pos, q


@pytest.mark.parametrize("which", ["small_periodic", "small_free"])
def test_energy_from_grids_equals_interpolated(which, request):
    # U^{1+} = 1/2 sum_l q~^l . (K^l q~^l) (grid form) must equal the
    # particle form 1/2 sum_i q_i phi^{1+}_i (eq. uoneplus_interpolation).
    o, pos, q = request.getfixturevalue(which)
    r = o.compute(pos, q)
    Ugrid = 0.5 * sum(np.sum(qg * eg) for qg, eg in r["grids"])
    assert 0.5 * np.dot(q, r["phi1"]) == pytest.approx(Ugrid, rel=1e-12)
    U0 = 0.5 * np.dot(q, r["phi0"]) - 0.5 * np.dot(q, q) * o.self_constant()
    assert r["E"] == pytest.approx(U0 + Ugrid, rel=1e-12)


@pytest.mark.parametrize("which", ["small_periodic", "small_free"])
def test_scaling_sign_permutation_reciprocity(which, request):
    o, pos, q = request.getfixturevalue(which)
    r = o.compute(pos, q)
    assert o.compute(pos, -q)["E"] == pytest.approx(r["E"], rel=1e-13)
    assert o.compute(pos, 2.5 * q)["E"] == pytest.approx(6.25 * r["E"], rel=1e-13)
    perm = np.random.default_rng(0).permutation(len(q))
    rp = o.compute(pos[perm], q[perm])
    assert rp["E"] == pytest.approx(r["E"], rel=1e-13)
    np.testing.assert_allclose(rp["F"], r["F"][perm], rtol=1e-11, atol=1e-13)
    # reciprocity: potential at j from a unit charge at i = potential at i from j
    i, j = 3, 17
    ei = np.zeros(len(q)); ei[i] = 1.0
    ej = np.zeros(len(q)); ej[j] = 1.0
    assert o.compute(pos, ei)["phi"][j] == pytest.approx(o.compute(pos, ej)["phi"][i], rel=1e-12)


def test_translation_by_top_spacing_is_exact(small_periodic):
    o, pos, q = small_periodic
    r = o.compute(pos, q)
    hL = o.spacing(o.L)
    rt = o.compute(pos + np.array([hL[0], 2 * hL[1], -hL[2]]), q)
    assert rt["E"] == pytest.approx(r["E"], rel=1e-12)
    np.testing.assert_allclose(rt["F"], r["F"], rtol=1e-10, atol=1e-12)
    # a generic translation is only approximately invariant (grids)
    rg = o.compute(pos + 0.1234, q)
    assert rg["E"] == pytest.approx(r["E"], rel=1e-2)
    # net force nearly vanishes (translation invariance broken only by grids)
    assert np.linalg.norm(r["F"].sum(0)) < 1e-2 * np.abs(r["F"]).sum()


@pytest.mark.parametrize("which", ["small_periodic", "small_free"])
def test_forces_and_potentials_are_energy_derivatives(which, request):
    o, pos, q = request.getfixturevalue(which)
    r = o.compute(pos, q)
    eps = 1e-5
    for i, k in ((0, 0), (5, 1), (11, 2), (29, 0)):
        pp, pm = pos.copy(), pos.copy()
        pp[i, k] += eps
        pm[i, k] -= eps
        fd = -(o.compute(pp, q)["E"] - o.compute(pm, q)["E"]) / (2 * eps)
        assert r["F"][i, k] == pytest.approx(fd, rel=1e-6, abs=1e-8)
        qp, qm = q.copy(), q.copy()
        qp[i] += eps
        qm[i] -= eps
        fdq = (o.compute(pos, qp)["E"] - o.compute(pos, qm)["E"]) / (2 * eps)
        assert r["phi"][i] == pytest.approx(fdq, rel=1e-7, abs=1e-9)


@pytest.mark.parametrize("which", ["small_periodic", "small_free"])
def test_force_vjp_matches_finite_differences(which, request):
    o, pos, q = request.getfixturevalue(which)
    v = WL.force_cotangent(len(q), seed=3)
    gE = 0.7
    gq, gr = o.backward(pos, q, gE, v)

    def Lfun(pp, qq):
        r = o.compute(pp, qq)
        return gE * r["E"] + np.sum(v * r["F"])

    eps = 1e-5
    for i, k in ((1, 0), (7, 2), (20, 1)):
        pp, pm = pos.copy(), pos.copy()
        pp[i, k] += eps
        pm[i, k] -= eps
        fd = (Lfun(pp, q) - Lfun(pm, q)) / (2 * eps)
        assert gr[i, k] == pytest.approx(fd, rel=1e-5, abs=1e-6)
        qp, qm = q.copy(), q.copy()
        qp[i] += eps
        qm[i] -= eps
        fdq = (Lfun(pos, qp) - Lfun(pos, qm)) / (2 * eps)
        assert gq[i] == pytest.approx(fdq, rel=1e-5, abs=1e-6)
