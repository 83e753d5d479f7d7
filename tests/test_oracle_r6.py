"""CPU pins of the oracle's MSM for the dispersion kernel k(r) = r^-6, the
paper's splitting applied to another power (Sec. Splitting for Coulomb
kernels; the package's core is meant to take other kernels): the softener's
contact with r^-6, the telescoping split, and the MSM against the exact
all-pairs sum (free space)."""
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


def test_periodic_r6_is_refused():
    with pytest.raises(AssertionError):
        O.OracleMSM((10.0,) * 3, (1, 1, 1), 4, 1.0, 3.0, 2, nu=NU)
