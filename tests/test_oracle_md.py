"""CPU pins of the oracle's charged Lennard-Jones model and velocity-Verlet
integrator (Sec. MD simulation of charged Lennard-Jonesium): the switch's
smoothness, forces as energy gradients, the textbook potential below the
switch, time reversibility, and the second-order energy error."""
import numpy as np
import pytest

from oracle import oracle as O

EPS, SIG, RC, RON = 1.0, 1.0, 3.0, 2.6
BOX = (7.0, 7.5, 8.0)


def _lattice(n_side, spacing, seed, jitter=0.05):
    rng = np.random.default_rng(seed)
    g = np.arange(n_side) * spacing + 0.5 * spacing
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos += rng.normal(scale=jitter, size=pos.shape)
    q = np.where(np.indices((n_side,) * 3).sum(0).ravel() % 2 == 0, 1.0, -1.0)
    return pos, q


def test_switch_is_twice_continuously_differentiable():
    S, dS = O.lj_switch([RON, RC, 0.5 * (RON + RC), 1.0, 5.0], RC, RON)
    assert S[0] == 1.0 and S[1] == 0.0 and S[2] == pytest.approx(0.5) and S[3] == 1.0
    assert S[4] == 0.0 and dS[0] == 0.0 and dS[1] == 0.0 and dS[3] == 0.0
    w = RC - RON
    for r in (RON, RC):  # S'' near both ends, by differences: it vanishes linearly
        for side in (-1.0, 1.0):
            for h in (1e-3, 1e-4):
                a, b, c = O.lj_switch([r, r + side * h, r + 2 * side * h], RC, RON)[0]
                assert abs(a - 2 * b + c) / h ** 2 <= 60.0 * (2 * h / w) / w ** 2 * 1.01
    r = np.linspace(RON - 0.1, RC + 0.1, 41)
    fd = (O.lj_switch(r + 1e-6, RC, RON)[0] - O.lj_switch(r - 1e-6, RC, RON)[0]) / 2e-6
    np.testing.assert_allclose(O.lj_switch(r, RC, RON)[1], fd, atol=1e-6)


def test_pair_below_the_switch_is_textbook_lennard_jones():
    for r in (0.95, 2 ** (1 / 6), 1.7, RON):
        E, F = O.lj_energy_forces((50.0,) * 3, (0, 0, 0), [[0, 0, 0], [r, 0, 0]], EPS, SIG, RC,
                                  RON)
        assert E == pytest.approx(4 * EPS * ((SIG / r) ** 12 - (SIG / r) ** 6), rel=1e-14)
        f = 24 * EPS * (2 * (SIG / r) ** 12 - (SIG / r) ** 6) / r
        assert F[1, 0] == pytest.approx(f, rel=1e-12) and F[0, 0] == pytest.approx(-f, rel=1e-12)
    E, F = O.lj_energy_forces((50.0,) * 3, (0, 0, 0), [[0, 0, 0], [RC + 1e-9, 0, 0]], EPS, SIG,
                              RC, RON)
    assert E == 0.0 and not F.any()


@pytest.mark.parametrize("periodic", [(1, 1, 1), (0, 0, 0)])
def test_lj_forces_are_energy_gradients(periodic):
    pos, _ = _lattice(4, 1.6, 1, jitter=0.15)
    E, F = O.lj_energy_forces(BOX, periodic, pos, EPS, SIG, RC, RON)
    eps = 1e-6
    for i, k in ((0, 0), (13, 1), (40, 2), (63, 0)):
        a, b = pos.copy(), pos.copy()
        a[i, k] += eps
        b[i, k] -= eps
        fd = -(O.lj_energy_forces(BOX, periodic, a, EPS, SIG, RC, RON)[0] -
               O.lj_energy_forces(BOX, periodic, b, EPS, SIG, RC, RON)[0]) / (2 * eps)
        assert F[i, k] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    # minimum image: moving a particle by a box vector changes nothing
    if periodic[0]:
        pos2 = pos.copy()
        pos2[5] += (BOX[0], -BOX[1], 0.0)
        E2, F2 = O.lj_energy_forces(BOX, periodic, pos2, EPS, SIG, RC, RON)
        assert E2 == pytest.approx(E, rel=1e-12)
        np.testing.assert_allclose(F2, F, atol=1e-10)


def _charged_lj(box):
    o = O.OracleMSM(box, (1, 1, 1), 4, 0.8, RC, 2)

    def forces(x, q):
        r = o.compute(x, q)
        El, Fl = O.lj_energy_forces(box, (1, 1, 1), x, EPS, SIG, RC, RON)
        return r["F"] + Fl, (El, r["E"])
    return forces


def test_velocity_verlet_is_time_reversible():
    pos, q = _lattice(4, 1.75, 2)
    q = q * 2.0
    m = np.full(len(q), 1.5)
    v = np.random.default_rng(3).normal(scale=0.3, size=pos.shape)
    f = _charged_lj(BOX)
    x1, v1, _ = O.velocity_verlet(pos, v, m, lambda x: f(x, q), 2e-3, 10)
    x0, v0, _ = O.velocity_verlet(x1, -v1, m, lambda x: f(x, q), 2e-3, 10)
    np.testing.assert_allclose(x0, pos, atol=1e-10)
    np.testing.assert_allclose(-v0, v, atol=1e-10)


def test_energy_error_is_second_order_in_the_step():
    """The total-energy excursion of a short trajectory falls about 4x when the
    step is halved (velocity Verlet with forces that are exact gradients)."""
    pos, q = _lattice(4, 1.75, 4)
    q = q * 2.0
    m = np.ones(len(q))
    v = np.random.default_rng(5).normal(scale=0.5, size=pos.shape)
    f = _charged_lj(BOX)
    E0 = sum(f(pos, q)[1]) + 0.5 * float(np.sum(v * v))
    dev = []
    for dt, steps in ((4e-3, 10), (2e-3, 20)):
        _, _, log = O.velocity_verlet(pos, v, m, lambda x: f(x, q), dt, steps)
        dev.append(max(abs(ke + sum(e) - E0) for ke, e in log))
    assert 3.0 < dev[0] / dev[1] < 5.0, dev
