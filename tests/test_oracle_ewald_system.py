"""CPU pins of the oracle's structure-factor Ewald sum (potentials and forces
of a whole 3-D periodic system), the exact reference of the periodic
cost-vs-accuracy sweep (Sec. Accuracy-performance tradeoff).  Its potentials
are compared with the pairwise lattice sum, itself pinned by the rock-salt
Madelung constant; its forces with central differences of its energy.
"""
import numpy as np
import pytest

from oracle import oracle as O

BOX = np.array([7.0, 8.0, 9.0])


def _system(n, seed):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3)) * BOX
    q = rng.uniform(-1.0, 1.0, n)
    q -= q.mean()
    return pos, q


@pytest.mark.parametrize("images", [True, False], ids=["images", "minimum-image"])
def test_potentials_equal_the_pairwise_lattice_sum(images):
    pos, q = _system(40, 1)
    ref = O.ewald_potentials(BOX, pos, q)
    alpha = O.ewald_alpha_3d(BOX) if images else None
    phi, _ = O.ewald3d_system(BOX, pos, q, alpha=alpha)
    np.testing.assert_allclose(phi, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_rock_salt_madelung_constant():
    """A 2 x 2 x 2 block of rock-salt unit cells (64 ions, nearest distance 1)."""
    pos, q = [], []
    for i in range(4):
        for j in range(4):
            for k in range(4):
                pos.append((i, j, k))
                q.append(1.0 if (i + j + k) % 2 == 0 else -1.0)
    pos, q = np.array(pos, dtype=float) + 0.25, np.array(q)
    with open(__file__.replace("test_oracle_ewald_system.py", "golden/nacl_madelung.txt")) as f:
        M = float([l for l in f if not l.startswith("#")][0])
    phi, F = O.ewald3d_system([4.0, 4.0, 4.0], pos, q)
    np.testing.assert_allclose(-q * phi, M, atol=5e-7)  # M is quoted to 6 decimals
    assert np.abs(F).max() < 1e-10  # every ion sits at a centre of symmetry


def test_forces_are_minus_the_energy_gradient():
    pos, q = _system(30, 2)
    alpha = O.ewald_alpha_3d(BOX)  # (the forces do not depend on it: next test)
    _, F = O.ewald3d_system(BOX, pos, q, alpha=alpha)

    def E(p):
        return 0.5 * float(np.dot(q, O.ewald3d_system(BOX, p, q, alpha=alpha)[0]))
    eps = 1e-5
    for i in (0, 13, 29):
        for k in range(3):
            a, b = pos.copy(), pos.copy()
            a[i, k] += eps
            b[i, k] -= eps
            assert -(E(a) - E(b)) / (2 * eps) == pytest.approx(F[i, k], rel=1e-7, abs=1e-9)


def test_splitting_and_lattice_invariance():
    pos, q = _system(50, 3)
    phi, F = O.ewald3d_system(BOX, pos, q)
    for alpha in (0.45, 1.9):  # the second with rc at half the shortest edge
        p2, F2 = O.ewald3d_system(BOX, pos, q, alpha=alpha)
        np.testing.assert_allclose(p2, phi, rtol=0, atol=1e-11)
        np.testing.assert_allclose(F2, F, rtol=0, atol=1e-11)
    shift = np.array([7.0, -16.0, 27.0])  # whole box vectors
    p3, F3 = O.ewald3d_system(BOX, pos + shift, q)
    np.testing.assert_allclose(p3, phi, rtol=0, atol=1e-11)
    np.testing.assert_allclose(F3, F, rtol=0, atol=1e-11)
    assert np.abs(F.sum(axis=0)).max() < 1e-10  # Newton's third law
