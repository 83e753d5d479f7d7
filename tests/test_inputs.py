"""CPU checks of the seeded input generators that have a stated property
beyond their distribution (Sec. Benchmarks: minimum distance 0.6 d, neutral
uniform charges)."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_2510_05961_amd import workloads as WL


@pytest.mark.parametrize("periodic", [True, False])
def test_spaced_charges_recipe(periodic):
    n, L = 3000, 30.0
    pos, q = WL.spaced_charges(n, L, periodic, seed=11)
    dmin = 0.6 * L / n ** (1.0 / 3.0)
    tree = cKDTree(pos, boxsize=L if periodic else None)
    assert len(tree.query_pairs(dmin * (1 - 1e-12))) == 0
    assert pos.shape == (n, 3) and pos.min() >= 0.0 and pos.max() < L
    assert abs(q.sum()) < 1e-10 and np.abs(q).max() <= 2.0
    # the recipe's uniform charges: mean removed from U[-1, 1]
    assert 0.5 < q.std() < 0.65
    pos2, q2 = WL.spaced_charges(n, L, periodic, seed=11)
    assert np.array_equal(pos, pos2) and np.array_equal(q, q2)
