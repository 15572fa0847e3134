"""Input recipes: the coastal workload has the shape its description gives
(square hull, mesh sizes graded from the coast, about 15% dry cells at rest
outside the uplift, the uplift's peak and extent), checked on a coarsened
copy of the recipe (every size x16)."""
import numpy as np
import pytest

from paper_2002_04889_amd import workloads as W


@pytest.fixture(scope="module")
def coast16():
    return W.coastal_case(scale=16)


def test_coastal_mesh_shape(coast16):
    c = coast16
    assert c.vx.min() == 0.0 and c.vy.min() == 0.0
    assert c.vx.max() == W.COAST_L and c.vy.max() == W.COAST_L
    t = c.tri
    area = 0.5 * ((c.vx[t[:, 1]] - c.vx[t[:, 0]]) * (c.vy[t[:, 2]] - c.vy[t[:, 0]])
                  - (c.vx[t[:, 2]] - c.vx[t[:, 0]]) * (c.vy[t[:, 1]] - c.vy[t[:, 0]]))
    assert (np.abs(area) > 0).all()
    assert abs(np.abs(area).sum() - W.COAST_L ** 2) <= 1e-9 * W.COAST_L ** 2
    cx, cy = c.centroids()
    # triangles are small near the coast, large far from it
    near = np.abs(cx - W.COAST_X0) < 2e3
    far = cx < 300e3
    assert np.sqrt(np.abs(area[near])).mean() * 4 < np.sqrt(np.abs(area[far])).mean()


def test_coastal_bathymetry_and_state(coast16):
    c = coast16
    cx, cy = c.centroids()
    assert 0.12 <= c.info["dry_fraction"] <= 0.18
    assert (c.h[cx < W.COAST_X0 - W.COAST_AMP - W.COAST_SHELF] == 4000.0).all()
    assert (c.h[cx > W.COAST_X0 + W.COAST_AMP + 15e3] < 0).all()
    eta = np.where(c.H > 0, c.H - c.h, 0.0)
    assert 2.8 < eta.max() <= 3.0
    up = eta > 0
    assert np.all(np.abs(cx[up] - 650e3) < 30e3) and np.all(np.abs(cy[up] - 500e3) < 75e3)
    assert np.all(c.HU == 0) and np.all(c.HV == 0)


def test_coastal_random_order_is_a_permutation(coast16):
    r = W.coastal_case(scale=16, ordering_seed=5)
    key = lambda c: np.lexsort(np.sort(c.tri, axis=1).T[::-1])
    a, b = key(coast16), key(r)
    assert np.array_equal(np.sort(coast16.tri, axis=1)[a], np.sort(r.tri, axis=1)[b])
    assert np.array_equal(coast16.h[a], r.h[b]) and np.array_equal(coast16.H[a], r.H[b])
