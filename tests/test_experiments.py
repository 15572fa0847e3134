"""Section 4 error decomposition: the closed form of C1..C3 printed in the
paper is the solution of the 3x3 system sum_p C_{p-1} (h / 2^(k-1))^p = E_k,
k = 1, 2, 3.  Pinned by building E_k from known components and by solving
the system with a library routine."""
import numpy as np
import pytest

from paper_2002_04889_amd.experiments import error_decomposition, find_cells
from paper_2002_04889_amd import workloads as W


def test_decomposition_recovers_known_components():
    rng = np.random.default_rng(4)
    h = 0.024
    C = rng.normal(size=(3, 50)) * np.array([[1e-1], [1e1], [1e3]])
    E = [sum(C[p - 2] * (h / 2 ** (k - 1)) ** p for p in (2, 3, 4)) for k in (1, 2, 3)]
    C1, C2, C3 = error_decomposition(*E, h)
    for got, want in zip((C1, C2, C3), C):
        assert np.allclose(got, want, rtol=1e-9, atol=0)


def test_decomposition_matches_linear_solve():
    h = 0.012
    A = np.array([[(h / 2 ** (k - 1)) ** p for p in (2, 3, 4)] for k in (1, 2, 3)])
    E = np.array([3e-4, 1e-4, 2.6e-5])
    want = np.linalg.solve(A, E)
    got = np.array([float(x) for x in error_decomposition(E[0], E[1], E[2], h)])
    assert np.allclose(got, want, rtol=1e-10)


def test_gauge_cells_contain_points():
    c = W.thacker_case(45)
    pts = [(2.0, 2.0), (2.5, 2.0), (3.0, 2.0)]
    cells = find_cells(c, pts)
    cx, cy = c.centroids()
    for (px, py), k in zip(pts, cells):
        assert (cx[k] - px) ** 2 + (cy[k] - py) ** 2 < (4 / 44) ** 2
