"""Values the paper prints (tests/golden/): Thacker's parameters of
Section 3.  The workload and the closed form use them, and the derived
constants follow from the definitions the same section gives."""
import json
import math
import os

import numpy as np

from paper_2002_04889_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "thacker_parameters.json")


def test_thacker_parameters_are_the_papers():
    p = json.load(open(GOLDEN))
    c = W.thacker_constants(9.81)
    assert (c["alpha"], c["r0"], c["h0"], c["L"]) == (p["alpha_m"], p["r0_m"], p["h0_m"], p["L_m"])
    assert c["omega"] == math.sqrt(8 * 9.81 * p["h0_m"]) / p["alpha_m"]
    assert c["A"] == (p["alpha_m"] ** 2 - p["r0_m"] ** 2) / (p["alpha_m"] ** 2 + p["r0_m"] ** 2)
    assert abs(c["A"] - 0.36 / 1.64) < 1e-15
    assert abs(p["periods_in_T"] * c["T1"] - 3 * 2 * math.pi / c["omega"]) < 1e-12


def test_thacker_initial_shoreline_and_centre():
    """At t = 0 the closed form is at rest with the surface
    eta(r) = h0 (sqrt(1 - A^2) / (1 - A) - 1 - r^2 / alpha^2 ((1 - A^2) / (1 - A)^2 - 1));
    the shoreline is where it meets the bowl z = -h0 (1 - r^2 / alpha^2)."""
    p = json.load(open(GOLDEN))
    A = W.thacker_constants()["A"]
    a, h0, L = p["alpha_m"], p["h0_m"], p["L_m"]
    k1 = math.sqrt(1 - A * A) / (1 - A) - 1
    k2 = (1 - A * A) / (1 - A) ** 2 - 1
    # eta(r) = z(r): h0 (k1 - r^2 k2) = -h0 (1 - r^2)  ->  r^2 = (k1 + 1) / (k2 + 1)
    r_shore = a * math.sqrt((k1 + 1) / (k2 + 1))
    x = L / 2 + np.array([0.0, 0.5 * r_shore, 0.999 * r_shore, 1.001 * r_shore])
    eta, H, u, v = W.thacker_exact(x, np.full(4, L / 2), 0.0)
    assert np.all(u == 0) and np.all(v == 0)
    assert H[0] > 0 and H[1] > 0 and H[2] > 0 and H[3] == 0.0
    assert abs(eta[0] - h0 * k1) < 1e-15
