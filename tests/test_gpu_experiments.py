"""Section 3's gauge experiment on the GPU against the oracle: Thacker's
paraboloid with virtual gauges at (0,0), (0.5,0), (1,0) m from the centre,
one period, at two mesh sizes (dx = 0.048 and 0.024 m).  The oracle steps
the same mesh from the same state with its own CFL time steps; the GPU
gauge series must equal the oracle's (the FP64 paths agree bit for bit, the
bar is 1e-12 of the depth scale), and against the closed form at the gauge
cells' centroids the error must fall between the two sizes at every gauge
at an observed order of at least one (measured with the oracle: 1.32,
1.10 and 1.51 over the first period)."""
import math
import sys

import numpy as np
import pytest

from paper_2002_04889_amd import experiments as E
from paper_2002_04889_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_gauges(orc, case, cells, t_fin):
    m = orc.Mesh.from_case(case)
    p = orc.params(g=case.g, cfl=case.cfl, h_threshold=case.h_threshold)
    H, HU, HV, t = case.H.copy(), case.HU.copy(), case.HV.copy(), 0.0
    ts, etas = [], []
    while t < t_fin:
        r = m.run(p, H, HU, HV, t, 1, t_fin)
        H, HU, HV, t = r["H"], r["HU"], r["HV"], r["t"]
        ts.append(t)
        etas.append(H[cells] - case.h[cells])
    return np.array(ts), np.array(etas)


def test_thacker_gauges_two_resolutions_against_oracle(orc):
    T = W.thacker_constants()["T1"]
    errs = {}
    for dx in (0.048, 0.024):
        r = E.thacker_gauge_run(dx, t_fin=T)
        assert r["rc"] == 0 and r["t"][-1] == T
        t_o, eta_o = oracle_gauges(orc, r["case"], r["cells"], T)
        say(f"dx {dx}: {r['nc']} cells, GPU {r['steps']} steps, oracle {len(t_o)} steps")
        assert len(t_o) == r["steps"]
        assert np.abs(t_o - r["t"]).max() <= 1e-12 * T
        d = np.abs(eta_o - r["eta"]).max()
        say(f"  max |GPU - oracle| over the gauge series: {d:.3e} m")
        assert d <= 1e-12 * W.THACKER_H0
        errs[dx] = np.abs(r["eta"] - r["exact_centroid"]).max(axis=0)
        say(f"  L-inf error at the gauge cells' centroids: {errs[dx]}")
    order = np.log(errs[0.048] / errs[0.024]) / math.log(2.0)
    say(f"observed orders (centre, mid, edge): {order}")
    assert np.all(order >= 1.0)
