import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU run")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.build(force=not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")))
    return oracle


def _oracle_run(orc, case, n):
    m = orc.Mesh.from_case(case)
    p = orc.params(g=case.g, cfl=case.cfl, h_threshold=case.h_threshold)
    return m.run(p, case.H, case.HU, case.HV, case.t0, n, check=False)


@pytest.fixture(scope="session")
def basin1m_oracle(orc):
    """The 1M-triangle basin and the oracle's run of its 2000 steps (on
    every host core; shared by the FP64 and FP32 parity tests)."""
    from paper_2002_04889_amd import workloads as W

    c = W.basin_case()
    print(f"[oracle] basin {c.nc} cells, 2000 steps on {orc.max_threads()} threads",
          flush=True)
    return c, _oracle_run(orc, c, 2000)


@pytest.fixture(scope="session")
def coastal12m():
    """The full 12M-triangle coastal mesh (generated once per session)."""
    from paper_2002_04889_amd import workloads as W

    c = W.coastal_case(scale=1.0, log=lambda m: print("[coastal]", m, flush=True))
    print(f"[coastal] {c.nc} cells, {c.info['dry_fraction'] * 100:.1f}% dry", flush=True)
    return c


@pytest.fixture(scope="session")
def coastal12m_oracle50(orc, coastal12m):
    """The oracle's run of 50 steps of the 12M-triangle coastal mesh."""
    print(f"[oracle] coastal {coastal12m.nc} cells, 50 steps on {orc.max_threads()} threads",
          flush=True)
    return _oracle_run(orc, coastal12m, 50)
