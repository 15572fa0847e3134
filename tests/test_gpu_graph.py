"""Graph modes: the step loop replayed from a captured pair of steps (mode 1)
or captured whole for the call's step count (mode 2) must give exactly the
results of direct launches (state, times, dt history, gauges), for FP64
(face-parallel and two-pass kernels) and FP32, odd and even step counts,
t_stop inside the run, ensembles, and over repeated calls with the
program's own eager work (state reads, synchronisation) between the
replays; changing t_stop, the step count or the gauges recaptures the
graph."""
import math
import sys

import numpy as np
import pytest

from paper_2002_04889_amd import vsw
from paper_2002_04889_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def session(case_or_cases, calls, graph, gauges=None, **kw):
    """Run a list of (n, t_stop) calls; after each, read the state (eager
    kernels + synchronisation) and the logs."""
    if isinstance(case_or_cases, list):
        s = vsw.Solver.for_ensemble(case_or_cases, **kw)
    else:
        s = vsw.Solver.for_case(case_or_cases, **kw)
    out = []
    try:
        vsw.vsw_set_graph(s.h, graph)
        if gauges is not None:
            vsw.vsw_set_gauges(s.h, gauges)
        for n, t_stop in calls:
            rc, done, t = s.step(n, t_stop, check=False)
            H, HU, HV, t2 = s.state()
            rec = {"rc": rc, "done": done, "t": t, "H": H, "HU": HU, "HV": HV,
                   "dts": vsw.vsw_dt_history(s.h), "status": vsw.vsw_scenario_status(s.h)}
            if gauges is not None:
                rec["gauges"] = vsw.vsw_get_gauges(s.h, len(gauges))
            out.append(rec)
    finally:
        s.close()
    return out


def assert_same(a, b):
    assert len(a) == len(b)
    for x, y in zip(a, b):
        assert x["rc"] == y["rc"] and x["done"] == y["done"] and x["t"] == y["t"]
        for k in ("H", "HU", "HV", "dts"):
            assert np.array_equal(x[k], y[k]), k
        for u, v in zip(x["status"], y["status"]):
            assert np.array_equal(u, v)
        if "gauges" in x:
            assert np.array_equal(x["gauges"][0], y["gauges"][0])
            assert np.array_equal(x["gauges"][1], y["gauges"][1])


CALLS = [(7, math.inf), (10, math.inf), (1, math.inf), (6, math.inf), (9, math.inf)]


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("config", ["fp64", "fp64-two-pass", "fp32"])
def test_graph_equals_direct_launches(config, mode):
    c = W.basin_case(scale=16)
    kw = {"precision": vsw.VSW_FP32 if config == "fp32" else vsw.VSW_FP64}
    gauges = np.array([1, 500, 2000], dtype=np.int32)
    if config == "fp64-two-pass":
        def run(graph):
            s = vsw.Solver.for_case(c, **kw)
            try:
                vsw.vsw_set_kernel_variant(s.h, vsw.VSW_KERNEL_TWO_PASS)
                vsw.vsw_set_graph(s.h, graph)
                res = []
                for n, ts in CALLS:
                    rc, done, t = s.step(n, ts, check=False)
                    H, HU, HV, _ = s.state()
                    res.append({"rc": rc, "done": done, "t": t, "H": H, "HU": HU, "HV": HV,
                                "dts": vsw.vsw_dt_history(s.h),
                                "status": vsw.vsw_scenario_status(s.h)})
                return res
            finally:
                s.close()
        a, b = run(0), run(mode)
    else:
        a = session(c, CALLS, 0, gauges, **kw)
        b = session(c, CALLS, mode, gauges, **kw)
    assert_same(a, b)
    say(config, "mode", mode, "t", b[-1]["t"], "steps", sum(r["done"] for r in b))


@pytest.mark.parametrize("mode", [1, 2])
def test_graph_t_stop_changes_recapture(mode):
    c = W.thacker_case(23)
    T = W.thacker_constants()["T1"]
    calls = [(40, 0.1 * T), (40, 0.1 * T), (200, 0.5 * T), (7, T), (400, T)]
    a = session(c, calls, 0, cfl=0.45, h_threshold=1e-5)
    b = session(c, calls, mode, cfl=0.45, h_threshold=1e-5)
    assert_same(a, b)
    assert b[1]["done"] == 0 and b[-1]["t"] == T


@pytest.mark.parametrize("mode", [1, 2])
def test_graph_ensemble(mode):
    ens, _ = W.ensemble_cases(n_scen=4, nmin=2e3, nmax=2e4)
    t_stop = 200.0
    calls = [(11, t_stop), (20, t_stop), (300, t_stop), (300, t_stop)]
    a = session(ens, calls, 0)
    b = session(ens, calls, mode)
    assert_same(a, b)
    say("ensemble steps per scenario", b[-1]["status"][2], "t", b[-1]["status"][0])


@pytest.mark.parametrize("precision", [vsw.VSW_FP64, vsw.VSW_FP32], ids=["fp64", "fp32"])
def test_autotune_keeps_state_and_results(precision):
    """The autotuner times every launch configuration, restores the state
    and keeps the fastest; every configuration gives the same bits."""
    c = W.basin_case(scale=16)
    ref = session(c, [(30, math.inf)], 0, precision=precision)
    s = vsw.Solver.for_case(c, precision=precision)
    try:
        before = s.state()
        chosen, ms = vsw.vsw_autotune(s.h, 10)
        say(f"precision {precision}: chosen {chosen} ({vsw.tune_config_name(chosen)}), "
            f"ms/step {np.round(ms, 4)}")
        assert 0 <= chosen < vsw.VSW_TUNE_CONFIGS and ms[chosen] == np.min(ms)
        # the two-pass organisation (configurations 36-41) is FP64 only
        cfg = np.arange(vsw.VSW_TUNE_CONFIGS)
        applies = (cfg < 36) | (precision == vsw.VSW_FP64)
        assert np.all(np.isfinite(ms[applies])) and np.all(np.isinf(ms[~applies]))
        after = s.state()
        for a, b in zip(before, after):
            assert np.array_equal(np.asarray(a), np.asarray(b))
        rc, done, t = s.step(30)
        H, HU, HV, _ = s.state()
    finally:
        s.close()
    assert done == 30 and t == ref[0]["t"]
    for k, v in (("H", H), ("HU", HU), ("HV", HV)):
        assert np.array_equal(v, ref[0][k])


@pytest.mark.parametrize("precision", [vsw.VSW_FP64, vsw.VSW_FP32], ids=["fp64", "fp32"])
def test_occupancy_caps_bitwise(precision):
    """Capping the resident workgroups per CU changes the launch, not the
    arithmetic."""
    c = W.basin_case(scale=16)
    out = []
    for occ in (0, 3, 2):
        s = vsw.Solver.for_case(c, precision=precision)
        try:
            for bad in (1, 4, -1):
                with pytest.raises(vsw.VswError, match="EINVAL"):
                    vsw.vsw_set_occupancy(s.h, bad)
            vsw.vsw_set_occupancy(s.h, occ)
            s.step(25)
            out.append(s.state())
        finally:
            s.close()
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert np.array_equal(np.asarray(a), np.asarray(b))


def test_tile_orders_bitwise():
    c = W.basin_case(scale=16)
    out = []
    for order in (0, 1):
        s = vsw.Solver.for_case(c)
        try:
            vsw.vsw_set_tile_order(s.h, order)
            s.step(25)
            out.append(s.state())
        finally:
            s.close()
    for a, b in zip(*out):
        assert np.array_equal(np.asarray(a), np.asarray(b))


def test_graph_mode_checked():
    s = vsw.Solver.for_case(W.thacker_case(23))
    try:
        for bad in (-1, 3):
            with pytest.raises(vsw.VswError, match="EINVAL"):
                vsw.vsw_set_graph(s.h, bad)
    finally:
        s.close()
