"""Ensembles: several scenarios (each its own mesh, dt and time) advanced in
the same kernel launches.  Each scenario of an ensemble must give exactly
what the same scenario gives alone: bit for bit against a solo GPU run (FP64
and FP32) and against the FP64 oracle, with its own dt sequence, and each
scenario stops on its own at t_stop.  The ensemble mixes the basin recipe at
small sizes with meshes smaller than one tile (padding) and a Thacker bowl
(wet/dry fronts).
"""
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


def tiny_case(kind, depth=10.0, eta=0.5):
    vx, vy, tri = W.tiny_mesh(kind)
    nc = len(tri)
    h = np.full(nc, depth)
    H = depth + eta * np.linspace(0.0, 1.0, nc)
    return W.Case(name=kind, vx=vx, vy=vy, tri=tri, h=h, H=H, HU=np.zeros(nc),
                  HV=np.zeros(nc), h_threshold=1e-3)


@pytest.fixture(scope="module")
def cases():
    ens, _ = W.ensemble_cases(n_scen=5, nmin=2e3, nmax=2e4)
    th = W.thacker_case(23, h_threshold=1e-3)
    out = ens[:2] + [tiny_case("square8"), th, tiny_case("square2")] + ens[2:]
    say("ensemble cells:", [c.nc for c in out])
    return out


def run_ensemble(cases, n, precision=vsw.VSW_FP64, t_stop=math.inf, **kw):
    s = vsw.Solver.for_ensemble(cases, precision=precision, **kw)
    try:
        rc, done, t = s.step(n, t_stop, check=False)
        H, HU, HV, _ = s.state()
        ts, dts, steps = vsw.vsw_scenario_status(s.h)
        hist = [vsw.vsw_scenario_dt_history(s.h, i) for i in range(len(cases))]
        out = []
        o = 0
        for i, c in enumerate(cases):
            sl = slice(o, o + c.nc)
            out.append({"H": H[sl], "HU": HU[sl], "HV": HV[sl], "t": ts[i], "steps": steps[i],
                        "dts": hist[i]})
            o += c.nc
        return rc, done, t, out
    finally:
        s.close()


def run_solo(case, n, precision=vsw.VSW_FP64, t_stop=math.inf, **kw):
    s = vsw.Solver.for_case(case, precision=precision, **kw)
    try:
        rc, done, t = s.step(n, t_stop, check=False)
        H, HU, HV, t = s.state()
        return {"H": H, "HU": HU, "HV": HV, "t": t, "steps": done, "rc": rc,
                "dts": vsw.vsw_dt_history(s.h)}
    finally:
        s.close()


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("H", "HU", "HV")) and a["t"] == b["t"] \
        and a["steps"] == b["steps"] and np.array_equal(a["dts"], b["dts"])


@pytest.mark.parametrize("precision", [vsw.VSW_FP64, vsw.VSW_FP32], ids=["fp64", "fp32"])
def test_ensemble_equals_solo_runs(cases, precision):
    n = 60
    rc, done, t, ens = run_ensemble(cases, n, precision)
    assert rc == 0 and done == n
    dts0 = []
    for c, e in zip(cases, ens):
        solo = run_solo(c, n, precision)
        assert solo["rc"] == 0
        assert same(e, solo), c.name
        dts0.append(e["dts"][0])
    say(f"precision {precision}: first dt per scenario", np.array(dts0))
    assert len(set(dts0)) >= 3  # the scenarios step with their own dt
    assert t == min(e["t"] for e in ens)


def test_ensemble_fp64_matches_oracle(cases, orc):
    n = 40
    rc, done, t, ens = run_ensemble(cases, n)
    assert rc == 0
    for c, e in zip(cases, ens):
        m = orc.Mesh.from_case(c)
        o = m.run(orc.params(g=c.g, cfl=c.cfl, h_threshold=c.h_threshold), c.H, c.HU, c.HV,
                  0.0, n, check=False)
        assert o["steps"] == e["steps"] == n
        for k in ("H", "HU", "HV"):
            scale = max(np.abs(o[k]).max(), 1e-300)
            assert np.abs(e[k] - o[k]).max() <= 1e-12 * scale, (c.name, k)
        assert np.abs(e["dts"] - o["dts"]).max() <= 1e-12 * o["dts"].max(), c.name
        say(c.name, "bitwise", all(np.array_equal(e[k], o[k]) for k in ("H", "HU", "HV")))


@pytest.mark.parametrize("precision", [vsw.VSW_FP64, vsw.VSW_FP32], ids=["fp64", "fp32"])
def test_ensemble_scenarios_stop_on_their_own(cases, precision):
    """With t_stop inside the run, scenarios with larger dt reach it in
    fewer steps; each stops there (last step shortened) and matches its solo
    run with the same t_stop."""
    solo = [run_solo(c, 200, precision) for c in cases]
    t_stop = 0.999 * float(min(r["t"] for r in solo))
    rc, done, t, ens = run_ensemble(cases, 400, precision, t_stop=t_stop)
    assert rc == 0
    steps = [e["steps"] for e in ens]
    say("t_stop", t_stop, "steps per scenario", steps)
    assert len(set(steps)) > 1
    for c, e in zip(cases, ens):
        assert e["t"] == t_stop
        assert same(e, run_solo(c, 400, precision, t_stop=t_stop)), c.name
    assert done == max(steps) and t == t_stop


def test_ensemble_gauges_and_chunked_calls(cases):
    """Gauges in two scenarios; two calls of 30 steps equal one of 60."""
    offs = np.cumsum([0] + [c.nc for c in cases])
    gauges = np.array([offs[0] + 3, offs[3] + 100, offs[5] + 7], dtype=np.int32)
    s = vsw.Solver.for_ensemble(cases)
    try:
        vsw.vsw_set_gauges(s.h, gauges)
        s.step(30)
        t1, eta1 = vsw.vsw_get_gauges(s.h, len(gauges))
        H1, _, _, _ = s.state()
        s.step(30)
        H2, _, _, _ = s.state()
    finally:
        s.close()
    assert eta1.shape == (30, 3)
    cat = lambda k: np.concatenate([c.H if k == "H" else c.h for c in cases])
    h = cat("h")
    assert np.array_equal(eta1[-1], H1[gauges] - h[gauges])
    rc, done, t, ens = run_ensemble(cases, 60)
    assert np.array_equal(H2, np.concatenate([e["H"] for e in ens]))


def test_single_scenario_ensemble_equals_mesh_upload(cases):
    c = cases[1]
    a = run_solo(c, 50)
    rc, done, t, ens = run_ensemble([c], 50)
    assert same(ens[0], a)


@pytest.fixture(scope="module")
def full_cases():
    """The benchmark's ensemble at full size (about 25 s to generate)."""
    cases, _ = W.ensemble_cases()
    say("full ensemble:", len(cases), "scenarios,", sum(c.nc for c in cases), "cells")
    return cases


@pytest.mark.parametrize("precision", [vsw.VSW_FP32, vsw.VSW_FP64], ids=["fp32", "fp64"])
def test_full_ensemble_in_bench_configuration(full_cases, precision, orc):
    """The ensemble workload at full size (64 scenarios, 50k-500k triangles,
    12M in all) in the launch configuration the autotuner picks, as the
    benchmark times it: the smallest, a middle and the largest scenario
    equal their solo runs bit for bit after 50 steps, and (FP64) the
    smallest matches the oracle within 1e-12."""
    cases = full_cases
    n = 50
    s = vsw.Solver.for_ensemble(cases, precision=precision)
    try:
        chosen, _ = vsw.vsw_autotune(s.h, 10)
        say(f"precision {precision}: autotuner chose {vsw.tune_config_name(chosen)}")
        rc, done, t = s.step(n, check=False)
        assert rc == 0 and done == n
        H, HU, HV, _ = s.state()
        ts, dts, steps = vsw.vsw_scenario_status(s.h)
        hist = {i: vsw.vsw_scenario_dt_history(s.h, i) for i in range(len(cases))}
    finally:
        s.close()
    off = np.concatenate([[0], np.cumsum([c.nc for c in cases])])
    sizes = np.array([c.nc for c in cases])
    picks = [int(np.argmin(sizes)), int(np.argsort(sizes)[len(sizes) // 2]), int(np.argmax(sizes))]
    for i in picks:
        c = cases[i]
        sl = slice(off[i], off[i + 1])
        e = {"H": H[sl], "HU": HU[sl], "HV": HV[sl], "t": ts[i], "steps": steps[i],
             "dts": hist[i]}
        solo = run_solo(c, n, precision)
        assert solo["rc"] == 0 and same(e, solo), (i, c.nc)
        say(f"scenario {i} ({c.nc} cells): ensemble == solo run, t {e['t']:.3f} s")
    if precision == vsw.VSW_FP64:
        i = picks[0]
        c = cases[i]
        m = orc.Mesh.from_case(c)
        o = m.run(orc.params(g=c.g, cfl=c.cfl, h_threshold=c.h_threshold), c.H, c.HU, c.HV,
                  0.0, n, check=False)
        sl = slice(off[i], off[i + 1])
        bitwise = True
        for k, v in (("H", H), ("HU", HU), ("HV", HV)):
            scale = max(np.abs(o[k]).max(), 1e-300)
            assert np.abs(v[sl] - o[k]).max() <= 1e-12 * scale, k
            bitwise = bitwise and np.array_equal(v[sl], o[k])
        say(f"scenario {i}: ensemble vs oracle after {n} steps within 1e-12, bitwise {bitwise}")
