"""The face-parallel stage kernels (VSW_KERNEL_FACES, the FP64 default)
against the cell-parallel ones (VSW_KERNEL_FUSED) and the oracle.

Both evaluate the same expressions in the same order (the face-parallel
kernel computes the face normals, lengths, midpoint offsets and areas from
the vertex coordinates exactly as the host computes the stored geometry, and
each face once for both of its cells), so the results must agree bit for
bit, for every tile size and cell order.
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


def run(case, n, variant, tile=256, t_stop=math.inf, **kw):
    d = dict(g=case.g, cfl=case.cfl, h_threshold=case.h_threshold)
    d.update(kw)
    s = vsw.Solver(**d)
    try:
        vsw.vsw_set_tile_size(s.h, tile)
        s.upload_mesh(case.vx, case.vy, case.tri, case.h)
        s.set_state(case.H, case.HU, case.HV, case.t0)
        vsw.vsw_set_kernel_variant(s.h, variant)
        rc, done, t = s.step(n, t_stop, check=False)
        H, HU, HV, t = s.state()
        return {"H": H, "HU": HU, "HV": HV, "t": t, "steps": done, "rc": rc,
                "dts": vsw.vsw_dt_history(s.h), "clamps": vsw.vsw_clamp_count(s.h)}
    finally:
        s.close()


def same(a, b):
    return (all(np.array_equal(a[k], b[k]) for k in ("H", "HU", "HV")) and a["t"] == b["t"]
            and a["steps"] == b["steps"] and np.array_equal(a["dts"], b["dts"])
            and a["clamps"] == b["clamps"])


CASES = {
    "thacker": lambda: W.thacker_case(45),
    "basin": lambda: W.basin_case(scale=8),
    "channel": lambda: W.channel_case(n_len=201, h_threshold=1e-3),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("tile", [128, 256, 512])
def test_faces_equal_cell_parallel(name, tile):
    c = CASES[name]()
    n = 300
    ref = run(c, n, vsw.VSW_KERNEL_FUSED)
    got = run(c, n, vsw.VSW_KERNEL_FACES, tile=tile)
    say(name, c.nc, "cells, tile", tile, "steps", got["steps"], "t", got["t"])
    assert got["rc"] == 0 and same(got, ref)


@pytest.mark.parametrize("ordering", [vsw.VSW_ORDER_RANDOM, vsw.VSW_ORDER_NONE,
                                      vsw.VSW_ORDER_BISECTION])
def test_faces_orderings(ordering):
    """Random order puts most faces on tile boundaries (halo lists of up to
    three faces per cell, several face rounds per thread)."""
    c = W.basin_case(scale=16)
    ref = run(c, 80, vsw.VSW_KERNEL_FUSED)
    for tile in (128, 512):
        got = run(c, 80, vsw.VSW_KERNEL_FACES, tile=tile, ordering=ordering, seed=3)
        assert same(got, ref), tile


@pytest.mark.parametrize("kind", ["single", "square2", "square8"])
def test_faces_tiny_meshes(orc, kind):
    if kind == "single":
        vx, vy, tri = np.array([0.0, 1.0, 0.2]), np.array([0.0, 0.1, 0.9]), np.array([[0, 2, 1]])
    else:
        vx, vy, tri = W.tiny_mesh(kind)
    nc = len(tri)
    rng = np.random.default_rng(21)
    h = rng.uniform(0.5, 2.0, nc)
    c = W.Case(name=kind, vx=vx, vy=vy, tri=np.asarray(tri, dtype=np.int32), h=h,
               H=h + rng.uniform(-0.1, 0.1, nc), HU=rng.normal(0, 0.3, nc),
               HV=rng.normal(0, 0.3, nc), cfl=0.45, h_threshold=1e-3)
    ref = run(c, 40, vsw.VSW_KERNEL_FUSED)
    for tile in (128, 256, 512):
        assert same(run(c, 40, vsw.VSW_KERNEL_FACES, tile=tile), ref), tile


def test_faces_lake_at_rest():
    c = W.basin_case(scale=16, eta_amp=0.0)
    g = run(c, 500, vsw.VSW_KERNEL_FACES)
    Hm = c.H.max()
    assert np.abs(g["H"] - c.H).max() <= 1e-12 * Hm
    vmax = 1e-12 * Hm * math.sqrt(c.g * Hm)
    assert np.abs(g["HU"]).max() <= vmax and np.abs(g["HV"]).max() <= vmax


@pytest.mark.parametrize("precision", [vsw.VSW_FP64, vsw.VSW_FP32], ids=["fp64", "fp32"])
def test_tile_size_change_keeps_the_run(precision):
    """Laying the mesh out again for another tile size mid-run moves the
    state records, time and gauges over: the run continues bitwise as
    without the change."""
    c = W.basin_case(scale=16)
    gauges = np.array([2, 700, 3000], dtype=np.int32)
    ref = run(c, 90, vsw.VSW_KERNEL_FACES, precision=precision)
    s = vsw.Solver.for_case(c, precision=precision)
    try:
        vsw.vsw_set_gauges(s.h, gauges)
        s.step(30)
        vsw.vsw_set_tile_size(s.h, 512)
        assert vsw.vsw_tile_size(s.h) == 512
        s.step(31)
        vsw.vsw_set_tile_size(s.h, 128)
        s.step(29)
        H, HU, HV, t = s.state()
        _, eta = vsw.vsw_get_gauges(s.h, len(gauges))
    finally:
        s.close()
    assert t == ref["t"]
    for a, k in ((H, "H"), (HU, "HU"), (HV, "HV")):
        assert np.array_equal(a, ref[k]), k
    # the gauges survive the relayouts (FP32: eta recorded as stored, H - h
    # in FP64 differs from it by rounding at the 1e-12 m level)
    assert eta.shape == (29, 3)
    assert np.abs(eta[-1] - (H - c.h)[gauges]).max() <= 1e-9


def test_faces_ensemble_equals_solo():
    cases = [W.basin_case(scale=s, k=10 + i) for i, s in enumerate((40, 25, 60))]
    cases.append(W.thacker_case(23))
    n = 50
    for tile in (128, 512):
        s = vsw.Solver(g=cases[0].g, cfl=cases[0].cfl, h_threshold=cases[0].h_threshold)
        try:
            vsw.vsw_set_tile_size(s.h, tile)
            s.upload_ensemble([(c.vx, c.vy, c.tri, c.h) for c in cases])
            s.set_state(np.concatenate([c.H for c in cases]),
                        np.concatenate([c.HU for c in cases]),
                        np.concatenate([c.HV for c in cases]))
            rc, done, t = s.step(n)
            H, HU, HV, t = s.state()
        finally:
            s.close()
        off = np.cumsum([0] + [c.nc for c in cases])
        for i, c in enumerate(cases):
            solo = run(c, n, vsw.VSW_KERNEL_FUSED, h_threshold=cases[0].h_threshold)
            sl = slice(off[i], off[i + 1])
            assert np.array_equal(H[sl], solo["H"]) and np.array_equal(HU[sl], solo["HU"]), \
                (tile, i)


def test_faces_coastal_equals_cell_parallel():
    c = W.coastal_case(scale=4.0)
    ref = run(c, 60, vsw.VSW_KERNEL_FUSED)
    got = run(c, 60, vsw.VSW_KERNEL_FACES)
    say("coastal x4", c.nc, "cells", got["t"])
    assert same(got, ref)


@pytest.mark.parametrize("name", ["thacker", "basin"])
@pytest.mark.parametrize("tile", [128, 256, 512])
def test_faces_fp32_equal_cell_parallel(name, tile):
    """The FP32 face-parallel kernel against the FP32 cell-parallel one."""
    c = CASES[name]()
    n = 300
    ref = run(c, n, vsw.VSW_KERNEL_FUSED, precision=vsw.VSW_FP32)
    got = run(c, n, vsw.VSW_KERNEL_FACES, tile=tile, precision=vsw.VSW_FP32)
    assert got["rc"] == 0 and same(got, ref)


def test_faces_fp32_random_order_and_ensemble():
    c = W.basin_case(scale=16)
    ref = run(c, 80, vsw.VSW_KERNEL_FUSED, precision=vsw.VSW_FP32)
    got = run(c, 80, vsw.VSW_KERNEL_FACES, tile=512, precision=vsw.VSW_FP32,
              ordering=vsw.VSW_ORDER_RANDOM, seed=5)
    assert same(got, ref)
