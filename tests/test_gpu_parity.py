"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs, element by element.

Bar (FP64): per field q in (H, HU, HV), max_K |q_gpu - q_oracle| <= 1e-12
max_K |q_oracle|, and the same for the time and every step's dt.  The
kernels take a quotient by a value used more than once as one reciprocal
and products, where the oracle divides as the scheme is written; the tests
print the largest difference and the share of bitwise-equal values.
"""
import math
import sys

import numpy as np
import pytest

from paper_2002_04889_amd import vsw
from paper_2002_04889_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_run(case, n, t_stop=math.inf, ordering=vsw.VSW_ORDER_HILBERT, chunks=None,
            variant=vsw.VSW_KERNEL_FACES, **kw):
    s = vsw.Solver.for_case(case, ordering=ordering, **kw)
    try:
        vsw.vsw_set_kernel_variant(s.h, variant)
        if chunks is None:
            rc, done, t = s.step(n, t_stop, check=False)
            dts = vsw.vsw_dt_history(s.h)
        else:
            done, dts, rc = 0, [], 0
            while done < n and rc == 0:
                rc, d, t = s.step(min(chunks, n - done), t_stop, check=False)
                dts.extend(vsw.vsw_dt_history(s.h))
                done += d
                if d == 0:
                    break
            dts = np.array(dts)
        H, HU, HV, t = s.state()
        return {"H": H, "HU": HU, "HV": HV, "t": t, "steps": done, "dts": dts, "rc": rc,
                "clamps": vsw.vsw_clamp_count(s.h)}
    finally:
        s.close()


def orc_run(orc, case, n, t_stop=math.inf, **kw):
    m = orc.Mesh.from_case(case)
    d = dict(g=case.g, cfl=case.cfl, h_threshold=case.h_threshold)
    d.update(kw)
    return m.run(orc.params(**d), case.H, case.HU, case.HV, case.t0, n, t_stop, check=False)


def assert_parity(g, o, label=""):
    assert g["steps"] == o["steps"], (g["steps"], o["steps"])
    report = []
    for k in ("H", "HU", "HV"):
        scale = max(np.abs(o[k]).max(), 1e-300)
        diff = np.abs(g[k] - o[k]).max()
        report.append(f"{k}: maxdiff {diff:.3e} rel {diff / scale:.3e} "
                      f"bitwise {np.mean(g[k] == o[k]) * 100:.2f}%")
        assert diff <= TOL * scale, (k, diff, scale)
    assert abs(g["t"] - o["t"]) <= TOL * max(abs(o["t"]), 1e-300)
    if len(o["dts"]):
        assert np.abs(g["dts"] - o["dts"]).max() <= TOL * o["dts"].max()
    say(label, "steps", g["steps"], "t", g["t"], "|", "; ".join(report))


def test_thacker_period(orc):
    c = W.thacker_case(45)
    say("thacker45", c.nc, "cells, one period")
    g = gpu_run(c, 5000, c.t_end)
    o = orc_run(orc, c, 5000, c.t_end)
    assert g["t"] == c.t_end
    assert_parity(g, o, "thacker45")


def test_thacker_chunked_calls_equal_one_call():
    c = W.thacker_case(23)
    a = gpu_run(c, 300)
    b = gpu_run(c, 300, chunks=37)
    for k in ("H", "HU", "HV"):
        assert np.array_equal(a[k], b[k])
    assert np.array_equal(a["dts"], b["dts"]) and a["t"] == b["t"]


@pytest.mark.parametrize("variant", [vsw.VSW_KERNEL_FACES, vsw.VSW_KERNEL_FUSED,
                                     vsw.VSW_KERNEL_TWO_PASS])
def test_basin_small(orc, variant):
    c = W.basin_case(scale=8)
    say("basin scale 8", c.nc, "cells, 300 steps, variant", variant)
    g = gpu_run(c, 300, variant=variant)
    o = orc_run(orc, c, 300)
    assert_parity(g, o, "basin-s8")
    assert g["clamps"] == o["clamps"]


def test_random_order_fused_matches_two_pass():
    """Random order: every tile's halo is large (up to 3 x 256 faces)."""
    c = W.basin_case(scale=16)
    a = gpu_run(c, 60, ordering=vsw.VSW_ORDER_RANDOM, seed=7)
    b = gpu_run(c, 60, ordering=vsw.VSW_ORDER_RANDOM, seed=7, variant=vsw.VSW_KERNEL_TWO_PASS)
    for k in ("H", "HU", "HV"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("ordering", [vsw.VSW_ORDER_NONE, vsw.VSW_ORDER_RANDOM,
                                      vsw.VSW_ORDER_BISECTION])
def test_orderings_bitwise(ordering):
    c = W.basin_case(scale=16)
    a = gpu_run(c, 100)
    b = gpu_run(c, 100, ordering=ordering, seed=99)
    for k in ("H", "HU", "HV"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("which", ["thacker", "basin"])
def test_lake_at_rest(which):
    c = W.thacker_case(45, still=True) if which == "thacker" else W.basin_case(scale=16,
                                                                               eta_amp=0.0)
    g = gpu_run(c, 500)
    Hm = c.H.max()
    assert np.abs(g["H"] - c.H).max() <= 1e-12 * Hm
    vmax = 1e-12 * Hm * math.sqrt(c.g * Hm)
    assert np.abs(g["HU"]).max() <= vmax and np.abs(g["HV"]).max() <= vmax


@pytest.mark.parametrize("kind", ["single", "square2", "square8"])
def test_tiny_meshes(orc, kind):
    if kind == "single":
        vx, vy, tri = np.array([0.0, 1.0, 0.2]), np.array([0.0, 0.1, 0.9]), np.array([[0, 2, 1]])
    else:
        vx, vy, tri = W.tiny_mesh(kind)
    nc = len(tri)
    rng = np.random.default_rng(21)
    h = rng.uniform(0.5, 2.0, nc)
    H = h + rng.uniform(-0.1, 0.1, nc)
    c = W.Case(name=kind, vx=vx, vy=vy, tri=np.asarray(tri, dtype=np.int32), h=h, H=H,
               HU=rng.normal(0, 0.3, nc), HV=rng.normal(0, 0.3, nc), cfl=0.45,
               h_threshold=1e-3)
    g = gpu_run(c, 40)
    o = orc_run(orc, c, 40)
    assert_parity(g, o, kind)


def test_tiny_momenta_bitwise(orc):
    """Momenta far below the normal range, as the tails a wave front leaves
    ahead of it decay through them: a third of the basin starts with
    momenta between 1e-322 and 1e-280 (subnormal ones among them), a third
    at rest, a third with ordinary small momenta.  The quotients and square
    roots whose operands leave the range of the kernels' short sequences
    take the plain operators, so fields and dts stay bit for bit the
    oracle's, and tiny momenta are still there at the end."""
    c = W.basin_case(scale=16)
    cx, _ = c.centroids()
    rng = np.random.default_rng(5)
    band = (cx - cx.min()) / (cx.max() - cx.min())
    tiny = 10.0 ** rng.uniform(-322.0, -280.0, c.nc) * rng.choice([-1.0, 1.0], c.nc)
    wet = c.H > c.h_threshold
    c2 = c.copy()
    c2.HU = np.where(wet & (band < 0.33), tiny,
                     np.where(wet & (band > 0.66), 1e-3 * rng.normal(size=c.nc), 0.0))
    c2.HV = np.where(wet & (band < 0.33), tiny[::-1], 0.0)
    g = gpu_run(c2, 50)
    o = orc_run(orc, c2, 50)
    assert_parity(g, o, "tiny momenta")
    for k in ("H", "HU", "HV"):
        assert np.array_equal(g[k], o[k]), k
    assert np.array_equal(g["dts"], o["dts"])
    small = (np.abs(g["HU"]) < 2.0 ** -900) & (g["HU"] != 0.0)
    say("cells with momenta in (0, 2^-900) after 50 steps:", int(small.sum()))
    assert small.sum() > 100


def test_dam_break_dry_bed(orc):
    c = W.channel_case(n_len=201, h_threshold=1e-3)
    g = gpu_run(c, 400)
    o = orc_run(orc, c, 400)
    assert_parity(g, o, "channel")
    assert g["clamps"] == o["clamps"]


def test_fixed_dt_and_t_stop(orc):
    c = W.thacker_case(23)
    g = gpu_run(c, 1000, 0.3, dt_fixed=2e-3)
    o = orc_run(orc, c, 1000, 0.3, dt_fixed=2e-3)
    assert g["t"] == 0.3
    assert_parity(g, o, "dt_fixed")


@pytest.mark.parametrize("mode", ["fused", "two_pass", "graph", "fp32"])
def test_unstable_run_reports_eunstable(orc, mode):
    """A fixed dt far above the stable one blows up.  The call returns
    VSW_EUNSTABLE with the number of good steps, and the solver keeps the
    state those steps reached: the input of the failing step (the oracle's
    state after the same number of steps)."""
    c = W.thacker_case(23)
    o = orc_run(orc, c, 400, dt_fixed=0.2)
    assert o["rc"] != 0
    done_o = o["steps"]
    prec = vsw.VSW_FP32 if mode == "fp32" else vsw.VSW_FP64
    s = vsw.Solver.for_case(c, precision=prec, dt_fixed=0.2)
    try:
        if mode == "two_pass":
            vsw.vsw_set_kernel_variant(s.h, vsw.VSW_KERNEL_TWO_PASS)
        if mode == "graph":
            vsw.vsw_set_graph(s.h, True)
        s.step(3)  # an odd count first: the next call starts from the other buffer
        rc, done, t = s.step(400, check=False)
        H, HU, HV, t = s.state()
        assert rc == vsw.VSW_EUNSTABLE
        say(mode, "EUNSTABLE after", 3 + done, "good steps; oracle", done_o)
        if mode == "fp32":
            assert 3 + done >= 1
            ref = vsw.Solver.for_case(c, precision=prec, dt_fixed=0.2)
            try:
                ref.step(3 + done)
                r = ref.state()
            finally:
                ref.close()
            for a, b in zip((H, HU, HV), r[:3]):
                assert np.array_equal(a, b)
            return
        assert 3 + done == done_o
        ref = orc_run(orc, c, done_o, dt_fixed=0.2)
        g = {"H": H, "HU": HU, "HV": HV, "t": t, "steps": done_o, "dts": ref["dts"]}
        assert np.isfinite(H).all() and np.isfinite(HU).all() and np.isfinite(HV).all()
        assert_parity(g, ref, f"eunstable-{mode}")
        # the solver goes on from there: the same failing step again
        rc2, done2, _ = s.step(5, check=False)
        assert rc2 == vsw.VSW_EUNSTABLE and done2 == 0
    finally:
        s.close()


def test_state_validation_and_order_errors():
    c = W.thacker_case(23)
    s = vsw.Solver(g=c.g, cfl=c.cfl, h_threshold=c.h_threshold)
    try:
        with pytest.raises(vsw.VswError, match="ESTATE"):
            s.set_state(c.H, c.HU, c.HV)
        s.upload_mesh(c.vx, c.vy, c.tri, c.h)
        with pytest.raises(vsw.VswError, match="ESTATE"):
            s.step(1)
        bad = c.H.copy()
        bad[3] = np.nan
        with pytest.raises(vsw.VswError, match="EINVAL"):
            s.set_state(bad, c.HU, c.HV)
        bad[3] = -1.0
        with pytest.raises(vsw.VswError, match="EINVAL"):
            s.set_state(bad, c.HU, c.HV)
        s.set_state(c.H, c.HU, c.HV)
        # device arrays are checked on the device, and a rejected state
        # leaves the solver's state as it was
        import torch

        dev = torch.device("cuda:0")
        good = [torch.tensor(a, device=dev) for a in (c.H, c.HU, c.HV)]
        for k, v, what in ((0, -1.0, "negative"), (1, np.nan, "non-finite"),
                           (2, np.inf, "non-finite")):
            arr = [g.clone() for g in good]
            arr[k][7] = v
            torch.cuda.synchronize()
            with pytest.raises(vsw.VswError, match="EINVAL"):
                vsw.vsw_set_state_device(s.h, *[a.data_ptr() for a in arr], 0.0)
            assert what in vsw.vsw_last_error()
            H, HU, HV, t = s.state()
            assert np.array_equal(H, c.H) and np.array_equal(HU, c.HU)
        vsw.vsw_set_state_device(s.h, *[a.data_ptr() for a in good], 0.0)
        rc, done, t = s.step(0)
        assert rc == 0 and done == 0 and t == 0.0
        nc, ne, nw = vsw.vsw_mesh_info(s.h)
        assert nc == c.nc and nw == 4 * 22 and ne == (3 * nc + nw) // 2
    finally:
        s.close()


def test_device_state_roundtrip_and_profiling():
    import torch

    c = W.thacker_case(23)
    s = vsw.Solver.for_case(c)
    try:
        dev = torch.device("cuda:0")
        st = torch.cuda.Stream()
        vsw.vsw_set_stream(s.h, st.cuda_stream)
        H = torch.tensor(c.H, device=dev)
        HU = torch.tensor(c.HU, device=dev)
        HV = torch.tensor(c.HV, device=dev)
        torch.cuda.synchronize()
        vsw.vsw_set_state_device(s.h, H.data_ptr(), HU.data_ptr(), HV.data_ptr(), 0.0)
        vsw.vsw_set_profiling(s.h, True)
        s.step(20)
        times = vsw.vsw_kernel_times(s.h)
        assert times["stage1_kernel"][1] == 20 and times["stage2_kernel"][1] == 20
        assert all(ms > 0 for ms, n in times.values() if n)
        outH = torch.empty_like(H)
        outU = torch.empty_like(H)
        outV = torch.empty_like(H)
        vsw.vsw_get_state_device(s.h, outH.data_ptr(), outU.data_ptr(), outV.data_ptr())
        h2, u2, v2, t = s.state()
        assert np.array_equal(outH.cpu().numpy(), h2) and np.array_equal(outU.cpu().numpy(), u2)
        vsw.vsw_set_stream(s.h, None)
    finally:
        s.close()


def test_basin_1m_bench_configuration(orc, basin1m_oracle):
    """The benchmark's workload (1M-triangle basin, Hilbert order, the
    launch configuration the benchmark times): full-field parity with the
    oracle after all 2000 steps (the oracle on every host core, bitwise the
    same as on one), every step's dt, mass and positivity; the fields and
    dts are in fact bit for bit the oracle's, which is asserted too."""
    c, o = basin1m_oracle
    say("basin", c.nc, "cells: 2000-step parity; oracle on", orc.max_threads(), "threads")
    g = gpu_run(c, 2000)
    assert_parity(g, o, "basin-1M-2000")
    # beyond the bar: the FP64 kernels round every operation as the oracle
    # does, so the fields and the dt sequence are the oracle's bits
    for k in ("H", "HU", "HV"):
        assert np.array_equal(g[k], o[k]), k
    assert np.array_equal(g["dts"], o["dts"])
    assert g["clamps"] == o["clamps"]
    m = orc.Mesh.from_case(c)
    area = m.geometry()["area"]
    m0, m1 = (area * c.H).sum(), (area * g["H"]).sum()
    say("basin 2000 steps: t", g["t"], "mass rel change", (m1 - m0) / m0, "clamps", g["clamps"])
    assert abs(m1 - m0) <= 1e-12 * m0
    assert (g["H"] >= 0).all()


@pytest.mark.parametrize("precision", [vsw.VSW_FP64, vsw.VSW_FP32])
def test_gauges_record_each_step(orc, precision):
    c = W.thacker_case(23)
    cells = np.array([5, 100, 400, 967], dtype=np.int32)
    s = vsw.Solver.for_case(c, precision=precision)
    try:
        vsw.vsw_set_gauges(s.h, cells)
        s.step(37)
        t1, e1 = vsw.vsw_get_gauges(s.h, len(cells))
        rc, done, t = s.step(23)
        t2, e2 = vsw.vsw_get_gauges(s.h, len(cells))
        H, HU, HV, tt = s.state()
        assert e1.shape == (37, 4) and e2.shape == (23, 4)
        assert t2[-1] == tt and np.all(np.diff(np.concatenate([t1, t2])) > 0)
        assert np.array_equal(e2[-1], H[cells] - c.h[cells])
        with pytest.raises(vsw.VswError, match="EINVAL"):
            vsw.vsw_set_gauges(s.h, np.array([c.nc], dtype=np.int32))
    finally:
        s.close()
    if precision == vsw.VSW_FP64:
        o = orc_run(orc, c, 60)
        ref = o["H"][cells] - c.h[cells]
        assert np.abs(e2[-1] - ref).max() <= TOL * np.abs(o["H"]).max()


@pytest.mark.parametrize("which", ["thacker", "basin"])
def test_resume_from_saved_state(which):
    """Save and resume: the state and time read back mid-run and loaded
    into a fresh solver continue bitwise as the uninterrupted run (the
    state is the whole of the scheme's memory; dt comes from it)."""
    c = W.thacker_case(23) if which == "thacker" else W.basin_case(scale=16)
    a = vsw.Solver.for_case(c)
    try:
        a.step(37)
        H, HU, HV, t = a.state()
        a.step(40)
        ref = a.state()
        ref_dts = vsw.vsw_dt_history(a.h)
    finally:
        a.close()
    b = vsw.Solver.for_case(c)
    try:
        b.set_state(H, HU, HV, t)
        b.step(40)
        out = b.state()
        dts = vsw.vsw_dt_history(b.h)
    finally:
        b.close()
    assert out[3] == ref[3]
    for x, y in zip(out[:3], ref[:3]):
        assert np.array_equal(np.asarray(x), np.asarray(y))
    assert np.array_equal(dts, ref_dts)
