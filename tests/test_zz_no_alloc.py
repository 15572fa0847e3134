"""vsw_step_noalloc (logs in the library's fixed device array) against
vsw_step on the same runs: the same kernels, so state, time, dt history,
gauge records and clamp count must agree bit for bit.  Two calls in a row on
one solver, the second shorter, then a run on a smaller mesh that follows
them on the same device array."""
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


def record(s, ng):
    H, HU, HV, t = s.state()
    _, eta = vsw.vsw_get_gauges(s.h, ng)
    return {"H": H, "HU": HU, "HV": HV, "t": t, "dts": vsw.vsw_dt_history(s.h),
            "eta": eta, "clamps": vsw.vsw_clamp_count(s.h)}


def run(case, gauges, calls, step, **kw):
    s = vsw.Solver.for_case(case, **kw)
    out = []
    try:
        vsw.vsw_set_gauges(s.h, gauges)
        for n in calls:
            rc, done, t = step(s.h, n, math.inf, check=False)
            assert rc == 0 and done == n
            out.append(record(s, len(gauges)))
    finally:
        s.close()
    return out


def same(a, b):
    return (all(np.array_equal(a[k], b[k]) for k in ("H", "HU", "HV", "dts", "eta"))
            and a["t"] == b["t"] and a["clamps"] == b["clamps"])


@pytest.mark.parametrize("precision", [vsw.VSW_FP64, vsw.VSW_FP32])
def test_noalloc_step_equals_step(precision):
    big = W.basin_case(scale=8)
    small = W.thacker_case(23)
    gb = np.array([3, 500, 1200, big.nc // 2, big.nc - 1], dtype=np.int32)
    gs = np.array([0, small.nc // 3, small.nc - 1], dtype=np.int32)
    say("noalloc: basin", big.nc, "cells, then thacker", small.nc, "cells, precision", precision)
    for case, gauges, calls in ((big, gb, (150, 37)), (small, gs, (60,))):
        ref = run(case, gauges, calls, vsw.vsw_step, precision=precision)
        got = run(case, gauges, calls, vsw.vsw_step_noalloc, precision=precision)
        for i, (a, b) in enumerate(zip(got, ref)):
            say(f"  {case.name} call {i}: {calls[i]} steps, t = {a['t']:.6g}")
            assert same(a, b), (case.name, i)


def test_noalloc_rejects_calls_beyond_its_array():
    case = W.thacker_case(23)
    s = vsw.Solver.for_case(case)
    try:
        vsw.vsw_set_gauges(s.h, np.arange(6, dtype=np.int32))
        n_max = vsw.VSW_NOALLOC_BYTES // 8 // (2 + 6)
        with pytest.raises(vsw.VswError) as e:
            vsw.vsw_step_noalloc(s.h, n_max + 1)
        assert e.value.code == vsw.VSW_EINVAL
        H0 = s.state()[0]
        rc, done, t = vsw.vsw_step_noalloc(s.h, 20)
        assert rc == 0 and done == 20
        assert not np.array_equal(s.state()[0], H0)
    finally:
        s.close()
