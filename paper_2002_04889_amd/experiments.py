"""The paper's own accuracy experiments, run on the GPU solver.

* Section 3: Thacker's paraboloid with virtual gauges at (0,0), (0.5,0),
  (1,0) m from the centre, mesh sizes 0.048 ... 0.003 m, t_fin = 10 s;
  the L-infinity error at the centre gauge against the closed form and the
  observed order of convergence.
* Section 3: time-step study, dt = (0.333, 1, 1.2) dx at dx = 0.006 m
  (and the same factors on the solver's CFL number).
* Section 4: decomposition of the gauge error into C1 h^2 + C2 h^3 + C3 h^4
  from three grids h, h/2, h/4 (closed form of Section 4).

python -m paper_2002_04889_amd.experiments convergence [--sizes 0.048 0.024 ...]
python -m paper_2002_04889_amd.experiments dtstudy
python -m paper_2002_04889_amd.experiments decompose
python -m paper_2002_04889_amd.experiments floor [--sizes ...] [--h-threshold H]

The mesh for size dx is the seeded jittered grid of the Thacker case with
round(4 / dx) + 1 points per side.  Time steps follow the CFL rule of the
solver (CFL 0.45) unless a fixed dt is asked for.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import workloads as W

GAUGES_FROM_CENTRE = ((0.0, 0.0), (0.5, 0.0), (1.0, 0.0))


def error_decomposition(E1, E2, E3, h):
    """Section 4: with E(t) ~ C1 h^2 + C2 h^3 + C3 h^4 measured on grids
    h, h/2, h/4 (E1, E2, E3), the three components in closed form."""
    E1, E2, E3 = (np.asarray(x, dtype=np.float64) for x in (E1, E2, E3))
    C1 = (E1 - 24.0 * E2 + 128.0 * E3) / (3.0 * h ** 2)
    C2 = -2.0 * (E1 - 20.0 * E2 + 64.0 * E3) / h ** 3
    C3 = 8.0 * (E1 - 12.0 * E2 + 32.0 * E3) / (3.0 * h ** 4)
    return C1, C2, C3


def find_cells(case, points):
    """Index of the triangle containing each point (barycentric test)."""
    t = case.tri
    x0, y0 = case.vx[t[:, 0]], case.vy[t[:, 0]]
    x1, y1 = case.vx[t[:, 1]], case.vy[t[:, 1]]
    x2, y2 = case.vx[t[:, 2]], case.vy[t[:, 2]]
    det = (y1 - y2) * (x0 - x2) + (x2 - x1) * (y0 - y2)
    out = []
    for (px, py) in points:
        a = ((y1 - y2) * (px - x2) + (x2 - x1) * (py - y2)) / det
        b = ((y2 - y0) * (px - x2) + (x0 - x2) * (py - y2)) / det
        c = 1.0 - a - b
        inside = (a >= -1e-12) & (b >= -1e-12) & (c >= -1e-12)
        idx = np.flatnonzero(inside)
        out.append(int(idx[0]) if len(idx) else int(np.argmin(
            (case.centroids()[0] - px) ** 2 + (case.centroids()[1] - py) ** 2)))
    return np.array(out, dtype=np.int32)


def progress(msg):
    """One line per phase on stderr (flushed), so that a long experiment is
    never silent between its steps."""
    print(f"[experiments {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def thacker_gauge_run(dx, t_fin=10.0, dt_factor=None, precision=None, chunk=4000, cfl=None,
                      h_threshold=None):
    """Run Thacker's paraboloid on the mesh of size dx to t_fin with gauges.

    Returns dict(t, eta [steps, 3], exact [steps, 3], exact_centroid [steps, 3]
    (the closed form at the gauge cells' centroids), cells, nc, steps)."""
    from . import vsw

    n = int(round(4.0 / dx)) + 1
    progress(f"dx={dx:g}: generating the {n}x{n}-point mesh")
    t0 = time.perf_counter()
    case = W.thacker_case(n)
    L = W.THACKER_L
    pts = [(L / 2 + gx, L / 2 + gy) for gx, gy in GAUGES_FROM_CENTRE]
    cells = find_cells(case, pts)
    progress(f"dx={dx:g}: {case.nc} cells, gauge cells {cells.tolist()} "
             f"({time.perf_counter() - t0:.1f} s); uploading")
    kw = {}
    if dt_factor is not None:
        kw["dt_fixed"] = dt_factor * dx
    if precision is not None:
        kw["precision"] = precision
    if cfl is not None:
        kw["cfl"] = cfl
    if h_threshold is not None:
        kw["h_threshold"] = h_threshold
    s = vsw.Solver.for_case(case, **kw)
    progress(f"dx={dx:g}: uploaded; stepping to t={t_fin:g} in calls of {chunk} steps")
    try:
        vsw.vsw_set_gauges(s.h, cells)
        ts, etas = [], []
        t = 0.0
        while t < t_fin:
            rc, done, t = s.step(chunk, t_fin, check=False)
            tt, ee = vsw.vsw_get_gauges(s.h, len(cells))
            ts.append(tt)
            etas.append(ee)
            print(f"  dx={dx:g} t={t:.3f} steps={sum(len(x) for x in ts)}", file=sys.stderr,
                  flush=True)
            if rc != 0 or done == 0:
                break
        t_arr = np.concatenate(ts)
        eta = np.concatenate(etas)
        H_fin = s.state()[0]
    finally:
        s.close()
    progress(f"dx={dx:g}: {len(t_arr)} steps done; closed form at the gauges")
    px = np.array([p[0] for p in pts])
    py = np.array([p[1] for p in pts])
    cx, cy = case.centroids()
    gx, gy = cx[cells], cy[cells]
    exact = np.stack([W.thacker_exact(px, py, tt)[0] for tt in t_arr]) if len(t_arr) else \
        np.zeros((0, 3))
    exact_c = np.stack([W.thacker_exact(gx, gy, tt)[0] for tt in t_arr]) if len(t_arr) else \
        np.zeros((0, 3))
    return {"t": t_arr, "eta": eta, "exact": exact, "exact_centroid": exact_c, "cells": cells,
            "nc": case.nc, "n": n, "dx": 4.0 / (n - 1), "rc": rc, "steps": len(t_arr),
            "case": case, "H_final": H_fin}


def convergence(sizes=(0.048, 0.024, 0.012, 0.006), t_fin=10.0, h_threshold=None):
    """Section 3: L-infinity norm of the centre-gauge error over [0, t_fin]
    and at t_fin, per mesh size, with the observed orders."""
    rows = []
    for dx in sizes:
        r = thacker_gauge_run(dx, t_fin, h_threshold=h_threshold)
        err = np.abs(r["eta"] - r["exact"])
        rows.append({"dx": r["dx"], "cells": r["nc"], "steps": r["steps"],
                     "linf_centre": float(err[:, 0].max()),
                     "linf_mid": float(err[:, 1].max()),
                     "final_centre": float(err[-1, 0])})
        print(json.dumps(rows[-1]), flush=True)
    for a, b in zip(rows, rows[1:]):
        b["order_centre"] = math.log(a["linf_centre"] / b["linf_centre"]) / math.log(a["dx"] / b["dx"])
        b["order_mid"] = math.log(a["linf_mid"] / b["linf_mid"]) / math.log(a["dx"] / b["dx"])
    return rows


def floor_study(sizes=(0.048, 0.024, 0.012, 0.006), t_fin=10.0, band=0.02, h_threshold=None):
    """Where the error floor of the convergence study comes from.  At t_fin
    the free surface of every cell is compared with the closed form at its
    centroid, in three classes: the interior of the wet region (exact depth
    at least `band` m, about 0.1 m from the shoreline), the shoreline band
    (exact depth below `band`, or wet in the model where the closed form is
    dry), and the centre gauge cell; the gauge series are compared with the
    closed form at the gauge cells' centroids (not at the gauge points, which
    lie up to half a cell away where eta has a slope).  L-infinity and
    area-weighted mean errors per class, with observed orders."""
    rows = []
    for dx in sizes:
        r = thacker_gauge_run(dx, t_fin, h_threshold=h_threshold)
        c = r["case"]
        cx, cy = c.centroids()
        eta_ex, H_ex, _, _ = W.thacker_exact(cx, cy, float(r["t"][-1]))
        H = r["H_final"]
        err = np.abs((H - c.h) - eta_ex)
        t = c.tri
        area = 0.5 * np.abs((c.vx[t[:, 1]] - c.vx[t[:, 0]]) * (c.vy[t[:, 2]] - c.vy[t[:, 0]])
                            - (c.vx[t[:, 2]] - c.vx[t[:, 0]]) * (c.vy[t[:, 1]] - c.vy[t[:, 0]]))
        interior = H_ex >= band
        shore = ((H_ex > 0.0) & (H_ex < band)) | ((H_ex == 0.0) & (H > 0.0))
        row = {"dx": r["dx"], "cells": r["nc"], "steps": r["steps"],
               "interior_linf": float(err[interior].max()),
               "interior_mean": float((err * area)[interior].sum() / area[interior].sum()),
               "shore_linf": float(err[shore].max()),
               "shore_mean": float((err * area)[shore].sum() / area[shore].sum()),
               "centre_cell": float(err[r["cells"][0]])}
        ge = np.abs(r["eta"] - r["exact_centroid"]).max(axis=0)
        row.update({"gauge_centre_linf": float(ge[0]), "gauge_mid_linf": float(ge[1]),
                    "gauge_edge_linf": float(ge[2])})
        rows.append(row)
        print(json.dumps(row), flush=True)
    keys = [k for k in rows[0] if k.endswith("_linf") or k.endswith("_mean")
            or k == "centre_cell"]
    for a, b in zip(rows, rows[1:]):
        for k in keys:
            if a[k] > 0.0 and b[k] > 0.0:
                b["order_" + k] = math.log(a[k] / b[k]) / math.log(a["dx"] / b["dx"])
    return rows


def dt_study(dx=0.006, factors=(0.333, 1.0, 1.2), t_fin=10.0):
    """Section 3: time-step study on one mesh.  (a) the literal fixed
    dt = factor * dx (the paper reports it stable with its own dx measure;
    with the edge-length dx here it exceeds the CFL limit, reported as
    unstable); (b) the same factors applied to the solver's CFL number
    0.45, i.e. dt scaled by 0.333, 1 and 1.2 within the stability limit."""
    rows = []
    for f in factors:
        r = thacker_gauge_run(dx, min(t_fin, 1.0), dt_factor=f)
        rows.append({"mode": "dt = f dx", "factor": f, "dt": f * r["dx"], "steps": r["steps"],
                     "stable": r["rc"] == 0 and bool(np.isfinite(r["eta"]).all())})
        print(json.dumps(rows[-1]), flush=True)
    ref = None
    for f in factors:
        r = thacker_gauge_run(dx, t_fin, cfl=0.45 * f)
        err = np.abs(r["eta"] - r["exact"])[:, 0]
        late = r["t"] >= t_fin - 1.5
        row = {"mode": "cfl = 0.45 f", "factor": f, "steps": r["steps"],
               "stable": r["rc"] == 0, "linf_centre": float(err.max()),
               "linf_centre_last_1.5s": float(err[late].max())}
        if ref is None:
            ref = r
        else:
            row["max_diff_to_f0.333"] = float(np.abs(
                np.interp(ref["t"], r["t"], r["eta"][:, 0]) - ref["eta"][:, 0]).max())
        rows.append(row)
        print(json.dumps(rows[-1]), flush=True)
    return rows


def decompose(h=0.024, t_fin=10.0):
    """Section 4: components C1 h^2, C2 h^3, C3 h^4 of the centre-gauge error
    from grids h, h/2, h/4, sampled on the coarsest grid's output times."""
    runs = [thacker_gauge_run(h / 2 ** k, t_fin) for k in range(3)]
    t = runs[0]["t"]
    E = [np.interp(t, r["t"], r["eta"][:, 0] - r["exact"][:, 0]) for r in runs]
    C1, C2, C3 = error_decomposition(E[0], E[1], E[2], h)
    out = {"h": h, "t": t.tolist()[:: max(1, len(t) // 200)]}
    for name, comp in (("C1h2", C1 * h ** 2), ("C2h3", C2 * h ** 3), ("C3h4", C3 * h ** 4),
                       ("E1", E[0])):
        out[name + "_max_abs"] = float(np.abs(comp).max())
    print(json.dumps({k: v for k, v in out.items() if k != "t"}), flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["convergence", "dtstudy", "decompose", "floor"])
    ap.add_argument("--sizes", type=float, nargs="*", default=[0.048, 0.024, 0.012, 0.006])
    ap.add_argument("--t-fin", type=float, default=None)
    ap.add_argument("--h-threshold", type=float, default=None)
    a = ap.parse_args(argv)
    if a.what == "convergence":
        rows = convergence(a.sizes, a.t_fin or 10.0, a.h_threshold)
        print(json.dumps(rows))
    elif a.what == "floor":
        print(json.dumps(floor_study(a.sizes, a.t_fin or 10.0, h_threshold=a.h_threshold)))
    elif a.what == "dtstudy":
        print(json.dumps(dt_study(t_fin=a.t_fin or 10.0)))
    else:
        decompose(t_fin=a.t_fin or 10.0)


if __name__ == "__main__":
    sys.exit(main())
