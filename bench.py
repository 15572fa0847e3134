"""Benchmark: SSP-RK(2,2) steps of the shallow-water finite-volume scheme on
the 1M-triangle synthetic ocean basin, FP64, one MI355X (default), or on the
12M-triangle coastal mesh in FP32 (--workload coastal).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                [--workload basin|coastal|ensemble|adjoint]

Prints one JSON line.  value = cell-updates/s (one cell advanced by one full
two-stage step) over the timed region, with the mesh and the state already
resident in HBM; the other legs (FP32 on the basin; FP64 and random cell
order on the coastal mesh) are reported beside it.  The roofline entry uses the dominant kernel's average
launch duration from HIP events recorded on the solver's stream around each
launch, in a second pass over the same number of steps; beside the
datasheet peak it carries copy_GBps, the bandwidth of a plain 1 GiB device
copy measured in the same run.  The basin line also carries the FP64 leg of
the 12M-triangle coastal mesh (far larger than the last-level cache, so its
roofline is an HBM one).  cpu_baseline times the FP64 oracle on a bounded
sample of the same workload, on every host thread and on one.  --workload ensemble
reports ensemble runs/s, --workload adjoint the adjoint/forward time ratio.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X datasheet HBM3E bandwidth

# Algorithmic bytes per cell for one stage (FP64): the state a stage must
# read and write, the still-water depth, the mesh connectivity (3 neighbour
# indices + 3 vertex indices, 24 B) and the vertex coordinates amortised
# over the cells (about one value per cell).
#   stage 1: read w^n (24) + h (8) + coords (8) + topology (24) + write w1 (24)
#   stage 2: read w1 (24) + w^n (24) + h (8) + coords (8) + topology (24)
#            + write w^{n+1} (24)
ALG_BYTES_STAGE1 = 88
ALG_BYTES_STAGE2 = 112
# Same count with 4-byte values (FP32 state): stage 1 8 values + 24 B,
# stage 2 11 values + 24 B.
ALG_BYTES_STAGE1_F32 = 56
ALG_BYTES_STAGE2_F32 = 68


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(case, steps_all, steps_one):
    """The FP64 oracle on the host: `steps_all` steps on every thread the
    oracle's OpenMP loops get (OMP_NUM_THREADS, else every core), and
    `steps_one` steps on one thread (bitwise the same results)."""
    import oracle

    m = oracle.Mesh.from_case(case)
    p = oracle.params(g=case.g, cfl=case.cfl, h_threshold=case.h_threshold)
    threads = oracle.max_threads()
    out = {}
    for label, n, th in (("all", steps_all, threads), ("one", steps_one, 1)):
        oracle.set_threads(th)
        t0 = time.perf_counter()
        r = m.run(p, case.H, case.HU, case.HV, 0.0, n)
        el = time.perf_counter() - t0
        out[label] = (case.nc * r["steps"] / el, r["steps"], el, th)
    oracle.set_threads(threads)
    v, n, el, th = out["all"]
    v1, n1, el1, _ = out["one"]
    model = cpu_model()
    return {"value": v, "unit": "cell-updates/s", "cores": th, "kind": "oracle",
            "sample": f"{n} steps of the same {case.nc}-cell mesh from its initial state, C "
                      f"oracle (gcc -O3, OpenMP) on {th} threads, {el:.1f} s; host {model}, "
                      f"{os.cpu_count()} logical CPUs",
            "single_thread": {"value": v1, "unit": "cell-updates/s", "cores": 1,
                              "sample": f"{n1} steps on one thread, {el1:.1f} s"},
            "cpu_model": model, "nproc": os.cpu_count()}


def kernel_roofline(vsw, s, steps, nc, bytes1, bytes2):
    """Per-launch HIP events on the solver's stream over `steps` more steps;
    roofline entry of the dominant stage kernel."""
    vsw.vsw_set_profiling(s.h, True)
    s.step(steps)
    kt = vsw.vsw_kernel_times(s.h)
    vsw.vsw_set_profiling(s.h, False)
    log("[bench] kernel times: " + ", ".join(
        f"{k} {v[0] / max(v[1], 1) * 1e3:.1f} us x{v[1]}" for k, v in kt.items() if v[1]))
    avg = {k: v[0] / v[1] for k, v in kt.items() if v[1]}
    st1, st2 = avg.get("stage1_kernel", 0.0), avg.get("stage2_kernel", 0.0)
    if st2 >= st1:
        dom, dur_ms, per_cell = "stage2_kernel", st2, bytes2
    else:
        dom, dur_ms, per_cell = "stage1_kernel", st1, bytes1
    achieved = per_cell * nc / (dur_ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": dom, "alg_bytes_per_cell": per_cell,
            "avg_launch_us": round(dur_ms * 1e3, 2)}


def copy_bandwidth(torch, dev):
    """A STREAM-like device copy of 1 GiB (four times the 256 MB last-level
    cache) on the current stream: read + write bytes per second of the best
    of five, in GB/s -- the HBM bandwidth a plain kernel attains on this GPU,
    reported beside the datasheet peak."""
    n = 128 * 1024 * 1024
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(5):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return round(2 * n * 8 / (best / 1e3) / 1e9, 1)


def kernel_symbol(kind, precision_name, variant, tile):
    """The device kernel behind a timed kind ("stage1_kernel", ...) of the
    given kernel organisation, as rocprofv3 names it; None for kinds that
    are not one kernel."""
    stage = kind[5]  # "stage1_kernel" -> "1"
    if variant == "faces":
        return (f"vsw::faces_stage_kernel<{tile}, {stage}>" if precision_name == "fp64"
                else f"vsw::faces_stage_f32_kernel<{tile}, {stage}>")
    if variant == "fused":
        return (f"vsw::stage_kernel<{stage}>" if precision_name == "fp64"
                else f"vsw::stage_f32_kernel<{stage}>")
    return None


# Vector issue rate of the chip: 256 CUs x 4 SIMDs, each issuing one
# wave instruction over 16 lanes per clock (a wave64 instruction in four
# clocks, FP64 and FP32 alike without packed math), at 2.4 GHz: lane
# operations per second.
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


def measured_counters(workload, ordering, symbol, cells):
    """The committed PMC record of kernel `symbol` (see measured_traffic),
    or None."""
    from paper_2002_04889_amd import profsum

    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{ordering}.json")
    if symbol is None or not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("digest") != profsum.source_digest() or d.get("cells") not in (None, cells):
        return None
    return d["kernels"].get(symbol)


def measured_traffic(workload, ordering, symbol, cells):
    """HBM bytes per launch of kernel `symbol` from the committed PMC summary
    (profiles/traffic_<workload>_<ordering>.json: FETCH_SIZE + WRITE_SIZE,
    scaled by a plain copy kernel), or None when there is none or the kernel
    sources or the mesh layout code have changed since the counters were
    taken."""
    k = measured_counters(workload, ordering, symbol, cells)
    if not k or "fetch_bytes" not in k or "write_bytes" not in k:
        return None
    return round(k["fetch_bytes"] + k["write_bytes"])


def add_measured(rf, workload, ordering, cells):
    """Measured HBM traffic and vector issue rate of the roofline's kernel."""
    tr = measured_traffic(workload, ordering, rf["kernel_symbol"], cells)
    rf["traffic"] = tr
    if tr is not None:
        rf["traffic_bytes_per_cell"] = round(tr / cells, 1)
        rf["traffic_GBps"] = round(tr / (rf["avg_launch_us"] * 1e-6) / 1e9, 1)
    k = measured_counters(workload, ordering, rf["kernel_symbol"], cells)
    if k and "sq_insts_valu" in k:
        ops = k["sq_insts_valu"] * 64 / (rf["avg_launch_us"] * 1e-6)
        rf["valu_issue"] = {"achieved": round(ops / 1e12, 2), "peak": VALU_PEAK_LANE_OPS / 1e12,
                            "unit": "T lane-ops/s",
                            "frac": round(ops / VALU_PEAK_LANE_OPS, 3),
                            "wave_insts_per_launch": round(k["sq_insts_valu"])}


def time_steps(torch, stream, s, steps):
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    rc, done, t = s.step(steps)
    ev1.record(stream)
    ev1.synchronize()
    torch.cuda.synchronize()
    assert done == steps, (rc, done)
    return ev0.elapsed_time(ev1)


def run_leg(torch, vsw, case, stream, dev, dH, dHU, dHV, precision, ordering, steps, warmup,
            bytes1, bytes2, label, kernel=None, tile=None, launch_modes=False):
    """Warm up and time `steps` steps of one solver configuration; returns
    (leg summary dict, solver handle still open)."""
    s = vsw.Solver(g=case.g, cfl=case.cfl, h_threshold=case.h_threshold, device=0,
                   precision=precision, ordering=ordering)
    vsw.vsw_set_stream(s.h, stream.cuda_stream)
    if tile:
        vsw.vsw_set_tile_size(s.h, tile)
    if kernel is not None and precision == vsw.VSW_FP64:
        vsw.vsw_set_kernel_variant(s.h, kernel)
    t0 = time.perf_counter()
    s.upload_mesh(case.vx, case.vy, case.tri, case.h)
    log(f"[bench] {label}: mesh uploaded in {time.perf_counter() - t0:.1f} s")
    nc, ne, nw = vsw.vsw_mesh_info(s.h)
    vsw.vsw_set_state_device(s.h, dH.data_ptr(), dHU.data_ptr(), dHV.data_ptr(), 0.0)
    rc, done, t = s.step(warmup)
    log(f"[bench] {label}: warmup {done} steps, t={t:.3f} s")
    w0 = time.perf_counter()
    ms = time_steps(torch, stream, s, steps)
    wall = time.perf_counter() - w0
    value = nc * steps / (ms / 1e3)
    log(f"[bench] {label}: timed {steps} steps: {ms:.1f} ms (host wall {wall * 1e3:.1f} ms), "
        f"{value:.3e} cell-updates/s")
    leg = {"value": value, "unit": "cell-updates/s", "ms_per_step": ms / steps,
           "roofline": kernel_roofline(vsw, s, steps, nc, bytes1, bytes2),
           "mesh": {"cells": nc, "edges": ne, "walls": nw},
           "tile": vsw.vsw_tile_size(s.h)}
    if launch_modes:
        # the same call length replayed from a captured step pair and from
        # one graph of the whole call (its first call captures it), against
        # the direct launches timed above
        modes = {"direct": {"value": value, "ms_per_step": ms / steps}}
        for mode, name in ((1, "pair_graph"), (2, "whole_call_graph")):
            vsw.vsw_set_graph(s.h, mode)
            s.step(steps)
            m = time_steps(torch, stream, s, steps)
            modes[name] = {"value": nc * steps / (m / 1e3), "ms_per_step": m / steps}
            log(f"[bench] {label}, {name}: {m:.1f} ms for {steps} steps")
        vsw.vsw_set_graph(s.h, 0)
        leg["launch_modes"] = modes
    return leg, s


def bench_ensemble(args, torch, vsw, W):
    """Uneven-size scenario ensemble: every scenario advances `steps` steps
    (one run) with its own dt, all scenarios in the same launches, FP32, in
    the launch configuration the autotuner picks.  value = ensemble runs/s =
    scenarios / seconds for the timed steps."""
    import numpy as np

    steps = args.steps if args.steps is not None else 500
    warmup = args.warmup if args.warmup is not None else 10
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    cases, info = W.ensemble_cases(size_scale=args.scale, log=None)
    nsc = len(cases)
    ncell = sum(c.nc for c in cases)
    log(f"[bench] ensemble: {nsc} scenarios, {ncell} cells ({min(c.nc for c in cases)}-"
        f"{max(c.nc for c in cases)}), generated in {time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.Stream(device=dev)

    def ensemble_leg(precision, label):
        s = vsw.Solver.for_ensemble(cases, precision=precision)
        try:
            vsw.vsw_set_stream(s.h, stream.cuda_stream)
            chosen, table = vsw.vsw_autotune(s.h, 40)
            log(f"[bench] {label}: autotuner chose {vsw.tune_config_name(chosen)}; ms/step "
                + ", ".join(f"{c}:{m:.3f}" for c, m in enumerate(table)))
            s.step(warmup)
            ms = time_steps(torch, stream, s, steps)
            ts, dts, st = vsw.vsw_scenario_status(s.h)
            assert (st == steps).all(), st
            leg = {"runs_per_s": nsc / (ms / 1e3), "ms_per_step": ms / steps,
                   "cell_updates_per_s": ncell * steps / (ms / 1e3),
                   "autotune": {"chosen": vsw.tune_config_name(chosen),
                                "ms_per_step": {vsw.tune_config_name(c): (round(m, 4) if
                                                np.isfinite(m) else None)
                                                for c, m in enumerate(table)}},
                   "scenario_dt_range_s": [float(dts.min()), float(dts.max())]}
            log(f"[bench] {label}: {steps} steps {ms:.1f} ms, {leg['runs_per_s']:.2f} runs/s, "
                f"{leg['cell_updates_per_s']:.3e} cell-updates/s")
            b1, b2 = ((ALG_BYTES_STAGE1, ALG_BYTES_STAGE2) if precision == vsw.VSW_FP64
                      else (ALG_BYTES_STAGE1_F32, ALG_BYTES_STAGE2_F32))
            leg["roofline"] = kernel_roofline(vsw, s, min(steps, 100), ncell, b1, b2)
            return leg
        finally:
            s.close()

    legs = {}
    legs["fp32"] = ensemble_leg(vsw.VSW_FP32, "ensemble fp32")
    if not args.no_fp64:
        legs["fp64"] = ensemble_leg(vsw.VSW_FP64, "ensemble fp64")
    copy_gbs = copy_bandwidth(torch, dev)
    log(f"[bench] 1 GiB device copy: {copy_gbs:.1f} GB/s (read + write)")
    for leg in legs.values():
        leg["roofline"]["copy_GBps"] = copy_gbs
    # the same runs one scenario after another on the same GPU, in each
    # launch mode: direct launches, the replayed step pair, one graph per
    # run (captured by the warm-up call of the same step count)
    seq_modes = {}
    for mode, name in ((0, "direct"), (1, "pair_graph"), (2, "whole_run_graph")):
        seq_ms = 0.0
        for c in cases:
            s = vsw.Solver.for_case(c, precision=vsw.VSW_FP32)
            try:
                vsw.vsw_set_stream(s.h, stream.cuda_stream)
                vsw.vsw_set_graph(s.h, mode)
                s.step(steps if mode == 2 else warmup)
                seq_ms += time_steps(torch, stream, s, steps)
            finally:
                s.close()
        seq_modes[name] = {"runs_per_s": nsc / (seq_ms / 1e3), "ms_total": seq_ms}
        log(f"[bench] sequential fp32, {name}: {nsc} runs in {seq_ms:.1f} ms, "
            f"{seq_modes[name]['runs_per_s']:.2f} runs/s")
    best_seq = max(seq_modes, key=lambda k: seq_modes[k]["runs_per_s"])
    seq = dict(seq_modes[best_seq], launch_mode=best_seq, modes=seq_modes)
    top = legs.pop("fp32")
    out = {"metric": "ensemble runs/s", "value": top["runs_per_s"], "unit": "runs/s",
           "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": top["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"uneven-size scenario ensemble: {nsc} basin-style meshes, "
                                  f"{ncell} triangles in total (log-uniform 50k-500k), own "
                                  "uplift and dt per scenario, one run = "
                                  f"{steps} steps", "scenarios": nsc, "cells": ncell,
                      "precision": "fp32 state, fp64 accumulation", "ordering": "hilbert",
                      "global_batch": ncell, "parallelism": "single-gpu"},
           "cell_updates_per_s": top["cell_updates_per_s"],
           "roofline": top["roofline"], "autotune": top["autotune"],
           "vs_sequential": top["runs_per_s"] / seq["runs_per_s"],
           "sequential_fp32": seq}
    out.update(legs)
    if not args.no_cpu_baseline:
        import oracle

        csteps = args.cpu_steps if args.cpu_steps is not None else 4
        el = 0.0
        for c in cases:
            m = oracle.Mesh.from_case(c)
            p = oracle.params(g=c.g, cfl=c.cfl, h_threshold=c.h_threshold)
            tt = time.perf_counter()
            m.run(p, c.H, c.HU, c.HV, 0.0, csteps)
            el += time.perf_counter() - tt
        out["cpu_baseline"] = {"value": nsc / (el * steps / csteps), "unit": "runs/s",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": f"{csteps} steps of each of the {nsc} scenarios, "
                                         f"C oracle (gcc -O3, OpenMP) on "
                                         f"{oracle.max_threads()} threads, {el:.1f} s, scaled "
                                         f"to {steps}-step runs; host {cpu_model()}"}
    print(json.dumps(out), flush=True)


def bench_adjoint(args, torch, vsw, W):
    """Twin experiment on the basin: observations at 20 seeded wet gauge
    cells over `steps` steps from a seeded true bed displacement (200
    Gaussian bumps over a 200 x 100 km source box, bed and initial surface
    raised together); the gradient of the misfit at zero displacement with
    respect to the initial state and the bed, by the discrete adjoint with
    checkpoints every 50 steps.  value = adjoint time / forward time."""
    import numpy as np

    from paper_2002_04889_amd.adjoint import displacement_basis

    steps = args.steps if args.steps is not None else 2000
    ckpt = 50
    case = W.basin_case(scale=args.scale)
    nc = case.nc
    cx, cy = case.centroids()
    rng = np.random.default_rng(W.SEED_BASE + 4)
    wet = np.flatnonzero(case.H > 100.0)
    gauges = np.sort(rng.choice(wet, 20, replace=False)).astype(np.int32)
    Phi = displacement_basis(cx, cy)
    a_true = rng.uniform(-1.0, 1.0, Phi.shape[1])
    h_true = case.h - Phi @ a_true
    log(f"[bench] adjoint: {nc} cells, {steps} steps, 20 gauges, checkpoints every {ckpt}")

    def forward(h, timed, precision=vsw.VSW_FP64):
        s = vsw.Solver(g=case.g, cfl=case.cfl, h_threshold=case.h_threshold, precision=precision)
        try:
            s.upload_mesh(case.vx, case.vy, case.tri, h)
            s.set_state(case.H, case.HU, case.HV, 0.0)
            vsw.vsw_set_gauges(s.h, gauges)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, done, _ = s.step(steps)
            el = time.perf_counter() - t0
            assert done == steps
            return vsw.vsw_get_gauges(s.h, len(gauges))[1], el
        finally:
            s.close()

    obs, _ = forward(h_true, False)
    _, t_fwd = forward(case.h, True)
    s = vsw.Solver.for_case(case)
    try:
        t0 = time.perf_counter()
        loss, gH, gU, gV, gh = vsw.vsw_adjoint_gauge_loss(s.h, nc, steps, ckpt, gauges, obs)
        t_adj = time.perf_counter() - t0
    finally:
        s.close()
    ga = -(Phi.T @ gh)
    log(f"[bench] forward {t_fwd * 1e3:.1f} ms, adjoint (forward + reverse) {t_adj * 1e3:.1f} ms, "
        f"ratio {t_adj / t_fwd:.2f}; loss {loss:.6e}, |dL/da| {np.abs(ga).max():.3e}")
    # the FP32 solver: FP32 forward and replay, FP64 reverse sweep
    _, t_fwd32 = forward(case.h, True, vsw.VSW_FP32)
    s = vsw.Solver.for_case(case, precision=vsw.VSW_FP32)
    try:
        t0 = time.perf_counter()
        loss32, gH32, _, _, gh32 = vsw.vsw_adjoint_gauge_loss(s.h, nc, steps, ckpt, gauges, obs)
        t_adj32 = time.perf_counter() - t0
    finally:
        s.close()
    ga32 = -(Phi.T @ gh32)
    rel = float(np.abs(ga32 - ga).max() / np.abs(ga).max())
    log(f"[bench] fp32 forward {t_fwd32 * 1e3:.1f} ms, adjoint {t_adj32 * 1e3:.1f} ms, ratio "
        f"{t_adj32 / t_fwd32:.2f}; max |dL/da fp32-forward - fp64| / max |dL/da| {rel:.2e}")
    out = {"metric": "adjoint/forward time", "value": t_adj / t_fwd, "unit": "ratio",
           "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": t_adj * 1e3 / steps,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"adjoint source inversion on the {nc}-triangle basin: "
                                  "gauge misfit at 20 seeded wet cells over "
                                  f"{steps} steps, gradient w.r.t. initial eta and 200 bed-"
                                  "displacement amplitudes, checkpoints every 50 steps",
                      "cells": nc, "precision": "fp64 forward and adjoint",
                      "global_batch": nc, "parallelism": "single-gpu"},
           "forward_ms": t_fwd * 1e3, "adjoint_ms": t_adj * 1e3, "loss": loss,
           "grad_amplitudes_max": float(np.abs(ga).max()),
           "fp32_forward": {"value": t_adj32 / t_fwd32, "unit": "ratio",
                            "forward_ms": t_fwd32 * 1e3, "adjoint_ms": t_adj32 * 1e3,
                            "loss": loss32, "grad_amplitudes_rel_diff_vs_fp64": rel,
                            "precision": "fp32 forward and replay, fp64 reverse sweep"}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 2000 basin, 1000 coastal)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps before timing (default 100 basin, 20 coastal)")
    ap.add_argument("--workload", choices=["basin", "coastal", "ensemble", "adjoint"],
                    default="basin",
                    help="basin: 1M-triangle ocean basin, FP64 (and the FP32 leg); coastal: "
                         "12M-triangle coastal mesh, FP32 and FP64 in Hilbert and random "
                         "cell order; ensemble: 64 uneven scenarios, ensemble runs/s; "
                         "adjoint: gauge-misfit gradient, adjoint/forward time")
    ap.add_argument("--no-fp64", action="store_true", help="ensemble: skip the FP64 leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-launch-modes", action="store_true",
                    help="skip timing the FP64 leg again in the two graph modes")
    ap.add_argument("--no-fp32", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--no-random", action="store_true",
                    help="coastal: skip the random-order legs")
    ap.add_argument("--legs", default=None,
                    help="comma-separated subset of fp64, fp32, fp64_random_order, "
                         "fp32_random_order (for profiling one configuration at a time)")
    ap.add_argument("--cpu-steps", type=int, default=None,
                    help="oracle steps for cpu_baseline on all threads (default 200 basin, 20 "
                         "coastal; a tenth of them on one thread)")
    ap.add_argument("--no-coastal", action="store_true",
                    help="basin: skip the 12M-triangle coastal FP64 leg")
    ap.add_argument("--kernel", choices=["faces", "fused", "two_pass"], default="faces",
                    help="FP64 stage kernel organisation (default: face-parallel)")
    ap.add_argument("--tile", type=int, choices=[128, 256, 512], default=None,
                    help="cells per tile of the FP64 face-parallel kernel (default 256)")
    ap.add_argument("--scale", type=float, default=1.0,
                    help="mesh size multiplier (1 = the named workload)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 512 MiB three times (reference "
                         "kernel for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "sharding of this solver is a design note, not a built path.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "adjoint":
        import torch

        from paper_2002_04889_amd import vsw
        from paper_2002_04889_amd import workloads as W

        assert torch.cuda.is_available(), "bench.py needs a GPU"
        bench_adjoint(args, torch, vsw, W)
        return
    if args.workload == "ensemble":
        import torch

        from paper_2002_04889_amd import vsw
        from paper_2002_04889_amd import workloads as W

        assert torch.cuda.is_available(), "bench.py needs a GPU"
        bench_ensemble(args, torch, vsw, W)
        return
    coastal = args.workload == "coastal"
    steps = args.steps if args.steps is not None else (1000 if coastal else 2000)
    warmup = args.warmup if args.warmup is not None else (20 if coastal else 100)
    cpu_steps = args.cpu_steps if args.cpu_steps is not None else (20 if coastal else 200)

    import torch

    from paper_2002_04889_amd import vsw
    from paper_2002_04889_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    if coastal:
        case = W.coastal_case(scale=args.scale, log=lambda m: log("[bench] " + m))
        desc = (f"large graded coastal mesh 1000x1000 km, {case.nc} triangles (50 m-5 km), "
                f"fractal coastline, {case.info['dry_fraction'] * 100:.1f}% dry, elliptical "
                "uplift 150x60 km 3 m, walls, CFL 0.45")
    else:
        case = W.basin_case(scale=args.scale)
        desc = (f"synthetic ocean basin 500x500 km, {case.nc} triangles "
                "(graded 250 m-2 km), Gaussian hump, walls, CFL 0.45")
    log(f"[bench] workload {case.name}: {case.nc} cells, generated in "
        f"{time.perf_counter() - t0:.1f} s")
    stream = torch.cuda.Stream(device=dev)
    dH = torch.tensor(case.H, device=dev)
    dHU = torch.tensor(case.HU, device=dev)
    dHV = torch.tensor(case.HV, device=dev)
    torch.cuda.synchronize()

    legs = [("fp64", vsw.VSW_FP64, vsw.VSW_ORDER_HILBERT)]
    if not args.no_fp32:
        legs.append(("fp32", vsw.VSW_FP32, vsw.VSW_ORDER_HILBERT))
    if coastal and not args.no_random:
        legs.append(("fp64_random_order", vsw.VSW_FP64, vsw.VSW_ORDER_RANDOM))
        if not args.no_fp32:
            legs.append(("fp32_random_order", vsw.VSW_FP32, vsw.VSW_ORDER_RANDOM))
    if args.legs:
        keep = args.legs.split(",")
        legs = [x for x in legs if x[0] in keep]
    kernel = {"faces": vsw.VSW_KERNEL_FACES, "fused": vsw.VSW_KERNEL_FUSED,
              "two_pass": vsw.VSW_KERNEL_TWO_PASS}[args.kernel]
    res = {}
    for name, prec, order in legs:
        b1, b2 = ((ALG_BYTES_STAGE1, ALG_BYTES_STAGE2) if prec == vsw.VSW_FP64
                  else (ALG_BYTES_STAGE1_F32, ALG_BYTES_STAGE2_F32))
        leg, s = run_leg(torch, vsw, case, stream, dev, dH, dHU, dHV, prec, order, steps,
                         warmup, b1, b2, name, kernel=kernel, tile=args.tile,
                         launch_modes=(name == "fp64" and not coastal
                                       and not args.no_launch_modes))
        s.close()
        leg["dtype"] = ("f64" if prec == vsw.VSW_FP64 else
                        "f32 state and fluxes, f64 depths/pressure/accumulation")
        leg["ordering"] = "hilbert" if order == vsw.VSW_ORDER_HILBERT else "random"
        rf = leg["roofline"]
        rf["kernel_symbol"] = kernel_symbol(rf["kernel"], name[:4], args.kernel, leg["tile"])
        add_measured(rf, args.workload + ("" if args.scale == 1.0 else f"x{args.scale:g}"),
                     leg["ordering"], leg["mesh"]["cells"])
        res[name] = leg
        torch.cuda.synchronize()

    if not args.copy_calibration:
        # (a counter-calibration run keeps its 512 MiB copy the largest one)
        copy_gbs = copy_bandwidth(torch, dev)
        log(f"[bench] 1 GiB device copy: {copy_gbs:.1f} GB/s (read + write)")
        for leg in res.values():
            leg["roofline"]["copy_GBps"] = copy_gbs
    # The basin is quoted in FP64 (the plain method), the coastal mesh in FP32.
    main_leg = "fp32" if coastal and "fp32" in res else "fp64"
    if main_leg not in res:
        main_leg = next(iter(res))
    top = res.pop(main_leg)
    mesh = top.pop("mesh")
    out = {"metric": "cell-updates/s", "value": top["value"], "unit": "cell-updates/s",
           "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": top["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if main_leg.startswith("fp64") else "f32",
           "data": "synthetic",
           "config": {"workload": desc, "cells": mesh["cells"], "edges": mesh["edges"],
                      "walls": mesh["walls"],
                      "precision": "fp64" if main_leg.startswith("fp64")
                      else "fp32 state, fp64 accumulation",
                      "ordering": top["ordering"], "global_batch": mesh["cells"],
                      "parallelism": "single-gpu"},
           "roofline": top["roofline"]}
    if "launch_modes" in top:
        out["launch_modes"] = top["launch_modes"]
    for name, leg in res.items():
        leg.pop("mesh")
        out[name] = leg
    if args.copy_calibration:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration"] = {"bytes_read": src.numel() * 8, "bytes_written": dst.numel() * 8,
                                   "launches": 3}
    if not coastal and not args.no_coastal:
        # the 12M-triangle coastal mesh: the state and mesh are far larger
        # than the last-level cache, so its traffic is HBM traffic
        t0 = time.perf_counter()
        cst = W.coastal_case(scale=args.scale, log=lambda m: log("[bench] " + m))
        log(f"[bench] coastal workload: {cst.nc} cells, generated in "
            f"{time.perf_counter() - t0:.1f} s")
        cH = torch.tensor(cst.H, device=dev)
        cU = torch.tensor(cst.HU, device=dev)
        cV = torch.tensor(cst.HV, device=dev)
        torch.cuda.synchronize()
        leg, s = run_leg(torch, vsw, cst, stream, dev, cH, cU, cV, vsw.VSW_FP64,
                         vsw.VSW_ORDER_HILBERT, steps, warmup, ALG_BYTES_STAGE1,
                         ALG_BYTES_STAGE2, "coastal fp64", kernel=kernel, tile=args.tile)
        s.close()
        del cH, cU, cV
        torch.cuda.empty_cache()
        rf = leg["roofline"]
        rf["kernel_symbol"] = kernel_symbol(rf["kernel"], "fp64", args.kernel, leg["tile"])
        add_measured(rf, "coastal" + ("" if args.scale == 1.0 else f"x{args.scale:g}"),
                     "hilbert", leg["mesh"]["cells"])
        rf["copy_GBps"] = out["roofline"].get("copy_GBps")
        mesh = leg.pop("mesh")
        leg["dtype"] = "f64"
        leg["workload"] = (f"large graded coastal mesh 1000x1000 km, {mesh['cells']} triangles "
                           "(50 m-5 km), fractal coastline, elliptical uplift, walls, CFL 0.45")
        out["coastal12m_fp64"] = leg
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle, {cpu_steps} steps on all threads, "
            f"{max(cpu_steps // 10, 1)} on one")
        out["cpu_baseline"] = cpu_baseline(case, cpu_steps, max(cpu_steps // 10, 1))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
