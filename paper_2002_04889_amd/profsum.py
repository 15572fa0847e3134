"""Summarise rocprofv3 CSV output (kernel stats, PMC counters) as markdown.

python -m paper_2002_04889_amd.profsum --stats DIR/run_kernel_stats.csv
python -m paper_2002_04889_amd.profsum --trace DIR/run_kernel_trace.csv
python -m paper_2002_04889_amd.profsum --pmc DIR/run_counter_collection.csv \
       [--copy-bytes N]

--copy-bytes: bytes one plain copy kernel moved (read and written); the
counter value that the copy kernel (rocclr copyBuffer) reports for its
largest dispatch gives the scale factor from counter units to bytes.

--traffic-json OUT --workload NAME: also write the scaled FETCH_SIZE and
WRITE_SIZE per launch of every kernel, in bytes (and SQ_INSTS_VALU, SQ_WAVES
per launch where a pass holds them), with a digest of the kernel sources;
the benchmark reports these as the measured HBM traffic and vector issue
rate only while the digest matches the sources it runs.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


# The files the stage kernels are compiled from (their code and headers),
# the host code that lays the mesh out in memory, and the compile flags: a
# change to any of them invalidates measured traffic.
STAGE_SOURCES = ("vsw_device.hpp", "vsw_common.hpp", "vsw_kernels.hpp", "vsw_kernels.hip",
                 "vsw_kernels_f32.hpp", "vsw_kernels_f32.hip", "vsw_faces.hpp", "vsw_faces.hip",
                 "vsw_mesh.hpp", "vsw_mesh.cpp")


def source_digest() -> str:
    """sha256 over the stage kernels' sources and the compile flags."""
    from . import build as libbuild

    h = hashlib.sha256()
    for f in STAGE_SOURCES:
        h.update(f.encode())
        h.update(open(os.path.join(CSRC, f), "rb").read())
    h.update(" ".join(libbuild.FLAGS).encode())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    name = re.sub(r"\(.*", "", name)
    return name.replace("void ", "").strip()


def stats(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['Percentage']):.1f} |")
    return "\n".join(out)


def trace(path: str) -> str:
    """Per-dispatch kernel trace grouped by run and kernel: a run starts at
    each state upload (a pack_state kernel), so that the legs of one
    benchmark (meshes, precisions, cell orders) are averaged separately."""
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    agg = collections.OrderedDict()
    run = 0
    for r in rows:
        name = short(r["Kernel_Name"])
        if name.startswith("vsw::pack_state"):
            run += 1
        wg = int(r["Workgroup_Size_X"]) * int(r["Workgroup_Size_Y"]) * int(r["Workgroup_Size_Z"])
        grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        agg.setdefault((run, name, grid // max(wg, 1)), []).append(dur)
    total = sum(sum(v) for v in agg.values())
    out = ["| run | kernel | workgroups | calls | avg us | min us | max us | share % |",
           "|---|---|---|---|---|---|---|---|"]
    for (rn, k, wgs), v in agg.items():
        if not k.startswith("vsw::") or 100.0 * sum(v) / total < 0.05:
            continue
        out.append(f"| {rn} | {k} | {wgs} | {len(v)} | {sum(v) / len(v):.2f} | {min(v):.2f} | "
                   f"{max(v):.2f} | {100.0 * sum(v) / total:.1f} |")
    return "\n".join(out)


def _agg(path):
    rows = list(csv.DictReader(open(path)))
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        agg[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return agg


def _scales(agg, counters, copy_bytes):
    scale = {}
    if copy_bytes:
        cp = [k for k in agg if "copyBuffer" in k]
        for c in counters:
            if cp and c in ("FETCH_SIZE", "WRITE_SIZE") and agg[cp[0]][c]:
                scale[c] = copy_bytes / 1024.0 / max(agg[cp[0]][c])
    return scale


def traffic(paths, copy_bytes: float, workload: str) -> dict:
    """Average scaled FETCH_SIZE / WRITE_SIZE per launch, in bytes."""
    out = {"digest": source_digest(), "workload": workload, "kernels": {}}
    for p in paths:
        agg = _agg(p)
        counters = sorted({c for v in agg.values() for c in v})
        scale = _scales(agg, counters, copy_bytes)
        for k, v in agg.items():
            if not k.startswith("vsw::"):
                continue
            for c in ("FETCH_SIZE", "WRITE_SIZE"):
                if c in v and c in scale:
                    out["kernels"].setdefault(k, {})[c.lower().replace("_size", "_bytes")] = \
                        sum(v[c]) / len(v[c]) * scale[c] * 1024.0
            # vector instructions issued per launch (wave instructions: one
            # per wavefront of 64 lanes), when that pass was taken
            for c in ("SQ_INSTS_VALU", "SQ_WAVES"):
                if c in v:
                    out["kernels"].setdefault(k, {})[c.lower()] = sum(v[c]) / len(v[c])
    return out


def pmc(path: str, copy_bytes: float | None) -> str:
    agg = _agg(path)
    counters = sorted({c for v in agg.values() for c in v})
    scale = _scales(agg, counters, copy_bytes)
    head = "| kernel | dispatches | " + " | ".join(
        f"{c} (avg{', x' + format(scale[c], '.4f') + ' = KiB' if c in scale else ''})"
        for c in counters) + " |"
    out = [head, "|" + "---|" * (len(counters) + 2)]
    for k, v in agg.items():
        n = max(len(x) for x in v.values())
        vals = []
        for c in counters:
            x = v.get(c, [])
            a = sum(x) / len(x) if x else float("nan")
            vals.append(f"{a * scale.get(c, 1.0):.1f}")
        out.append(f"| {k} | {n} | " + " | ".join(vals) + " |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats")
    ap.add_argument("--trace")
    ap.add_argument("--pmc", action="append", default=[])
    ap.add_argument("--copy-bytes", type=float)
    ap.add_argument("--traffic-json")
    ap.add_argument("--workload", default="")
    a = ap.parse_args()
    if a.stats:
        print(stats(a.stats))
    if a.trace:
        print(trace(a.trace))
    for p in a.pmc:
        print()
        print(pmc(p, a.copy_bytes))
    if a.traffic_json:
        with open(a.traffic_json, "w") as f:
            json.dump(traffic(a.pmc, a.copy_bytes, a.workload), f, indent=1)


if __name__ == "__main__":
    main()
