"""Summaries of rocprofv3 output for the solver's kernels.

    python -m paper_2603_14040_amd.profiling stats DIR [--top N]
        per-kernel call count, total and mean duration from a
        ``rocprofv3 --kernel-trace --stats --output-format csv`` directory
        (markdown table)

    python -m paper_2603_14040_amd.profiling traffic FETCH_DIR WRITE_DIR \
            --kernel REGEX --copy-bytes N [--grid G] [--json OUT]
        HBM traffic per launch of the kernels whose name matches REGEX, from
        one ``--pmc FETCH_SIZE`` and one ``--pmc WRITE_SIZE`` run (CSV), each
        counter scaled by what it reads for the largest plain device copy in
        the same run (N bytes read and N written), so that the figure is in
        true bytes

Only the standard library is used; nothing here touches the GPU.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import re
import sys
from typing import Dict, List, Tuple


def short_name(n: str) -> str:
    n = n.replace("void ", "")
    for ns in ("tph::(anonymous namespace)::", "tph::msw::", "tph::dev::", "tph::"):
        n = n.replace(ns, "")
    m = re.match(r"([A-Za-z_0-9]+)(<[^()]*>)?", n)
    s = (m.group(1) + (m.group(2) or "")) if m else n[:60]
    return s.replace("float", "f32").replace("double", "f64").replace(" ", "")[:72]


def _find(dirname: str, suffix: str) -> List[str]:
    return sorted(glob.glob(os.path.join(dirname, "**", f"*{suffix}"), recursive=True))


def kernel_stats(dirname: str) -> List[Tuple[str, int, float, float]]:
    """(kernel, calls, total ms, mean us) from the kernel trace, largest total first."""
    files = _find(dirname, "kernel_trace.csv")
    if not files:
        raise FileNotFoundError(f"no *kernel_trace.csv under {dirname}")
    agg: Dict[str, List[float]] = collections.defaultdict(lambda: [0, 0.0])
    for fn in files:
        with open(fn) as fh:
            for row in csv.DictReader(fh):
                k = short_name(row["Kernel_Name"])
                d = float(row["End_Timestamp"]) - float(row["Start_Timestamp"])
                agg[k][0] += 1
                agg[k][1] += d
    out = [(k, int(c), s / 1e6, s / c / 1e3) for k, (c, s) in agg.items()]
    return sorted(out, key=lambda r: -r[2])


def counters(dirname: str, name: str) -> Dict[Tuple[str, int], List[float]]:
    """Counter values per dispatch, keyed by (full kernel name, grid size)."""
    files = _find(dirname, "counter_collection.csv")
    if not files:
        raise FileNotFoundError(f"no *counter_collection.csv under {dirname}")
    per: Dict[Tuple[str, str], float] = collections.defaultdict(float)
    key_of: Dict[str, Tuple[str, int]] = {}
    for fn in files:
        with open(fn) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] != name:
                    continue
                d = row["Dispatch_Id"]
                key_of[d] = (row["Kernel_Name"], int(float(row["Grid_Size"])))
                per[d] += float(row["Counter_Value"])      # summed over dimensions (e.g. XCDs)
    out: Dict[Tuple[str, int], List[float]] = collections.defaultdict(list)
    for d, v in per.items():
        out[key_of[d]].append(v)
    return out


def copy_reading(c: Dict[Tuple[str, int], List[float]]) -> float:
    """Mean counter value (KiB) of the largest-grid plain copy kernel."""
    cands = [(g, vals) for (k, g), vals in c.items() if "copyBuffer" in k and "Rect" not in k]
    if not cands:
        raise ValueError("no device copy kernel in the counter run")
    g, vals = max(cands, key=lambda t: t[0])
    return sum(vals) / len(vals)


# the files that hold the code of the finest-level smoothing kernels (bodies,
# stencils, reductions, launchers); kernels.h only declares launchers and is
# left out, so adding an unrelated kernel does not invalidate the counters
SMOOTHER_SOURCES = ("common.h", "stencil.h", "reduce.h", "fused_dev.h", "msweep.h", "msweep_f32.hip",
                    "msweep_f64.hip", "fused.hip")


# the files that hold the code of the Uzawa link pass (kernel, cell body,
# stencils) and of its launcher
LINK_SOURCES = ("common.h", "stencil.h", "stencil_dev.h", "stencil.hip")

# sources whose hash a committed counter summary carries, by the kernel class
# bench.py reports in its roofline entry
KERNEL_SOURCES = {"smooth": SMOOTHER_SOURCES, "link": LINK_SOURCES}


def sources_hash(files=SMOOTHER_SOURCES) -> str:
    """SHA-256 over the sources of the profiled kernel (which code the counters belong to)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for fn in sorted(files):
        h.update(fn.encode())
        with open(os.path.join(csrc, fn), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic(fetch_dir: str, write_dir: str, kernel: str, copy_bytes: float, grid: int = 0,
            sources=SMOOTHER_SOURCES) -> dict:
    rx = re.compile(kernel)
    res = {}
    for tag, d, cname in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        c = counters(d, cname)
        calib = copy_bytes / (copy_reading(c) * 1024.0)          # true bytes per counted byte
        vals = [v for (k, g), vs in c.items() if rx.search(k) and (grid <= 0 or g == grid) for v in vs]
        if not vals:
            raise ValueError(f"no dispatch of {kernel!r} in {d}")
        raw = sum(vals) / len(vals) * 1024.0
        res[tag] = {"launches": len(vals), "raw_bytes": raw, "calibration": calib, "bytes": raw * calib}
    res["bytes_per_launch"] = res["fetch"]["bytes"] + res["write"]["bytes"]
    res["kernel"] = kernel
    res["grid"] = grid
    res["sources_sha256"] = sources_hash(sources)
    res["sources"] = list(sources)
    return res


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s1 = sub.add_parser("stats")
    s1.add_argument("dir")
    s1.add_argument("--top", type=int, default=25)
    s2 = sub.add_parser("traffic")
    s2.add_argument("fetch_dir")
    s2.add_argument("write_dir")
    s2.add_argument("--kernel", required=True)
    s2.add_argument("--copy-bytes", type=float, required=True)
    s2.add_argument("--grid", type=int, default=0, help="only dispatches of this grid size (work items)")
    s2.add_argument("--json", default=None)
    s2.add_argument("--sources", choices=sorted(KERNEL_SOURCES), default="smooth",
                    help="kernel class whose source files the summary's hash covers")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        rows = kernel_stats(a.dir)
        tot = sum(r[2] for r in rows)
        print(f"| kernel | calls | total ms | mean us | % |\n|---|---:|---:|---:|---:|")
        for k, c, s, m in rows[:a.top]:
            print(f"| `{k}` | {c} | {s:.2f} | {m:.2f} | {100 * s / tot:.1f} |")
        print(f"\nall kernels: {tot:.2f} ms")
        return 0
    r = traffic(a.fetch_dir, a.write_dir, a.kernel, a.copy_bytes, a.grid, KERNEL_SOURCES[a.sources])
    print(f"kernel /{a.kernel}/: {r['fetch']['launches']} launches; FETCH {r['fetch']['raw_bytes'] / 1e6:.2f} MB raw x "
          f"{r['fetch']['calibration']:.3f} = {r['fetch']['bytes'] / 1e6:.2f} MB; WRITE "
          f"{r['write']['raw_bytes'] / 1e6:.2f} MB raw x {r['write']['calibration']:.3f} = "
          f"{r['write']['bytes'] / 1e6:.2f} MB; traffic {r['bytes_per_launch'] / 1e6:.2f} MB per launch")
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(r, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
