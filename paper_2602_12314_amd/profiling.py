"""Summaries of rocprofv3 CSV output for the library's kernels.

    python -m paper_2602_12314_amd.profiling stats DIR [--by-grid] [--top N]
        per-kernel calls, total and average duration from a
        ``rocprofv3 --kernel-trace --stats --output-format csv -d DIR`` run
        (markdown table); with --by-grid, from the kernel trace per (kernel,
        grid size), so that one launch shape's average is not mixed with the
        same kernel's launches at other sizes.

    python -m paper_2602_12314_amd.profiling counters DIR [KERNEL_PREFIX]
        mean value per dispatch of every counter of a ``--pmc`` run, by kernel.

    python -m paper_2602_12314_amd.profiling traffic --workload NAME \\
            --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR --copy-bytes N [--only STAGES]
            [--largest-grid] [--options JSON]
        HBM bytes per launch of each kernel from two ``--pmc FETCH_SIZE`` /
        ``--pmc WRITE_SIZE`` runs, each counter scaled by what it reads for a
        plain device copy of N bytes (``bench.py --copy-calibration N`` under the
        same counter).  Prints a markdown table and, with ``--json FILE``, merges
        the figures into FILE keyed by workload and the bench's stage names,
        together with the hash of the kernel sources they were taken on.

    python -m paper_2602_12314_amd.profiling timeline DIR [--step K]
        the launches of one step of a ``--kernel-trace`` run in start order,
        from the K-th projection launch (``k_preprocess``; default the third
        from last) to the next: start and end relative to the step's first
        launch and the duration, in microseconds.  Launches on the two streams
        of a step interleave, so overlapping rows show what ran beside what.

Counter values are KiB per dispatch (rocprofv3's derived FETCH_SIZE and
WRITE_SIZE).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")

# bench stage name -> (kernel name prefix in the trace, source files it is built from)
STAGES = {
    "decode_rows": ("k_dec_rows", ["decode.hip", "common.h", "kernels.h"]),
    "decode_tn": ("k_dec_dv", ["decode.hip", "common.h", "kernels.h"]),
    "raster_fwd": ("k_raster_fwd", ["render.hip", "common.h", "kernels.h"]),
    "raster_bwd": ("k_raster_bwd", ["render.hip", "common.h", "kernels.h"]),
    "kmeans_assign": ("k_km_assign", ["kmeans.hip", "kmeans.h", "common.h", "kernels.h"]),
}


def source_hash(files) -> str:
    """Hash of the named files under csrc/ (what a counter figure was taken on)."""
    h = hashlib.sha256()
    for name in sorted(files):
        with open(os.path.join(CSRC, name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    name = name.replace("lam::", "").replace("km::", "").replace("void ", "")
    i = name.find("(")
    return name[:i] if i > 0 else name


def _one(d, pattern):
    f = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not f:
        raise FileNotFoundError(f"no {pattern} under {d}")
    return f[0]


def kernel_stats(d):
    rows = list(csv.DictReader(open(_one(d, "*kernel_stats.csv"))))
    return [(short(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
             float(r["AverageNs"]) / 1e3, float(r["Percentage"])) for r in rows]


def kernel_stats_by_grid(d):
    """(kernel, grid threads, calls, total us, average us) from the kernel trace."""
    acc = defaultdict(list)
    for r in csv.DictReader(open(_one(d, "*kernel_trace.csv"))):
        g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        acc[(short(r["Kernel_Name"]), g)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    rows = [(k, g, len(v), sum(v), sum(v) / len(v)) for (k, g), v in acc.items()]
    return sorted(rows, key=lambda x: -x[3])


def counter_means(d, counter, largest_grid=False):
    """Mean counter value per dispatch, by kernel (with largest_grid, over the
    dispatches of the kernel's largest grid only)."""
    acc = defaultdict(list)
    for r in csv.DictReader(open(_one(d, "*counter_collection.csv"))):
        if r.get("Counter_Name") == counter:
            acc[short(r["Kernel_Name"])].append((int(r.get("Grid_Size") or 0), float(r["Counter_Value"])))
    out = {}
    for k, v in acc.items():
        if largest_grid:
            gmax = max(g for g, _ in v)
            v = [x for x in v if x[0] == gmax]
        out[k] = sum(x for _, x in v) / len(v)
    return out


def copy_factor(d, counter, copy_bytes):
    """Bytes per KiB of counter for the plain copy kernel (true bytes / counted)."""
    m = counter_means(d, counter)
    ks = [k for k in m if "copyBuffer" in k]
    if not ks:
        raise RuntimeError(f"no copy kernel in {d}")
    return copy_bytes / (m[ks[0]] * 1024.0)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--by-grid", action="store_true")
    s.add_argument("--top", type=int, default=0)
    c = sub.add_parser("counters")
    c.add_argument("dir")
    c.add_argument("prefix", nargs="?", default="")
    tl = sub.add_parser("timeline")
    tl.add_argument("dir")
    tl.add_argument("--step", type=int, default=-3)
    t = sub.add_parser("traffic")
    t.add_argument("--workload", required=True)
    for k in ("fetch", "write", "copy-fetch", "copy-write"):
        t.add_argument("--" + k, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--json", default=None)
    t.add_argument("--only", default=None, help="comma-separated stage names to record (default: all found)")
    t.add_argument("--largest-grid", action="store_true",
                   help="average only the dispatches of each kernel's largest grid")
    t.add_argument("--options", default=None, metavar="JSON",
                   help="launch options the counter runs were pinned to (tile, decode shape, "
                        "split count), recorded beside the figures")
    a = ap.parse_args(argv)
    if a.cmd == "stats" and a.by_grid:
        rows = kernel_stats_by_grid(a.dir)
        tot = sum(r[3] for r in rows)
        print("| kernel | grid (threads) | calls | total us | avg us | % |")
        print("|---|---|---|---|---|---|")
        for k, g, calls, t, avg in rows[:a.top or None]:
            print(f"| {k} | {g} | {calls} | {t:.1f} | {avg:.2f} | {100 * t / tot:.1f} |")
        return 0
    if a.cmd == "stats":
        print("| kernel | calls | total us | avg us | % |")
        print("|---|---|---|---|---|")
        for k, calls, tot, avg, pct in kernel_stats(a.dir):
            print(f"| {k} | {calls} | {tot:.1f} | {avg:.2f} | {pct:.1f} |")
        return 0
    if a.cmd == "timeline":
        rows = sorted(csv.DictReader(open(_one(a.dir, "*kernel_trace.csv"))), key=lambda r: int(r["Start_Timestamp"]))
        pre = [i for i, r in enumerate(rows) if short(r["Kernel_Name"]) == "k_preprocess"]
        if len(pre) < 2:
            raise SystemExit("fewer than two k_preprocess launches in the trace")
        k = a.step % len(pre)
        if k + 1 >= len(pre):
            raise SystemExit("the chosen step has no following k_preprocess launch")
        i, j = pre[k], pre[k + 1]
        t0 = int(rows[i]["Start_Timestamp"])
        print("| start us | end us | duration us | kernel | grid (threads) |")
        print("|---|---|---|---|---|")
        for r in rows[i:j]:
            s0, e0 = int(r["Start_Timestamp"]) - t0, int(r["End_Timestamp"]) - t0
            print(f"| {s0 / 1e3:.2f} | {e0 / 1e3:.2f} | {(e0 - s0) / 1e3:.2f} | {short(r['Kernel_Name'])} "
                  f"| {r['Grid_Size_X']} |")
        print(f"\nnext step's projection starts at {(int(rows[j]['Start_Timestamp']) - t0) / 1e3:.2f} us")
        return 0
    if a.cmd == "counters":
        acc = defaultdict(lambda: defaultdict(list))
        for r in csv.DictReader(open(_one(a.dir, "*counter_collection.csv"))):
            k = short(r["Kernel_Name"])
            if k.startswith(a.prefix):
                acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
        for k in sorted(acc):
            print(f"{k}: " + ", ".join(f"{c}={sum(v) / len(v):.6g}" for c, v in sorted(acc[k].items())))
        return 0
    ff = copy_factor(a.copy_fetch, "FETCH_SIZE", a.copy_bytes)
    fw = copy_factor(a.copy_write, "WRITE_SIZE", a.copy_bytes)
    fetch = counter_means(a.fetch, "FETCH_SIZE", a.largest_grid)
    write = counter_means(a.write, "WRITE_SIZE", a.largest_grid)
    print(f"copy calibration: FETCH_SIZE x {ff:.3f}, WRITE_SIZE x {fw:.3f} "
          f"({a.copy_bytes} bytes copied per launch)")
    print("| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes per launch (scaled) |")
    print("|---|---|---|---|")
    for k in sorted(set(fetch) | set(write)):
        b = fetch.get(k, 0.0) * 1024 * ff + write.get(k, 0.0) * 1024 * fw
        print(f"| {k} | {fetch.get(k, 0.0):.1f} | {write.get(k, 0.0):.1f} | {b:.4g} |")
    if a.json:
        try:
            rec = json.load(open(a.json))
        except (OSError, ValueError):
            rec = {}
        ent = rec.setdefault(a.workload, {})
        only = set(a.only.split(",")) if a.only else None
        for stage, (prefix, files) in STAGES.items():
            if only is not None and stage not in only:
                continue
            ks = [k for k in set(fetch) & set(write) if k.startswith(prefix)]
            if len(ks) != 1:
                continue
            k = ks[0]
            ent[stage] = {"kernel": k, "fetch_kib": fetch[k], "write_kib": write[k],
                          "fetch_factor": ff, "write_factor": fw,
                          "bytes_per_launch": fetch[k] * 1024 * ff + write[k] * 1024 * fw,
                          "source_hash": source_hash(files)}
            if a.options:
                ent[stage]["options"] = json.loads(a.options)
        with open(a.json, "w") as fh:
            json.dump(rec, fh, indent=1, sort_keys=True)
            fh.write("\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
