"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_1604_06043_amd.prof KT_DIR FETCH_DIR WRITE_DIR OUT.md \
        --kernel k_spmv --command "..." [--json OUT.json]

KT_DIR holds a ``--kernel-trace --stats --output-format csv`` run, FETCH_DIR and
WRITE_DIR one ``--pmc FETCH_SIZE`` and one ``--pmc WRITE_SIZE`` run of the same
command.  The byte counters are scaled by what they read for the largest
device-to-device copy in the same run (a plain copy of known size: reads and
writes each equal the copied bytes), so ``traffic`` is in real HBM bytes.

The JSON record carries the SHA-256 of the kernel source it was taken with
(kernels.hpp by default); bench.py reports the traffic only while that file
is unchanged.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
# the solver's kernels live in kernels.hpp (solver.hip holds the host side)
KERNEL_SOURCES = [os.path.join(HERE, "csrc", "kernels.hpp")]


def sources_digest(files=None) -> str:
    h = hashlib.sha256()
    for f in (files or KERNEL_SOURCES):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _find(d: str, suffix: str) -> str:
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffix} under {d}")


def kernel_stats(kt_dir: str):
    rows = list(csv.DictReader(open(_find(kt_dir, "kernel_stats.csv"))))
    out = []
    for r in rows:
        out.append({"name": r["Name"], "calls": int(r["Calls"]),
                    "avg_us": float(r["AverageNs"]) / 1e3, "min_us": float(r["MinNs"]) / 1e3,
                    "max_us": float(r["MaxNs"]) / 1e3, "pct": float(r["Percentage"])})
    return out


def counters(pmc_dir: str):
    per = defaultdict(list)
    for r in csv.DictReader(open(_find(pmc_dir, "counter_collection.csv"))):
        per[r["Kernel_Name"]].append(float(r["Counter_Value"]))   # KiB per dispatch
    return per


def calibration(per: dict, copy_bytes: int) -> float:
    """Factor that turns the counter's KiB into bytes, from the largest copy."""
    best = 0.0
    for name, vals in per.items():
        if "copyBuffer" in name or "elementwise" in name:
            best = max(best, max(vals))
    if best <= 0:
        raise ValueError("no copy kernel in the counter run")
    return copy_bytes / best


def summarize(kt_dir, fetch_dir, write_dir, kernel, command, copy_bytes=256 << 20, sources=None):
    stats = kernel_stats(kt_dir)
    fetch, write = counters(fetch_dir), counters(write_dir)
    fs, ws = calibration(fetch, copy_bytes), calibration(write, copy_bytes)
    sel = [s for s in stats if kernel in s["name"]]
    traffic = {}
    for name in {n for n in fetch if kernel in n} | {n for n in write if kernel in n}:
        f = statistics.mean(fetch.get(name, [0.0])) * fs
        w = statistics.mean(write.get(name, [0.0])) * ws
        traffic[name] = {"fetch_bytes": f, "write_bytes": w, "traffic_bytes": f + w,
                         "dispatches": len(fetch.get(name, []))}
    return {"command": command, "kernel": kernel, "stats": stats, "selected": sel,
            "fetch_scale": fs, "write_scale": ws, "traffic": traffic,
            "sources_sha256": sources_digest(sources)}


def write_md(summary: dict, path: str, title: str):
    lines = [f"# {title}", "", "Command (from the repository root, on an MI355X):", "",
             "```", summary["command"], "```", "",
             "## Kernel durations (rocprofv3 --kernel-trace --stats)", "",
             "| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for s in summary["stats"][:14]:
        lines.append(f"| `{s['name'][:90]}` | {s['calls']} | {s['avg_us']:.2f} | {s['min_us']:.2f} | "
                     f"{s['max_us']:.2f} | {s['pct']:.2f} |")
    lines += ["", "## HBM bytes per dispatch (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)", "",
              f"Scale factors from the 256 MiB device copy in the same run: FETCH x{summary['fetch_scale']:.3f}, "
              f"WRITE x{summary['write_scale']:.3f} (KiB counter -> bytes).", "",
              "| kernel | dispatches | read MB | written MB | traffic MB |", "|---|---|---|---|---|"]
    for name, t in sorted(summary["traffic"].items()):
        lines.append(f"| `{name[:90]}` | {t['dispatches']} | {t['fetch_bytes'] / 1e6:.1f} | "
                     f"{t['write_bytes'] / 1e6:.1f} | {t['traffic_bytes'] / 1e6:.1f} |")
    lines += ["", f"Kernel sources SHA-256: `{summary['sources_sha256']}`", ""]
    with open(path, "w") as fh:
        fh.write("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("kt_dir")
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("out_md")
    ap.add_argument("--kernel", default="k_spmv")
    ap.add_argument("--command", required=True)
    ap.add_argument("--title", default="Kernel profile")
    ap.add_argument("--json")
    ap.add_argument("--sources", nargs="*", help="kernel source files (under csrc/) of the digest")
    a = ap.parse_args()
    srcs = [os.path.join(HERE, "csrc", f) for f in a.sources] if a.sources else None
    s = summarize(a.kt_dir, a.fetch_dir, a.write_dir, a.kernel, a.command, sources=srcs)
    write_md(s, a.out_md, a.title)
    if a.json:
        rec = {"kernel": a.kernel, "sources_sha256": s["sources_sha256"], "command": a.command,
               "traffic": s["traffic"],
               "avg_us": {x["name"]: x["avg_us"] for x in s["selected"]}}
        with open(a.json, "w") as fh:
            json.dump(rec, fh, indent=1)


if __name__ == "__main__":
    main()
