"""Summaries of rocprofv3 output for the step kernel (measurement helper).

    python -m paper_1211_6932_amd.prof trace DIR
        kernel-trace statistics (rocprofv3 --kernel-trace --stats --output-format csv)

    python -m paper_1211_6932_amd.prof traffic FETCH_DIR WRITE_DIR --store f32 --sites N [--out FILE]
        HBM bytes per step launch from two counter runs (--pmc FETCH_SIZE, --pmc WRITE_SIZE),
        each scaled by what the same counter reports for the 1 GiB copy probe of the same
        run (read 1 GiB, write 1 GiB); optionally records the result for bench.py.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the kernel sources and the build script that fixes their compiler flags
KERNEL_SOURCES = ["paper_1211_6932_amd/csrc/d2q9_core.hpp", "paper_1211_6932_amd/csrc/d2q9_kernels.hip",
                  "paper_1211_6932_amd/build.py"]
COPY_BYTES = 1 << 30


def kernel_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _find(d, suffix):
    hits = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def trace(d):
    path = _find(d, "kernel_stats.csv")
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        out.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                    float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    out.sort(key=lambda t: -t[5])
    lines = [f"{'kernel':70s} {'calls':>6s} {'avg_us':>9s} {'min_us':>9s} {'max_us':>9s} {'pct':>6s}"]
    for n, c, a, mn, mx, p in out:
        lines.append(f"{n[:70]:70s} {c:6d} {a:9.2f} {mn:9.2f} {mx:9.2f} {p:6.2f}")
    return "\n".join(lines), out


def _counter_by_kernel(d, counter):
    path = _find(d, "counter_collection.csv")
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def _is_step_kernel(name):
    """A time-step kernel: d2q9_strip<store, walls, MODE = 0, psi form>, or the
    two-columns-per-lane d2q9_pair<walls, psi form>."""
    if re.search(r"d2q9_pair(<|I)", name):  # the profiler may leave this name mangled
        return True
    m = re.search(r"d2q9_strip<(\d+), (true|false), (\d+), (\d+)>", name)
    return bool(m) and m.group(3) == "0"


def traffic(fetch_dir, write_dir, store, sites):
    res = {}
    for counter, d, key in (("FETCH_SIZE", fetch_dir, "read"), ("WRITE_SIZE", write_dir, "write")):
        vals = _counter_by_kernel(d, counter)
        step = [v for k, v in vals.items() if _is_step_kernel(k)]
        copy = [v for k, v in vals.items() if "copy_probe" in k]
        if not step or not copy:
            raise RuntimeError(f"{counter}: step or copy-probe dispatches missing in {d}")
        step_kib = statistics.median(step[0])
        copy_kib = statistics.median(copy[0])
        scale = COPY_BYTES / (copy_kib * 1024.0)
        res[key] = dict(counter_kib_per_launch=step_kib, copy_counter_kib=copy_kib, scale=scale,
                        bytes_per_launch=step_kib * 1024.0 * scale)
    bps = {"f32": 72, "f16": 36, "bf16": 36, "f16local": 44, "bf16local": 44, "f16dest": 40}[store]
    total = res["read"]["bytes_per_launch"] + res["write"]["bytes_per_launch"]
    return dict(store=store, sites=sites, kernel_sha=kernel_hash(), bytes_per_launch=total,
                algorithmic_bytes=bps * sites, ratio=total / (bps * sites), detail=res)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    f = sub.add_parser("traffic")
    f.add_argument("fetch_dir")
    f.add_argument("write_dir")
    f.add_argument("--store", default="f32")
    f.add_argument("--sites", type=int, required=True)
    f.add_argument("--out", default=None, help="JSON file to record the result in (keyed by store)")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace(a.dir)[0])
    else:
        r = traffic(a.fetch_dir, a.write_dir, a.store, a.sites)
        print(json.dumps(r, indent=1))
        if a.out:
            doc = {}
            if os.path.exists(a.out):
                with open(a.out) as fh:
                    doc = json.load(fh)
            doc[a.store] = r
            with open(a.out, "w") as fh:
                json.dump(doc, fh, indent=1)


if __name__ == "__main__":
    sys.exit(main())
