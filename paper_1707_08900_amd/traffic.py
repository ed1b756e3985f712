"""HBM traffic of a kernel from two rocprofv3 counter passes.

rocprofv3 --pmc FETCH_SIZE (one run) and --pmc WRITE_SIZE (another run) of the
same command write per-dispatch counter values in KiB.  The command also runs
a plain 1 GiB device copy (bench.py --calibrate-copy), whose true traffic is
1 GiB read and 1 GiB written; the ratio to what the counters report for it is
the scale applied to every kernel's values.  This module turns the two CSV
files into per-kernel bytes per dispatch, and adds (or replaces) the record
of that kernel shape, z-chunk and layout in the file bench.py reads for its
roofline's `traffic`.

    python -m paper_1707_08900_amd.traffic FETCH_DIR WRITE_DIR --match substep55_sweep \\
        --alg-bytes-per-launch 7158278826.67 [--record profiles/traffic_....json ...]
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import statistics
import sys
from collections import defaultdict

COPY_KERNEL = "copyBuffer"  # the runtime's device-to-device copy kernel
COPY_KIB = 1 << 20          # 1 GiB moved each way by the calibration copy


def read_counters(path: str, counter: str):
    """{kernel name: [value per dispatch]} from a counter-collection CSV (or a
    directory searched for one)."""
    files = [path] if os.path.isfile(path) else glob.glob(
        os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {path}")
    out = defaultdict(list)
    for fn in files:
        with open(fn, newline="") as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name") == counter:
                    out[row["Kernel_Name"]].append(float(row["Counter_Value"]))
    return out


def scale_of(values, expect_kib):
    """Counter scale from the calibration copy: the largest dispatches of the
    runtime's copy kernel (the same kernel also serves the program's smaller
    device copies, which are left out)."""
    copy = [v for k, vs in values.items() if COPY_KERNEL in k for v in vs]
    if not copy:
        raise ValueError("the calibration copy kernel is missing (run with --calibrate-copy)")
    top = max(copy)
    return expect_kib / statistics.median([v for v in copy if v >= 0.9 * top])


def summarize(fetch_dir, write_dir, match):
    fetch = read_counters(fetch_dir, "FETCH_SIZE")
    write = read_counters(write_dir, "WRITE_SIZE")
    fs, ws = scale_of(fetch, COPY_KIB), scale_of(write, COPY_KIB)
    kernels = {}
    for name in sorted(set(fetch) | set(write)):
        if match not in name:
            continue
        f, w = fetch.get(name, []), write.get(name, [])
        kernels[name] = {"dispatches": max(len(f), len(w)),
                         "fetch_kib": statistics.mean(f) if f else 0.0,
                         "write_kib": statistics.mean(w) if w else 0.0,
                         "read_bytes": (statistics.mean(f) if f else 0.0) * fs * 1024,
                         "write_bytes": (statistics.mean(w) if w else 0.0) * ws * 1024}
    return {"fetch_scale": fs, "write_scale": ws, "kernels": kernels}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("fetch_dir")
    ap.add_argument("write_dir")
    ap.add_argument("--match", required=True, help="substring of the kernel names to report")
    ap.add_argument("--alg-bytes-per-launch", type=float, default=None)
    ap.add_argument("--record", default=None, help="write the bench.py traffic record here")
    ap.add_argument("--record-field", action="append", default=[],
                    help="extra key=value pairs for the record (kernel, workload, tile, ...)")
    a = ap.parse_args(argv)
    s = summarize(a.fetch_dir, a.write_dir, a.match)
    tot = []
    for name, k in s["kernels"].items():
        b = k["read_bytes"] + k["write_bytes"]
        tot.append(b)
        extra = (f", {b / a.alg_bytes_per_launch:.3f}x algorithmic"
                 if a.alg_bytes_per_launch else "")
        print(f"{name}: {k['dispatches']} dispatches, FETCH {k['fetch_kib']:.0f} KiB, WRITE "
              f"{k['write_kib']:.0f} KiB -> read {k['read_bytes'] / 1e9:.3f} GB, write "
              f"{k['write_bytes'] / 1e9:.3f} GB per dispatch{extra}")
    print(f"scales: FETCH {s['fetch_scale']:.4f}, WRITE {s['write_scale']:.4f}")
    if a.record and tot:
        rec = {"traffic_bytes_per_launch": sum(tot) / len(tot),
               "per_kernel_bytes": {n: k["read_bytes"] + k["write_bytes"]
                                    for n, k in s["kernels"].items()},
               "fetch_scale": s["fetch_scale"], "write_scale": s["write_scale"]}
        for kv in a.record_field:
            k, v = kv.split("=", 1)
            rec[k] = int(v) if v.lstrip("-").isdigit() else v
        # one record per (kernel shape, z-chunk, layout): replace that one
        try:
            with open(a.record) as f:
                doc = json.load(f)
            records = doc.get("records", []) if isinstance(doc, dict) else []
        except (OSError, ValueError):
            records = []
        key = lambda r: (r.get("tile"), r.get("zchunk"), r.get("layout"))  # noqa: E731
        records = [r for r in records if key(r) != key(rec)] + [rec]
        with open(a.record, "w") as f:
            json.dump({"records": records}, f, indent=1)
            f.write("\n")
        print(f"record written to {a.record}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
