"""Summaries of rocprofv3 output for the solver's kernels.

`stats_summary` condenses a `--kernel-trace --stats --output-format csv` run
(the *_kernel_stats.csv file) into a short text table; `traffic_summary` turns two
`--pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs (the *_counter_collection.csv files)
into HBM bytes per launch for each kernel, scaled by what the same counters read
for a plain device copy of known size that ran in the same process.

    python -m paper_2411_18341_amd.profiling stats <kernel_stats.csv> <command...>
    python -m paper_2411_18341_amd.profiling traffic <fetch.csv> <write.csv> <copy_bytes> <out.json> <workload> [sources...]

(`traffic` adds its kernels to <out.json> when that file holds a measurement of the
same kernel sources and workload, else replaces it; the sources default to the RK4
kernels' files.)
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# sources whose change invalidates a stored counter measurement of the RK4 kernels
KERNEL_SOURCES = ["paper_2411_18341_amd/csrc/rk4.hip", "paper_2411_18341_amd/csrc/stencil.h",
                  "paper_2411_18341_amd/csrc/phx_kernels.h", "paper_2411_18341_amd/csrc/rk4_step.hip",
                  "paper_2411_18341_amd/csrc/step_body.h", "paper_2411_18341_amd/csrc/stream_body.h",
                  "paper_2411_18341_amd/csrc/stream_wide.h", "paper_2411_18341_amd/csrc/rk4_stream_wide.hip"]


def kernel_source_hash(sources=None) -> str:
    """Hash of the kernel sources a counter record was taken on (default: the RK4
    kernels' sources)."""
    h = hashlib.sha256()
    for p in (KERNEL_SOURCES if sources is None else sources):
        path = os.path.join(ROOT, p)
        if os.path.exists(path):
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def kernel_kind(name: str) -> str:
    """Kernel kind as the solver's timing API names it (rk4_stage2, dp_stage7, ...),
    the whole-step kernel with its shape (rk4_step_8x6: 8 waves x 6 rows; the
    streaming form rk4_step_1x40: bands of 40 rows; the wide streaming form
    rk4_step_wide8 / rk4_step_wide12 by its input ring, whatever its band height),
    or a shortened name for other kernels."""
    m = re.search(r"(rk4_stage_kernel|dp_stage_kernel)<[^>]*?(\d+)>", name)
    if m:
        return ("rk4_stage" if m.group(1).startswith("rk4") else "dp_stage") + m.group(2)
    m = re.search(r"rk4_stream_wide_kernel<[^>]*?, (\d+), \d+, \d+(?:, (?:true|false))*>", name)
    if m:  # wide streaming form: named by its input ring (8: shapes 2 x B, 12: shapes 3 x B)
        return f"rk4_step_wide{m.group(1)}"
    m = re.search(r"rk4_step_kernel<[^>]*?(\d+), (\d+)>", name)
    if m:
        return f"rk4_step_{m.group(1)}x{m.group(2)}"
    m = re.search(r"rk4_stream(?:_drive)?_kernel<[^>]*?, (\d+)(?:, (?:true|false))?>", name)
    if m:  # streaming form (also with the drive or in imaginary time): shape 1 x band rows
        return f"rk4_step_1x{m.group(1)}"
    named = {"rk4_step_kernel": "rk4_step", "batch_step_kernel": "batch_step", "dp_restart_kernel": "dp_restart",
             "dp_err_sum_kernel": "dp_error", "obs_pass1": "obs_pass1", "obs_pass2": "obs_pass2",
             "conv_fwd_kernel": "conv_fwd", "conv_bwd_weight_kernel": "conv_bwd_weight",
             "wiener_noise_kernel": "wiener_noise"}
    for k, v in named.items():
        if k in name:
            return v
    return name[:60]


def read_stats(path: str):
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append({"name": r["Name"], "calls": int(r["Calls"]),
                         "total_ns": float(r["TotalDurationNs"]), "avg_ns": float(r["AverageNs"]),
                         "pct": float(r["Percentage"]), "min_ns": float(r["MinNs"]),
                         "max_ns": float(r["MaxNs"])})
    return sorted(rows, key=lambda r: -r["total_ns"])


def stats_summary(path: str, command: str, top: int = 12) -> str:
    rows = read_stats(path)
    out = [f"command: {command}", "",
           f"{'kernel':70s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}"]
    for r in rows[:top]:
        out.append(f"{r['name'][:70]:70s} {r['calls']:6d} {r['avg_ns'] / 1e3:10.2f} "
                   f"{r['min_ns'] / 1e3:10.2f} {r['max_ns'] / 1e3:10.2f} {r['pct']:6.2f}")
    return "\n".join(out) + "\n"


def read_counter(path: str, counter: str):
    """{kernel name: [value per dispatch]} for one counter (summed over its
    dimensions, as rocprofv3 reports one row per dispatch and counter)."""
    per = defaultdict(lambda: defaultdict(float))
    with open(path) as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter:
                continue
            per[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return {k: list(v.values()) for k, v in per.items()}


def traffic_summary(fetch_csv: str, write_csv: str, copy_bytes: float, workload: str, sources=None):
    """Bytes per launch (read, write, total) per kernel, each counter scaled by
    copy_bytes over the counter's mean reading for the copy kernel (a copy reads
    and writes copy_bytes each)."""
    fetch = read_counter(fetch_csv, "FETCH_SIZE")
    write = read_counter(write_csv, "WRITE_SIZE")
    copy_f = [v for k, vs in fetch.items() if "copy" in k for v in vs]
    copy_w = [v for k, vs in write.items() if "copy" in k for v in vs]
    if not copy_f or not copy_w:
        raise RuntimeError("no copy kernel found in the counter runs")
    # FETCH_SIZE and WRITE_SIZE are in KiB
    med = lambda v: sorted(v)[len(v) // 2]
    f_scale = copy_bytes / (1024.0 * med(copy_f))
    w_scale = copy_bytes / (1024.0 * med(copy_w))
    # dispatches of every instantiation of one kernel kind are pooled (the wide
    # streaming kernel has a variant that also tests for non-finite values)
    by_kind_f, by_kind_w = defaultdict(list), defaultdict(list)
    for k in sorted(set(fetch) | set(write)):
        if "copy" in k or not fetch.get(k) or not write.get(k):
            continue
        by_kind_f[kernel_kind(k)] += fetch[k]
        by_kind_w[kernel_kind(k)] += write[k]
    kernels = {}
    for kind in sorted(by_kind_f):
        fr, wr = by_kind_f[kind], by_kind_w[kind]
        rd = sum(fr) / len(fr) * 1024.0 * f_scale
        wb = sum(wr) / len(wr) * 1024.0 * w_scale
        kernels[kind] = {"read_bytes": rd, "write_bytes": wb, "bytes_per_launch": rd + wb,
                         "dispatches": len(fr), "fetch_kib_raw": sum(fr) / len(fr),
                         "write_kib_raw": sum(wr) / len(wr)}
    return {"workload": workload, "source_hash": kernel_source_hash(sources), "fetch_scale": f_scale,
            "write_scale": w_scale, "copy_bytes": copy_bytes, "kernels": kernels}


def main(argv):
    if argv[0] == "stats":
        sys.stdout.write(stats_summary(argv[1], " ".join(argv[2:])))
    elif argv[0] == "traffic":
        # merges into an existing file taken on the same sources and workload
        t = traffic_summary(argv[1], argv[2], float(argv[3]), argv[5], argv[6:] or None)
        if os.path.exists(argv[4]):
            with open(argv[4]) as f:
                old = json.load(f)
            if old.get("source_hash") == t["source_hash"] and old.get("workload") == t["workload"]:
                old["kernels"].update(t["kernels"])
                t["kernels"] = old["kernels"]
        with open(argv[4], "w") as f:
            json.dump(t, f, indent=1)
        print(json.dumps(t, indent=1))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
