"""Summaries of rocprofv3 runs of the benchmark (kernel statistics and the
HBM traffic counters of one whole global trade).

    python -m paper_1804_08487_amd.rocprof_summary --workload large \\
        --trace <dir>/trace_kernel_stats.csv \\
        --fetch <dir>/fetch_counter_collection.csv --write <dir>/write_counter_collection.csv \\
        --copy-fetch <dir>/cfetch_counter_collection.csv --copy-write <dir>/cwrite_counter_collection.csv \\
        --copy-bytes 1073741824 --commands commands.txt

writes profiles/<kernel-or-step>_<workload>_rocprofv3.md and
profiles/traffic_<workload>.json. The counter runs time one warm-up and one
measured round; the round summed here is the last one (every dispatch of the
library's kernels from the last per-round reset on). FETCH_SIZE and
WRITE_SIZE are KiB per dispatch; each is scaled by what it reads for a plain
device copy of known size (the copy reads and writes --copy-bytes).
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def short(name: str) -> str:
    base = name.split("(")[0]
    return base.replace("void ", "").strip()


def kernel_stats(path):
    rows = list(csv.DictReader(open(path)))
    return [(short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e6, float(r["MinNs"]) / 1e6,
             float(r["MaxNs"]) / 1e6, float(r["Percentage"])) for r in rows]


def last_round(path):
    """Per-kernel KiB of the last round (dispatches from the last reset on)."""
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    start = max(i for i, r in enumerate(rows) if "k_round_reset" in r["Kernel_Name"])
    out = {}
    for r in rows[start:]:
        if "cbx::" not in r["Kernel_Name"]:
            continue
        k = short(r["Kernel_Name"])
        out[k] = out.get(k, 0.0) + float(r["Counter_Value"])
    return out


def copy_kib(path):
    rows = list(csv.DictReader(open(path)))
    vals = [float(r["Counter_Value"]) for r in rows if "copy" in r["Kernel_Name"].lower()]
    return max(vals)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-bytes", type=int, required=True)
    ap.add_argument("--commands", required=True, help="text file: the commands that made the inputs")
    ap.add_argument("--out-dir", default=os.path.join(ROOT, "profiles"))
    a = ap.parse_args(argv)
    sys.path.insert(0, ROOT)
    from bench import kernel_source_digest

    stats = kernel_stats(a.trace)
    fetch = last_round(a.fetch)
    write = last_round(a.write)
    cf, cw = copy_kib(a.copy_fetch), copy_kib(a.copy_write)
    fscale = a.copy_bytes / (cf * 1024.0)
    wscale = a.copy_bytes / (cw * 1024.0)
    kernels = {}
    for k in sorted(set(fetch) | set(write)):
        kernels[k] = fetch.get(k, 0.0) * 1024.0 * fscale + write.get(k, 0.0) * 1024.0 * wscale
    step = sum(kernels.values())
    commands = [c.strip() for c in open(a.commands) if c.strip()]
    rec = {"workload": a.workload, "source_sha1": kernel_source_digest(), "kernels": kernels,
           "step_bytes": step, "fetch_kib": fetch, "write_kib": write,
           "copy_calibration": {"bytes": a.copy_bytes, "fetch_kib": cf, "write_kib": cw,
                                "fetch_scale": fscale, "write_scale": wscale},
           "commands": commands}
    os.makedirs(a.out_dir, exist_ok=True)
    with open(os.path.join(a.out_dir, f"traffic_{a.workload}.json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    lines = [f"# rocprofv3: one global trade, {a.workload} workload", "",
             "Commands (run from `/tmp` with `TMPDIR=/tmp`):", ""]
    lines += [f"    {c}" for c in commands]
    lines += ["", "## Kernel statistics", "", "| kernel | calls | avg ms | min ms | max ms | share |",
              "|---|---|---|---|---|---|"]
    lines += [f"| {k} | {c} | {av:.3f} | {mn:.3f} | {mx:.3f} | {p:.2f}% |" for k, c, av, mn, mx, p in stats]
    lines += ["", "## HBM traffic of one round (FETCH_SIZE, WRITE_SIZE; last round of the counter runs)", "",
              f"Copy calibration: a {a.copy_bytes} B device copy reads FETCH_SIZE {cf:.4g} KiB and WRITE_SIZE "
              f"{cw:.4g} KiB, so FETCH_SIZE is scaled by {fscale:.3f} and WRITE_SIZE by {wscale:.3f}.", "",
              "| kernel | FETCH KiB | WRITE KiB | bytes (scaled) |", "|---|---|---|---|"]
    for k in sorted(kernels, key=lambda x: -kernels[x]):
        lines.append(f"| {k} | {fetch.get(k, 0):.4g} | {write.get(k, 0):.4g} | {kernels[k]:.4g} |")
    lines += ["", f"Whole round: {step:.4g} bytes.",
              f"Kernel source digest (bench.py compares it before using these numbers): `{rec['source_sha1']}`.", ""]
    with open(os.path.join(a.out_dir, f"superstep_{a.workload}_rocprofv3.md"), "w") as f:
        f.write("\n".join(lines))
    print(json.dumps({"step_bytes": step, "kernels": len(kernels)}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
