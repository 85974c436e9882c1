"""Summaries of rocprofv3 output for the spatial pooler kernels.

``python -m paper_1608_01966_amd.profiling summarize --trace DIR [--fetch DIR]
[--write DIR] --kernel NAME --workload TEXT --command TEXT > profiles/<file>.md``

reads the CSV files rocprofv3 writes with ``-f csv`` (kernel stats from
``--kernel-trace --stats``; per-dispatch counters from ``--pmc FETCH_SIZE``
and ``--pmc WRITE_SIZE``) and prints a short Markdown summary.  Memory
counters are calibrated against the elementwise int32 copy the benchmark
launches with ``--calibration-copy-mb``: the copy's known byte count divided
by what each counter reports for it is that counter's scale factor.

The summary ends with a JSON block (per-launch counter bytes and the SHA-256
of the kernel source they were taken from) that ``bench.py`` reads to report
measured HBM traffic, and ignores once the source has changed.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
# the source files each profiled kernel is compiled from
KERNEL_SOURCES = {
    "k_sp_persistent_w": ("sp_kernels.hip", "sp_device.h", "sp_internal.h"),
    "k_pair_frames": ("sp_kernels.hip", "sp_device.h", "sp_internal.h"),
    "k_sp_persistent_local": ("sp_local.hip", "sp_device.h", "sp_internal.h"),
    "k_sp_persistent_local2": ("sp_local.hip", "sp_device.h", "sp_internal.h"),
    "k_sp_persistent_boost": ("sp_boost.hip", "sp_device.h", "sp_internal.h"),
    "k_infer_gather": ("sp_infer.hip", "sp_device.h", "sp_internal.h"),
    "k_infer_gather_db": ("sp_infer.hip", "sp_device.h", "sp_internal.h"),
    "k_topk_batch": ("sp_infer.hip", "sp_device.h", "sp_internal.h"),
    "k_infer_mfma": ("sp_infer_mfma.hip", "sp_device.h", "sp_internal.h"),
    "k_mfma_reduce": ("sp_infer_mfma.hip", "sp_device.h", "sp_internal.h"),
    "k_sp_many": ("sp_many.hip", "sp_device.h", "sp_internal.h"),
    "k_encode": ("sp_encode.hip", "sp_device.h", "sp_internal.h"),
    "k_zero": ("sp_encode.hip", "sp_device.h", "sp_internal.h"),
}
COPY_KERNEL = "vectorized_elementwise_kernel"


def kernels_of(spec: str) -> list[str]:
    """'a+b' -> ['a', 'b']: a profiled unit may be several kernels launched
    back to back by one library call."""
    return [k for k in spec.split("+") if k]


def source_sha256(spec: str) -> str:
    files = []
    for k in kernels_of(spec):
        files += [f for f in KERNEL_SOURCES[k] if f not in files]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(PKG, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise FileNotFoundError(pattern)
    return hits[0]


def kernel_stats(trace_dir: str) -> list[dict]:
    with open(_one(os.path.join(trace_dir, "**", "*kernel_stats.csv"))) as f:
        return list(csv.DictReader(f))


def counters(pmc_dir: str, name: str) -> list[dict]:
    with open(_one(os.path.join(pmc_dir, "**", "*counter_collection.csv"))) as f:
        return [r for r in csv.DictReader(f) if r["Counter_Name"] == name]


def calibrated(pmc_dir: str, name: str, kernel: str, copy_bytes: int):
    """(KiB per launch of `kernel`, scale factor from the copy kernel)."""
    rows = counters(pmc_dir, name)
    copy = [float(r["Counter_Value"]) for r in rows if r["Kernel_Name"].startswith(COPY_KERNEL)]
    # the copy is the elementwise kernel that moves the most data
    factor = copy_bytes / 1024.0 / max(copy) if copy and max(copy) > 0 else None
    kib, n = 0.0, None
    for k in kernels_of(kernel):
        ours = [float(r["Counter_Value"]) for r in rows if r["Kernel_Name"] == k]
        if not ours:
            return None, factor, 0
        kib += sum(ours) / len(ours)
        n = len(ours) if n is None else min(n, len(ours))
    return kib, factor, n


def summarize(args) -> str:
    out = [f"# rocprofv3 summary: `{args.kernel}`, {args.workload}", ""]
    out += ["Command (from the repository root):", "", "```", args.command, "```", ""]
    stats = kernel_stats(args.trace)
    out += ["## Kernel trace statistics (`--kernel-trace --stats`)", "",
            "| kernel | calls | average (us) | min (us) | max (us) | share |",
            "|---|---|---|---|---|---|"]
    for r in stats:
        out.append(f"| {r['Name']} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['Percentage']):.1f}% |")
    out.append("")
    block = {"kernel": args.kernel, "workload": args.workload,
             "source_sha256": source_sha256(args.kernel)}
    avg = [float(r["AverageNs"]) for k in kernels_of(args.kernel) for r in stats
           if r["Name"] == k]
    if len(avg) == len(kernels_of(args.kernel)):
        block["trace_avg_ms"] = sum(avg) / 1e6
    copy_bytes = args.copy_mb * (1 << 20)
    if args.fetch and args.write:
        fk, ff, nf = calibrated(args.fetch, "FETCH_SIZE", args.kernel, copy_bytes)
        wk, wf, nw = calibrated(args.write, "WRITE_SIZE", args.kernel, copy_bytes)
        out += ["## Memory counters (`--pmc FETCH_SIZE`, then `--pmc WRITE_SIZE`)", "",
                f"Calibration: an elementwise int32 copy of {args.copy_mb} MiB reads and writes "
                f"{args.copy_mb} MiB; FETCH_SIZE scale factor {ff:.3f}, WRITE_SIZE scale factor "
                f"{wf:.3f}.", "",
                "| counter | KiB per launch (raw) | launches | scaled bytes per launch |",
                "|---|---|---|---|",
                f"| FETCH_SIZE | {fk:.1f} | {nf} | {fk * ff * 1024:.4g} |",
                f"| WRITE_SIZE | {wk:.1f} | {nw} | {wk * wf * 1024:.4g} |", ""]
        block.update({"fetch_kib_per_launch": fk, "write_kib_per_launch": wk,
                      "fetch_factor": ff, "write_factor": wf,
                      "hbm_bytes_per_launch": fk * ff * 1024 + wk * wf * 1024})
    out += ["## Machine-readable", "", "```json", json.dumps(block, indent=1), "```", ""]
    return "\n".join(out)


def read_block(md_path: str) -> dict | None:
    """The JSON block of a summary, or None."""
    try:
        text = open(md_path).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    return json.loads(m.group(1)) if m else None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("summarize")
    s.add_argument("--trace", required=True)
    s.add_argument("--fetch")
    s.add_argument("--write")
    s.add_argument("--kernel", required=True, help="kernel name, or names joined by '+'")
    s.add_argument("--workload", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--copy-mb", type=int, default=256)
    args = ap.parse_args()
    print(summarize(args))


if __name__ == "__main__":
    main()
