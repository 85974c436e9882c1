"""Benchmark: HTM spatial pooler steps on one MI355X.

A step is one pass of the whole hot path (overlap, global top-k inhibition,
permanence learning) over one batch of synthetic frames: 1000 sequential
learning frames of a 960x540 binary input (~5% on, as random 8x8 blobs)
through one spatial pooler of 1024 columns x 256 potential synapses,
min_overlap 4, 40 winners, threshold 0.5, inc 8/256, dec 4/256.  Frames are
resident in HBM before the timed region starts.

Prints one JSON line (rank 0) with frames/s, the roofline of the dominant
kernel (the persistent step) and the oracle timed on the host as a CPU
baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
PROFILE = os.path.join(ROOT, "profiles", "k_sp_persistent_960x540_1024c_256s.md")


def algorithmic_bytes(cfg: dict, winners: np.ndarray) -> int:
    """Bytes one spatial pooler frame must move at minimum in the library's
    layout, summed over frames: the packed frame, idx + perm of every
    potential synapse (overlap), read-modify-write of perm plus the idx read
    for each winner's synapses (learning), overlaps and winners written."""
    W = (cfg["input_bits"] + 31) // 32
    C, S, k = cfg["num_columns"], cfg["synapses_per_column"], cfg["winners"]
    F = winners.shape[0]
    n_win = int((winners >= 0).sum())
    return F * (4 * W + 8 * C * S + 4 * C + 4 * k) + 12 * S * n_win


def cpu_baseline(w, budget_s: float) -> dict:
    """The oracle, single-threaded, on the first frames of the same workload
    (as many as fit the time budget, doubling from 25)."""
    import oracle
    n = 25
    while True:
        t0 = time.perf_counter()
        oracle.run(w.cfg, w.idx, w.perm, w.frames[:n], learn=True, want_overlaps=False)
        dt = time.perf_counter() - t0
        if dt > budget_s / 3 or n >= w.frames.shape[0]:
            break
        n = min(2 * n, w.frames.shape[0])
    return {"value": n / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} frames of the same 1000-frame learning workload "
                      f"from the same initial state, {dt:.2f} s single-threaded"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--frames", type=int, default=1000)
    ap.add_argument("--columns", type=int, default=1024)
    ap.add_argument("--synapses", type=int, default=256)
    ap.add_argument("--plain-frames", type=int, default=200,
                    help="frames timed through the one-frame-per-launch path (0: skip)")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibration-copy-mb", type=int, default=0,
                    help="before timing, run one elementwise int32 copy of this many MiB "
                         "(reads and writes that many bytes) to calibrate memory counters")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the spatial pooler step is benchmarked on "
              "a single device and no multi-GPU path exists", file=sys.stderr)
        return 2

    import torch
    import paper_1608_01966_amd as sp
    from paper_1608_01966_amd import synth

    torch.cuda.set_device(0)
    w = synth.workload_paper_scale(frames=args.frames, columns=args.columns,
                                   synapses=args.synapses)
    cfg = w.cfg
    C, S, k = cfg["num_columns"], cfg["synapses_per_column"], cfg["winners"]
    frames = torch.from_numpy(np.ascontiguousarray(w.frames).view(np.int32)).cuda()
    F = frames.shape[0]

    if args.calibration_copy_mb > 0:
        n = args.calibration_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.add(src, 1, out=dst)
        torch.cuda.synchronize()
        del src, dst

    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    perm0 = pool.perm.clone()
    stream = torch.cuda.current_stream()
    ov = torch.empty((F, C), dtype=torch.int32, device="cuda")
    win = torch.empty((F, k), dtype=torch.int32, device="cuda")

    # Every step learns the same frames from the same initial state (without
    # boosting, a pooler that keeps learning on random frames disconnects most
    # synapses, and later steps would time a different workload).  The 1 MB
    # reset copy stays inside the timed region.
    def step():
        pool.perm.copy_(perm0)
        sp.sp_step(pool.handle, cfg, frames, True, ov, win, stream)

    for _ in range(args.warmup):
        step()
    pool.sync()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        pool.perm.copy_(perm0)
        starts[i].record(stream)
        sp.sp_step(pool.handle, cfg, frames, True, ov, win, stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pool.sync()
    wall_s = t1 - t0
    kernel_ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
    ms_per_step = wall_s / args.steps * 1e3
    fps = args.steps * F / wall_s

    win_np = win.cpu().numpy()
    abytes = algorithmic_bytes(cfg, win_np)
    achieved = abytes / (kernel_ms * 1e-3) / 1e9

    # Measured HBM traffic from the committed counter summary, only while the
    # kernel source is the one the counters were taken from.
    from paper_1608_01966_amd import profiling
    traffic, traffic_bytes = None, None
    blk = profiling.read_block(PROFILE)
    if (blk and blk.get("source_sha256") == profiling.source_sha256()
            and (C, S, F) == (1024, 256, 1000) and "hbm_bytes_per_launch" in blk):
        traffic_bytes = blk["hbm_bytes_per_launch"]
        traffic = traffic_bytes / (kernel_ms * 1e-3) / 1e9

    plain = None
    if args.plain_frames > 0:
        pf = min(args.plain_frames, F)
        ppool = sp.SpatialPooler(cfg, w.idx, w.perm)
        pov = torch.empty((pf, C), dtype=torch.int32, device="cuda")
        pwin = torch.empty((pf, k), dtype=torch.int32, device="cuda")
        sp.sp_step_plain(ppool.handle, cfg, frames[:pf], True, pov, pwin, stream)
        ppool.perm.copy_(perm0)
        ppool.sync()
        tp0 = time.perf_counter()
        sp.sp_step_plain(ppool.handle, cfg, frames[:pf], True, pov, pwin, stream)
        ppool.sync()
        plain = pf / (time.perf_counter() - tp0)
        ppool.close()

    cpu = None if args.no_cpu_baseline else cpu_baseline(w, args.cpu_budget)

    line = {
        "metric": "SP frames/s (1024 columns x 256 synapses, learning on)",
        "value": fps,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"960x540 blob frames (~5% on), {C} columns x {S} synapses, "
                               f"min_overlap {cfg['min_overlap']}, {k} winners, "
                               f"{F} sequential learning frames per step",
                   "frames_per_step": F, "columns": C, "synapses": S,
                   "input_bits": cfg["input_bits"], "winners": k,
                   "path": "persistent" if pool.persistent else "plain"},
        "synapse_updates_per_s": fps * C * S,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_sp_persistent", "kernel_ms_per_launch": kernel_ms,
                     "algorithmic_bytes_per_launch": abytes,
                     "counter_bytes_per_launch": traffic_bytes},
        "plain_one_frame_per_launch_frames_per_s": plain,
        "cpu_baseline": cpu,
    }
    pool.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    rc = main()
    if rc:
        sys.exit(rc)
