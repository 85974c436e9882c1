"""Benchmark: HTM spatial pooler steps on one MI355X.

Default workload (``--workload learn``): a step is one pass of the whole hot
path (overlap, global top-k inhibition, permanence learning) over one batch
of synthetic frames: 1000 sequential learning frames of a 960x540 binary
input (~5% on, as random 8x8 blobs) through one spatial pooler of 1024
columns x 256 potential synapses, min_overlap 4, 40 winners, threshold 0.5,
inc 8/256, dec 4/256.

``--workload infer``: a step is one batched-inference call over 4096
independent 960x540 Bernoulli(0.05) frames through a frozen pooler of the
same shape.

Frames are resident in HBM before the timed region starts.  Prints one JSON
line with frames/s, the roofline of the dominant kernel and the oracle timed
on the host as a CPU baseline.
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
PROFILES = os.path.join(ROOT, "profiles")


def frame_bytes(cfg: dict) -> int:
    return 4 * ((cfg["input_bits"] + 31) // 32)


def algorithmic_bytes_learn(cfg: dict, winners: np.ndarray) -> int:
    """Bytes the learning step must move per launch at minimum in the
    library's layout, summed over frames: the packed frame, idx + perm of
    every potential synapse (overlap), read-modify-write of perm plus the idx
    read for each winner's synapses (learning), overlaps and winners out."""
    C, S, k = cfg["num_columns"], cfg["synapses_per_column"], cfg["winners"]
    F = winners.shape[0]
    n_win = int((winners >= 0).sum())
    return F * (frame_bytes(cfg) + 8 * C * S + 4 * C + 4 * k) + 12 * S * n_win


def algorithmic_bytes_infer(cfg: dict, F: int) -> int:
    """Batched inference with frozen state: every frame read once, the state
    (idx + perm) read once, overlaps and winners written once."""
    C, S, k = cfg["num_columns"], cfg["synapses_per_column"], cfg["winners"]
    return F * (frame_bytes(cfg) + 4 * C + 4 * k) + 8 * C * S


def measured_traffic(profile: str, kernel_ms: float):
    """Counter bytes per launch from a committed summary, while the kernel
    source still matches the one the counters were taken from."""
    from paper_1608_01966_amd import profiling
    blk = profiling.read_block(os.path.join(PROFILES, profile))
    if not blk or blk.get("source_sha256") != profiling.source_sha256():
        return None, None
    b = blk.get("hbm_bytes_per_launch")
    if b is None:
        return None, None
    return b / (kernel_ms * 1e-3) / 1e9, b


def cpu_baseline(w, learn: bool, budget_s: float, what: str) -> dict:
    """The oracle, single-threaded, on the first frames of the same workload
    (as many as fit the time budget, doubling from 25)."""
    import oracle
    F = w.frames.shape[0]
    n = min(25, F)
    while True:
        t0 = time.perf_counter()
        oracle.run(w.cfg, w.idx, w.perm, w.frames[:n], learn=learn, want_overlaps=False)
        dt = time.perf_counter() - t0
        if dt > budget_s / 3 or n >= F:
            break
        n = min(2 * n, F)
    return {"value": n / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} frames of the same {what} from the same state, "
                      f"{dt:.2f} s single-threaded"}


def timed(run, steps: int):
    """Wall time of `steps` calls, and the mean time per call between the
    events each call records on the launch stream."""
    import torch
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        run(starts[i], ends[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = float(np.mean([s.elapsed_time(e) for s, e in zip(starts, ends)]))
    return wall, ms


def warm_clock(fn, seconds: float):
    """Keeps the GPU busy for a moment so that its clocks have ramped up."""
    t_end = time.perf_counter() + seconds
    while time.perf_counter() < t_end:
        fn()


def bench_learn(args, torch, sp, synth):
    w = synth.workload_paper_scale(frames=args.frames, columns=args.columns,
                                   synapses=args.synapses)
    cfg = w.cfg
    C, S, k = cfg["num_columns"], cfg["synapses_per_column"], cfg["winners"]
    frames = torch.from_numpy(np.ascontiguousarray(w.frames).view(np.int32)).cuda()
    F = frames.shape[0]

    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    perm0 = pool.perm.clone()
    stream = torch.cuda.current_stream()
    ov = torch.empty((F, C), dtype=torch.int32, device="cuda")
    win = torch.empty((F, k), dtype=torch.int32, device="cuda")

    # Every step learns the same frames from the same initial state (without
    # boosting, a pooler that keeps learning on random frames disconnects most
    # synapses, and later steps would time a different workload).  The 1 MB
    # reset copy stays inside the timed region.
    def run(ev0=None, ev1=None):
        pool.perm.copy_(perm0)
        if ev0 is not None:
            ev0.record(stream)
        sp.sp_step(pool.handle, cfg, frames, True, ov, win, stream)
        if ev1 is not None:
            ev1.record(stream)

    for _ in range(args.warmup):
        run()
    pool.sync()
    warm_clock(lambda: (run(), pool.sync()), args.warm_seconds)
    wall_s, kernel_ms = timed(run, args.steps)
    pool.sync()
    fps = args.steps * F / wall_s

    abytes = algorithmic_bytes_learn(cfg, win.cpu().numpy())
    achieved = abytes / (kernel_ms * 1e-3) / 1e9
    traffic, traffic_bytes = (None, None)
    if (C, S, F) == (1024, 256, 1000):
        traffic, traffic_bytes = measured_traffic("k_sp_persistent_960x540_1024c_256s.md",
                                                  kernel_ms)

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

    cpu = None if args.no_cpu_baseline else cpu_baseline(
        w, True, args.cpu_budget, f"{F}-frame learning workload")
    line = {
        "metric": "SP frames/s (1024 columns x 256 synapses, learning on)",
        "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_s / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
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
    return line


def bench_infer(args, torch, sp, synth):
    w = synth.workload_batched_inference(frames=args.infer_frames)
    cfg = w.cfg
    C, S, k = cfg["num_columns"], cfg["synapses_per_column"], cfg["winners"]
    frames = torch.from_numpy(np.ascontiguousarray(w.frames).view(np.int32)).cuda()
    F = frames.shape[0]
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    stream = torch.cuda.current_stream()
    ov = torch.empty((F, C), dtype=torch.int32, device="cuda")
    win = torch.empty((F, k), dtype=torch.int32, device="cuda")

    def run(ev0=None, ev1=None):
        if ev0 is not None:
            ev0.record(stream)
        sp.sp_infer(pool.handle, cfg, frames, sp.SP_INFER_GATHER, ov, win, stream)
        if ev1 is not None:
            ev1.record(stream)

    for _ in range(args.warmup):
        run()
    pool.sync()
    warm_clock(lambda: (run(), pool.sync()), args.warm_seconds)
    wall_s, call_ms = timed(run, args.steps)
    pool.sync()
    fps = args.steps * F / wall_s
    abytes = algorithmic_bytes_infer(cfg, F)
    achieved = abytes / (call_ms * 1e-3) / 1e9
    traffic, traffic_bytes = measured_traffic("k_infer_gather_960x540_1024c_256s.md", call_ms)

    # the same frames one launch sequence at a time, and through the
    # persistent sequential step with learning off
    comp = {}
    pf = min(args.plain_frames, F) if args.plain_frames > 0 else 0
    if pf:
        pov = torch.empty((pf, C), dtype=torch.int32, device="cuda")
        pwin = torch.empty((pf, k), dtype=torch.int32, device="cuda")
        for name, fn in (("plain_one_frame_per_launch", sp.sp_step_plain),
                         ("persistent_sequential", sp.sp_step)):
            fn(pool.handle, cfg, frames[:pf], False, pov, pwin, stream)
            pool.sync()
            t0 = time.perf_counter()
            fn(pool.handle, cfg, frames[:pf], False, pov, pwin, stream)
            pool.sync()
            comp[name + "_frames_per_s"] = pf / (time.perf_counter() - t0)

    cpu = None if args.no_cpu_baseline else cpu_baseline(
        w, False, args.cpu_budget, f"{F}-frame inference batch")
    line = {
        "metric": "SP frames/s (1024 columns x 256 synapses, batched inference, learning off)",
        "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_s / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{F} independent 960x540 Bernoulli(0.05) frames per step, "
                               f"frozen {C} columns x {S} synapses, min_overlap "
                               f"{cfg['min_overlap']}, {k} winners",
                   "frames_per_step": F, "columns": C, "synapses": S,
                   "input_bits": cfg["input_bits"], "winners": k, "path": "gather"},
        "synapse_updates_per_s": fps * C * S,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_infer_gather + k_topk_batch", "kernel_ms_per_launch": call_ms,
                     "algorithmic_bytes_per_launch": abytes,
                     "counter_bytes_per_launch": traffic_bytes},
        **comp,
        "cpu_baseline": cpu,
    }
    pool.close()
    return line


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["learn", "infer"], default="learn")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--warm-seconds", type=float, default=1.0,
                    help="untimed busy time before the timed steps (GPU clock ramp-up)")
    ap.add_argument("--frames", type=int, default=1000)
    ap.add_argument("--infer-frames", type=int, default=4096)
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
    if args.calibration_copy_mb > 0:
        n = args.calibration_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.add(src, 1, out=dst)
        torch.cuda.synchronize()
        del src, dst

    fn = bench_learn if args.workload == "learn" else bench_infer
    line = fn(args, torch, sp, synth)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    rc = main()
    if rc:
        sys.exit(rc)
