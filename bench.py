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
INT8_PEAK_TOPS = 5000.0  # MI355X dense int8 matrix throughput, published (TOP/s)
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


def measured_traffic(profile: str, kernel: str, kernel_ms: float):
    """Counter bytes per launch from a committed summary, while the kernel
    source still matches the one the counters were taken from."""
    from paper_1608_01966_amd import profiling
    blk = profiling.read_block(os.path.join(PROFILES, profile))
    if not blk or blk.get("source_sha256") != profiling.source_sha256(kernel):
        return None, None
    b = blk.get("hbm_bytes_per_launch")
    if b is None:
        return None, None
    return b / (kernel_ms * 1e-3) / 1e9, b


def host_cores() -> int:
    return len(os.sched_getaffinity(0))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _sample(fn, F: int, budget_s: float):
    """Frames (doubling from 25, at most F) that fn(n) takes at least
    budget_s / 3 on; returns (n, seconds)."""
    n = min(25, F)
    while True:
        t0 = time.perf_counter()
        fn(n)
        dt = time.perf_counter() - t0
        if dt > budget_s / 3 or n >= F:
            return n, dt
        n = min(2 * n, F)


def cpu_baseline(w, learn: bool, budget_s: float, what: str) -> dict:
    """The oracle on the first frames of the same workload (as many as fit
    the time budget): on every host core the process may use (columns split
    over threads, the inhibition on one), and single-threaded."""
    import oracle
    F = w.frames.shape[0]
    cores = host_cores()
    n1, dt1 = _sample(lambda n: oracle.run(w.cfg, w.idx, w.perm, w.frames[:n], learn=learn,
                                           want_overlaps=False), F, budget_s)
    nm, dtm = _sample(lambda n: oracle.run_threads(w.cfg, w.idx, w.perm, w.frames[:n], cores,
                                                   learn=learn, want_overlaps=False),
                      F, budget_s)
    return {"value": nm / dtm, "unit": "frames/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"first {nm} frames of the same {what} from the same state, "
                      f"{dtm:.2f} s on {cores} threads (columns split per frame, "
                      f"inhibition on one thread)",
            "single_thread": {"value": n1 / dt1, "unit": "frames/s", "cores": 1,
                              "sample": f"first {n1} frames, {dt1:.2f} s"}}


def copy_peak(torch, mib: int = 1024, reps: int = 5) -> float:
    """Device-to-device copy rate (GB/s, bytes read plus bytes written) of a
    `mib` MiB buffer, best of `reps`: the HBM bandwidth a plain streaming
    kernel reaches on this device, measured in the same run."""
    n = mib * (1 << 20) // 4
    # (contents do not matter; no fill kernel, which the memory-counter
    # calibration would take for its copy)
    src = torch.empty(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    return 2 * n * 4 / (best * 1e-3) / 1e9


def with_measured_peak(roof: dict, peak_gbs: float) -> dict:
    """Adds the copy rate measured in this run beside the published peak."""
    if roof is not None and roof.get("unit") == "GB/s":
        roof["measured_copy_peak"] = peak_gbs
        roof["frac_of_measured_peak"] = roof["achieved"] / peak_gbs
    elif roof is not None:
        roof["measured_copy_peak_gbs"] = peak_gbs
    return roof


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
    kname = pool.kernel
    # a persistent step is the pairing pass, then the persistent kernel
    kspec = "k_pair_frames+k_sp_persistent_w" if kname == "k_sp_persistent_w" else kname
    traffic, traffic_bytes = (None, None)
    if (C, S, F) == (1024, 256, 1000):
        traffic, traffic_bytes = measured_traffic(f"{kname}_960x540_1024c_256s.md", kspec,
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

    # End to end: the frames start in pinned host memory and are uploaded
    # on the same stream before the step (the paper's timing with transfers).
    host = torch.from_numpy(np.ascontiguousarray(w.frames).view(np.int32)).pin_memory()
    dev2 = torch.empty_like(frames)

    def run_e2e(ev0=None, ev1=None):
        pool.perm.copy_(perm0)
        if ev0 is not None:
            ev0.record(stream)
        dev2.copy_(host, non_blocking=True)
        sp.sp_step(pool.handle, cfg, dev2, True, ov, win, stream)
        if ev1 is not None:
            ev1.record(stream)

    run_e2e()
    pool.sync()
    e2e_wall, e2e_ms = timed(run_e2e, max(1, args.steps // 2))
    pool.sync()
    e2e = {"frames_per_s": max(1, args.steps // 2) * F / e2e_wall, "ms_per_step": e2e_ms,
           "upload_bytes_per_step": int(host.numel() * 4),
           "what": "pinned host frames uploaded on the step's stream, then the step"}

    sweep = []
    if args.sweep:
        for sc in (256, 512, 1024, 2048):
            for ss in (32, 64, 128, 256):
                if (sc, ss) == (C, S):
                    continue
                ws = synth.workload_paper_scale(frames=args.sweep_frames, columns=sc,
                                                synapses=ss)
                sfr = torch.from_numpy(np.ascontiguousarray(ws.frames).view(np.int32)).cuda()
                sp2 = sp.SpatialPooler(ws.cfg, ws.idx, ws.perm)
                sp0 = sp2.perm.clone()
                sov = torch.empty((args.sweep_frames, sc), dtype=torch.int32, device="cuda")
                swin = torch.empty((args.sweep_frames, ws.cfg["winners"]), dtype=torch.int32,
                                   device="cuda")

                def srun(ev0=None, ev1=None, sp2=sp2, sp0=sp0, ws=ws, sfr=sfr, sov=sov,
                         swin=swin):
                    sp2.perm.copy_(sp0)
                    if ev0 is not None:
                        ev0.record(stream)
                    sp.sp_step(sp2.handle, ws.cfg, sfr, True, sov, swin, stream)
                    if ev1 is not None:
                        ev1.record(stream)

                srun()
                sp2.sync()
                swall, sms = timed(srun, 3)
                sp2.sync()
                sab = algorithmic_bytes_learn(ws.cfg, swin.cpu().numpy())
                sweep.append({"columns": sc, "synapses": ss, "frames": args.sweep_frames,
                              "frames_per_s": 3 * args.sweep_frames / swall,
                              "synapse_updates_per_s": 3 * args.sweep_frames * sc * ss / swall,
                              "kernel_ms_per_launch": sms, "path": sp2.kernel,
                              "roofline_frac": sab / (sms * 1e-3) / 1e9 / HBM_PEAK_GBS})
                sp2.close()
        sweep.append({"columns": C, "synapses": S, "frames": F, "frames_per_s": fps,
                      "synapse_updates_per_s": fps * C * S, "kernel_ms_per_launch": kernel_ms,
                      "path": kname, "roofline_frac": achieved / HBM_PEAK_GBS})
        sweep.sort(key=lambda r: (r["columns"], r["synapses"]))

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
                   "path": kname},
        "synapse_updates_per_s": fps * C * S,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kspec.replace("+", " + "), "kernel_ms_per_launch": kernel_ms,
                     "algorithmic_bytes_per_launch": abytes,
                     "counter_bytes_per_launch": traffic_bytes},
        "plain_one_frame_per_launch_frames_per_s": plain,
        "end_to_end_pinned_upload": e2e,
        "sweep": sweep,
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

    mfma = args.infer_mode == "mfma"
    mode = sp.SP_INFER_MFMA_I8 if mfma else sp.SP_INFER_GATHER

    def run(ev0=None, ev1=None):
        if ev0 is not None:
            ev0.record(stream)
        sp.sp_infer(pool.handle, cfg, frames, mode, ov, win, stream)
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
    hbm_achieved = abytes / (call_ms * 1e-3) / 1e9
    if mfma:
        # the dense product: 2 F N C int8 operations (multiply and add) per call
        aops = 2 * F * cfg["input_bits"] * C
        achieved = aops / (call_ms * 1e-3) / 1e12
        traffic, traffic_bytes = measured_traffic("k_infer_mfma_960x540_1024c_256s.md",
                                                  "k_infer_mfma+k_mfma_reduce+k_topk_batch",
                                                  call_ms)
        roof = {"bound": "mfma", "achieved": achieved, "peak": INT8_PEAK_TOPS,
                "unit": "TOP/s", "frac": achieved / INT8_PEAK_TOPS, "traffic": traffic,
                "kernel": "k_infer_mfma + k_mfma_reduce + k_topk_batch",
                "kernel_ms_per_launch": call_ms, "algorithmic_ops_per_launch": aops,
                "algorithmic_bytes_per_launch": abytes, "hbm_achieved_gbs": hbm_achieved,
                "counter_bytes_per_launch": traffic_bytes}
    else:
        traffic, traffic_bytes = measured_traffic("k_infer_gather_960x540_1024c_256s.md",
                                                  "k_infer_gather_db+k_topk_batch",
                                                  call_ms)
        roof = {"bound": "hbm", "achieved": hbm_achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": hbm_achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "k_infer_gather_db + k_topk_batch", "kernel_ms_per_launch": call_ms,
                "algorithmic_bytes_per_launch": abytes,
                "counter_bytes_per_launch": traffic_bytes}

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

    # end to end: the frames uploaded from pinned host memory before the call
    host = torch.from_numpy(np.ascontiguousarray(w.frames).view(np.int32)).pin_memory()
    dev2 = torch.empty_like(frames)

    def run_e2e(ev0=None, ev1=None):
        if ev0 is not None:
            ev0.record(stream)
        dev2.copy_(host, non_blocking=True)
        sp.sp_infer(pool.handle, cfg, dev2, mode, ov, win, stream)
        if ev1 is not None:
            ev1.record(stream)

    run_e2e()
    pool.sync()
    e2e_wall, e2e_ms = timed(run_e2e, max(1, args.steps // 2))
    comp["end_to_end_pinned_upload"] = {
        "frames_per_s": max(1, args.steps // 2) * F / e2e_wall, "ms_per_step": e2e_ms,
        "upload_bytes_per_step": int(host.numel() * 4),
        "what": "pinned host frames uploaded on the call's stream, then the call"}

    cpu = None if args.no_cpu_baseline else cpu_baseline(
        w, False, args.cpu_budget, f"{F}-frame inference batch")
    line = {
        "metric": "SP frames/s (1024 columns x 256 synapses, batched inference, learning off"
                  + (", dense int8 matrix product)" if mfma else ")"),
        "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_s / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8" if mfma else "u32", "data": "synthetic",
        "config": {"workload": f"{F} independent 960x540 Bernoulli(0.05) frames per step, "
                               f"frozen {C} columns x {S} synapses, min_overlap "
                               f"{cfg['min_overlap']}, {k} winners",
                   "frames_per_step": F, "columns": C, "synapses": S,
                   "input_bits": cfg["input_bits"], "winners": k,
                   "path": "mfma_i8" if mfma else "gather"},
        "synapse_updates_per_s": fps * C * S,
        "roofline": roof,
        **comp,
        "cpu_baseline": cpu,
    }
    pool.close()
    return line


def bench_multi(args, torch, sp, synth):
    ws = synth.workload_multi(instances=args.instances, frames=args.multi_frames)
    stream = torch.cuda.current_stream()
    pools = [sp.SpatialPooler(w.cfg, w.idx, w.perm) for w in ws]
    perm0 = [p.perm.clone() for p in pools]
    frames = [torch.from_numpy(np.ascontiguousarray(w.frames).view(np.int32)).cuda() for w in ws]
    wins = [torch.empty((w.frames.shape[0], w.cfg["winners"]), dtype=torch.int32, device="cuda")
            for w in ws]
    handles = [p.handle for p in pools]
    cfgs = [w.cfg for w in ws]
    total = sum(w.frames.shape[0] for w in ws)

    def reset():
        for p, p0 in zip(pools, perm0):
            p.perm.copy_(p0)

    # Every step learns the same frames from the same initial states; the
    # resets (one device copy per instance) stay inside the timed region.
    def run(ev0=None, ev1=None):
        reset()
        if ev0 is not None:
            ev0.record(stream)
        sp.sp_step_many(handles, cfgs, frames, True, None, wins, stream)
        if ev1 is not None:
            ev1.record(stream)

    for _ in range(args.warmup):
        run()
    pools[0].sync()
    warm_clock(lambda: (run(), pools[0].sync()), args.warm_seconds)
    wall_s, call_ms = timed(run, args.steps)
    pools[0].sync()
    ips = args.steps * total / wall_s

    nsyn = sum(w.cfg["num_columns"] * w.cfg["synapses_per_column"] for w in ws)
    abytes = 0
    for w, wn in zip(ws, wins):
        cfg = dict(w.cfg)
        F = w.frames.shape[0]
        nw = int((wn.cpu().numpy() >= 0).sum())
        S = cfg["synapses_per_column"]
        abytes += F * (frame_bytes(cfg) + 8 * cfg["num_columns"] * S + 4 * cfg["winners"])
        abytes += 12 * S * nw
    achieved = abytes / (call_ms * 1e-3) / 1e9
    traffic, traffic_bytes = measured_traffic("k_sp_many_64_instances.md", "k_sp_many", call_ms)

    # the same instances stepped one after another by the single-instance path
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, w, f, wn in zip(pools, ws, frames, wins):
        sp.sp_step(p.handle, w.cfg, f, True, None, wn, stream)
    torch.cuda.synchronize()
    seq = total / (time.perf_counter() - t0)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores = host_cores()

        def sample(threads):
            n, dt = 2, 0.0
            while True:
                t0 = time.perf_counter()
                for w in ws:
                    if threads == 1:
                        oracle.run(w.cfg, w.idx, w.perm, w.frames[:n], learn=True,
                                   want_overlaps=False)
                    else:
                        oracle.run_threads(w.cfg, w.idx, w.perm, w.frames[:n], threads,
                                           learn=True, want_overlaps=False)
                dt = time.perf_counter() - t0
                if dt > args.cpu_budget / 3 or n >= args.multi_frames:
                    return n, dt
                n = min(2 * n, args.multi_frames)

        n1, dt1 = sample(1)
        nm, dtm = sample(cores)
        cpu = {"value": nm * len(ws) / dtm, "unit": "instance-frames/s", "cores": cores,
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"first {nm} frames of each of the {len(ws)} instances from the same "
                         f"states, {dtm:.2f} s on {cores} threads (each instance's columns "
                         f"split per frame)",
               "single_thread": {"value": n1 * len(ws) / dt1, "unit": "instance-frames/s",
                                 "cores": 1, "sample": f"first {n1} frames, {dt1:.2f} s"}}
    line = {
        "metric": "SP instance-frames/s, 64 uneven instances, learning on",
        "value": ips, "unit": "instance-frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_s / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{len(ws)} independent poolers (columns 256-4096, synapses "
                               f"32-512, inputs 64x64-960x540 at 2-10% density), "
                               f"{args.multi_frames} learning frames each per step",
                   "instances": len(ws), "frames_per_instance": args.multi_frames,
                   "synapses_total": nsyn, "path": "many"},
        "synapse_updates_per_s": args.steps * sum(
            w.frames.shape[0] * w.cfg["num_columns"] * w.cfg["synapses_per_column"]
            for w in ws) / wall_s,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_sp_many", "kernel_ms_per_launch": call_ms,
                     "algorithmic_bytes_per_launch": abytes,
                     "counter_bytes_per_launch": traffic_bytes},
        "sequential_single_instance_launches_instance_frames_per_s": seq,
        "cpu_baseline": cpu,
    }
    for p in pools:
        p.close()
    return line


def bench_encode(args, torch, sp, synth):
    """The adaptive video encoder on a batch of 960x540 colour frames."""
    F, W, H = args.encode_frames, 960, 540
    rgb_h = synth.rgb_frames(synth.rng(14, 6), min(F, 16), W, H)
    reps = (F + rgb_h.shape[0] - 1) // rgb_h.shape[0]
    rgb = torch.from_numpy(np.concatenate([rgb_h] * reps)[:F]).cuda()
    bits = sp.sp_encoded_bits(W, H, args.encode_factor)
    out = torch.empty((F, (bits + 31) // 32), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def run(ev0=None, ev1=None):
        if ev0 is not None:
            ev0.record(stream)
        sp.sp_encode(rgb, args.encode_factor, 11, 2, out=out, stream=stream)
        if ev1 is not None:
            ev1.record(stream)

    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    warm_clock(lambda: (run(), torch.cuda.synchronize()), args.warm_seconds)
    wall_s, call_ms = timed(run, args.steps)
    torch.cuda.synchronize()
    fps = args.steps * F / wall_s
    abytes = F * (W * H * 3 + out.shape[1] * 4)
    achieved = abytes / (call_ms * 1e-3) / 1e9
    # rows of a whole number of words are stored whole (no zeroing kernel)
    kernels = "k_encode" if (W // args.encode_factor) % 32 == 0 else "k_zero+k_encode"
    traffic, traffic_bytes = measured_traffic(
        f"k_encode_960x540_f{args.encode_factor}.md", kernels, call_ms)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        n, dt = 1, 0.0
        while True:
            t0 = time.perf_counter()
            oracle.enc_frames(rgb_h[:n], args.encode_factor, 11, 2)
            dt = time.perf_counter() - t0
            if dt > args.cpu_budget / 3 or n >= rgb_h.shape[0]:
                break
            n = min(2 * n, rgb_h.shape[0])
        cpu = {"value": n / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
               "sample": f"first {n} of the frames, {dt:.2f} s single-threaded"}
    return {
        "metric": "adaptive video encoder frames/s (960x540 RGB to packed SP input)",
        "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_s / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"{F} synthetic 960x540 RGB frames per step, reduction factor "
                               f"{args.encode_factor}, 11x11 binomial window, offset 2",
                   "frames_per_step": F, "path": "encode"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernels.replace("+", " + "),
                     "kernel_ms_per_launch": call_ms, "algorithmic_bytes_per_launch": abytes,
                     "counter_bytes_per_launch": traffic_bytes},
        "cpu_baseline": cpu,
    }


def bench_local(args, torch, sp, synth):
    """Learning with local inhibition (Algorithm 2 with the paper's initial
    inhibition radius 80 over a 1-D column line): 960x540 blob frames, 1024
    columns x 256 synapses, n = 6 per neighbourhood (about the 40-in-1024
    density of the global step)."""
    F = args.local_frames
    w = synth.workload_paper_scale(frames=F, columns=1024, synapses=256)
    cfg = dict(w.cfg)
    cfg["winners"] = 6
    C, S = cfg["num_columns"], cfg["synapses_per_column"]
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    perm0 = pool.perm.clone()
    frames = torch.from_numpy(w.frames.view(np.int32)).cuda()
    act = torch.empty((F, C), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()

    def run(ev0=None, ev1=None):
        pool.perm.copy_(perm0)
        if ev0 is not None:
            ev0.record(stream)
        sp.sp_step_local(pool.handle, cfg, frames, True, 1024, 80, None, act, stream)
        if ev1 is not None:
            ev1.record(stream)

    for _ in range(args.warmup):
        run()
    pool.sync()
    warm_clock(lambda: (run(), pool.sync()), args.warm_seconds)
    wall_s, call_ms = timed(run, args.steps)
    pool.sync()
    fps = args.steps * F / wall_s
    n_act = int(act.sum().item())
    abytes = F * (frame_bytes(cfg) + 8 * C * S + 4 * C + C) + 12 * S * n_act
    achieved = abytes / (call_ms * 1e-3) / 1e9
    kname = pool.local_kernel_for(1024, 80)
    # the two-frame kernel runs after the pass that pairs the frames
    kspec = "k_pair_frames+" + kname if kname == "k_sp_persistent_local2" else kname
    traffic, traffic_bytes = (None, None)
    if kname != "plain" and F == 1000:
        traffic, traffic_bytes = measured_traffic(f"{kname}_960x540_1024c_256s_radius80.md",
                                                  kspec, call_ms)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        n, dt = 8, 0.0
        while True:
            t0 = time.perf_counter()
            oracle.run_local(cfg, w.idx, w.perm, w.frames[:n], 1024, 80, 6, want_overlaps=False)
            dt = time.perf_counter() - t0
            if dt > args.cpu_budget / 3 or n >= F:
                break
            n = min(2 * n, F)
        cpu = {"value": n / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
               "sample": f"first {n} frames from the same state, {dt:.2f} s single-threaded"}
    return {
        "metric": "SP frames/s with local inhibition (radius 80, 1024 columns x 256 synapses, "
                  "learning on)",
        "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_s / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"960x540 blob frames, 1024 columns in a line, radius 80, n = 6 "
                               f"per neighbourhood, {F} sequential learning frames per step",
                   "frames_per_step": F, "active_per_frame": n_act / F, "path": "local"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": (kspec.replace("+", " + ") if kname != "plain" else
                                "k_overlap_plain + k_inhibit_local + k_learn_active"),
                     "kernel_ms_per_launch": call_ms, "algorithmic_bytes_per_launch": abytes,
                     "counter_bytes_per_launch": traffic_bytes},
        "cpu_baseline": cpu,
    }


def bench_boost(args, torch, sp, synth):
    """Learning with boosting and duty cycles: 960x540 blob frames, 1024
    columns x 256 synapses, 40 winners, duty-cycle period 1024, minimum duty
    0.01 of the maximum, boost up to 10, permanence raise 13/256."""
    F = args.local_frames
    w = synth.workload_paper_scale(frames=F, columns=1024, synapses=256)
    cfg = w.cfg
    bc = {"period_log2": 10, "min_pct_q16": 655, "max_boost_q8": 2560, "bump_q8": 13}
    C, S, k = cfg["num_columns"], cfg["synapses_per_column"], cfg["winners"]
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    perm0 = pool.perm.clone()
    frames = torch.from_numpy(w.frames.view(np.int32)).cuda()
    win = torch.empty((F, k), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def run(ev0=None, ev1=None):
        pool.perm.copy_(perm0)
        sp.sp_boost_reset(pool.handle, stream)
        if ev0 is not None:
            ev0.record(stream)
        sp.sp_step_boost(pool.handle, cfg, bc, frames, True, None, win, stream)
        if ev1 is not None:
            ev1.record(stream)

    for _ in range(args.warmup):
        run()
    pool.sync()
    warm_clock(lambda: (run(), pool.sync()), args.warm_seconds)
    wall_s, call_ms = timed(run, args.steps)
    pool.sync()
    fps = args.steps * F / wall_s
    abytes = algorithmic_bytes_learn(cfg, win.cpu().numpy()) + F * 12 * C
    achieved = abytes / (call_ms * 1e-3) / 1e9
    kname = pool.boost_kernel
    traffic, traffic_bytes = (None, None)
    if kname != "plain" and F == 1000:
        traffic, traffic_bytes = measured_traffic(f"{kname}_960x540_1024c_256s.md", kname,
                                                  call_ms)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        n, dt = 8, 0.0
        while True:
            t0 = time.perf_counter()
            oracle.run_boost(cfg, bc, w.idx, w.perm, w.frames[:n], want_overlaps=False)
            dt = time.perf_counter() - t0
            if dt > args.cpu_budget / 3 or n >= F:
                break
            n = min(2 * n, F)
        cpu = {"value": n / dt, "unit": "frames/s", "cores": 1, "kind": "oracle",
               "sample": f"first {n} frames from the same state, {dt:.2f} s single-threaded"}
    return {
        "metric": "SP frames/s with boosting and duty cycles (1024 columns x 256 synapses, "
                  "learning on)",
        "value": fps, "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_s / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"960x540 blob frames, 1024 columns x 256 synapses, 40 winners, "
                               f"duty period 1024, min duty 0.01, max boost 10, raise 13/256, "
                               f"{F} sequential learning frames per step",
                   "frames_per_step": F, "path": "boost"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": (kname if kname != "plain" else
                                "k_overlap_plain + k_topk_plain + k_learn_plain + k_boost_update"),
                     "kernel_ms_per_launch": call_ms, "algorithmic_bytes_per_launch": abytes,
                     "counter_bytes_per_launch": traffic_bytes},
        "cpu_baseline": cpu,
    }


def bench_serve(args, torch, sp, synth):
    """The serving scheduler on 256 streams of 960x540 frames at 30 fps
    (Poisson), every stream live for the whole window: in real time with the
    budget holding every stream's state; in real time with a budget of half
    of it (streams evicted to host checkpoints after a residency quantum and
    re-admitted); and with the arrival times compressed until throughput
    stops growing (saturation), where the roofline is taken."""
    from paper_1608_01966_amd import serve
    P = args.pool_frames
    frames = synth.blob_frames(synth.rng(5, 2), P, 960, 540, 0.05)
    pool = torch.from_numpy(frames.view(np.int32)).cuda()
    specs = serve.make_streams(args.streams, fps=args.fps, window=args.window, pool_frames=P)
    offered = sum(len(s.arrivals) for s in specs)
    W = (960 * 540 + 31) // 32

    def serve_once(scale: float, budget_frac: float, quantum, frames_tick: int,
                   preadmit: bool = False):
        sc = [serve.StreamSpec(s.sid, s.cfg, s.idx, s.perm, s.arrivals / scale, s.frame_ids)
              for s in specs]
        be = serve.GpuBackend(pool, sc, keep_outputs=False, max_frames=frames_tick)
        total = sum(be.stream_bytes(s) for s in sc)
        srv = serve.Server(be, sc, budget_bytes=int(total * budget_frac),
                           max_frames_per_tick=frames_tick, quantum=quantum)
        if preadmit:
            srv.preadmit()
            torch.cuda.synchronize()
        t0 = time.perf_counter()
        srv.run()
        be.stream.synchronize()
        wall = time.perf_counter() - t0
        lat = srv.latencies(skip_before=1.0 / scale)
        # algorithmic bytes of every stream-frame: the frame, idx + perm of
        # every synapse, winners out, and the winners' learning (their count
        # from each stream's histogram)
        abytes = 0
        for i, s in enumerate(sc):
            C, S, k = s.cfg["num_columns"], s.cfg["synapses_per_column"], s.cfg["winners"]
            nwin = int(be.histogram(i).sum().item())
            abytes += len(s.arrivals) * (4 * W + 8 * C * S + 4 * k) + 12 * S * nwin
        gpu_s = float(np.sum(be.gpu_ms)) * 1e-3
        achieved = abytes / gpu_s / 1e9
        out = {"arrival_scale": scale, "budget_frac": budget_frac, "preadmitted": preadmit,
               "residency_quantum_s": quantum, "max_frames_per_stream_per_batch": frames_tick,
               "frames_per_s": offered / srv.last_completion(),
               "p50_ms": float(np.percentile(lat, 50) * 1e3),
               "p99_ms": float(np.percentile(lat, 99) * 1e3), "max_ms": float(lat.max() * 1e3),
               "batches": len(srv.batch_sizes),
               "mean_batch_frames": float(np.mean(srv.batch_sizes)),
               "mean_batch_streams": float(np.mean(srv.batch_streams)),
               "mean_batch_gpu_ms": float(np.mean(be.gpu_ms)),
               "mean_batch_wall_ms": float(np.mean(be.batch_wall) * 1e3),
               "gpu_busy_s": gpu_s, "wall_s": wall, "gpu_busy_frac": gpu_s / wall,
               "peak_resident_bytes": srv.peak_used, "budget_bytes": srv.budget,
               "state_bytes_all_streams": total,
               "evictions": srv.evictions, "readmissions": srv.readmissions,
               "max_admission_wait_ms": float(max(srv.admit_waits, default=0.0) * 1e3),
               "algorithmic_bytes": abytes, "achieved_GBps": achieved}
        del srv, be
        torch.cuda.synchronize()
        return out

    # real time, every stream resident
    rt = serve_once(1.0, 1.0, None, args.max_frames_tick)
    # real time, half the state's budget: time-sliced residency
    half = serve_once(1.0, 0.5, args.quantum, args.max_frames_tick)
    # saturation: the same arrivals compressed
    # (streams connected before the burst: 256 admissions would otherwise
    # take most of a window compressed to a fraction of a second)
    sat = [serve_once(scale, 1.0, None, args.sat_frames_tick, preadmit=True)
           for scale in args.saturation_scales]
    best = max(sat, key=lambda r: r["frames_per_s"]) if sat else None
    roof = None
    if best is not None:
        roof = {"bound": "hbm", "achieved": best["achieved_GBps"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": best["achieved_GBps"] / HBM_PEAK_GBS, "traffic": None,
                "kernel": "k_sp_many",
                "basis": "algorithmic bytes of every stream-frame / GPU time of the batches "
                         "(events around each sp_step_many) in the saturated run"}
    line = {
        "metric": "SP serve: p99 frame latency at 30 fps per stream, and saturated frames/s",
        "value": rt["p99_ms"], "unit": "ms", "n_gpus": 1, "steps": 2 + len(sat),
        "warmup": 0, "ms_per_step": rt["wall_s"] * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{args.streams} streams live for {args.window:.0f} s, 960x540 "
                               f"blob frames (~5% on) at {args.fps:g} fps Poisson per stream, "
                               f"poolers 256-4096 columns x 32-512 synapses, learning on",
                   "streams": args.streams, "frames_offered": offered,
                   "offered_frames_per_s": offered / args.window, "path": "serve"},
        "real_time": rt,
        "real_time_half_budget": half,
        "saturation": sat,
        "saturated_frames_per_s": best["frames_per_s"] if best else None,
        "roofline": roof,
    }
    return line


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload",
                    choices=["learn", "infer", "multi", "serve", "encode", "local", "boost"],
                    default="learn")
    ap.add_argument("--local-frames", type=int, default=1000)
    ap.add_argument("--encode-frames", type=int, default=256)
    ap.add_argument("--encode-factor", type=int, default=1)
    ap.add_argument("--streams", type=int, default=256)
    ap.add_argument("--fps", type=float, default=30.0)
    ap.add_argument("--window", type=float, default=10.0)
    ap.add_argument("--pool-frames", type=int, default=512)
    ap.add_argument("--max-frames-tick", type=int, default=8)
    ap.add_argument("--saturation-scales", type=float, nargs="*", default=[40.0, 160.0, 1000.0])
    ap.add_argument("--sat-frames-tick", type=int, default=32,
                    help="frames of one stream per batch in the saturated serving runs")
    ap.add_argument("--quantum", type=float, default=1.0,
                    help="residency quantum (s) of the half-budget serving run")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--multi-frames", type=int, default=500)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--warm-seconds", type=float, default=1.0,
                    help="untimed busy time before the timed steps (GPU clock ramp-up)")
    ap.add_argument("--frames", type=int, default=1000)
    ap.add_argument("--infer-frames", type=int, default=4096)
    ap.add_argument("--infer-mode", choices=["gather", "mfma"], default="gather",
                    help="sp_infer mode of --workload infer")
    ap.add_argument("--columns", type=int, default=1024)
    ap.add_argument("--synapses", type=int, default=256)
    ap.add_argument("--plain-frames", type=int, default=200,
                    help="frames timed through the one-frame-per-launch path (0: skip)")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-sweep", dest="sweep", action="store_false",
                    help="skip the column x synapse sweep of --workload learn")
    ap.add_argument("--sweep-frames", type=int, default=200)
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

    fn = {"learn": bench_learn, "infer": bench_infer, "multi": bench_multi,
          "serve": bench_serve, "encode": bench_encode, "local": bench_local,
          "boost": bench_boost}[args.workload]
    peak = copy_peak(torch)
    line = fn(args, torch, sp, synth)
    with_measured_peak(line.get("roofline"), peak)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    rc = main()
    if rc:
        sys.exit(rc)
