"""Serving spatial poolers to many video streams with continuous batching.

The paper feeds video frame by frame through a spatial pooler (Section 2)
and, in its 'Multiple HTMs' setup, runs one pooler per category (Section
3.1).  Here every stream owns one pooler whose state stays resident on the
GPU while the stream is live; frames arrive on their own schedule, and each
scheduler tick steps the oldest pending frames of every resident stream
together in one batched call (``sp_step_many``), so work that arrives while
a batch runs joins the next one.  Frames of one stream are processed strictly
in arrival order (learning makes each frame depend on the previous one);
batches are issued in order on one device stream, so a stream may have frames
in two consecutive batches at once.

Admission: a stream becomes resident when its state (synapse indices and
permanences) plus the library's workspace fit the remaining device-memory
budget; it leaves when its last frame is done, which frees budget for
streams waiting to be admitted.

Backends provide ``stream_bytes(spec)``, ``open(spec)``, ``close(handle)``,
``launch(items) -> token`` and ``finished(token) -> completion time or
None``, times in seconds on the server's clock.  ``GpuBackend`` runs the HIP
library; tests without a GPU use a backend built on the oracle.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class StreamSpec:
    """One video stream: its pooler and the frames it will send."""
    sid: int
    cfg: dict
    idx: np.ndarray                 # uint32 [C][S] initial pools
    perm: np.ndarray                # float32 [C][S] initial permanences
    arrivals: np.ndarray            # float64 [F] seconds after start, non-decreasing
    frame_ids: np.ndarray           # int64 [F] index of each frame in the frame pool


@dataclass
class StreamState:
    spec: StreamSpec
    resident: bool = False
    finished: bool = False
    handle: object = None
    next_frame: int = 0             # first frame not yet handed to a batch
    done: int = 0                   # frames completed
    bytes: int = 0
    completions: list = field(default_factory=list)   # (frame index, completion time)


class Server:
    """Continuous-batching scheduler over a backend.

    ``max_frames_per_tick`` bounds how many pending frames of one stream join
    one batch; ``max_inflight`` batches may be queued on the device at once."""

    def __init__(self, backend, specs, budget_bytes: int, max_frames_per_tick: int = 4,
                 max_inflight: int = 2):
        self.backend = backend
        self.streams = [StreamState(s) for s in specs]
        self.budget = int(budget_bytes)
        self.used = 0
        self.peak_used = 0
        self.max_frames = int(max_frames_per_tick)
        self.max_inflight = int(max_inflight)
        order = sorted(range(len(specs)),
                       key=lambda i: specs[i].arrivals[0] if len(specs[i].arrivals) else 0.0)
        self.waiting = deque(i for i in order if len(specs[i].arrivals))
        for i in order:
            if not len(specs[i].arrivals):
                self.streams[i].finished = True
        self.inflight = deque()      # (token, [(stream index, first frame, count)])
        self.batch_sizes = []
        self.admit_waits = []        # admission time minus first arrival, per stream

    def _admit(self, now: float):
        while self.waiting:
            i = self.waiting[0]
            st = self.streams[i]
            if st.spec.arrivals[0] > now:
                break
            need = self.backend.stream_bytes(st.spec)
            if need > self.budget:
                raise ValueError(f"stream {st.spec.sid} needs {need} bytes, over the budget")
            if self.used + need > self.budget:
                break
            self.waiting.popleft()
            st.handle = self.backend.open(st.spec)
            st.bytes = need
            st.resident = True
            self.used += need
            self.peak_used = max(self.peak_used, self.used)
            self.admit_waits.append(now - st.spec.arrivals[0])

    def _retire(self, st: StreamState):
        self.backend.close(st.handle)
        st.handle = None
        st.resident = False
        st.finished = True
        self.used -= st.bytes

    def _complete(self, now: float):
        while self.inflight:
            token, parts = self.inflight[0]
            t_done = self.backend.finished(token)
            if t_done is None:
                return
            self.inflight.popleft()
            for i, first, count in parts:
                st = self.streams[i]
                for f in range(first, first + count):
                    st.completions.append((f, t_done))
                st.done += count
                if st.done == len(st.spec.arrivals):
                    self._retire(st)

    def _pending(self, st: StreamState, now: float) -> int:
        arrived = int(np.searchsorted(st.spec.arrivals, now, side="right"))
        n = min(arrived - st.next_frame, self.max_frames)
        if n > 1:
            # one call reads consecutive pool frames
            ids = st.spec.frame_ids[st.next_frame:st.next_frame + n]
            breaks = np.flatnonzero(np.diff(ids) != 1)
            if breaks.size:
                n = int(breaks[0]) + 1
        return max(n, 0)

    def poll(self, now: float) -> bool:
        """Advances the scheduler to time `now`.  False once every stream is done."""
        self._complete(now)
        self._admit(now)
        if len(self.inflight) < self.max_inflight:
            parts = []
            for i, st in enumerate(self.streams):
                if st.resident:
                    n = self._pending(st, now)
                    if n > 0:
                        parts.append((i, st.next_frame, n))
            if parts:
                items = [(self.streams[i].handle, self.streams[i].spec, first, n)
                         for i, first, n in parts]
                token = self.backend.launch(items)
                for i, first, n in parts:
                    self.streams[i].next_frame += n
                self.inflight.append((token, parts))
                self.batch_sizes.append(sum(n for _, _, n in parts))
        return not all(st.finished for st in self.streams)

    def run(self, clock=None):
        """Polls until every stream is done, against `clock()` (seconds since
        the start; the wall clock by default)."""
        if clock is None:
            t_start = time.perf_counter()
            if hasattr(self.backend, "set_start"):
                self.backend.set_start(t_start)
            clock = lambda: time.perf_counter() - t_start  # noqa: E731
        while self.poll(clock()):
            pass

    def latencies(self, skip_before: float = 0.0) -> np.ndarray:
        """Completion minus arrival of every frame that arrived at or after
        `skip_before`."""
        out = []
        for st in self.streams:
            arr = st.spec.arrivals
            for f, t_done in st.completions:
                if arr[f] >= skip_before:
                    out.append(t_done - arr[f])
        return np.asarray(out, dtype=np.float64)


class GpuBackend:
    """Batches through the HIP library: one ``sp_step_many`` per batch on a
    dedicated device stream; a batch's completion time comes from a GPU
    event; winners are kept per stream on the device."""

    def __init__(self, frame_pool, keep_outputs: bool = True):
        import torch
        from . import sp_step_many, sp_workspace_bytes
        self.torch = torch
        self._step_many = sp_step_many
        self._ws_bytes = sp_workspace_bytes
        self.pool = frame_pool              # int32 [P][W] frames on the device
        self.stream = torch.cuda.Stream()
        self.keep = keep_outputs
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(self.stream)
        self.ref.synchronize()
        self.ref_host = time.perf_counter()
        self.t_start = self.ref_host

    def set_start(self, host_t0: float):
        self.t_start = host_t0

    def stream_bytes(self, spec: StreamSpec) -> int:
        C, S = spec.cfg["num_columns"], spec.cfg["synapses_per_column"]
        return 8 * C * S + 4 * C + int(self._ws_bytes(spec.cfg))

    def open(self, spec: StreamSpec):
        from . import SpatialPooler
        pool = SpatialPooler(spec.cfg, spec.idx, spec.perm, stream=self.stream)
        win = (self.torch.empty((len(spec.arrivals), spec.cfg["winners"]),
                                dtype=self.torch.int32, device="cuda") if self.keep else None)
        # the stream's SDR histogram (Section 2's per-video feature vector)
        hist = self.torch.zeros(spec.cfg["num_columns"], dtype=self.torch.int32, device="cuda")
        self.torch.cuda.current_stream().synchronize()
        pool.set_histogram(hist)
        return {"pool": pool, "win": win, "hist": hist}

    def close(self, h):
        h["pool"].close()

    def launch(self, items):
        torch = self.torch
        handles, cfgs, frames, wins = [], [], [], []
        for h, spec, first, n in items:
            f0 = int(spec.frame_ids[first])
            handles.append(h["pool"].handle)
            cfgs.append(spec.cfg)
            frames.append(self.pool[f0:f0 + n])
            if self.keep:
                wins.append(h["win"][first:first + n])
            else:
                # allocated on the current stream, written on ours: the
                # allocator must not hand the block out again before our
                # stream is past this batch
                wn = torch.empty((n, spec.cfg["winners"]), dtype=torch.int32, device="cuda")
                wn.record_stream(self.stream)
                wins.append(wn)
        self._step_many(handles, cfgs, frames, True, None, wins, self.stream)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        return ev

    def finished(self, ev):
        if not ev.query():
            return None
        return self.ref_host + self.ref.elapsed_time(ev) * 1e-3 - self.t_start

    def winners(self, h):
        return h["win"]


def poisson_arrivals(g: np.random.Generator, rate: float, start: float, duration: float):
    """Arrival times of a Poisson process of `rate` per second in
    [start, start + duration)."""
    n = max(16, int(rate * duration * 1.5) + 16)
    t = start + np.cumsum(g.exponential(1.0 / rate, size=n))
    while t[-1] < start + duration:
        t = np.concatenate([t, t[-1] + np.cumsum(g.exponential(1.0 / rate, size=n))])
    return t[t < start + duration]


def make_streams(n_streams: int, fps: float, window: float, pool_frames: int, seed: int = 5,
                 columns=(256, 512, 1024, 2048, 4096), synapses=(32, 64, 128, 256, 512),
                 input_bits: int = 960 * 540, min_len: float = 2.0, max_len: float = 8.0):
    """Streams with pooler sizes drawn like the multi-instance workload,
    a random start in the window and a length of min_len..max_len seconds of
    Poisson(fps) frames; each stream reads consecutive frames of a shared
    pool from a random offset."""
    from . import synth
    g = synth.rng(seed, 0)
    specs = []
    for s in range(n_streams):
        C, S = int(g.choice(columns)), int(g.choice(synapses))
        cfg = synth.sp_config(input_bits, C, S, 4, max(1, 10 * C // 256))
        length = float(g.uniform(min_len, max_len))
        start = float(g.uniform(0.0, max(0.0, window - length)))
        arr = poisson_arrivals(synth.rng(seed * 1000 + s, 3), fps, start, length)
        off = int(g.integers(0, pool_frames))
        ids = (off + np.arange(len(arr))) % pool_frames
        idx = synth.pools(synth.rng(seed * 1000 + s, 0), input_bits, C, S)
        perm = synth.q_to_float(synth.permanences_q(synth.rng(seed * 1000 + s, 1), C, S))
        specs.append(StreamSpec(s, cfg, idx, perm, arr, ids))
    return specs
