"""Serving spatial poolers to many video streams with continuous batching.

The paper feeds video frame by frame through a spatial pooler (Section 2)
and, in its 'Multiple HTMs' setup, runs one pooler per category (Section
3.1).  Here every stream owns one pooler whose state stays resident on the
GPU while the stream is admitted; frames arrive on their own schedule, and
each scheduler tick steps the oldest pending frames of every resident stream
together in one batched call (``sp_step_many``), so work that arrives while
a batch runs joins the next one.  Frames of one stream are processed strictly
in arrival order (learning makes each frame depend on the previous one);
batches are issued in order on one device stream, so a stream may have frames
in two consecutive batches at once.

Admission: a stream with pending frames becomes resident when its state
(synapse indices and permanences) plus the library's workspace fit the
remaining device-memory budget, oldest pending frame first; it leaves when
its last frame is done.  With a residency ``quantum``, a stream that waits
for budget may evict resident streams that have held their place for at
least the quantum and have nothing in flight: an evicted stream's
permanences go to host memory (a checkpoint, ``sp_get_state``) and come back
when it is re-admitted (Section 3.2.1's pooler that keeps learning across
sessions), so its results are those of stepping it alone.

The scheduler's bookkeeping is vectorised over streams (numpy arrays indexed
by the stream's position in ``specs``), so a tick costs the same few array
operations for 4 or 400 streams.

Backends provide ``stream_bytes(spec)``, ``open(i, spec, checkpoint)``,
``evict(handle) -> checkpoint``, ``close(handle)``, ``launch(ids, firsts,
counts) -> token`` and ``finished(token) -> completion time or None``, times
in seconds on the server's clock.  ``GpuBackend`` runs the HIP library; tests
without a GPU use a backend built on the oracle.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass

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


def _ranges(starts: np.ndarray, counts: np.ndarray) -> np.ndarray:
    """Concatenation of arange(s, s + c) over the pairs."""
    counts = np.asarray(counts, dtype=np.int64)
    tot = int(counts.sum())
    if tot == 0:
        return np.zeros(0, dtype=np.int64)
    ends = np.cumsum(counts)
    base = np.repeat(np.asarray(starts, dtype=np.int64) - (ends - counts), counts)
    return base + np.arange(tot, dtype=np.int64)


class Server:
    """Continuous-batching scheduler over a backend.

    ``max_frames_per_tick`` bounds how many pending frames of one stream join
    one batch; ``max_inflight`` batches may be queued on the device at once;
    ``quantum`` (seconds, or None for no eviction) is the residency after
    which a stream may be evicted for one that waits for budget."""

    def __init__(self, backend, specs, budget_bytes: int, max_frames_per_tick: int = 4,
                 max_inflight: int = 2, quantum: float | None = None):
        self.backend = backend
        self.specs = list(specs)
        n = len(self.specs)
        self.budget = int(budget_bytes)
        self.max_frames = int(max_frames_per_tick)
        self.max_inflight = int(max_inflight)
        self.quantum = quantum
        self.nframes = np.array([len(s.arrivals) for s in self.specs], dtype=np.int64)
        self.need = np.array([backend.stream_bytes(s) for s in self.specs], dtype=np.int64)
        self.off = np.concatenate([[0], np.cumsum(self.nframes)]).astype(np.int64)
        arr = [np.asarray(s.arrivals, dtype=np.float64) for s in self.specs]
        self.arr = np.concatenate(arr) if n else np.zeros(0)
        # end (exclusive) of the run of consecutive pool frames each frame is in
        runend = np.zeros(self.arr.size, dtype=np.int64)
        for i, s in enumerate(self.specs):
            ids = np.asarray(s.frame_ids, dtype=np.int64)
            if ids.size:
                brk = np.flatnonzero(np.diff(ids) != 1) + 1
                ends = np.concatenate([brk, [ids.size]])
                runend[self.off[i]:self.off[i + 1]] = np.repeat(ends, np.diff(
                    np.concatenate([[0], ends])))
        self.runend = runend
        sid = np.repeat(np.arange(n, dtype=np.int64), self.nframes)
        order = np.argsort(self.arr, kind="stable")
        self.ev_t = self.arr[order]
        self.ev_sid = sid[order]
        self.ev_pos = 0
        self.arrived = np.zeros(n, dtype=np.int64)
        self.next = np.zeros(n, dtype=np.int64)
        self.done = np.zeros(n, dtype=np.int64)
        self.busy = np.zeros(n, dtype=np.int64)        # batches in flight holding the stream
        self.resident = np.zeros(n, dtype=bool)
        self.finished = self.nframes == 0
        self.admitted_at = np.zeros(n, dtype=np.float64)
        self.handles = [None] * n
        self.ckpt = [None] * n
        self.comp = np.full(self.arr.size, np.nan)
        self.used = 0
        self.peak_used = 0
        self.inflight = deque()      # (token, ids, firsts, counts)
        self.batch_sizes = []
        self.batch_streams = []
        self.admit_waits = []        # admission time minus the oldest pending arrival
        self.evictions = 0
        self.readmissions = 0

    # -- bookkeeping ---------------------------------------------------------
    def _complete(self):
        while self.inflight:
            token, ids, firsts, counts = self.inflight[0]
            t_done = self.backend.finished(token)
            if t_done is None:
                return
            self.inflight.popleft()
            self.done[ids] += counts
            self.busy[ids] -= 1
            self.comp[_ranges(self.off[ids] + firsts, counts)] = t_done
            for i in ids[self.done[ids] == self.nframes[ids]]:
                self._retire(int(i))

    def _retire(self, i: int):
        self.backend.close(self.handles[i])
        self.handles[i] = None
        self.ckpt[i] = None
        self.resident[i] = False
        self.finished[i] = True
        self.used -= int(self.need[i])

    def _evict(self, i: int):
        self.ckpt[i] = self.backend.evict(self.handles[i])
        self.handles[i] = None
        self.resident[i] = False
        self.used -= int(self.need[i])
        self.evictions += 1

    def _arrive(self, now: float):
        end = int(np.searchsorted(self.ev_t, now, side="right"))
        if end > self.ev_pos:
            self.arrived += np.bincount(self.ev_sid[self.ev_pos:end], minlength=len(self.specs))
            self.ev_pos = end

    def _admit(self, now: float):
        waiting = np.flatnonzero(~self.resident & ~self.finished & (self.arrived > self.next))
        if waiting.size == 0:
            return
        oldest = self.arr[self.off[waiting] + self.next[waiting]]
        for i in waiting[np.argsort(oldest, kind="stable")]:
            i = int(i)
            need = int(self.need[i])
            if need > self.budget:
                raise ValueError(f"stream {self.specs[i].sid} needs {need} bytes, over the budget")
            if self.used + need > self.budget and self.quantum is not None:
                self._make_room(need, now)
            if self.used + need > self.budget:
                break  # first come, first served: later streams wait too
            ck = self.ckpt[i]
            self.handles[i] = self.backend.open(i, self.specs[i], ck)
            self.ckpt[i] = None
            self.readmissions += ck is not None
            self.resident[i] = True
            self.admitted_at[i] = now
            self.used += need
            self.peak_used = max(self.peak_used, self.used)
            self.admit_waits.append(now - float(self.arr[self.off[i] + self.next[i]]))

    def preadmit(self):
        """Admits, before the clock starts, every stream that fits the budget
        in order of first arrival (streams already connected when their
        frames start to arrive); the rest are admitted as usual."""
        order = np.argsort(np.array([s.arrivals[0] if len(s.arrivals) else np.inf
                                     for s in self.specs]), kind="stable")
        for i in order:
            i = int(i)
            if self.finished[i] or self.resident[i]:
                continue
            need = int(self.need[i])
            if self.used + need > self.budget:
                break
            self.handles[i] = self.backend.open(i, self.specs[i], None)
            self.resident[i] = True
            self.admitted_at[i] = 0.0
            self.used += need
            self.peak_used = max(self.peak_used, self.used)

    def _make_room(self, need: int, now: float):
        cand = np.flatnonzero(self.resident & (self.busy == 0) &
                              (now - self.admitted_at >= self.quantum))
        if cand.size == 0:
            return
        # streams with nothing pending first, then the longest resident
        pending = (self.arrived[cand] > self.next[cand]).astype(np.int64)
        order = np.lexsort((self.admitted_at[cand], pending))
        for i in cand[order]:
            if self.used + need <= self.budget:
                return
            self._evict(int(i))

    def _batch(self):
        if len(self.inflight) >= self.max_inflight:
            return
        res = np.flatnonzero(self.resident)
        if res.size == 0:
            return
        nxt = self.next[res]
        n = np.minimum(self.arrived[res] - nxt, self.max_frames)
        live = n > 0
        if not live.any():
            return
        res, nxt, n = res[live], nxt[live], n[live]
        # one call reads consecutive pool frames of a stream
        n = np.minimum(n, self.runend[self.off[res] + nxt] - nxt)
        token = self.backend.launch(res, nxt, n)
        self.next[res] += n
        self.busy[res] += 1
        self.inflight.append((token, res, nxt, n))
        self.batch_sizes.append(int(n.sum()))
        self.batch_streams.append(int(res.size))

    def poll(self, now: float) -> bool:
        """Advances the scheduler to time `now`.  False once every stream is done."""
        self._complete()
        self._arrive(now)
        self._admit(now)
        self._batch()
        return not bool(self.finished.all())

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

    # -- results -------------------------------------------------------------
    def completions(self, i: int) -> np.ndarray:
        """Completion time of every frame of stream i (NaN: not done)."""
        return self.comp[self.off[i]:self.off[i + 1]]

    def latencies(self, skip_before: float = 0.0) -> np.ndarray:
        """Completion minus arrival of every frame that arrived at or after
        `skip_before`."""
        keep = self.arr >= skip_before
        return self.comp[keep] - self.arr[keep]

    def last_completion(self) -> float:
        return float(np.nanmax(self.comp)) if self.comp.size else 0.0


class GpuBackend:
    """Batches through the HIP library: one ``sp_step_many`` per batch on a
    dedicated device stream, its arrays built with numpy from per-stream
    tables; admission, eviction and retirement run on a side stream, so they
    never wait for the batches in flight.  A batch's completion time and GPU
    time come from events around it; winners (if kept) and each stream's SDR
    histogram stay on the device across evictions."""

    def __init__(self, frame_pool, specs, keep_outputs: bool = True, max_frames: int = 8):
        import torch
        from . import sp_workspace_bytes
        self.torch = torch
        self._ws_bytes = sp_workspace_bytes
        self.pool = frame_pool              # int32 [P][W] frames on the device
        self.specs = list(specs)
        n = len(self.specs)
        W = int(frame_pool.shape[1])
        for s in self.specs:
            if (s.cfg["input_bits"] + 31) // 32 != W:
                raise ValueError(f"stream {s.sid}: frames have {W} words, the pooler reads "
                                 f"{(s.cfg['input_bits'] + 31) // 32}")
        self.row_bytes = 4 * W
        self.fbase = int(frame_pool.data_ptr())
        lens = np.array([len(s.frame_ids) for s in self.specs], dtype=np.int64)
        self.foff = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        self.fids = (np.concatenate([np.asarray(s.frame_ids, dtype=np.int64) for s in self.specs])
                     if n else np.zeros(0, dtype=np.int64))
        self.hptr = np.zeros(n, dtype=np.uint64)
        self.winp = np.zeros(n, dtype=np.uint64)
        self.wrow = np.array([4 * s.cfg["winners"] for s in self.specs], dtype=np.uint64)
        self.keep = keep_outputs
        self.max_frames = int(max_frames)
        self.win = [None] * n
        self.hist = [None] * n
        self.stream = torch.cuda.Stream()
        self.side = torch.cuda.Stream()
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(self.stream)
        self.ref.synchronize()
        self.ref_host = time.perf_counter()
        self.t_start = self.ref_host
        self.gpu_ms = []         # GPU time of each batch
        self.batch_wall = []     # completion minus launch, host clock, each batch
        self.frames_done = 0

    def set_start(self, host_t0: float):
        self.t_start = host_t0

    def stream_bytes(self, spec: StreamSpec) -> int:
        C, S = spec.cfg["num_columns"], spec.cfg["synapses_per_column"]
        return 8 * C * S + int(self._ws_bytes(spec.cfg))

    def open(self, i: int, spec: StreamSpec, checkpoint=None):
        torch = self.torch
        from . import SpatialPooler
        perm = spec.perm if checkpoint is None else checkpoint
        with torch.cuda.stream(self.side):
            if self.hist[i] is None:
                # per-stream outputs, kept across evictions: winners of every
                # frame (or a scratch row block) and the SDR histogram
                # (Section 2's per-video feature vector)
                rows = len(spec.arrivals) if self.keep else self.max_frames
                self.win[i] = torch.empty((rows, spec.cfg["winners"]), dtype=torch.int32,
                                          device="cuda")
                self.hist[i] = torch.zeros(spec.cfg["num_columns"], dtype=torch.int32,
                                           device="cuda")
            # creation synchronises the side stream only (its state check)
            pool = SpatialPooler(spec.cfg, spec.idx, perm, stream=self.side)
        pool.set_histogram(self.hist[i])
        self.hptr[i] = pool.handle
        self.winp[i] = self.win[i].data_ptr()
        return {"i": i, "pool": pool}

    def evict(self, h):
        """Checkpoint of the permanences (the pools never change), then the
        handle is destroyed; the stream has no batch in flight."""
        _, perm, _ = h["pool"].get_state(stream=self.side, with_idx=False)
        self.close(h)
        return perm

    def close(self, h):
        h["pool"].close()
        self.hptr[h["i"]] = 0

    def launch(self, ids, firsts, counts):
        torch = self.torch
        from . import sp_step_many_raw
        fp = self.fbase + self.fids[self.foff[ids] + firsts].astype(np.uint64) * self.row_bytes
        wp = self.winp[ids]
        if self.keep:
            wp = wp + firsts.astype(np.uint64) * self.wrow[ids]
        elif int(counts.max()) > self.max_frames:
            # (winners not kept: each batch of a stream overwrites its block
            # of max_frames rows)
            raise ValueError(f"a batch holds {int(counts.max())} frames of one stream; "
                             f"the backend keeps rows for {self.max_frames}")
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(self.stream)
        sp_step_many_raw(self.hptr[ids], fp, counts.astype(np.uint32), True, None, wp,
                         self.stream)
        ev1.record(self.stream)
        return (ev0, ev1, time.perf_counter(), int(counts.sum()))

    def finished(self, token):
        ev0, ev1, t_launch, nfr = token
        if not ev1.query():
            return None
        t_done = self.ref_host + self.ref.elapsed_time(ev1) * 1e-3
        self.gpu_ms.append(ev0.elapsed_time(ev1))
        self.batch_wall.append(t_done - t_launch)
        self.frames_done += nfr
        return t_done - self.t_start

    def winners(self, i: int):
        return self.win[i]

    def histogram(self, i: int):
        return self.hist[i]


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
                 input_bits: int = 960 * 540, min_len: float | None = None,
                 max_len: float | None = None):
    """Streams with pooler sizes drawn like the multi-instance workload, each
    sending Poisson(fps) frames.  By default every stream is live for the
    whole window (a random phase comes from the first exponential gap); with
    min_len/max_len a stream lasts a uniform length in that range from a
    uniform start inside the window.  Each stream reads consecutive frames of
    a shared pool from a random offset."""
    from . import synth
    g = synth.rng(seed, 0)
    specs = []
    for s in range(n_streams):
        C, S = int(g.choice(columns)), int(g.choice(synapses))
        cfg = synth.sp_config(input_bits, C, S, 4, max(1, 10 * C // 256))
        if min_len is None:
            length, start = float(window), 0.0
        else:
            length = float(g.uniform(min_len, max_len))
            start = float(g.uniform(0.0, max(0.0, window - length)))
        arr = poisson_arrivals(synth.rng(seed * 1000 + s, 3), fps, start, length)
        off = int(g.integers(0, pool_frames))
        ids = (off + np.arange(len(arr))) % pool_frames
        idx = synth.pools(synth.rng(seed * 1000 + s, 0), input_bits, C, S)
        perm = synth.q_to_float(synth.permanences_q(synth.rng(seed * 1000 + s, 1), C, S))
        specs.append(StreamSpec(s, cfg, idx, perm, arr, ids))
    return specs
