"""The serving scheduler without a GPU: a backend that steps each stream's
frames with the oracle shows admission by budget, strict per-stream order,
batching of concurrent streams, and that every stream's results equal
stepping it alone."""
import numpy as np
import pytest

import oracle
from paper_1608_01966_amd import serve, synth


class OracleBackend:
    """Runs a batch at launch time with the oracle; the batch completes
    `latency` seconds of server time later.  Eviction checkpoints the
    permanences; every stream's outputs accumulate across evictions."""

    def __init__(self, pool, specs, clock, latency=0.002):
        self.pool = pool            # uint32 [P][W]
        self.specs = specs
        self.clock = clock
        self.latency = latency
        self.open_count = 0
        self.max_open = 0
        self.open_bytes = 0
        self.max_open_bytes = 0
        self.launches = []
        self.live = {}
        self.win = {s.sid: [] for s in specs}
        self.ov = {s.sid: [] for s in specs}
        self.final = {}
        self.opened_from_ckpt = 0

    def stream_bytes(self, spec):
        return 8 * spec.cfg["num_columns"] * spec.cfg["synapses_per_column"]

    def open(self, i, spec, ckpt):
        assert i not in self.live
        self.open_count += 1
        self.max_open = max(self.max_open, self.open_count)
        self.open_bytes += self.stream_bytes(spec)
        self.max_open_bytes = max(self.max_open_bytes, self.open_bytes)
        self.opened_from_ckpt += ckpt is not None
        perm = (spec.perm if ckpt is None else ckpt).astype(np.float64)
        self.live[i] = {"i": i, "perm": perm, "bytes": self.stream_bytes(spec)}
        return self.live[i]

    def close(self, h):
        self.final[h["i"]] = h["perm"]
        del self.live[h["i"]]
        self.open_count -= 1
        self.open_bytes -= h["bytes"]

    def evict(self, h):
        perm = h["perm"].astype(np.float32)
        self.close(h)
        return perm

    def launch(self, ids, firsts, counts):
        self.launches.append([(int(i), int(f), int(n)) for i, f, n in zip(ids, firsts, counts)])
        for i, first, n in zip(ids, firsts, counts):
            spec, h = self.specs[i], self.live[int(i)]
            fids = spec.frame_ids[first:first + n]
            assert np.all(np.diff(fids) == 1)
            ov, win, h["perm"] = oracle.run(spec.cfg, spec.idx, h["perm"], self.pool[fids])
            self.win[spec.sid].append(win)
            self.ov[spec.sid].append(ov)
        return self.clock() + self.latency

    def finished(self, t_done):
        return t_done if self.clock() >= t_done else None


class FakeClock:
    def __init__(self, step=0.001):
        self.t = 0.0
        self.step = step

    def __call__(self):
        self.t += self.step
        return self.t


def small_streams(n, seed=3):
    return serve.make_streams(n, fps=200.0, window=0.5, pool_frames=40, seed=seed,
                              columns=(8, 16, 32), synapses=(4, 8, 16), input_bits=300,
                              min_len=0.05, max_len=0.2)


def pool(seed=4):
    return synth.bernoulli_frames(synth.rng(seed, 2), 40, 300, 0.2)


def check_alone(specs, fr, be):
    for spec in specs:
        e_ov, e_win, e_perm = oracle.run(spec.cfg, spec.idx, spec.perm, fr[spec.frame_ids])
        assert np.array_equal(np.concatenate(be.win[spec.sid]), e_win), f"stream {spec.sid}"
        assert np.array_equal(np.concatenate(be.ov[spec.sid]), e_ov), f"stream {spec.sid}"
        assert np.array_equal(be.final[spec.sid], e_perm), f"stream {spec.sid}"


def test_every_stream_equals_alone():
    specs = small_streams(12)
    fr = pool()
    clock = FakeClock()
    be = OracleBackend(fr, specs, clock)
    srv = serve.Server(be, specs, budget_bytes=10 ** 9)
    srv.run(clock)
    check_alone(specs, fr, be)
    # streams overlapped in time, so batches held several streams
    assert max(len(b) for b in be.launches) > 1
    assert srv.evictions == 0


def test_eviction_and_readmission_equal_alone():
    """Budget for a third of the streams, all live for the whole window:
    streams are evicted after their quantum (permanences checkpointed) and
    re-admitted later, and every stream's results still equal stepping it
    alone."""
    specs = serve.make_streams(9, fps=100.0, window=0.6, pool_frames=40, seed=8,
                               columns=(8, 16, 32), synapses=(4, 8, 16), input_bits=300)
    fr = pool()
    clock = FakeClock()
    be = OracleBackend(fr, specs, clock)
    need = [be.stream_bytes(s) for s in specs]
    budget = sum(sorted(need)[-3:])
    srv = serve.Server(be, specs, budget_bytes=budget, quantum=0.05)
    srv.run(clock)
    assert srv.evictions > 0 and srv.readmissions > 0
    assert be.opened_from_ckpt == srv.readmissions
    assert srv.peak_used <= budget and be.max_open_bytes <= budget
    assert be.max_open < len(specs)
    assert srv.finished.all()
    check_alone(specs, fr, be)


def test_frames_in_order_and_complete():
    specs = small_streams(8, seed=5)
    clock = FakeClock()
    be = OracleBackend(pool(), specs, clock)
    srv = serve.Server(be, specs, budget_bytes=10 ** 9, max_frames_per_tick=3)
    srv.run(clock)
    seen = {i: [] for i in range(len(specs))}
    for batch in be.launches:
        ids = [i for i, _, _ in batch]
        assert len(ids) == len(set(ids)), "a stream appears twice in one batch"
        for i, first, n in batch:
            assert 1 <= n <= 3
            seen[i].extend(range(first, first + n))
    for i, s in enumerate(specs):
        assert seen[i] == list(range(len(s.arrivals)))
        # a frame completes after it arrives
        assert np.all(srv.completions(i) > s.arrivals)
    lat = srv.latencies()
    assert lat.size == sum(len(s.arrivals) for s in specs) and np.all(lat > 0)
    assert srv.finished.all() and np.array_equal(srv.done, srv.nframes)


def test_admission_respects_budget():
    specs = small_streams(20, seed=6)
    need = [8 * s.cfg["num_columns"] * s.cfg["synapses_per_column"] for s in specs]
    budget = max(need) + min(need)   # far less than all streams together
    clock = FakeClock()
    be = OracleBackend(pool(), specs, clock)
    srv = serve.Server(be, specs, budget_bytes=budget)
    srv.run(clock)
    assert srv.peak_used <= budget and be.max_open_bytes <= budget
    assert be.max_open < len(specs)
    assert srv.finished.all()
    assert max(srv.admit_waits) > 0  # some stream had to wait for budget


def test_stream_over_budget_is_rejected():
    specs = small_streams(2, seed=7)
    be = OracleBackend(pool(), specs, FakeClock())
    srv = serve.Server(be, specs, budget_bytes=1)
    with pytest.raises(ValueError, match="over the budget"):
        srv.run(FakeClock())


def test_poisson_arrivals_rate():
    g = np.random.default_rng(0)
    t = serve.poisson_arrivals(g, 30.0, 1.0, 100.0)
    assert np.all(np.diff(t) > 0) and t[0] >= 1.0 and t[-1] < 101.0
    assert abs(len(t) - 3000) < 200


def test_ranges_helper():
    got = serve._ranges(np.array([5, 0, 10]), np.array([2, 0, 3]))
    assert got.tolist() == [5, 6, 10, 11, 12]


def test_streams_live_for_the_whole_window_by_default():
    specs = serve.make_streams(6, fps=30.0, window=10.0, pool_frames=64, seed=5,
                               columns=(8,), synapses=(4,), input_bits=300)
    for s in specs:
        assert s.arrivals[0] < 1.0 and s.arrivals[-1] > 9.0
        assert 200 < len(s.arrivals) < 400


def test_preadmit_within_budget():
    specs = small_streams(10, seed=9)
    clock = FakeClock()
    fr = pool()
    be = OracleBackend(fr, specs, clock)
    need = [be.stream_bytes(s) for s in specs]
    budget = sum(need) - min(need)   # all but (at least) one stream
    srv = serve.Server(be, specs, budget_bytes=budget)
    srv.preadmit()
    assert 0 < srv.resident.sum() < len(specs) and srv.used <= budget
    srv.run(clock)
    assert srv.finished.all() and srv.peak_used <= budget
    check_alone(specs, fr, be)
