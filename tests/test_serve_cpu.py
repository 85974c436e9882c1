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
    `latency` seconds of server time later."""

    def __init__(self, pool, clock, latency=0.002):
        self.pool = pool            # uint32 [P][W]
        self.clock = clock
        self.latency = latency
        self.open_count = 0
        self.max_open = 0
        self.launches = []

    def stream_bytes(self, spec):
        return 8 * spec.cfg["num_columns"] * spec.cfg["synapses_per_column"]

    def open(self, spec):
        self.open_count += 1
        self.max_open = max(self.max_open, self.open_count)
        self.open_bytes = getattr(self, "open_bytes", 0) + self.stream_bytes(spec)
        self.max_open_bytes = max(getattr(self, "max_open_bytes", 0), self.open_bytes)
        return {"perm": spec.perm.astype(np.float64), "win": [], "ov": [],
                "bytes": self.stream_bytes(spec)}

    def close(self, h):
        self.open_count -= 1
        self.open_bytes -= h["bytes"]

    def launch(self, items):
        self.launches.append([(spec.sid, first, n) for _, spec, first, n in items])
        for h, spec, first, n in items:
            ids = spec.frame_ids[first:first + n]
            assert np.all(np.diff(ids) == 1)
            ov, win, h["perm"] = oracle.run(spec.cfg, spec.idx, h["perm"], self.pool[ids])
            h["win"].append(win)
            h["ov"].append(ov)
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


def test_every_stream_equals_alone():
    specs = small_streams(12)
    fr = pool()
    clock = FakeClock()
    be = OracleBackend(fr, clock)
    srv = serve.Server(be, specs, budget_bytes=10 ** 9)
    handles = {}
    orig_open = be.open

    def open_(spec):
        h = orig_open(spec)
        handles[spec.sid] = h
        return h
    be.open = open_
    srv.run(clock)
    for spec in specs:
        h = handles[spec.sid]
        e_ov, e_win, e_perm = oracle.run(spec.cfg, spec.idx, spec.perm, fr[spec.frame_ids])
        assert np.array_equal(np.concatenate(h["win"]), e_win)
        assert np.array_equal(np.concatenate(h["ov"]), e_ov)
        assert np.array_equal(h["perm"], e_perm)
    # streams overlapped in time, so batches held several streams
    assert max(len(b) for b in be.launches) > 1


def test_frames_in_order_and_complete():
    specs = small_streams(8, seed=5)
    clock = FakeClock()
    be = OracleBackend(pool(), clock)
    srv = serve.Server(be, specs, budget_bytes=10 ** 9, max_frames_per_tick=3)
    srv.run(clock)
    seen = {s.sid: [] for s in specs}
    for batch in be.launches:
        sids = [sid for sid, _, _ in batch]
        assert len(sids) == len(set(sids)), "a stream appears twice in one batch"
        for sid, first, n in batch:
            assert 1 <= n <= 3
            seen[sid].extend(range(first, first + n))
    for s in specs:
        assert seen[s.sid] == list(range(len(s.arrivals)))
    lat = srv.latencies()
    assert lat.size == sum(len(s.arrivals) for s in specs) and np.all(lat > 0)
    for st in srv.streams:
        assert st.finished and st.done == len(st.spec.arrivals)


def test_admission_respects_budget():
    specs = small_streams(20, seed=6)
    need = [8 * s.cfg["num_columns"] * s.cfg["synapses_per_column"] for s in specs]
    budget = max(need) + min(need)   # far less than all streams together
    clock = FakeClock()
    be = OracleBackend(pool(), clock)
    srv = serve.Server(be, specs, budget_bytes=budget)
    srv.run(clock)
    assert srv.peak_used <= budget and be.max_open_bytes <= budget
    assert be.max_open < len(specs)
    assert all(st.finished for st in srv.streams)
    assert max(srv.admit_waits) > 0  # some stream had to wait for budget


def test_stream_over_budget_is_rejected():
    specs = small_streams(2, seed=7)
    be = OracleBackend(pool(), FakeClock())
    srv = serve.Server(be, specs, budget_bytes=1)
    with pytest.raises(ValueError, match="over the budget"):
        srv.run(FakeClock())


def test_poisson_arrivals_rate():
    g = np.random.default_rng(0)
    t = serve.poisson_arrivals(g, 30.0, 1.0, 100.0)
    assert np.all(np.diff(t) > 0) and t[0] >= 1.0 and t[-1] < 101.0
    assert abs(len(t) - 3000) < 200
