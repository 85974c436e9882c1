"""Per-stream SDR histograms on the GPU (Section 2's per-video histogram of
the pooler output) against the oracle's histogram of the oracle's winners,
for every execution path; accumulation over calls; switching off."""
import numpy as np
import pytest

import oracle
import paper_1608_01966_amd as sp
from paper_1608_01966_amd import synth

pytestmark = pytest.mark.gpu


def _hist(C):
    import torch
    return torch.zeros(C, dtype=torch.int32, device="cuda")


@pytest.mark.parametrize("path", ["persistent", "plain", "infer"])
def test_paths(path):
    cfg = synth.sp_config(100_000, 700, 96, 3, 30)
    w = synth.random_instance(31, cfg, 60, density=0.08)
    learn = path != "infer"
    _, e_win, _ = oracle.run(cfg, w.idx, w.perm, w.frames, learn=learn, want_overlaps=False)
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    h = _hist(cfg["num_columns"])
    pool.set_histogram(h)
    if path == "infer":
        _, win = pool.infer(w.frames, overlaps=False)
    else:
        _, win = pool.step(w.frames, learn=True, overlaps=False, plain=path == "plain")
    pool.sync()
    assert np.array_equal(win.cpu().numpy(), e_win)
    assert np.array_equal(h.cpu().numpy().astype(np.uint32), oracle.histogram(e_win, 700))
    pool.close()


def test_accumulates_then_stops():
    w = synth.workload_plain_32x32(frames=40)
    _, e_win, _ = oracle.run(w.cfg, w.idx, w.perm, w.frames, learn=True, want_overlaps=False)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    h = _hist(256)
    pool.set_histogram(h)
    pool.step(w.frames[:15])
    pool.step(w.frames[15:30])
    pool.set_histogram(None)
    pool.step(w.frames[30:])
    pool.sync()
    assert np.array_equal(h.cpu().numpy().astype(np.uint32), oracle.histogram(e_win[:30], 256))
    pool.close()


def test_many_instances():
    import torch
    ws = [synth.random_instance(40 + i, synth.sp_config(n, c, s, 4, max(1, c // 32)), f,
                                density=0.06)
          for i, (n, c, s, f) in enumerate([(4096, 256, 32, 25), (20000, 1024, 128, 40),
                                             (50000, 3000, 64, 7)])]
    pools = [sp.SpatialPooler(w.cfg, w.idx, w.perm) for w in ws]
    hists = [_hist(w.cfg["num_columns"]) for w in ws]
    for p, h in zip(pools, hists):
        p.set_histogram(h)
    frames = [torch.from_numpy(w.frames.view(np.int32)).cuda() for w in ws]
    wins = [torch.empty((w.frames.shape[0], w.cfg["winners"]), dtype=torch.int32, device="cuda")
            for w in ws]
    stream = torch.cuda.current_stream()
    sp.sp_step_many([p.handle for p in pools], [w.cfg for w in ws], frames, True, None, wins,
                    stream)
    pools[0].sync()
    for w, h, wn in zip(ws, hists, wins):
        _, e_win, _ = oracle.run(w.cfg, w.idx, w.perm, w.frames, learn=True, want_overlaps=False)
        assert np.array_equal(wn.cpu().numpy(), e_win)
        assert np.array_equal(h.cpu().numpy().astype(np.uint32),
                              oracle.histogram(e_win, w.cfg["num_columns"]))
    for p in pools:
        p.close()


@pytest.mark.parametrize("C", [700, 1500])  # persistent boosted step, and the plain sequence
def test_boosted_step(C):
    import torch
    bc = {"period_log2": 6, "min_pct_q16": 16384, "max_boost_q8": 2560, "bump_q8": 13}
    cfg = synth.sp_config(100_000, C, 96, 3, 30)
    w = synth.random_instance(37 + C, cfg, 24, density=0.08)
    _, e_win, _, _ = oracle.run_boost(cfg, bc, w.idx, w.perm, w.frames, want_overlaps=False)
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    assert pool.boost_kernel == ("k_sp_persistent_boost" if C <= 1024 else "plain")
    h = _hist(C)
    pool.set_histogram(h)
    frames = torch.from_numpy(w.frames.view(np.int32)).cuda()
    win = torch.empty((24, 30), dtype=torch.int32, device="cuda")
    sp.sp_step_boost(pool.handle, cfg, bc, frames, True, None, win)
    pool.sync()
    assert np.array_equal(win.cpu().numpy(), e_win)
    assert np.array_equal(h.cpu().numpy().astype(np.uint32), oracle.histogram(e_win, C))
    pool.close()


@pytest.mark.parametrize("persistent", [True, False])
def test_local_step(persistent):
    """sp_step_local adds each frame's active columns (its output is an
    active mask, not a winner list) on the persistent and the per-frame
    executions; two calls accumulate."""
    import torch
    if persistent:
        w = synth.workload_paper_scale(frames=24, columns=1024, synapses=128)
        w.cfg["winners"] = 4
        grid_w, radius = 32, 3
    else:
        # more columns than one persistent launch exchanges: per-frame launches
        cfg = synth.sp_config(20_000, 5000, 16, 2, 3)
        w = synth.random_instance(7, cfg, 12, density=0.1)
        grid_w, radius = 100, 2
    cfg = w.cfg
    C, F = cfg["num_columns"], w.frames.shape[0]
    _, e_act, _ = oracle.run_local(cfg, w.idx, w.perm, w.frames, grid_w, radius, cfg["winners"])
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    assert (pool.local_kernel == "k_sp_persistent_local") == persistent
    h = _hist(C)
    pool.set_histogram(h)
    frames = torch.from_numpy(np.ascontiguousarray(w.frames).view(np.int32)).cuda()
    act = torch.empty((F, C), dtype=torch.uint8, device="cuda")
    half = F // 2
    sp.sp_step_local(pool.handle, cfg, frames[:half], True, grid_w, radius, None, act[:half])
    sp.sp_step_local(pool.handle, cfg, frames[half:], True, grid_w, radius, None, act[half:])
    pool.sync()
    want = e_act.astype(np.int64).sum(axis=0)
    assert want.sum() > 0
    assert np.array_equal(h.cpu().numpy().astype(np.int64), want)
    pool.close()
