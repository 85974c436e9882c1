"""The persistent steps' failure path, forced from the host: sp_test_stall
makes the next persistent launch wait for exchange entries that are never
written, under a small spin limit.  Every wave must give up within its own
bounded wait and the launch must drain; sp_sync then reports SP_EDEVICE, the
handle refuses further steps (SP_EBROKEN) and can still be destroyed."""
import numpy as np
import pytest

import paper_1608_01966_amd as sp
from paper_1608_01966_amd import synth

pytestmark = pytest.mark.gpu

BC = {"period_log2": 6, "min_pct_q16": 16384, "max_boost_q8": 2560, "bump_q8": 13}


def _step(kind, pool, cfg, frames, F):
    import torch
    C, k = cfg["num_columns"], cfg["winners"]
    if kind == "global":
        sp.sp_step(pool.handle, cfg, frames, True, None,
                   torch.empty((F, k), dtype=torch.int32, device="cuda"))
    elif kind == "local":
        # two frames per exchange
        sp.sp_step_local(pool.handle, cfg, frames, True, 1024, 80, None,
                         torch.empty((F, C), dtype=torch.uint8, device="cuda"))
    elif kind == "local_one_frame":
        # a 64 x 64 grid whose radius-40 windows are too large for two frames
        # per exchange
        sp.sp_step_local(pool.handle, cfg, frames, True, 64, 40, None,
                         torch.empty((F, C), dtype=torch.uint8, device="cuda"))
    else:
        sp.sp_step_boost(pool.handle, cfg, BC, frames, True, None,
                         torch.empty((F, k), dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("kind", ["global", "local", "local_one_frame", "boost"])
def test_stalled_exchange_drains_and_reports(kind):
    import torch
    if kind == "local_one_frame":
        w = synth.workload_paper_scale(frames=8, columns=4096, synapses=64)
    else:
        w = synth.workload_paper_scale(frames=8, columns=1024, synapses=256)
    cfg = w.cfg
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    assert {"global": pool.kernel, "local": pool.local_kernel_for(1024, 80),
            "local_one_frame": pool.local_kernel_for(64, 40),
            "boost": pool.boost_kernel}[kind] == {
                "global": "k_sp_persistent_w", "local": "k_sp_persistent_local2",
                "local_one_frame": "k_sp_persistent_local",
                "boost": "k_sp_persistent_boost"}[kind]
    frames = torch.from_numpy(w.frames.view(np.int32)).cuda()
    sp.sp_test_stall(pool.handle, 200)
    _step(kind, pool, cfg, frames, 8)
    with pytest.raises(sp.SpError) as e:
        pool.sync()
    assert e.value.code == sp.SP_EDEVICE
    with pytest.raises(sp.SpError) as e:
        _step(kind, pool, cfg, frames, 8)
    assert e.value.code == sp.SP_EBROKEN
    pool.close()


def test_stall_applies_to_one_launch_only():
    """A stall request is consumed by one launch: a fresh handle that never
    had one runs the same frames to the same results as before."""
    import torch
    w = synth.workload_paper_scale(frames=6, columns=1024, synapses=256)
    cfg = w.cfg
    frames = torch.from_numpy(w.frames.view(np.int32)).cuda()
    a = sp.SpatialPooler(cfg, w.idx, w.perm)
    with pytest.raises(sp.SpError):
        sp.sp_test_stall(a.handle, 0)
    ov, win = a.step(frames)
    a.sync()
    b = sp.SpatialPooler(cfg, w.idx, w.perm)
    ov2, win2 = b.step(frames)
    b.sync()
    assert torch.equal(win, win2) and torch.equal(ov, ov2)
    a.close()
    b.close()


def test_many_instance_stall_marks_every_handle():
    """One handle of a sp_step_many launch waits for entries that are never
    written: every wait of the launch gives up and the launch drains.  The
    stalled handle reports SP_EDEVICE on sp_sync and refuses further steps;
    every other handle either reports SP_EDEVICE too (its steps may have been
    cut short) or took all its steps and holds the oracle's results.  A later
    launch over fresh handles is unaffected (the error word belongs to one
    launch)."""
    import torch
    import oracle
    ws = [synth.random_instance(60 + i, synth.sp_config(4096, 256 * (i + 1), 64, 2, 10),
                                frames=6, density=0.2) for i in range(3)]

    def step_all(pools):
        wins = [torch.empty((6, w.cfg["winners"]), dtype=torch.int32, device="cuda") for w in ws]
        fr = [torch.from_numpy(w.frames.view(np.int32)).cuda() for w in ws]
        sp.sp_step_many([p.handle for p in pools], [w.cfg for w in ws], fr, True, None, wins)
        return wins

    def expect(w):
        return oracle.run(w.cfg, w.idx, w.perm, w.frames, learn=True, want_overlaps=False)

    pools = [sp.SpatialPooler(w.cfg, w.idx, w.perm) for w in ws]
    sp.sp_test_stall(pools[1].handle, 200)
    wins = step_all(pools)
    torch.cuda.synchronize()
    for i, (p, w, wn) in enumerate(zip(pools, ws, wins)):
        try:
            p.sync()
        except sp.SpError as e:
            assert e.code == sp.SP_EDEVICE
            with pytest.raises(sp.SpError) as e2:
                sp.sp_step(p.handle, w.cfg, torch.from_numpy(w.frames.view(np.int32)).cuda(),
                           True, None, torch.empty((6, w.cfg["winners"]), dtype=torch.int32,
                                                   device="cuda"))
            assert e2.value.code == sp.SP_EBROKEN
            continue
        assert i != 1, "the stalled handle reported no failure"
        _, e_win, e_perm = expect(w)
        assert np.array_equal(wn.cpu().numpy(), e_win), i
        assert np.array_equal(p.perm.cpu().numpy().astype(np.float64), e_perm), i
    for p in pools:
        p.close()
    fresh = [sp.SpatialPooler(w.cfg, w.idx, w.perm) for w in ws]
    wins = step_all(fresh)
    for p in fresh:
        p.sync()
    for w, wn in zip(ws, wins):
        _, e_win, _ = expect(w)
        assert np.array_equal(wn.cpu().numpy(), e_win)
    for p in fresh:
        p.close()
