"""Checkpoint and resume through the C ABI (sp_get_state / sp_set_state and
the boost state's getter and setter): a pooler that learns 500 frames, is
saved, destroyed, re-created from other state and restored, then learns 500
more, ends bit for bit where one that learned all 1000 frames uninterrupted
ends -- for sp_step, sp_step_boost and sp_step_many -- and the setters refuse
bad contents without changing anything."""
import numpy as np
import pytest

import oracle
import paper_1608_01966_amd as sp
from paper_1608_01966_amd import synth

pytestmark = pytest.mark.gpu

BC = {"period_log2": 10, "min_pct_q16": 655, "max_boost_q8": 2560, "bump_q8": 13}


def _dev(frames):
    import torch
    return torch.from_numpy(np.ascontiguousarray(frames).view(np.int32)).cuda()


def test_resume_step_equals_uninterrupted():
    """The paper-scale learning workload: 960x540 blob frames, 1024 x 256."""
    w = synth.workload_paper_scale(frames=1000, columns=1024, synapses=256)
    frames = _dev(w.frames)
    a = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    ov_a, win_a = a.step(frames)
    a.sync()

    b = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    ov1, win1 = b.step(frames[:500])
    idx, perm, seen = b.get_state()
    assert seen == 500
    b.close()
    # a new handle over other state, then the checkpoint
    other = synth.random_instance(99, w.cfg, frames=1)
    c = sp.SpatialPooler(w.cfg, other.idx, other.perm)
    c.set_state(idx, perm, seen)
    ov2, win2 = c.step(frames[500:])
    c.sync()
    assert np.array_equal(np.concatenate([win1.cpu().numpy(), win2.cpu().numpy()]),
                          win_a.cpu().numpy())
    assert np.array_equal(np.concatenate([ov1.cpu().numpy(), ov2.cpu().numpy()]),
                          ov_a.cpu().numpy())
    assert np.array_equal(c.perm.cpu().numpy(), a.perm.cpu().numpy())
    assert np.array_equal(c.idx.cpu().numpy(), a.idx.cpu().numpy())
    assert c.get_state()[2] == 1000
    # and the uninterrupted run is the oracle's
    _, e_win, e_perm = oracle.run(w.cfg, w.idx, w.perm, w.frames, learn=True,
                                  want_overlaps=False)
    assert np.array_equal(win_a.cpu().numpy(), e_win)
    assert np.array_equal(a.perm.cpu().numpy().astype(np.float64), e_perm)
    a.close()
    c.close()


def _boost_run(pool, cfg, frames):
    import torch
    F = frames.shape[0]
    ov = torch.empty((F, cfg["num_columns"]), dtype=torch.int32, device="cuda")
    win = torch.empty((F, cfg["winners"]), dtype=torch.int32, device="cuda")
    sp.sp_step_boost(pool.handle, cfg, BC, frames, True, ov, win)
    return ov, win


def test_resume_boost_equals_uninterrupted():
    w = synth.workload_paper_scale(frames=1000, columns=1024, synapses=256)
    cfg, frames = w.cfg, _dev(w.frames)
    a = sp.SpatialPooler(cfg, w.idx, w.perm)
    ov_a, win_a = _boost_run(a, cfg, frames)
    a.sync()
    b = sp.SpatialPooler(cfg, w.idx, w.perm)
    ov1, win1 = _boost_run(b, cfg, frames[:500])
    b.sync()
    idx, perm, seen = b.get_state()
    boost_state = sp.sp_get_boost_state(b.handle, cfg["num_columns"])
    assert seen == 500
    b.close()
    c = sp.SpatialPooler(cfg, w.idx, w.perm)
    c.set_state(idx, perm, seen)
    sp.sp_set_boost_state(c.handle, *boost_state)
    ov2, win2 = _boost_run(c, cfg, frames[500:])
    c.sync()
    assert np.array_equal(np.concatenate([win1.cpu().numpy(), win2.cpu().numpy()]),
                          win_a.cpu().numpy())
    assert np.array_equal(np.concatenate([ov1.cpu().numpy(), ov2.cpu().numpy()]),
                          ov_a.cpu().numpy())
    assert np.array_equal(c.perm.cpu().numpy(), a.perm.cpu().numpy())
    for x, y in zip(sp.sp_get_boost_state(c.handle, cfg["num_columns"]),
                    sp.sp_get_boost_state(a.handle, cfg["num_columns"])):
        assert np.array_equal(x, y)
    a.close()
    c.close()


def test_resume_many_equals_uninterrupted():
    """Eight instances of the multi-instance workload, 100 frames each, stepped
    together; checkpointed after 50."""
    import torch
    ws = synth.workload_multi(instances=8, frames=100)
    fr = [_dev(w.frames) for w in ws]
    cfgs = [w.cfg for w in ws]

    def many(pools, lo, hi):
        wins = [torch.empty((hi - lo, w.cfg["winners"]), dtype=torch.int32, device="cuda")
                for w in ws]
        sp.sp_step_many([p.handle for p in pools], cfgs, [f[lo:hi] for f in fr], True, None,
                        wins)
        pools[0].sync()
        return [x.cpu().numpy() for x in wins]

    a = [sp.SpatialPooler(w.cfg, w.idx, w.perm) for w in ws]
    win_a = many(a, 0, 100)
    b = [sp.SpatialPooler(w.cfg, w.idx, w.perm) for w in ws]
    win1 = many(b, 0, 50)
    ck = [p.get_state() for p in b]
    for p in b:
        p.close()
    c = [sp.SpatialPooler(w.cfg, w.idx, w.perm) for w in ws]
    for p, (idx, perm, seen) in zip(c, ck):
        assert seen == 50
        p.set_state(idx, perm, seen)
    win2 = many(c, 50, 100)
    for i in range(len(ws)):
        assert np.array_equal(np.concatenate([win1[i], win2[i]]), win_a[i]), i
        assert np.array_equal(c[i].perm.cpu().numpy(), a[i].perm.cpu().numpy()), i
        assert c[i].get_state()[2] == 100
    for p in a + c:
        p.close()


def test_setters_refuse_bad_contents():
    w = synth.random_instance(31, synth.sp_config(2000, 64, 32, 2, 5), frames=4)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    idx0, perm0, _ = pool.get_state()
    bad_perm = perm0.copy()
    bad_perm[3, 7] = 0.3
    with pytest.raises(sp.SpError, match=r"perm\[103\]") as e:
        pool.set_state(idx0, bad_perm)
    assert e.value.code == sp.SP_EINVAL
    bad_idx = idx0.copy()
    bad_idx[1, 2] = 2000
    with pytest.raises(sp.SpError, match=r"idx\[34\]") as e:
        pool.set_state(bad_idx, perm0)
    assert e.value.code == sp.SP_EINVAL
    idx1, perm1, _ = pool.get_state()
    assert np.array_equal(idx1, idx0) and np.array_equal(perm1, perm0)
    C = w.cfg["num_columns"]
    adc, odc, boost = sp.sp_get_boost_state(pool.handle, C)
    assert not adc.any() and not odc.any() and (boost == 256).all()
    for arrays, what in [((adc, odc, np.full(C, 255, np.uint32)), "boost"),
                         ((adc, np.full(C, 65537, np.uint32), boost), "duty"),
                         ((adc, odc, np.full(C, 4097, np.uint32)), "boost")]:
        with pytest.raises(sp.SpError, match=what) as e:
            sp.sp_set_boost_state(pool.handle, *arrays)
        assert e.value.code == sp.SP_EINVAL
    # a good boost state round-trips
    g = np.random.default_rng(3)
    st = (g.integers(0, 65537, C).astype(np.uint32), g.integers(0, 65537, C).astype(np.uint32),
          g.integers(256, 4097, C).astype(np.uint32))
    sp.sp_set_boost_state(pool.handle, *st)
    for x, y in zip(sp.sp_get_boost_state(pool.handle, C), st):
        assert np.array_equal(x, y)
    # idx None keeps the pools; the frame count is the caller's
    perm2 = np.full_like(perm0, 0.5)
    pool.set_state(None, perm2, 12345)
    idx3, perm3, seen3 = pool.get_state()
    assert np.array_equal(idx3, idx0) and np.array_equal(perm3, perm2) and seen3 == 12345
    pool.close()


def test_inference_sees_restored_state():
    """Both inference modes rebuild what they derive from the state after a
    restore."""
    w = synth.random_instance(32, synth.sp_config(3000, 128, 40, 2, 8), frames=12, density=0.2)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    for mode in (sp.SP_INFER_GATHER, sp.SP_INFER_MFMA_I8):
        pool.infer(w.frames, mode=mode)
    other = synth.random_instance(33, w.cfg, frames=1)
    pool.set_state(other.idx, other.perm)
    e_ov, e_win, _ = oracle.run(w.cfg, other.idx, other.perm, w.frames, learn=False)
    for mode in (sp.SP_INFER_GATHER, sp.SP_INFER_MFMA_I8):
        ov, win = pool.infer(w.frames, mode=mode)
        pool.sync()
        assert np.array_equal(ov.cpu().numpy(), e_ov), mode
        assert np.array_equal(win.cpu().numpy(), e_win), mode
    pool.close()
