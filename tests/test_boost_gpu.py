"""Boosting and duty cycles on the GPU against the oracle (readings B1-B7):
boosted overlaps, winners, permanences and the whole boost state, bit for
bit, across calls, with learning off, and after a reset."""
import json
import os

import numpy as np
import pytest

import oracle
import paper_1608_01966_amd as sp
from paper_1608_01966_amd import synth

pytestmark = pytest.mark.gpu

# a minimum duty cycle of a quarter of the maximum keeps boosts and raises
# active on these short runs
BC = {"period_log2": 6, "min_pct_q16": 16384, "max_boost_q8": 2560, "bump_q8": 13}
GOLD = os.path.join(os.path.dirname(__file__), "golden", "boost_3col.json")


def _run(pool, cfg, bc, frames_np, learn=True):
    import torch
    F = frames_np.shape[0]
    frames = torch.from_numpy(np.ascontiguousarray(frames_np).view(np.int32)).cuda()
    ov = torch.empty((F, cfg["num_columns"]), dtype=torch.int32, device="cuda")
    win = torch.empty((F, cfg["winners"]), dtype=torch.int32, device="cuda")
    sp.sp_step_boost(pool.handle, cfg, bc, frames, learn, ov, win)
    pool.sync()
    return ov.cpu().numpy(), win.cpu().numpy()


def _state(pool, C):
    return tuple(t.cpu().numpy().view(np.uint32) for t in sp.sp_boost_state(pool.handle, C))


def _same(got, want, what):
    bad = np.argwhere(np.asarray(got) != np.asarray(want))
    assert bad.size == 0, f"{what}: {bad[:5].tolist()}"


def test_handworked():
    with open(GOLD) as f:
        g = json.load(f)
    idx = np.array(g["idx"], dtype=np.uint32)
    perm = (np.array(g["perm_q_before"], dtype=np.float32) / 256).astype(np.float32)
    pool = sp.SpatialPooler(g["config"], idx, perm)
    ov, win = _run(pool, g["config"], g["boost"], np.array(g["frames"], dtype=np.uint32))
    assert ov.tolist() == g["boosted_overlaps"] and win.tolist() == g["winners"]
    adc, odc, boost = _state(pool, 3)
    assert adc.tolist() == g["active_duty_q16"] and odc.tolist() == g["overlap_duty_q16"]
    assert boost.tolist() == g["boost_q8"]
    assert (pool.perm.cpu().numpy() * 256).tolist() == g["perm_q_after"]
    pool.close()


@pytest.mark.parametrize("name", ["32x32", "960x540"])
def test_workloads_across_calls(name):
    if name == "32x32":
        w = synth.workload_plain_32x32(frames=120)
    else:
        w = synth.workload_paper_scale(frames=150, columns=1024, synapses=256)
    cfg = w.cfg
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    half = w.frames.shape[0] // 2
    ov1, win1 = _run(pool, cfg, BC, w.frames[:half])
    ov2, win2 = _run(pool, cfg, BC, w.frames[half:])
    e_ov, e_win, e_perm, e_state = oracle.run_boost(cfg, BC, w.idx, w.perm, w.frames)
    _same(np.concatenate([ov1, ov2]), e_ov, "boosted overlaps")
    _same(np.concatenate([win1, win2]), e_win, "winners")
    _same(pool.perm.cpu().numpy().astype(np.float64), e_perm, "permanences")
    for got, want, what in zip(_state(pool, cfg["num_columns"]), e_state,
                               ("active duty", "overlap duty", "boost")):
        _same(got, want, what)
    assert e_state[2].max() > 256  # boosting took effect
    pool.close()


def test_learning_off_and_reset():
    w = synth.workload_plain_32x32(frames=40)
    cfg = w.cfg
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    _run(pool, cfg, BC, w.frames[:20])
    st = _state(pool, 256)
    perm = pool.perm.cpu().numpy().copy()
    ov, win = _run(pool, cfg, BC, w.frames[20:], learn=False)
    _, e_state = oracle.run_boost(cfg, BC, w.idx, w.perm, w.frames[:20])[2:]
    e_ov, e_win, _, _ = oracle.run_boost(cfg, BC, w.idx, perm, w.frames[20:], learn=False,
                                         state=e_state)
    _same(ov, e_ov, "boosted overlaps, learning off")
    _same(win, e_win, "winners, learning off")
    assert np.array_equal(pool.perm.cpu().numpy(), perm)
    assert all(np.array_equal(a, b) for a, b in zip(_state(pool, 256), st))
    sp.sp_boost_reset(pool.handle)
    adc, odc, boost = _state(pool, 256)
    assert adc.max() == 0 and odc.max() == 0 and np.all(boost == 256)
    pool.close()
