"""Pin: the oracle against a hand-worked two-frame, eight-column example
(Section 1.1, Algorithms 1 and 2, and the learning rule; derivation notes in
tests/golden/handworked_8col.json)."""
import json
import os

import numpy as np

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "handworked_8col.json")


def _gold():
    with open(GOLD) as f:
        return json.load(f)


def test_frame_by_frame():
    g = _gold()
    cfg = g["config"]
    idx = np.array(g["idx"], dtype=np.uint32)
    perm = np.array(g["perm_q_before"], dtype=np.float64) / 256.0
    after = [g["perm_q_after_frame1"], g["perm_q_after_frame2"]]
    for t, frame in enumerate(g["frames"]):
        frame = np.array(frame, dtype=np.uint32)
        ov = oracle.overlap(cfg, idx, perm, frame)
        assert ov.tolist() == g["overlaps"][t]
        win, active = oracle.inhibit(cfg, ov)
        assert win.tolist() == g["winners"][t]
        assert np.flatnonzero(active).tolist() == g["winners"][t]
        perm = oracle.learn(cfg, idx, perm, frame, active)
        assert (perm * 256).tolist() == after[t]


def test_run_two_frames():
    g = _gold()
    cfg = g["config"]
    idx = np.array(g["idx"], dtype=np.uint32)
    perm = (np.array(g["perm_q_before"], dtype=np.float32) / 256).astype(np.float32)
    frames = np.array(g["frames"], dtype=np.uint32)
    ov, win, p = oracle.run(cfg, idx, perm, frames, learn=True)
    assert ov.tolist() == g["overlaps"]
    assert win.tolist() == g["winners"]
    assert (p * 256).tolist() == g["perm_q_after_frame2"]
    # the final column 2 as float32 values
    assert p[2].astype(np.float32).tolist() == [0.5703125, 0.5625, 0.6484375, 0.640625]


def test_learn_off_is_identity():
    g = _gold()
    cfg = g["config"]
    idx = np.array(g["idx"], dtype=np.uint32)
    perm = np.array(g["perm_q_before"], dtype=np.float64) / 256.0
    frames = np.array(g["frames"], dtype=np.uint32)
    ov, win, p = oracle.run(cfg, idx, perm, frames, learn=False)
    assert np.array_equal(p, perm)
    # without learning, frame 2 sees the initial state: column 0 counts 3
    assert ov[1].tolist() == [3, 0, 2, 0, 0, 2, 0, 2]
    assert win.tolist()[0] == g["winners"][0]
