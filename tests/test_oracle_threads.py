"""The oracle on several host threads (the all-cores CPU baseline) against
the single-threaded oracle: identical overlaps, winners and permanences for
thread counts that split the columns evenly, unevenly and into empty
ranges, with learning on and off."""
import numpy as np
import pytest

import oracle
from paper_1608_01966_amd import synth


@pytest.mark.parametrize("threads", [1, 2, 3, 7, 16])
@pytest.mark.parametrize("shape", [(1024, 256, 64, 4, 20), (300, 5, 33, 2, 3),
                                   (50000, 700, 96, 3, 30)])
@pytest.mark.parametrize("learn", [True, False])
def test_equals_single_thread(threads, shape, learn):
    N, C, S, m, k = shape
    w = synth.random_instance(41 + C, synth.sp_config(N, C, S, m, k), frames=25, density=0.1)
    e_ov, e_win, e_perm = oracle.run(w.cfg, w.idx, w.perm, w.frames, learn=learn)
    ov, win, perm = oracle.run_threads(w.cfg, w.idx, w.perm, w.frames, threads, learn=learn)
    assert np.array_equal(ov, e_ov)
    assert np.array_equal(win, e_win)
    assert np.array_equal(perm, e_perm)
    if learn and C > 5:
        assert not np.array_equal(perm, w.perm.astype(np.float64))


def test_hand_worked_example():
    """The hand-worked 8-column example gives the same winners threaded."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "handworked_8col.json")))
    cfg = g["config"]
    idx = np.array(g["idx"], dtype=np.uint32)
    perm = np.array(g["perm_q_before"], dtype=np.float64) / 256.0
    frames = np.array(g["frames"], dtype=np.uint32)
    ov, win, p = oracle.run_threads(cfg, idx, perm, frames, 3)
    assert ov.tolist() == g["overlaps"]
    assert win.tolist() == g["winners"]
    assert (p * 256).tolist() == g["perm_q_after_frame2"]


def test_rejects_bad_thread_count():
    w = synth.random_instance(3, synth.sp_config(100, 4, 5, 1, 2), frames=2)
    with pytest.raises(ValueError):
        oracle.run_threads(w.cfg, w.idx, w.perm, w.frames, 0)
