"""Pin: the oracle against an independent vectorised form of the step
(integer matrix product, lexsort, clip) on random instances, parameter
extremes and the plain 32x32 workload."""
import numpy as np
import pytest

import oracle
from paper_1608_01966_amd import synth
from tests.dense_reference import dense_run


def _check(w, learn=True):
    ov, win, p = oracle.run(w.cfg, w.idx, w.perm, w.frames, learn=learn)
    dov, dwin, dq = dense_run(w.cfg, w.idx, w.perm_q, w.frames, learn=learn)
    assert np.array_equal(ov, dov)
    assert np.array_equal(win, dwin)
    assert np.array_equal(p * 256, dq)
    assert np.all(p * 256 == np.round(p * 256))


@pytest.mark.parametrize("seed", range(40))
def test_random_tiny(seed):
    g = np.random.default_rng(1000 + seed)
    N = int(g.integers(1, 200))
    C = int(g.integers(1, 24))
    S = int(g.integers(1, min(N, 12) + 1))
    k = int(g.integers(1, C + 1))
    m = int(g.integers(0, S + 2))
    cfg = synth.sp_config(N, C, S, m, k, connected_q8=int(g.integers(0, 257)),
                          inc_q8=int(g.integers(0, 40)), dec_q8=int(g.integers(0, 40)))
    w = synth.random_instance(seed, cfg, frames=int(g.integers(0, 12)),
                              density=float(g.uniform(0, 1)))
    _check(w, learn=bool(seed % 4 != 3))


@pytest.mark.parametrize("case", [
    dict(connected_q8=0), dict(connected_q8=256), dict(inc_q8=256, dec_q8=256),
    dict(inc_q8=0, dec_q8=0), dict(min_overlap=0), dict(winners=64), dict(winners=1),
])
def test_extremes(case):
    base = synth.sp_config(300, 64, 16, 2, 8)
    base.update(case)
    w = synth.random_instance(7, base, frames=15, density=0.3)
    _check(w)


def test_plain_32x32_workload():
    _check(synth.workload_plain_32x32(100))


def test_paper_frame_shape_subset():
    """The 960x540 blob input with a reduced column count (the full
    1024x256 case is compared the same way, at GPU-test time)."""
    w = synth.workload_paper_scale(frames=6, columns=48, synapses=256)
    _check(w)
