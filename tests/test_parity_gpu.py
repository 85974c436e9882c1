"""Parity of the HIP path with the oracle, element by element: overlaps,
winners and final permanences must be identical (integer results; the
permanences are exact multiples of 1/256, so float equality is exact)."""
import json
import os

import numpy as np
import pytest

import oracle
import paper_1608_01966_amd as sp
from paper_1608_01966_amd import synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "handworked_8col.json")


def gpu_run(w, learn=True, plain=False, chunks=None, want_ov=True):
    import torch
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    frames = torch.from_numpy(np.ascontiguousarray(w.frames).view(np.int32)).cuda()
    F = frames.shape[0]
    bounds = [0] + list(chunks or []) + [F]
    ovs, wins = [], []
    for a, b in zip(bounds[:-1], bounds[1:]):
        ov, win = pool.step(frames[a:b], learn=learn, overlaps=want_ov, plain=plain)
        ovs.append(ov)
        wins.append(win)
    pool.sync()
    out = (torch.cat(ovs).cpu().numpy() if want_ov else None,
           torch.cat(wins).cpu().numpy(), pool.perm.cpu().numpy(), pool.persistent)
    pool.close()
    return out


def check(w, learn=True, plain=False, chunks=None, want_ov=True, expect_persistent=None):
    e_ov, e_win, e_perm = oracle.run(w.cfg, w.idx, w.perm, w.frames, learn=learn)
    ov, win, perm, persistent = gpu_run(w, learn, plain, chunks, want_ov)
    if want_ov:
        bad = np.argwhere(ov != e_ov)
        assert bad.size == 0, f"overlap mismatch at (frame, column) {bad[:5].tolist()}"
    bad = np.argwhere(win != e_win)
    assert bad.size == 0, f"winner mismatch at (frame, slot) {bad[:5].tolist()}"
    bad = np.argwhere(perm.astype(np.float64) != e_perm)
    assert bad.size == 0, f"permanence mismatch at (column, synapse) {bad[:5].tolist()}"
    if expect_persistent is not None and not plain:
        assert persistent == expect_persistent
    return persistent


@pytest.mark.parametrize("plain", [False, True])
def test_handworked(plain):
    g = json.load(open(GOLD))
    w = synth.Workload("handworked", g["config"], np.array(g["idx"], dtype=np.uint32),
                       np.array(g["perm_q_before"], dtype=np.uint16),
                       np.array(g["frames"], dtype=np.uint32))
    check(w, plain=plain)
    ov, win, perm, _ = gpu_run(w, plain=plain)
    assert win.tolist() == g["winners"]
    assert (perm * 256).astype(int).tolist() == g["perm_q_after_frame2"]


# (N, C, S, m, k, theta, inc, dec, frames, density): several tiles and ragged
# tails in every dimension.
SHAPES = [
    (1, 1, 1, 0, 1, 128, 8, 4, 5, 0.5),
    (31, 3, 7, 1, 2, 0, 8, 4, 9, 0.4),
    (33, 5, 33, 2, 5, 256, 16, 8, 9, 0.6),
    (1000, 257, 65, 3, 17, 128, 8, 4, 12, 0.2),
    (4097, 1000, 100, 4, 40, 100, 24, 12, 10, 0.15),
    (20000, 4100, 64, 2, 160, 128, 8, 4, 6, 0.1),
    (100000, 300, 512, 6, 30, 128, 8, 4, 8, 0.05),
    (70000, 130, 1000, 8, 13, 128, 256, 256, 6, 0.03),
    (5000, 2048, 32, 1, 200, 128, 8, 4, 10, 0.2),
    (3000, 64, 129, 0, 64, 128, 0, 0, 6, 0.3),
]


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("shape", SHAPES, ids=[f"N{s[0]}_C{s[1]}_S{s[2]}" for s in SHAPES])
def test_random_shapes(shape, plain):
    N, C, S, m, k, th, inc, dec, F, d = shape
    cfg = synth.sp_config(N, C, S, m, k, th, inc, dec)
    w = synth.random_instance(11, cfg, frames=F, density=d)
    check(w, plain=plain)


@pytest.mark.parametrize("plain", [False, True])
def test_plain_32x32_workload(plain):
    """32x32 Bernoulli(0.10) input, 256 x 64, 100 learning frames."""
    check(synth.workload_plain_32x32(100), plain=plain, expect_persistent=True)


def test_paper_scale_1000_frames_persistent():
    """The 960x540 blob input, 1024 columns x 256 synapses, 1000 learning
    frames in one persistent launch, as the benchmark runs it."""
    w = synth.workload_paper_scale(frames=1000)
    check(w, expect_persistent=True)


def test_paper_scale_plain_200_frames():
    check(synth.workload_paper_scale(frames=200), plain=True)


SWEEP = [(c, s) for c in (256, 512, 1024, 2048) for s in (32, 64, 128, 256)]


@pytest.mark.parametrize("C,S", SWEEP, ids=[f"C{c}_S{s}" for c, s in SWEEP])
def test_paper_scale_sweep_points(C, S):
    """Every point of the column x synapse sweep the benchmark times, at 960x540."""
    check(synth.workload_paper_scale(frames=41, columns=C, synapses=S), expect_persistent=True)


# One shape per instance of the one-column-group-per-wave persistent kernel
# (rows per column, exchange words per lane, rows per wave), each picked so
# that the planner lands on it: (C, S) with 7 frames (an odd count, so the
# last exchange carries one frame).
WAVE_SHAPES = [
    (64, 40), (300, 64), (1000, 50), (2000, 33), (4096, 64),          # 1 row per column
    (200, 100), (500, 128), (1024, 65), (2048, 128), (3000, 100),     # 2
    (256, 256), (400, 200), (1000, 256), (1500, 256), (4000, 200),    # 4
    (100, 512), (512, 300), (1024, 512), (2048, 400),                 # 8
    (200, 1000), (300, 1024), (1024, 700),                            # 16
]


@pytest.mark.parametrize("C,S", WAVE_SHAPES, ids=[f"C{c}_S{s}" for c, s in WAVE_SHAPES])
def test_persistent_instances(C, S):
    cfg = synth.sp_config(20000, C, S, 3, max(1, C // 25))
    w = synth.random_instance(900 + C + S, cfg, frames=7, density=0.08)
    check(w, expect_persistent=True)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    assert pool.kernel == "k_sp_persistent_w"
    pool.close()


def test_split_launches_equal_one_launch():
    w = synth.workload_paper_scale(frames=60, columns=512, synapses=128)
    check(w, chunks=[1, 2, 3, 10, 11, 40])


def test_mixed_plain_and_persistent_calls():
    import torch
    w = synth.workload_plain_32x32(30)
    e_ov, e_win, e_perm = oracle.run(w.cfg, w.idx, w.perm, w.frames)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    fr = torch.from_numpy(w.frames.view(np.int32)).cuda()
    outs = [pool.step(fr[0:7], plain=True), pool.step(fr[7:19]), pool.step(fr[19:20], plain=True),
            pool.step(fr[20:30])]
    pool.sync()
    assert np.array_equal(torch.cat([o[0] for o in outs]).cpu().numpy(), e_ov)
    assert np.array_equal(torch.cat([o[1] for o in outs]).cpu().numpy(), e_win)
    assert np.array_equal(pool.perm.cpu().numpy().astype(np.float64), e_perm)
    pool.close()


@pytest.mark.parametrize("plain", [False, True])
def test_learn_off_leaves_state(plain):
    w = synth.workload_paper_scale(frames=20, columns=512, synapses=64)
    check(w, learn=False, plain=plain)
    _, _, perm, _ = gpu_run(w, learn=False, plain=plain)
    assert np.array_equal(perm, w.perm)


@pytest.mark.parametrize("plain", [False, True])
def test_without_overlap_output(plain):
    check(synth.workload_plain_32x32(25), plain=plain, want_ov=False)


@pytest.mark.parametrize("kind", ["zeros", "ones"])
def test_degenerate_frames(kind):
    cfg = synth.sp_config(2000, 300, 40, 0, 25)
    w = synth.random_instance(12, cfg, frames=4)
    if kind == "zeros":
        w.frames[:] = 0
    else:
        w.frames[:] = 0xFFFFFFFF
    check(w)
    check(w, plain=True)


@pytest.mark.parametrize("case", [dict(winners=300), dict(winners=1), dict(min_overlap=41),
                                  dict(connected_q8=0), dict(connected_q8=256),
                                  dict(inc_q8=256, dec_q8=256), dict(min_overlap=0)])
def test_parameter_extremes(case):
    cfg = synth.sp_config(2000, 300, 40, 2, 25)
    cfg.update(case)
    w = synth.random_instance(13, cfg, frames=12, density=0.3)
    check(w)
    check(w, plain=True)


def test_max_columns_persistent():
    """4096 columns is the largest count the persistent exchange holds."""
    cfg = synth.sp_config(50000, 4096, 64, 3, 400)
    check(synth.random_instance(14, cfg, frames=6, density=0.1), expect_persistent=True)


def test_columns_past_persistent_limit():
    cfg = synth.sp_config(50000, 4097, 64, 3, 400)
    check(synth.random_instance(14, cfg, frames=4, density=0.1), expect_persistent=False)
    cfg = synth.sp_config(50000, 16384, 64, 3, 400)
    check(synth.random_instance(14, cfg, frames=4, density=0.1), expect_persistent=False)


def test_max_columns_plain_only():
    cfg = synth.sp_config(50000, 65536, 4, 1, 1000)
    check(synth.random_instance(15, cfg, frames=3, density=0.3), expect_persistent=False)


def test_max_synapses():
    cfg = synth.sp_config(100000, 40, 4096, 10, 8)
    check(synth.random_instance(16, cfg, frames=5, density=0.05), expect_persistent=False)


def test_max_synapses_persistent():
    """1024 synapses (16 rows of 64) is the most one persistent workgroup holds."""
    cfg = synth.sp_config(100000, 300, 1024, 10, 24)
    check(synth.random_instance(18, cfg, frames=8, density=0.05), expect_persistent=True)
    cfg = synth.sp_config(100000, 300, 1025, 10, 24)
    check(synth.random_instance(18, cfg, frames=3, density=0.05), expect_persistent=False)


def test_max_input_bits():
    cfg = synth.sp_config(1 << 23, 256, 128, 1, 20)
    w = synth.random_instance(17, cfg, frames=3, density=0.02)
    check(w)


def test_step_longer_than_one_launch():
    """At 2^23 input bits one persistent launch takes 64 frames (its paired
    copy of the frames is bounded), so 151 frames run as launches of 64, 64
    and 23 frames: the results must be those of stepping frame by frame."""
    cfg = synth.sp_config(1 << 23, 256, 64, 2, 10)
    w = synth.random_instance(31, cfg, frames=151, density=0.02)
    check(w, expect_persistent=True)


def test_zero_frames_is_noop():
    import torch
    w = synth.workload_plain_32x32(1)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    empty = torch.empty((0, 32), dtype=torch.int32, device="cuda")
    pool.step(empty)
    pool.step(empty, plain=True)
    pool.sync()
    assert np.array_equal(pool.perm.cpu().numpy(), w.perm)
    pool.close()


def test_create_rejects_bad_state():
    import torch
    cfg = synth.sp_config(100, 4, 8, 1, 2)
    w = synth.random_instance(1, cfg, frames=1)
    idx = torch.from_numpy(w.idx.view(np.int32).copy()).cuda()
    perm = torch.from_numpy(w.perm.copy()).cuda()
    h = sp.sp_create(cfg, idx, perm)
    sp.sp_destroy(h)
    idx[1, 2] = 100
    with pytest.raises(sp.SpError, match="indices >= input_bits") as e:
        sp.sp_create(cfg, idx, perm)
    assert e.value.code == sp.SP_EINVAL
    idx[1, 2] = 5
    perm[3, 0] = 0.3
    with pytest.raises(sp.SpError, match="off the 1/256 grid"):
        sp.sp_create(cfg, idx, perm)
    perm[3, 0] = 0.5
    h = sp.sp_create(cfg, idx, perm)
    perm[0, 0] = float("nan")
    with pytest.raises(sp.SpError, match="off the 1/256 grid"):
        sp.sp_check_state(h)
    sp.sp_destroy(h)
