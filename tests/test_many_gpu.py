"""Parity of the many-instance step (sp_step_many) with the oracle run on
each instance alone: overlaps, winners and final permanences element by
element, bit-exact."""
import numpy as np
import pytest

import oracle
import paper_1608_01966_amd as sp
from paper_1608_01966_amd import synth

pytestmark = pytest.mark.gpu


def run_many(ws, learn=True, frames_per=None, want_ov=True, calls=1):
    import torch
    pools = [sp.SpatialPooler(w.cfg, w.idx, w.perm) for w in ws]
    n = len(ws)
    Fs = [w.frames.shape[0] if frames_per is None else frames_per[i] for i, w in enumerate(ws)]
    dev_frames = [torch.from_numpy(np.ascontiguousarray(w.frames[:F]).view(np.int32)).cuda()
                  for w, F in zip(ws, Fs)]
    ovs = [[] for _ in range(n)]
    wins = [[] for _ in range(n)]
    # split every instance's frames over `calls` consecutive calls
    cuts = [np.linspace(0, F, calls + 1).astype(int) for F in Fs]
    for c in range(calls):
        fr, ov, wn = [], [], []
        for i in range(n):
            a, b = cuts[i][c], cuts[i][c + 1]
            fr.append(dev_frames[i][a:b])
            ov.append(torch.empty((b - a, ws[i].cfg["num_columns"]), dtype=torch.int32,
                                  device="cuda") if want_ov else None)
            wn.append(torch.empty((b - a, ws[i].cfg["winners"]), dtype=torch.int32, device="cuda"))
        sp.sp_step_many([p.handle for p in pools], [w.cfg for w in ws], fr, learn,
                        ov if want_ov else None, wn)
        for i in range(n):
            if want_ov:
                ovs[i].append(ov[i])
            wins[i].append(wn[i])
    pools[0].sync()
    out = []
    for i in range(n):
        o = torch.cat(ovs[i]).cpu().numpy() if want_ov else None
        out.append((o, torch.cat(wins[i]).cpu().numpy(), pools[i].perm.cpu().numpy()))
        pools[i].close()
    return out, Fs


def check(ws, **kw):
    out, Fs = run_many(ws, **kw)
    learn = kw.get("learn", True)
    for i, (w, (ov, win, perm)) in enumerate(zip(ws, out)):
        e_ov, e_win, e_perm = oracle.run(w.cfg, w.idx, w.perm, w.frames[:Fs[i]], learn=learn)
        if ov is not None:
            bad = np.argwhere(ov != e_ov)
            assert bad.size == 0, f"instance {i}: overlap mismatch {bad[:5].tolist()}"
        bad = np.argwhere(win != e_win)
        assert bad.size == 0, f"instance {i}: winner mismatch {bad[:5].tolist()}"
        bad = np.argwhere(perm.astype(np.float64) != e_perm)
        assert bad.size == 0, f"instance {i}: permanence mismatch {bad[:5].tolist()}"


def mixed(seed, n, frames):
    g = np.random.default_rng(seed)
    ws = []
    for i in range(n):
        N = int(g.integers(1, 60000))
        C = int(g.integers(1, 1500))
        S = int(g.integers(1, min(N, 700) + 1))
        cfg = synth.sp_config(N, C, S, int(g.integers(0, 6)), int(g.integers(1, C + 1)))
        ws.append(synth.random_instance(seed * 100 + i, cfg, frames=frames,
                                        density=float(g.uniform(0.02, 0.5))))
    return ws


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_mixed_shapes(seed):
    check(mixed(seed, 7, 12))


def test_learning_off():
    check(mixed(4, 5, 9), learn=False)


def test_uneven_frame_counts_and_empty_instances():
    ws = mixed(5, 6, 15)
    check(ws, frames_per=[15, 0, 3, 1, 15, 7])


def test_split_calls_equal_one_call():
    check(mixed(6, 4, 20), calls=3)


def test_without_overlaps():
    check(mixed(7, 3, 8), want_ov=False)


def test_aligned_synapse_counts_ragged_columns():
    """Only S that are multiples of 64 (the aligned kernel), including S that
    are not powers of two, with ragged column counts and input sizes."""
    g = np.random.default_rng(12)
    ws = []
    for i, S in enumerate([64, 192, 320, 128, 448, 64]):
        N = int(g.integers(S, 90000))
        C = int(g.integers(1, 2500))
        cfg = synth.sp_config(N, C, S, int(g.integers(0, 6)), int(g.integers(1, C + 1)))
        ws.append(synth.random_instance(1200 + i, cfg, frames=10,
                                        density=float(g.uniform(0.02, 0.3))))
    check(ws)


def test_largest_instances():
    """4096 columns x 512 synapses and the 960x540 input in one batch with
    small instances."""
    ws = [synth.random_instance(80, synth.sp_config(960 * 540, 4096, 512, 4, 160), 6, 0.05),
          synth.random_instance(81, synth.sp_config(64 * 64, 256, 32, 4, 10), 6, 0.1),
          synth.random_instance(82, synth.sp_config(240 * 134, 2048, 128, 4, 80), 6, 0.03)]
    check(ws)


def test_input_sizes_from_4m_pixels_down():
    """One launch over a 4M-pixel input, one-synapse columns (the widest
    tiles), the 960x540 input and an input that is not a whole number of
    four-word groups."""
    ws = [synth.random_instance(90, synth.sp_config(1 << 22, 300, 40, 2, 12), 5, 0.05),
          synth.random_instance(91, synth.sp_config(5000, 700, 1, 0, 30), 5, 0.3),
          synth.random_instance(92, synth.sp_config(33007, 512, 96, 3, 20), 5, 0.1),
          synth.random_instance(93, synth.sp_config(960 * 540, 256, 64, 4, 10), 5, 0.05)]
    check(ws)


def test_multi_workload_subset():
    """The 64-instance workload's instances, 12 steps each, all compared."""
    check(synth.workload_multi(64, 12))


def test_many_tiny_instances():
    """600 instances of at most 64 columns: the top-k workgroups then hold
    several instances per wave."""
    g = np.random.default_rng(21)
    ws = []
    for i in range(600):
        C = int(g.integers(1, 65))
        S = int(g.integers(1, 40))
        cfg = synth.sp_config(int(g.integers(S, 3000)), C, S, int(g.integers(0, 4)),
                              int(g.integers(1, C + 1)))
        ws.append(synth.random_instance(3000 + i, cfg, frames=int(g.integers(1, 5)),
                                        density=float(g.uniform(0.05, 0.4))))
    check(ws)


def test_split_over_launches():
    """260 instances of 1024 columns x 256 synapses are more tiles than one
    launch holds, so the call is split; every instance still matches."""
    ws = [synth.random_instance(4000 + i, synth.sp_config(4096, 1024, 256, 3, 40), 3, 0.1)
          for i in range(260)]
    check(ws)


def test_same_as_single_instance_step():
    import torch
    w = synth.workload_paper_scale(frames=30, columns=512, synapses=128)
    a = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    b = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    fr = torch.from_numpy(w.frames.view(np.int32)).cuda()
    ov_a, win_a = a.step(fr)
    ov_b = torch.empty_like(ov_a)
    win_b = torch.empty_like(win_a)
    sp.sp_step_many([b.handle], [w.cfg], [fr], True, [ov_b], [win_b])
    a.sync()
    b.sync()
    assert torch.equal(ov_a, ov_b) and torch.equal(win_a, win_b) and torch.equal(a.perm, b.perm)
    a.close()
    b.close()


def test_rejects_duplicates_and_large():
    import torch
    w = synth.workload_plain_32x32(2)
    p = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    fr = torch.from_numpy(w.frames.view(np.int32)).cuda()
    win = torch.empty((2, 20), dtype=torch.int32, device="cuda")
    with pytest.raises(sp.SpError, match="repeats"):
        sp.sp_step_many([p.handle, p.handle], [w.cfg, w.cfg], [fr, fr], True, None, [win, win])
    big = synth.random_instance(9, synth.sp_config(5000, 4097, 4, 1, 10), 1)
    q = sp.SpatialPooler(big.cfg, big.idx, big.perm)
    with pytest.raises(sp.SpError, match="at most 4096"):
        sp.sp_step_many([q.handle], [big.cfg],
                        [torch.from_numpy(big.frames.view(np.int32)).cuda()], True, None,
                        [torch.empty((1, 10), dtype=torch.int32, device="cuda")])
    p.close()
    q.close()
