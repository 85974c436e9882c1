"""Local inhibition on the GPU (Algorithm 2 with a column neighbourhood)
against the oracle: the inhibition kernel alone on random overlaps (LDS and
device-memory paths, 1-D and 2-D grids, ragged last rows), and the learning
step built on it, bit for bit."""
import numpy as np
import pytest

import oracle
import paper_1608_01966_amd as sp
from paper_1608_01966_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("C,grid_w,radius,n", [
    (1, 1, 0, 1), (7, 7, 1, 1), (9, 3, 1, 2), (100, 10, 2, 3), (1000, 33, 4, 5),
    (1024, 1024, 80, 6), (1024, 32, 80, 40), (4097, 64, 3, 2), (16384, 128, 2, 4),
    (20000, 141, 1, 2), (3000, 1, 5, 3),
])
def test_inhibit_local(C, grid_w, radius, n):
    import torch
    g = np.random.default_rng(C + radius)
    F = 5
    ov = g.integers(0, 12, size=(F, C)).astype(np.int32)
    ov[ov < 3] = 0  # gated overlaps: many zeros
    act = sp.sp_inhibit_local(torch.from_numpy(ov).cuda(), grid_w, radius, n)
    torch.cuda.synchronize()
    got = act.cpu().numpy()
    for f in range(F):
        want = oracle.inhibit_local(ov[f], grid_w, radius, n)
        bad = np.flatnonzero(got[f] != want)
        assert bad.size == 0, f"frame {f}: columns {bad[:5].tolist()}"


@pytest.mark.parametrize("name", ["32x32", "960x540_1d_radius80", "960x540_2d"])
def test_step_local(name):
    import torch
    if name == "32x32":
        w = synth.workload_plain_32x32(frames=40)
        grid_w, radius = 16, 2
    elif name == "960x540_1d_radius80":
        w = synth.workload_paper_scale(frames=60, columns=1024, synapses=256)
        w.cfg["winners"] = 6
        grid_w, radius = 1024, 80
    else:
        w = synth.workload_paper_scale(frames=30, columns=1024, synapses=128)
        w.cfg["winners"] = 3
        grid_w, radius = 32, 3
    cfg = w.cfg
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    frames = torch.from_numpy(w.frames.view(np.int32)).cuda()
    F, C = w.frames.shape[0], cfg["num_columns"]
    ov = torch.empty((F, C), dtype=torch.int32, device="cuda")
    act = torch.empty((F, C), dtype=torch.uint8, device="cuda")
    sp.sp_step_local(pool.handle, cfg, frames, True, grid_w, radius, ov, act)
    pool.sync()
    e_ov, e_act, e_perm = oracle.run_local(cfg, w.idx, w.perm, w.frames, grid_w, radius,
                                           cfg["winners"])
    assert np.array_equal(ov.cpu().numpy(), e_ov)
    assert np.array_equal(act.cpu().numpy(), e_act)
    assert np.array_equal(pool.perm.cpu().numpy().astype(np.float64), e_perm)
    assert e_act.sum() > 0
    assert pool.local_kernel == "k_sp_persistent_local"
    pool.close()


def run_local_gpu(w, grid_w, radius, learn=True, want_ov=True, cuts=()):
    """sp_step_local over the frames, split at `cuts` into consecutive calls."""
    import torch
    cfg = w.cfg
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    frames = torch.from_numpy(np.ascontiguousarray(w.frames).view(np.int32)).cuda()
    F, C = w.frames.shape[0], cfg["num_columns"]
    ov = torch.full((F, C), -1, dtype=torch.int32, device="cuda")
    act = torch.full((F, C), 7, dtype=torch.uint8, device="cuda")
    b = [0, *cuts, F]
    for a0, a1 in zip(b[:-1], b[1:]):
        sp.sp_step_local(pool.handle, cfg, frames[a0:a1], learn, grid_w, radius,
                         ov[a0:a1] if want_ov else None, act[a0:a1])
    pool.sync()
    out = (ov.cpu().numpy(), act.cpu().numpy(), pool.perm.cpu().numpy(), pool.local_kernel)
    pool.close()
    return out


# (N, C, S, m, n, grid_w, radius, frames): every instance family of the
# persistent local step (rows per column 1..16, exchange words 1..16), 2-D
# grids with ragged last rows, and shapes past its limits (per-frame launches).
LOCAL_SHAPES = [
    (4000, 60, 40, 2, 2, 60, 5, 9), (20000, 1000, 50, 3, 4, 37, 3, 8),
    (20000, 4096, 64, 3, 5, 4096, 40, 5), (30000, 2048, 128, 3, 3, 64, 4, 6),
    (30000, 500, 200, 4, 3, 500, 30, 7), (50000, 1500, 256, 4, 6, 1500, 80, 6),
    (60000, 4000, 200, 4, 5, 63, 2, 4), (80000, 512, 300, 5, 4, 23, 6, 6),
    (90000, 2048, 400, 5, 3, 2048, 100, 4), (100000, 300, 1024, 8, 4, 17, 2, 5),
    (100000, 1024, 700, 8, 6, 1024, 80, 4), (20000, 5000, 16, 1, 3, 100, 2, 4),
    (20000, 200, 1100, 8, 2, 200, 10, 3),
]


@pytest.mark.parametrize("shape", LOCAL_SHAPES,
                         ids=[f"C{s[1]}_S{s[2]}_w{s[5]}_r{s[6]}" for s in LOCAL_SHAPES])
def test_step_local_shapes(shape):
    N, C, S, m, n, grid_w, radius, F = shape
    cfg = synth.sp_config(N, C, S, m, n)
    w = synth.random_instance(5000 + C + S, cfg, frames=F, density=0.1)
    ov, act, perm, kern = run_local_gpu(w, grid_w, radius)
    e_ov, e_act, e_perm = oracle.run_local(cfg, w.idx, w.perm, w.frames, grid_w, radius, n)
    assert np.array_equal(ov, e_ov)
    assert np.array_equal(act, e_act)
    assert np.array_equal(perm.astype(np.float64), e_perm)
    assert kern == ("plain" if C > 4096 or S > 1024 else "k_sp_persistent_local")


def test_step_local_kernel_choice():
    """Two frames per exchange wherever every workgroup's halo (the bounding
    box of its columns' neighbourhoods) and every window are small enough;
    one frame per exchange otherwise; per-frame launches past the persistent
    shapes."""
    w = synth.workload_paper_scale(frames=1, columns=1024, synapses=256)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    assert pool.local_kernel_for(1024, 80) == "k_sp_persistent_local2"
    assert pool.local_kernel_for(32, 20) == "k_sp_persistent_local2"
    pool.close()
    w = synth.workload_paper_scale(frames=1, columns=4096, synapses=64)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    assert pool.local_kernel_for(64, 2) == "k_sp_persistent_local2"
    assert pool.local_kernel_for(64, 40) == "k_sp_persistent_local"   # 4096-column windows
    assert pool.local_kernel_for(4096, 1200) == "k_sp_persistent_local"  # 2401-column windows
    with pytest.raises(sp.SpError):
        pool.local_kernel_for(0, 2)
    pool.close()
    cfg = synth.sp_config(20000, 5000, 16, 1, 3)
    w = synth.random_instance(3, cfg, frames=1, density=0.1)
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    assert pool.local_kernel_for(100, 2) == "plain"
    pool.close()


def test_step_local_one_and_two_frame_exchanges_alternate():
    """Calls on one handle switching between the two persistent kernels
    (radius 2 and 40 on a 64 x 64 grid), with odd frame counts: each keeps
    its own exchange region and sequence, and the state carries over."""
    import torch
    cfg = synth.sp_config(30000, 4096, 64, 3, 5)
    w = synth.random_instance(77, cfg, frames=13, density=0.1)
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    frames = torch.from_numpy(np.ascontiguousarray(w.frames).view(np.int32)).cuda()
    C = cfg["num_columns"]
    ov = torch.empty((13, C), dtype=torch.int32, device="cuda")
    act = torch.empty((13, C), dtype=torch.uint8, device="cuda")
    plan = [(0, 5, 2), (5, 8, 40), (8, 9, 2), (9, 12, 2), (12, 13, 40)]
    kinds = set()
    for a0, a1, r in plan:
        kinds.add(pool.local_kernel_for(64, r))
        sp.sp_step_local(pool.handle, cfg, frames[a0:a1], True, 64, r, ov[a0:a1], act[a0:a1])
    pool.sync()
    assert kinds == {"k_sp_persistent_local", "k_sp_persistent_local2"}
    perm = w.perm
    for a0, a1, r in plan:
        e_ov, e_act, e_perm = oracle.run_local(cfg, w.idx, perm, w.frames[a0:a1], 64, r, 5)
        assert np.array_equal(ov[a0:a1].cpu().numpy(), e_ov), (a0, a1, r)
        assert np.array_equal(act[a0:a1].cpu().numpy(), e_act), (a0, a1, r)
        perm = e_perm
    assert np.array_equal(pool.perm.cpu().numpy().astype(np.float64), perm)
    assert act.cpu().numpy().sum() > 0
    pool.close()


def test_step_local_learning_off_and_no_overlaps():
    w = synth.workload_paper_scale(frames=9, columns=1024, synapses=256)
    w.cfg["winners"] = 6
    ov, act, perm, _ = run_local_gpu(w, 1024, 80, learn=False, want_ov=False)
    e_ov, e_act, e_perm = oracle.run_local(w.cfg, w.idx, w.perm, w.frames, 1024, 80, 6,
                                           learn=False)
    assert np.array_equal(act, e_act)
    assert (ov == -1).all()
    assert np.array_equal(perm.astype(np.float64), e_perm)


def test_step_local_split_and_interleaved_with_global():
    """Consecutive local calls (one of a single frame), then a global step on
    the same handle, then local again: each path keeps its own exchange
    sequence, and the state carries over exactly."""
    import torch
    w = synth.workload_paper_scale(frames=14, columns=1024, synapses=256)
    cfg = dict(w.cfg)
    cfg["winners"] = 6
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    frames = torch.from_numpy(w.frames.view(np.int32)).cuda()
    C = cfg["num_columns"]
    act = torch.empty((14, C), dtype=torch.uint8, device="cuda")
    win = torch.empty((4, cfg["winners"]), dtype=torch.int32, device="cuda")
    sp.sp_step_local(pool.handle, cfg, frames[0:1], True, 1024, 80, None, act[0:1])
    sp.sp_step_local(pool.handle, cfg, frames[1:6], True, 1024, 80, None, act[1:6])
    sp.sp_step(pool.handle, cfg, frames[6:10], True, None, win)
    sp.sp_step_local(pool.handle, cfg, frames[10:14], True, 1024, 80, None, act[10:14])
    pool.sync()
    _, a1, p1 = oracle.run_local(cfg, w.idx, w.perm, w.frames[0:6], 1024, 80, 6)
    _, wg, p2 = oracle.run(cfg, w.idx, p1.astype(np.float32), w.frames[6:10])
    _, a3, p3 = oracle.run_local(cfg, w.idx, p2.astype(np.float32), w.frames[10:14], 1024, 80, 6)
    got = act.cpu().numpy()
    assert np.array_equal(got[0:6], a1)
    assert np.array_equal(win.cpu().numpy(), wg)
    assert np.array_equal(got[10:14], a3)
    assert np.array_equal(pool.perm.cpu().numpy().astype(np.float64), p3)
    pool.close()


def test_rejects_bad_arguments():
    import torch
    ov = torch.zeros((2, 10), dtype=torch.int32, device="cuda")
    for kw in ({"grid_w": 0}, {"grid_w": 11}, {"n": 0}):
        args = {"grid_w": 5, "radius": 1, "n": 1}
        args.update(kw)
        with pytest.raises(sp.SpError):
            sp.sp_inhibit_local(ov, **args)


ADAPT = [
    # (name, N, in_w, C, S, grid_w, radius0, n, frames, density)
    ("960x540_32x32_grid", 960 * 540, 960, 1024, 128, 32, 8, 3, 16, 0.05),
    ("ragged_grid_and_rows", 37 * 23 - 11, 37, 301, 40, 17, 3, 4, 14, 0.2),
    ("one_row_grid", 4000, 80, 500, 64, 500, 80, 6, 10, 0.1),
]


@pytest.mark.parametrize("case", ADAPT, ids=[a[0] for a in ADAPT])
@pytest.mark.parametrize("learn", [True, False])
def test_step_local_adaptive(case, learn):
    """The radius adapted after every learning frame (reading L5): overlaps,
    active columns, permanences, every frame's radius and the final radius
    against the oracle."""
    import torch
    name, N, in_w, C, S, grid_w, r0, n, F, d = case
    cfg = synth.sp_config(N, C, S, 2, n)
    blobs = name.startswith("960")
    w = synth.random_instance(61, cfg, F, density=d,
                              shape=(960, 540) if blobs else None, blobs=blobs)
    e_ov, e_act, e_perm, e_radii, e_r = oracle.run_local_adaptive(
        cfg, w.idx, w.perm, w.frames, in_w, grid_w, r0, n, learn=learn)
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    frames = torch.from_numpy(np.ascontiguousarray(w.frames).view(np.int32)).cuda()
    ov = torch.full((F, C), -1, dtype=torch.int32, device="cuda")
    act = torch.full((F, C), 7, dtype=torch.uint8, device="cuda")
    radius = torch.tensor([r0], dtype=torch.int32, device="cuda")
    radii = torch.zeros(F, dtype=torch.int32, device="cuda")
    half = F // 2
    for a0, a1 in ((0, half), (half, F)):
        sp.sp_step_local_adaptive(pool.handle, cfg, frames[a0:a1], learn, in_w, grid_w, radius,
                                  ov[a0:a1], act[a0:a1], radii[a0:a1])
    pool.sync()
    assert np.array_equal(ov.cpu().numpy(), e_ov)
    assert np.array_equal(act.cpu().numpy(), e_act)
    assert np.array_equal(pool.perm.cpu().numpy().astype(np.float64), e_perm)
    assert np.array_equal(radii.cpu().numpy().astype(np.uint32), e_radii)
    assert int(radius.item()) == e_r
    if learn and name != "one_row_grid":
        assert len(set(e_radii.tolist())) > 1, "the radius should move on this workload"
    pool.close()


def test_step_local_longer_than_one_launch():
    """At 2^23 input bits one launch of the two-frame local kernel takes 64
    frames (its paired copy of the frames is bounded): 151 frames run as
    launches of 64, 64 and 23 frames, with the results of one frame at a
    time."""
    import torch
    cfg = synth.sp_config(1 << 23, 256, 64, 2, 3)
    w = synth.random_instance(41, cfg, frames=151, density=0.02)
    pool = sp.SpatialPooler(cfg, w.idx, w.perm)
    assert pool.local_kernel_for(16, 2) == "k_sp_persistent_local2"
    frames = torch.from_numpy(np.ascontiguousarray(w.frames).view(np.int32)).cuda()
    F, C = w.frames.shape[0], cfg["num_columns"]
    ov = torch.empty((F, C), dtype=torch.int32, device="cuda")
    act = torch.empty((F, C), dtype=torch.uint8, device="cuda")
    sp.sp_step_local(pool.handle, cfg, frames, True, 16, 2, ov, act)
    pool.sync()
    perm = pool.perm.cpu().numpy()
    pool.close()
    e_ov, e_act, e_perm = oracle.run_local(cfg, w.idx, w.perm, w.frames, 16, 2, 3)
    assert np.array_equal(ov.cpu().numpy(), e_ov)
    assert np.array_equal(act.cpu().numpy(), e_act)
    assert np.array_equal(perm.astype(np.float64), e_perm)

