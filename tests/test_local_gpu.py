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
    pool.close()


def test_rejects_bad_arguments():
    import torch
    ov = torch.zeros((2, 10), dtype=torch.int32, device="cuda")
    for kw in ({"grid_w": 0}, {"grid_w": 11}, {"n": 0}):
        args = {"grid_w": 5, "radius": 1, "n": 1}
        args.update(kw)
        with pytest.raises(sp.SpError):
            sp.sp_inhibit_local(ov, **args)
