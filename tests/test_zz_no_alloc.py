"""sp_infer_noalloc, the inference entry point that allocates nothing (its
lists live in the library's fixed per-GPU scratch array), called through the
C ABI and checked against sp_infer in gather mode on the same inputs, bit
for bit: two calls in a row, the second with a smaller input, then a third
that goes back to the first handle after the second rewrote the scratch."""
import ctypes

import numpy as np
import pytest

import paper_1608_01966_amd as sp
from paper_1608_01966_amd import synth

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _both(pool, w, frames):
    """(overlaps, winners) of sp_infer_noalloc and of sp_infer on `frames`."""
    import torch
    lib = sp.lib()
    F, C, k = frames.shape[0], w.cfg["num_columns"], w.cfg["winners"]
    ov = torch.full((F, C), -7, dtype=torch.int32, device="cuda")
    win = torch.full((F, k), -7, dtype=torch.int32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.sp_infer_noalloc(ctypes.c_void_p(pool.handle), _ptr(frames), F, _ptr(ov), _ptr(win),
                              s)
    assert rc == sp.SP_OK, sp.sp_last_error()
    ov2 = torch.empty((F, C), dtype=torch.int32, device="cuda")
    win2 = torch.empty((F, k), dtype=torch.int32, device="cuda")
    rc = lib.sp_infer(ctypes.c_void_p(pool.handle), _ptr(frames), F, sp.SP_INFER_GATHER, _ptr(ov2),
                      _ptr(win2), s)
    assert rc == sp.SP_OK, sp.sp_last_error()
    pool.sync()
    return ov.cpu().numpy(), win.cpu().numpy(), ov2.cpu().numpy(), win2.cpu().numpy()


def _dev(frames):
    import torch
    return torch.from_numpy(np.ascontiguousarray(frames).view(np.int32)).cuda()


def test_noalloc_matches_sp_infer_on_consecutive_calls():
    import oracle
    big = synth.workload_batched_inference(frames=256)
    small = synth.workload_plain_32x32(40)
    pa = sp.SpatialPooler(big.cfg, big.idx, big.perm)
    pb = sp.SpatialPooler(small.cfg, small.idx, small.perm)
    for pool, w in ((pa, big), (pb, small), (pa, big)):
        fr = _dev(w.frames)
        ov, win, ov2, win2 = _both(pool, w, fr)
        assert np.array_equal(ov, ov2) and np.array_equal(win, win2), w.name
        e_ov, e_win, _ = oracle.run(w.cfg, w.idx, w.perm, w.frames, learn=False)
        assert np.array_equal(ov, e_ov) and np.array_equal(win, e_win), w.name
    # fewer frames of the same handle, after learning changed its state
    pb.step(small.frames[:10], learn=True)
    ov, win, ov2, win2 = _both(pb, small, _dev(small.frames[10:17]))
    assert np.array_equal(ov, ov2) and np.array_equal(win, win2)
    pa.close()
    pb.close()


def test_noalloc_refuses_what_the_scratch_cannot_hold():
    import torch
    lib = sp.lib()
    assert lib.sp_infer_noalloc_max_bytes() == 16 << 20
    # lists of 65536 x 64 entries: 16.8 MB > 16 MiB
    w = synth.random_instance(41, synth.sp_config(70000, 65536, 64, 1, 10), frames=2)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    fr = _dev(w.frames)
    ov = torch.empty((2, 65536), dtype=torch.int32, device="cuda")
    win = torch.empty((2, 10), dtype=torch.int32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.sp_infer_noalloc(ctypes.c_void_p(pool.handle), _ptr(fr), 2, _ptr(ov), _ptr(win), s)
    assert rc == sp.SP_EINVAL and "scratch" in sp.sp_last_error()
    rc = lib.sp_infer_noalloc(ctypes.c_void_p(pool.handle), _ptr(fr), 2, None, _ptr(win), s)
    assert rc == sp.SP_EINVAL
    pool.close()
