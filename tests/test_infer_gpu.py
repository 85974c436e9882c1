"""Parity of batched inference (sp_infer, learning off) with the oracle run
with learning off: overlaps and winners element by element, bit-exact, and
the state unchanged, for the gather mode and the int8 matrix-product mode."""
import numpy as np
import pytest

import oracle
import paper_1608_01966_amd as sp
from paper_1608_01966_amd import synth

pytestmark = pytest.mark.gpu


MODES = [sp.SP_INFER_GATHER, sp.SP_INFER_MFMA_I8]
MODE_IDS = ["gather", "mfma"]


def check_infer(w, want_ov=True, mode=sp.SP_INFER_GATHER):
    import torch
    e_ov, e_win, e_perm = oracle.run(w.cfg, w.idx, w.perm, w.frames, learn=False)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    ov, win = pool.infer(w.frames, overlaps=want_ov, mode=mode)
    pool.sync()
    if want_ov:
        bad = np.argwhere(ov.cpu().numpy() != e_ov)
        assert bad.size == 0, f"overlap mismatch at (frame, column) {bad[:5].tolist()}"
    bad = np.argwhere(win.cpu().numpy() != e_win)
    assert bad.size == 0, f"winner mismatch at (frame, slot) {bad[:5].tolist()}"
    assert np.array_equal(pool.perm.cpu().numpy(), w.perm)
    pool.close()


SHAPES = [
    (1, 1, 1, 0, 1, 5, 0.5),
    (33, 5, 33, 2, 5, 9, 0.6),
    (1000, 257, 65, 3, 17, 12, 0.2),
    (4097, 1000, 100, 4, 40, 33, 0.15),
    (20000, 4096, 64, 2, 160, 7, 0.1),
    (100000, 300, 256, 6, 30, 20, 0.05),
    (5000, 2048, 32, 1, 200, 10, 0.2),
]


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
@pytest.mark.parametrize("shape", SHAPES, ids=[f"N{s[0]}_C{s[1]}_S{s[2]}" for s in SHAPES])
def test_random_shapes(shape, mode):
    N, C, S, m, k, F, d = shape
    w = synth.random_instance(21, synth.sp_config(N, C, S, m, k), frames=F, density=d)
    check_infer(w, mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_plain_32x32_workload(mode):
    check_infer(synth.workload_plain_32x32(100), mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_without_overlap_output(mode):
    check_infer(synth.workload_plain_32x32(40), want_ov=False, mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_960x540_bernoulli_1024x256(mode):
    """The batched-inference workload's shape: 960x540 Bernoulli(0.05)
    frames through 1024 columns x 256 synapses (fewer frames than the
    benchmark's 4096, all of them compared)."""
    cfg = synth.sp_config(960 * 540, 1024, 256, 4, 40)
    w = synth.random_instance(3, cfg, frames=512, density=0.05)
    check_infer(w, mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_960x540_full_batch_as_benchmarked(mode):
    """The benchmark's batch exactly: the batched-inference workload's 4096
    frames in one call, every overlap and winner against the oracle."""
    w = synth.workload_batched_inference(frames=4096)
    check_infer(w, mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_columns_past_batch_topk(mode):
    """More than 4096 columns: the top-k falls back to one workgroup per frame."""
    w = synth.random_instance(22, synth.sp_config(30000, 5000, 48, 2, 300), frames=6, density=0.2)
    check_infer(w, mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_frames_too_large_for_lds(mode):
    """N = 2^23: frames are read from global memory instead of LDS (gather);
    a 256 x 262 144-word mask (matrix product)."""
    w = synth.random_instance(23, synth.sp_config(1 << 23, 256, 128, 1, 20), frames=3, density=0.03)
    check_infer(w, mode=mode)


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_unaligned_frames(mode):
    """Frames starting one row into a buffer whose rows are not a multiple of
    16 bytes (W = 129 words)."""
    import torch
    w = synth.random_instance(25, synth.sp_config(4100, 300, 40, 2, 12), frames=9, density=0.3)
    e_ov, e_win, _ = oracle.run(w.cfg, w.idx, w.perm, w.frames[1:], learn=False)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    fr = torch.from_numpy(w.frames.view(np.int32)).cuda()[1:]
    assert fr.data_ptr() % 16 != 0
    ov, win = pool.infer(fr, mode=mode)
    pool.sync()
    assert np.array_equal(ov.cpu().numpy(), e_ov)
    assert np.array_equal(win.cpu().numpy(), e_win)
    pool.close()


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_lists_rebuilt_after_learning(mode):
    import torch
    w = synth.workload_plain_32x32(30)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    ov0, win0 = pool.infer(w.frames[20:], mode=mode)
    pool.step(w.frames[:20], learn=True)
    ov1, win1 = pool.infer(w.frames[20:], mode=mode)
    pool.sync()
    _, _, p20 = oracle.run(w.cfg, w.idx, w.perm, w.frames[:20], learn=True)
    e_ov, e_win, _ = oracle.run(w.cfg, w.idx, p20, w.frames[20:], learn=False)
    assert np.array_equal(ov1.cpu().numpy(), e_ov)
    assert np.array_equal(win1.cpu().numpy(), e_win)
    e0_ov, _, _ = oracle.run(w.cfg, w.idx, w.perm, w.frames[20:], learn=False)
    assert np.array_equal(ov0.cpu().numpy(), e0_ov)
    pool.close()


@pytest.mark.parametrize("case", ["all_connected_300", "s512_960x540", "4096_global_frame"])
def test_gather_lists_longer_than_registers(case):
    """Columns with more than 256 connected synapses: the gather mode reads
    their lists from device memory (frames staged in LDS, or read from device
    memory when a frame is larger than LDS) with the same results."""
    if case == "all_connected_300":
        cfg = synth.sp_config(5000, 16, 300, 1, 4, connected_q8=0)
        w = synth.random_instance(24, cfg, frames=5, density=0.2)
    elif case == "s512_960x540":
        # the batched-training and serving poolers go up to 512 synapses
        cfg = synth.sp_config(960 * 540, 640, 512, 4, 25)
        w = synth.random_instance(25, cfg, frames=9, density=0.05, shape=(960, 540), blobs=True)
    else:
        cfg = synth.sp_config(1 << 21, 300, 4096, 2, 12, connected_q8=0)
        w = synth.random_instance(28, cfg, frames=3, density=0.02)
    check_infer(w, mode=sp.SP_INFER_GATHER)


def test_matrix_product_any_connected_count():
    """The matrix-product mode has no per-column list: 4096 synapses, every
    one connected."""
    cfg = synth.sp_config(20000, 24, 4096, 1, 5, connected_q8=0)
    w = synth.random_instance(26, cfg, frames=4, density=0.3)
    check_infer(w, mode=sp.SP_INFER_MFMA_I8)


def test_matrix_product_rejects_repeated_pixels():
    """Two connected synapses of one column on one pixel: the 0/1 mask cannot
    count them, so the matrix-product mode refuses (the gather mode counts
    both, like the oracle)."""
    w = synth.random_instance(27, synth.sp_config(500, 8, 10, 1, 3, connected_q8=0), frames=3)
    idx = w.idx.copy()
    idx[5, 3] = idx[5, 7]
    w2 = synth.Workload("repeated_pixel", w.cfg, idx, w.perm_q, w.frames)
    check_infer(w2, mode=sp.SP_INFER_GATHER)
    pool = sp.SpatialPooler(w.cfg, idx, w.perm)
    with pytest.raises(sp.SpError, match="repeat a pixel") as e:
        pool.infer(w.frames, mode=sp.SP_INFER_MFMA_I8)
    assert e.value.code == sp.SP_EINVAL
    pool.close()


def test_modes_interleaved_with_learning():
    """Gather and matrix-product calls alternate with learning steps on one
    handle; each inference sees the state the steps left."""
    w = synth.random_instance(28, synth.sp_config(3000, 200, 50, 2, 10), frames=40, density=0.2)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    perm = w.perm.astype(np.float64)
    for i, t in enumerate(range(0, 40, 10)):
        pool.step(w.frames[t:t + 5], learn=True)
        _, _, perm = oracle.run(w.cfg, w.idx, perm, w.frames[t:t + 5], learn=True)
        for mode in (MODES if i % 2 == 0 else MODES[::-1]):
            ov, win = pool.infer(w.frames[t + 5:t + 10], mode=mode)
            pool.sync()
            e_ov, e_win, _ = oracle.run(w.cfg, w.idx, perm, w.frames[t + 5:t + 10], learn=False)
            assert np.array_equal(ov.cpu().numpy(), e_ov), (t, mode)
            assert np.array_equal(win.cpu().numpy(), e_win), (t, mode)
    pool.close()


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_zero_frames(mode):
    import torch
    w = synth.workload_plain_32x32(1)
    pool = sp.SpatialPooler(w.cfg, w.idx, w.perm)
    ov, win = pool.infer(torch.empty((0, 32), dtype=torch.int32, device="cuda"), mode=mode)
    pool.sync()
    assert ov.shape == (0, 256) and win.shape == (0, 20)
    pool.close()
