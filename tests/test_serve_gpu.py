"""Serving on the GPU: every stream's winners, final permanences and SDR
histogram equal the oracle stepping that stream alone, while batches mixed
many streams -- with staggered streams under a budget of half their state,
and with every stream live at once under a budget that forces evictions and
re-admissions from checkpoints."""
import numpy as np
import pytest

import oracle
from paper_1608_01966_amd import serve, synth

pytestmark = pytest.mark.gpu


def _run_and_check(specs, frames, pool, budget_frac, quantum):
    be = serve.GpuBackend(pool, specs)
    need = [be.stream_bytes(s) for s in specs]
    srv = serve.Server(be, specs, budget_bytes=int(sum(need) * budget_frac), quantum=quantum)
    finals = {}
    orig_close = be.close

    def close_(h):
        # the library waits for the handle's own work only; read its final
        # permanences on the side stream before it goes
        if srv.finished[h["i"]] or srv.done[h["i"]] == srv.nframes[h["i"]]:
            finals[h["i"]] = h["pool"].get_state(stream=be.side, with_idx=False)[1]
        orig_close(h)
    be.close = close_
    srv.run()
    be.stream.synchronize()
    assert max(srv.batch_streams) > 1
    assert srv.peak_used <= srv.budget
    for i, spec in enumerate(specs):
        e_ov, e_win, e_perm = oracle.run(spec.cfg, spec.idx, spec.perm, frames[spec.frame_ids])
        win = be.winners(i).cpu().numpy()
        hist = be.histogram(i).cpu().numpy()
        assert np.array_equal(win, e_win), f"stream {spec.sid}"
        assert np.array_equal(finals[i].astype(np.float64), e_perm), f"stream {spec.sid}"
        assert np.array_equal(hist.astype(np.uint32),
                              oracle.histogram(e_win, spec.cfg["num_columns"])), f"stream {spec.sid}"
    lat = srv.latencies()
    assert lat.size == sum(len(s.arrivals) for s in specs) and np.all(lat > 0)
    assert len(be.gpu_ms) == len(srv.batch_sizes) and min(be.gpu_ms) > 0
    return srv


def test_staggered_streams_equal_alone_in_the_mix():
    import torch
    P = 64
    frames = synth.blob_frames(synth.rng(9, 2), P, 240, 134, 0.05)
    pool = torch.from_numpy(frames.view(np.int32)).cuda()
    specs = serve.make_streams(24, fps=300.0, window=0.6, pool_frames=P, seed=11,
                               columns=(256, 512, 1024), synapses=(32, 64, 128),
                               input_bits=240 * 134, min_len=0.1, max_len=0.4)
    _run_and_check(specs, frames, pool, budget_frac=0.5, quantum=None)


def test_evictions_equal_alone_in_the_mix():
    import torch
    P = 48
    frames = synth.blob_frames(synth.rng(10, 2), P, 240, 134, 0.05)
    pool = torch.from_numpy(frames.view(np.int32)).cuda()
    specs = serve.make_streams(16, fps=120.0, window=0.5, pool_frames=P, seed=12,
                               columns=(256, 512, 1024), synapses=(32, 64, 256, 512),
                               input_bits=240 * 134)
    srv = _run_and_check(specs, frames, pool, budget_frac=0.4, quantum=0.02)
    assert srv.evictions > 0 and srv.readmissions > 0
