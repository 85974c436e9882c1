"""Serving on the GPU: every stream's winners and final permanences equal
the oracle stepping that stream alone, while batches mixed many streams."""
import numpy as np
import pytest

import oracle
from paper_1608_01966_amd import serve, synth

pytestmark = pytest.mark.gpu


def test_streams_equal_alone_in_the_mix():
    import torch
    P = 64
    frames = synth.blob_frames(synth.rng(9, 2), P, 240, 134, 0.05)
    pool = torch.from_numpy(frames.view(np.int32)).cuda()
    specs = serve.make_streams(24, fps=300.0, window=0.6, pool_frames=P, seed=11,
                               columns=(256, 512, 1024), synapses=(32, 64, 128),
                               input_bits=240 * 134, min_len=0.1, max_len=0.4)
    be = serve.GpuBackend(pool)
    need = [be.stream_bytes(s) for s in specs]
    srv = serve.Server(be, specs, budget_bytes=sum(need) // 2)
    handles = {}
    orig_open = be.open

    def open_(spec):
        h = orig_open(spec)
        handles[spec.sid] = h
        return h
    be.open = open_
    orig_close = be.close
    finals = {}

    def close_(h):
        h["pool"].sync(be.stream)
        finals[id(h)] = (h["win"].cpu().numpy(), h["pool"].perm.cpu().numpy(),
                         h["hist"].cpu().numpy())
        orig_close(h)
    be.close = close_
    srv.run()
    assert max(srv.batch_sizes) > 1
    assert srv.peak_used <= srv.budget
    for spec in specs:
        win, perm, hist = finals[id(handles[spec.sid])]
        e_ov, e_win, e_perm = oracle.run(spec.cfg, spec.idx, spec.perm, frames[spec.frame_ids])
        assert np.array_equal(win, e_win), f"stream {spec.sid}"
        assert np.array_equal(perm.astype(np.float64), e_perm), f"stream {spec.sid}"
        assert np.array_equal(hist.astype(np.uint32),
                              oracle.histogram(e_win, spec.cfg["num_columns"])), f"stream {spec.sid}"
    lat = srv.latencies()
    assert lat.size == sum(len(s.arrivals) for s in specs) and np.all(lat > 0)
