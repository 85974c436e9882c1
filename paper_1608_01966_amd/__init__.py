"""htmsp -- the HTM spatial pooler step (Wielgosz & Pietron, arXiv 1608.01966,
Section 1.1) on AMD Instinct MI355X.

Thin Python binding over the C ABI of ``libhtmsp.so`` (``include/sp.h``):
each ``sp_*`` function here has the C function's name and only marshals
arguments (torch device tensors -> device pointers, torch streams -> HIP
streams).  Every step of the computation runs in the library's HIP kernels.

Tensor conventions (all on the GPU, contiguous):
  idx     int32  [C][S]  input pixel per potential synapse (uint32 bits)
  perm    float32[C][S]  permanences on the 1/256 grid
  frames  int32  [F][W]  packed frames, W = ceil(N/32) (uint32 bits)
  overlaps int32 [F][C]
  winners  int32 [F][k]  ascending, -1 padded
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native, synth
from ._native import (SP_EBROKEN, SP_EDEVICE, SP_EINVAL, SP_ENOMEM, SP_INFER_GATHER,
                      SP_INFER_MFMA_I8, SP_OK, SpConfig, lib)

__all__ = [
    "SpError", "SpatialPooler", "synth", "sp_config_check", "sp_frame_words",
    "sp_workspace_bytes", "sp_check_state_host", "sp_create", "sp_check_state", "sp_step",
    "sp_step_plain", "sp_infer", "sp_step_many", "sp_step_many_raw", "sp_set_histogram", "sp_encode",
    "sp_inhibit_local", "sp_step_local", "sp_step_local_adaptive", "sp_step_boost", "sp_boost_state", "sp_boost_reset",
    "sp_encoded_bits", "sp_step_is_persistent", "sp_step_kernel", "sp_step_local_kernel",
    "sp_step_local_kernel_for", "LOCAL_KERNELS",
    "sp_step_boost_kernel", "sp_test_stall", "STEP_KERNELS", "sp_state_bytes", "sp_get_state",
    "sp_set_state", "sp_get_boost_state", "sp_set_boost_state",
    "sp_sync",
    "sp_destroy",
    "sp_last_error", "SP_OK", "SP_EINVAL", "SP_ENOMEM", "SP_EDEVICE", "SP_EBROKEN",
    "SP_INFER_GATHER", "SP_INFER_MFMA_I8",
]


class SpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def sp_last_error() -> str:
    return lib().sp_last_error().decode()


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise SpError(rc, f"{what}: {sp_last_error()}")
    return rc


def _cfg(cfg) -> SpConfig:
    return cfg if isinstance(cfg, SpConfig) else SpConfig.from_dict(cfg)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev(t, dtype, shape, name):
    """Device pointer of a contiguous CUDA tensor of the given dtype/shape."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def sp_config_check(cfg) -> None:
    c = _cfg(cfg)
    _check(lib().sp_config_check(ctypes.byref(c)), "sp_config_check")


def sp_frame_words(cfg) -> int:
    c = _cfg(cfg)
    return int(lib().sp_frame_words(ctypes.byref(c)))


def sp_workspace_bytes(cfg) -> int:
    c = _cfg(cfg)
    return int(lib().sp_workspace_bytes(ctypes.byref(c)))


def sp_check_state_host(cfg, idx: np.ndarray, perm: np.ndarray) -> None:
    c = _cfg(cfg)
    n = c.num_columns * c.synapses_per_column
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    perm = np.ascontiguousarray(perm, dtype=np.float32)
    if idx.size != n or perm.size != n:
        raise ValueError("idx and perm must hold num_columns * synapses_per_column entries")
    _check(lib().sp_check_state_host(ctypes.byref(c), idx.ctypes.data_as(ctypes.c_void_p),
                                     perm.ctypes.data_as(ctypes.c_void_p)), "sp_check_state_host")


def sp_create(cfg, idx, perm, stream=None) -> int:
    """Returns an opaque handle (int).  idx and perm are borrowed: keep them
    alive until sp_destroy."""
    import torch
    c = _cfg(cfg)
    shape = (c.num_columns, c.synapses_per_column)
    pi = _dev(idx, torch.int32, shape, "idx")
    pp = _dev(perm, torch.float32, shape, "perm")
    out = ctypes.c_void_p()
    _check(lib().sp_create(ctypes.byref(c), pi, pp, _stream(stream), ctypes.byref(out)),
           "sp_create")
    return int(out.value)


def sp_check_state(h: int, stream=None) -> None:
    _check(lib().sp_check_state(ctypes.c_void_p(h), _stream(stream)), "sp_check_state")


def _step(fn, name, h, cfg, frames, learn, overlaps, winners, stream):
    import torch
    c = _cfg(cfg)
    F = int(frames.shape[0]) if frames is not None else 0
    W = (c.input_bits + 31) // 32
    pf = _dev(frames, torch.int32, (F, W), "frames")
    po = _dev(overlaps, torch.int32, (F, c.num_columns), "overlaps")
    pw = _dev(winners, torch.int32, (F, c.winners), "winners")
    _check(fn(ctypes.c_void_p(h), pf, F, int(bool(learn)), po, pw, _stream(stream)), name)


def sp_step(h: int, cfg, frames, learn: bool, overlaps, winners, stream=None) -> None:
    _step(lib().sp_step, "sp_step", h, cfg, frames, learn, overlaps, winners, stream)


def sp_step_plain(h: int, cfg, frames, learn: bool, overlaps, winners, stream=None) -> None:
    _step(lib().sp_step_plain, "sp_step_plain", h, cfg, frames, learn, overlaps, winners, stream)


def sp_infer(h: int, cfg, frames, mode: int, overlaps, winners, stream=None) -> None:
    """Batched inference (learning off); overlaps may be None."""
    import torch
    c = _cfg(cfg)
    F = int(frames.shape[0])
    W = (c.input_bits + 31) // 32
    pf = _dev(frames, torch.int32, (F, W), "frames")
    po = _dev(overlaps, torch.int32, (F, c.num_columns), "overlaps")
    pw = _dev(winners, torch.int32, (F, c.winners), "winners")
    _check(lib().sp_infer(ctypes.c_void_p(h), pf, F, int(mode), po, pw, _stream(stream)),
           "sp_infer")


def sp_step_many(handles, cfgs, frames, learn: bool, overlaps, winners, stream=None) -> None:
    """Steps several handles in one launch.  frames[i] is an int32 GPU tensor
    [F_i][W_i] (F_i may be 0); overlaps[i] may be None (or overlaps None);
    winners[i] is [F_i][k_i]."""
    import torch
    n = len(handles)
    H = (ctypes.c_void_p * n)(*[ctypes.c_void_p(h) for h in handles])
    FR = (ctypes.c_void_p * n)()
    NF = (ctypes.c_uint32 * n)()
    OV = (ctypes.c_void_p * n)()
    WN = (ctypes.c_void_p * n)()
    for i in range(n):
        c = _cfg(cfgs[i])
        F = int(frames[i].shape[0])
        W = (c.input_bits + 31) // 32
        NF[i] = F
        FR[i] = _dev(frames[i], torch.int32, (F, W), f"frames[{i}]")
        ov = overlaps[i] if overlaps is not None else None
        OV[i] = _dev(ov, torch.int32, (F, c.num_columns), f"overlaps[{i}]")
        WN[i] = _dev(winners[i], torch.int32, (F, c.winners), f"winners[{i}]")
    _check(lib().sp_step_many(H, n, FR, NF, int(bool(learn)), OV, WN, _stream(stream)),
           "sp_step_many")


def sp_step_many_raw(handles: np.ndarray, frames: np.ndarray, num_frames: np.ndarray,
                     learn: bool, overlaps, winners: np.ndarray, stream=None) -> None:
    """sp_step_many with its arrays already built: handles, frames and
    winners are uint64 numpy arrays of handles and device addresses,
    num_frames a uint32 array, overlaps a uint64 array or None (marshalling
    only, for schedulers that batch hundreds of handles per call)."""
    n = len(handles)
    arrs = [np.ascontiguousarray(handles, dtype=np.uint64),
            np.ascontiguousarray(frames, dtype=np.uint64),
            np.ascontiguousarray(num_frames, dtype=np.uint32),
            np.ascontiguousarray(winners, dtype=np.uint64)]
    if any(len(a) != n for a in arrs[1:]):
        raise ValueError("handles, frames, num_frames and winners must have one entry each")
    ov = None
    if overlaps is not None:
        ov = np.ascontiguousarray(overlaps, dtype=np.uint64)
        if len(ov) != n:
            raise ValueError("overlaps must have one entry per handle")
    _check(lib().sp_step_many(_host_ptr(arrs[0]), n, _host_ptr(arrs[1]), _host_ptr(arrs[2]),
                              int(bool(learn)), _host_ptr(ov) if ov is not None else None,
                              _host_ptr(arrs[3]), _stream(stream)), "sp_step_many")


def _boost_cfg(b: dict):
    return _native.BoostCfg(int(b["period_log2"]), int(b["min_pct_q16"]),
                            int(b["max_boost_q8"]), int(b["bump_q8"]))


def sp_step_boost(h: int, cfg: dict, bcfg: dict, frames, learn: bool, overlaps, winners,
                  stream=None) -> None:
    """Frames in order with boosting; bcfg has period_log2, min_pct_q16,
    max_boost_q8, bump_q8; overlaps (boosted, may be None) and winners are
    GPU tensors [F][C] and [F][k]."""
    b = _boost_cfg(bcfg)
    _check(lib().sp_step_boost(ctypes.c_void_p(h), ctypes.byref(b),
                               ctypes.c_void_p(frames.data_ptr()), int(frames.shape[0]),
                               int(bool(learn)),
                               ctypes.c_void_p(overlaps.data_ptr()) if overlaps is not None
                               else None, ctypes.c_void_p(winners.data_ptr()), _stream(stream)),
           "sp_step_boost")


def sp_boost_state(h: int, num_columns: int, stream=None):
    """(active duty, overlap duty, boost) as int32 GPU tensors [C]."""
    import torch
    out = [torch.empty(num_columns, dtype=torch.int32, device="cuda") for _ in range(3)]
    _check(lib().sp_boost_state(ctypes.c_void_p(h), *(ctypes.c_void_p(t.data_ptr()) for t in out),
                                _stream(stream)), "sp_boost_state")
    return tuple(out)


def sp_boost_reset(h: int, stream=None) -> None:
    _check(lib().sp_boost_reset(ctypes.c_void_p(h), _stream(stream)), "sp_boost_reset")


def sp_inhibit_local(overlaps, grid_w: int, radius: int, n: int, active=None, stream=None):
    """overlaps: int32 GPU tensor [F][C].  Returns (or fills) the uint8 GPU
    tensor [F][C] of active flags (Algorithm 2 with a neighbourhood)."""
    import torch
    assert overlaps.is_cuda and overlaps.dtype == torch.int32 and overlaps.dim() == 2
    overlaps = overlaps.contiguous()
    F, C = (int(x) for x in overlaps.shape)
    if active is None:
        active = torch.empty((F, C), dtype=torch.uint8, device=overlaps.device)
    assert active.is_contiguous() and active.shape == (F, C) and active.dtype == torch.uint8
    _check(lib().sp_inhibit_local(ctypes.c_void_p(overlaps.data_ptr()), F, C, int(grid_w),
                                  int(radius), int(n), ctypes.c_void_p(active.data_ptr()),
                                  _stream(stream)), "sp_inhibit_local")
    return active


def sp_step_local(h: int, cfg: dict, frames, learn: bool, grid_w: int, radius: int,
                  overlaps, active, stream=None) -> None:
    """Frames in order with local inhibition (n = cfg winners); overlaps may
    be None; active: uint8 GPU tensor [F][C]."""
    F = int(frames.shape[0])
    assert active.shape == (F, cfg["num_columns"])
    _check(lib().sp_step_local(ctypes.c_void_p(h), ctypes.c_void_p(frames.data_ptr()), F,
                               int(bool(learn)), int(grid_w), int(radius),
                               ctypes.c_void_p(overlaps.data_ptr()) if overlaps is not None
                               else None, ctypes.c_void_p(active.data_ptr()),
                               _stream(stream)), "sp_step_local")


def sp_step_local_adaptive(h: int, cfg: dict, frames, learn: bool, input_w: int, grid_w: int,
                           radius, overlaps, active, radii=None, stream=None) -> None:
    """sp_step_local with the radius adapted after each learning frame.
    radius: int32 GPU tensor [1] (the first frame's radius in, the last
    radius out); radii: int32 GPU tensor [F] of each frame's radius, or None."""
    import torch
    F = int(frames.shape[0])
    C = cfg["num_columns"]
    pr = _dev(radius, torch.int32, (1,), "radius")
    pa = _dev(active, torch.uint8, (F, C), "active")
    po = _dev(overlaps, torch.int32, (F, C), "overlaps")
    prs = _dev(radii, torch.int32, (F,), "radii")
    _check(lib().sp_step_local_adaptive(ctypes.c_void_p(h), ctypes.c_void_p(frames.data_ptr()), F,
                                        int(bool(learn)), int(input_w), int(grid_w), pr, po, pa,
                                        prs, _stream(stream)), "sp_step_local_adaptive")


def _enc_cfg(width: int, height: int, factor: int = 1, block: int = 11, offset: int = 2):
    return _native.EncCfg(int(width), int(height), int(factor), int(block), int(offset))


def sp_encoded_bits(width: int, height: int, factor: int = 1, block: int = 11,
                    offset: int = 2) -> int:
    """Input bits of one encoded frame (0 for a bad configuration)."""
    return int(lib().sp_encoded_bits(ctypes.byref(_enc_cfg(width, height, factor, block,
                                                           offset))))


def sp_encode(rgb, factor: int = 1, block: int = 11, offset: int = 2, out=None, stream=None):
    """rgb: uint8 GPU tensor [F][H][W][3].  Returns (or fills) the int32 GPU
    tensor [F][ceil(bits / 32)] of packed binary frames."""
    import torch
    assert rgb.is_cuda and rgb.dtype == torch.uint8 and rgb.dim() == 4 and rgb.shape[3] == 3
    rgb = rgb.contiguous()
    F, H, W = (int(x) for x in rgb.shape[:3])
    c = _enc_cfg(W, H, factor, block, offset)
    bits = int(lib().sp_encoded_bits(ctypes.byref(c)))
    if bits == 0:
        raise SpError(SP_EINVAL, f"sp_encoded_bits: {sp_last_error()}")
    if out is None:
        out = torch.empty((F, (bits + 31) // 32), dtype=torch.int32, device=rgb.device)
    assert out.is_contiguous() and out.shape == (F, (bits + 31) // 32)
    _check(lib().sp_encode(ctypes.byref(c), ctypes.c_void_p(rgb.data_ptr()), F,
                           ctypes.c_void_p(out.data_ptr()), _stream(stream)), "sp_encode")
    return out


def sp_set_histogram(h: int, hist=None) -> None:
    """hist: uint32-sized int32 GPU tensor [C] that every later call of this
    handle adds its winners to, or None to stop."""
    if hist is not None:
        assert hist.is_cuda and hist.is_contiguous() and hist.element_size() == 4
    ptr = ctypes.c_void_p(hist.data_ptr()) if hist is not None else None
    _check(lib().sp_set_histogram(ctypes.c_void_p(h), ptr), "sp_set_histogram")


def sp_step_is_persistent(h: int) -> bool:
    return bool(_check(lib().sp_step_is_persistent(ctypes.c_void_p(h)), "sp_step_is_persistent"))


# sp_step_kernel codes, and the HIP kernel each one runs.
STEP_KERNELS = {0: "plain", 2: "k_sp_persistent_w"}


def sp_step_kernel(h: int) -> str:
    """The execution sp_step uses for this handle: a STEP_KERNELS value."""
    return STEP_KERNELS[_check(lib().sp_step_kernel(ctypes.c_void_p(h)), "sp_step_kernel")]


def sp_step_local_kernel(h: int) -> str:
    """The execution sp_step_local uses: "plain" or "k_sp_persistent_local"."""
    code = _check(lib().sp_step_local_kernel(ctypes.c_void_p(h)), "sp_step_local_kernel")
    return "k_sp_persistent_local" if code == 2 else "plain"


# sp_step_local_kernel_for codes, and the HIP kernel each one runs.
LOCAL_KERNELS = {0: "plain", 2: "k_sp_persistent_local", 3: "k_sp_persistent_local2"}


def sp_step_local_kernel_for(h: int, grid_w: int, radius: int) -> str:
    """The execution sp_step_local uses with this grid width and radius: a
    LOCAL_KERNELS value."""
    code = _check(lib().sp_step_local_kernel_for(ctypes.c_void_p(h), int(grid_w), int(radius)),
                  "sp_step_local_kernel_for")
    return LOCAL_KERNELS[code]


def sp_step_boost_kernel(h: int) -> str:
    """The execution sp_step_boost uses: "plain" or "k_sp_persistent_boost"."""
    code = _check(lib().sp_step_boost_kernel(ctypes.c_void_p(h)), "sp_step_boost_kernel")
    return "k_sp_persistent_boost" if code == 2 else "plain"


def sp_test_stall(h: int, spin_limit: int) -> None:
    """Failure-path tests only: the next persistent launch on this handle
    stalls on its exchange and gives up after `spin_limit` polls."""
    _check(lib().sp_test_stall(ctypes.c_void_p(h), spin_limit), "sp_test_stall")


def _host_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def sp_state_bytes(cfg) -> int:
    """Bytes of a handle's idx plus perm (0 for a bad configuration)."""
    c = _cfg(cfg)
    return int(lib().sp_state_bytes(ctypes.byref(c)))


def sp_get_state(h: int, cfg, stream=None, with_idx: bool = True):
    """(idx uint32 [C][S] or None, perm float32 [C][S], frames_seen) in host
    memory."""
    c = _cfg(cfg)
    shape = (c.num_columns, c.synapses_per_column)
    idx = np.empty(shape, dtype=np.uint32) if with_idx else None
    perm = np.empty(shape, dtype=np.float32)
    seen = ctypes.c_uint64()
    _check(lib().sp_get_state(ctypes.c_void_p(h), _host_ptr(idx) if with_idx else None,
                              _host_ptr(perm), ctypes.byref(seen), _stream(stream)),
           "sp_get_state")
    return idx, perm, int(seen.value)


def sp_set_state(h: int, cfg, idx, perm, frames_seen: int = 0, stream=None) -> None:
    """Loads host arrays idx (or None: keep the pools) and perm into the
    handle's device state."""
    c = _cfg(cfg)
    n = c.num_columns * c.synapses_per_column
    perm = np.ascontiguousarray(perm, dtype=np.float32)
    if perm.size != n:
        raise ValueError("perm must hold num_columns * synapses_per_column entries")
    pi = None
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.uint32)
        if idx.size != n:
            raise ValueError("idx must hold num_columns * synapses_per_column entries")
        pi = _host_ptr(idx)
    _check(lib().sp_set_state(ctypes.c_void_p(h), pi, _host_ptr(perm), int(frames_seen),
                              _stream(stream)), "sp_set_state")


def sp_get_boost_state(h: int, num_columns: int, stream=None):
    """(active duty, overlap duty, boost) as uint32 host arrays [C]."""
    out = [np.empty(num_columns, dtype=np.uint32) for _ in range(3)]
    _check(lib().sp_get_boost_state(ctypes.c_void_p(h), *(_host_ptr(a) for a in out),
                                    _stream(stream)), "sp_get_boost_state")
    return tuple(out)


def sp_set_boost_state(h: int, active_duty, overlap_duty, boost, stream=None) -> None:
    """Loads the boost state from uint32 host arrays [C]."""
    arrs = [np.ascontiguousarray(a, dtype=np.uint32) for a in (active_duty, overlap_duty, boost)]
    _check(lib().sp_set_boost_state(ctypes.c_void_p(h), *(_host_ptr(a) for a in arrs),
                                    _stream(stream)), "sp_set_boost_state")


def sp_sync(h: int, stream=None) -> None:
    _check(lib().sp_sync(ctypes.c_void_p(h), _stream(stream)), "sp_sync")


def sp_destroy(h: int) -> None:
    _check(lib().sp_destroy(ctypes.c_void_p(h) if h else None), "sp_destroy")


def _keep_for(stream, *tensors) -> None:
    """Tensors allocated on the current stream but used by a call enqueued on
    another `stream`: the caching allocator must not hand their memory to new
    work before that stream has passed the call."""
    import torch
    if stream is None or not isinstance(stream, torch.cuda.Stream):
        return
    if stream == torch.cuda.current_stream(stream.device):
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


class SpatialPooler:
    """One spatial pooler instance whose state lives in GPU memory.

    ``cfg`` is a dict with the fields of ``sp_config``; ``idx`` (uint32 or
    int32 [C][S]) and ``perm`` (float32 [C][S], 1/256 grid) may be numpy
    arrays or GPU tensors; they are copied to GPU tensors owned by the
    instance."""

    def __init__(self, cfg: dict, idx, perm, device="cuda", stream=None):
        import torch
        self.cfg = dict(cfg)
        if isinstance(idx, np.ndarray):
            idx = torch.from_numpy(np.ascontiguousarray(idx).astype(np.uint32).view(np.int32))
        if isinstance(perm, np.ndarray):
            perm = torch.from_numpy(np.ascontiguousarray(perm, dtype=np.float32))
        self.idx = idx.to(device=device, dtype=torch.int32).contiguous()
        self.perm = perm.to(device=device, dtype=torch.float32).contiguous()
        if stream is not None:
            # the copies above ran on the current stream; sp_create checks
            # the state on `stream`
            torch.cuda.current_stream(self.idx.device).synchronize()
        self.handle = sp_create(self.cfg, self.idx, self.perm, stream)

    @property
    def persistent(self) -> bool:
        return sp_step_is_persistent(self.handle)

    @property
    def kernel(self) -> str:
        """The execution sp_step uses (a STEP_KERNELS value)."""
        return sp_step_kernel(self.handle)

    @property
    def local_kernel(self) -> str:
        """The execution sp_step_local uses."""
        return sp_step_local_kernel(self.handle)

    def local_kernel_for(self, grid_w: int, radius: int) -> str:
        """The execution sp_step_local uses with this grid width and radius."""
        return sp_step_local_kernel_for(self.handle, grid_w, radius)

    @property
    def boost_kernel(self) -> str:
        """The execution sp_step_boost uses."""
        return sp_step_boost_kernel(self.handle)

    def step(self, frames, learn: bool = True, overlaps: bool = True, plain: bool = False,
             stream=None):
        """frames: int32 GPU tensor [F][W] (or uint32 numpy).  Returns
        (overlaps [F][C] or None, winners [F][k]) GPU tensors, valid after the
        stream synchronises."""
        import torch
        if isinstance(frames, np.ndarray):
            frames = torch.from_numpy(np.ascontiguousarray(frames, dtype=np.uint32).view(np.int32))
        frames = frames.to(device=self.idx.device).contiguous()
        F = frames.shape[0]
        ov = torch.empty((F, self.cfg["num_columns"]), dtype=torch.int32,
                         device=self.idx.device) if overlaps else None
        win = torch.empty((F, self.cfg["winners"]), dtype=torch.int32, device=self.idx.device)
        fn = sp_step_plain if plain else sp_step
        fn(self.handle, self.cfg, frames, learn, ov, win, stream)
        _keep_for(stream, frames, ov, win)
        return ov, win

    def infer(self, frames, overlaps: bool = True, mode: int = SP_INFER_GATHER, stream=None):
        """Batched inference over F independent frames; returns (overlaps or
        None, winners) GPU tensors; the state is not changed."""
        import torch
        if isinstance(frames, np.ndarray):
            frames = torch.from_numpy(np.ascontiguousarray(frames, dtype=np.uint32).view(np.int32))
        frames = frames.to(device=self.idx.device).contiguous()
        F = frames.shape[0]
        ov = torch.empty((F, self.cfg["num_columns"]), dtype=torch.int32,
                         device=self.idx.device) if overlaps else None
        win = torch.empty((F, self.cfg["winners"]), dtype=torch.int32, device=self.idx.device)
        sp_infer(self.handle, self.cfg, frames, mode, ov, win, stream)
        _keep_for(stream, frames, ov, win)
        return ov, win

    def get_state(self, stream=None, with_idx: bool = True):
        """Checkpoint: (idx or None, perm, frames_seen) in host memory."""
        return sp_get_state(self.handle, self.cfg, stream, with_idx)

    def set_state(self, idx, perm, frames_seen: int = 0, stream=None) -> None:
        """Resume from a checkpoint taken by get_state (idx None keeps the pools)."""
        sp_set_state(self.handle, self.cfg, idx, perm, frames_seen, stream)

    def set_histogram(self, hist=None) -> None:
        """Accumulate every later call's winners into `hist` (GPU int32 [C],
        kept alive here), or stop with None."""
        sp_set_histogram(self.handle, hist)
        self.hist = hist

    def sync(self, stream=None) -> None:
        sp_sync(self.handle, stream)

    def close(self) -> None:
        if self.handle:
            sp_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
