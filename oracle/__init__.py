"""Oracle for the HTM spatial pooler step -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper over ``sp_oracle.c`` (plain C, double-precision permanences),
a direct implementation of Section 1.1 of Wielgosz & Pietron (arXiv
1608.01966): Algorithm 1 (overlap), Algorithm 2 (inhibition, global form)
and the learning rule the paper takes from the Numenta CLA whitepaper.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The GPU library never does, and this
module imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_lib", "libsp_oracle.so")


def build() -> str:
    """Compile the oracle with gcc (portable flags: the library also runs on
    hosts other than the one that built it)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call([
        "gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-Werror", "-fPIC", "-shared", "-pthread",
        os.path.join(_HERE, "sp_oracle.c"), os.path.join(_HERE, "sp_oracle_mt.c"),
        os.path.join(_HERE, "enc_oracle.c"), "-o", tmp,
    ])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("input_bits", ctypes.c_uint32),
        ("num_columns", ctypes.c_uint32),
        ("synapses_per_column", ctypes.c_uint32),
        ("min_overlap", ctypes.c_uint32),
        ("winners", ctypes.c_uint32),
        ("connected_perm", ctypes.c_double),
        ("perm_inc", ctypes.c_double),
        ("perm_dec", ctypes.c_double),
    ]


class _Boost(ctypes.Structure):
    _fields_ = [
        ("period_log2", ctypes.c_uint32),
        ("min_pct_q16", ctypes.c_uint32),
        ("max_boost_q8", ctypes.c_uint32),
        ("bump_q8", ctypes.c_uint32),
    ]


class _EncCfg(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_uint32),
        ("height", ctypes.c_uint32),
        ("factor", ctypes.c_uint32),
        ("block", ctypes.c_uint32),
        ("offset", ctypes.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.spo_overlap.argtypes = [ctypes.POINTER(_Cfg), P, P, P, P]
        lib.spo_overlap.restype = None
        lib.spo_inhibit.argtypes = [ctypes.POINTER(_Cfg), P, P, P]
        lib.spo_inhibit.restype = ctypes.c_int
        lib.spo_learn.argtypes = [ctypes.POINTER(_Cfg), P, P, P, P]
        lib.spo_learn.restype = None
        lib.spo_run.argtypes = [ctypes.POINTER(_Cfg), P, P, P, ctypes.c_uint32, ctypes.c_int, P, P]
        lib.spo_run.restype = ctypes.c_int
        lib.spo_run_threads.argtypes = [ctypes.POINTER(_Cfg), P, P, P, ctypes.c_uint32,
                                        ctypes.c_int, P, P, ctypes.c_uint32]
        lib.spo_run_threads.restype = ctypes.c_int
        lib.spo_histogram.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, P]
        lib.spo_histogram.restype = ctypes.c_int
        lib.spo_run_boost.argtypes = [ctypes.POINTER(_Cfg), ctypes.POINTER(_Boost), P, P, P,
                                      ctypes.c_uint32, ctypes.c_int, P, P, P, P, P]
        lib.spo_run_boost.restype = ctypes.c_int
        lib.spo_inhibit_local.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                          ctypes.c_uint32, P]
        lib.spo_inhibit_local.restype = ctypes.c_int
        lib.spo_run_local.argtypes = [ctypes.POINTER(_Cfg), P, P, P, ctypes.c_uint32, ctypes.c_int,
                                      ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, P, P]
        lib.spo_run_local.restype = ctypes.c_int
        lib.spo_adapt_radius.argtypes = [ctypes.POINTER(_Cfg), P, P, ctypes.c_uint32,
                                         ctypes.c_uint32, ctypes.c_uint32]
        lib.spo_adapt_radius.restype = ctypes.c_uint32
        lib.spo_run_local_adaptive.argtypes = [ctypes.POINTER(_Cfg), P, P, P, ctypes.c_uint32,
                                               ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32,
                                               ctypes.c_uint32, ctypes.c_uint32, P, P, P]
        lib.spo_run_local_adaptive.restype = ctypes.c_uint32
        lib.enc_reduce.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, P]
        lib.enc_reduce.restype = None
        lib.enc_gray.argtypes = [P, ctypes.c_uint32, P]
        lib.enc_gray.restype = None
        lib.enc_threshold.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_int32, P]
        lib.enc_threshold.restype = None
        lib.enc_pack.argtypes = [P, ctypes.c_uint32, P]
        lib.enc_pack.restype = None
        lib.enc_frames.argtypes = [ctypes.POINTER(_EncCfg), P, ctypes.c_uint32, P]
        lib.enc_frames.restype = ctypes.c_int
        _lib = lib
    return _lib


def _cfg(cfg: dict) -> _Cfg:
    """cfg uses the integer 1/256-unit parameters of the library's config."""
    return _Cfg(
        int(cfg["input_bits"]), int(cfg["num_columns"]), int(cfg["synapses_per_column"]),
        int(cfg["min_overlap"]), int(cfg["winners"]),
        cfg["connected_q8"] / 256.0, cfg["inc_q8"] / 256.0, cfg["dec_q8"] / 256.0,
    )


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _words(cfg) -> int:
    return (int(cfg["input_bits"]) + 31) // 32


def overlap(cfg: dict, idx: np.ndarray, perm: np.ndarray, frame: np.ndarray) -> np.ndarray:
    """Algorithm 1 for one packed frame; returns int32[C]."""
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    perm = np.ascontiguousarray(perm, dtype=np.float64)
    frame = np.ascontiguousarray(frame, dtype=np.uint32).reshape(-1)
    assert frame.size == _words(cfg)
    out = np.zeros(int(cfg["num_columns"]), dtype=np.int32)
    c = _cfg(cfg)
    _load().spo_overlap(ctypes.byref(c), _ptr(idx), _ptr(perm), _ptr(frame), _ptr(out))
    return out


def inhibit(cfg: dict, ov: np.ndarray):
    """Algorithm 2 (global form); returns (winners int32[k] -1 padded, active uint8[C])."""
    ov = np.ascontiguousarray(ov, dtype=np.int32)
    assert ov.size == int(cfg["num_columns"])
    active = np.zeros(int(cfg["num_columns"]), dtype=np.uint8)
    win = np.zeros(int(cfg["winners"]), dtype=np.int32)
    c = _cfg(cfg)
    _load().spo_inhibit(ctypes.byref(c), _ptr(ov), _ptr(active), _ptr(win))
    return win, active


def learn(cfg: dict, idx: np.ndarray, perm: np.ndarray, frame: np.ndarray,
          active: np.ndarray) -> np.ndarray:
    """Learning on the active columns; returns the updated float64 permanences."""
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    perm = np.array(perm, dtype=np.float64, order="C", copy=True)
    frame = np.ascontiguousarray(frame, dtype=np.uint32).reshape(-1)
    active = np.ascontiguousarray(active, dtype=np.uint8)
    c = _cfg(cfg)
    _load().spo_learn(ctypes.byref(c), _ptr(idx), _ptr(perm), _ptr(frame), _ptr(active))
    return perm


def run(cfg: dict, idx: np.ndarray, perm: np.ndarray, frames: np.ndarray, learn: bool = True,
        want_overlaps: bool = True):
    """F frames in order.  perm may be float32 or float64 on the 1/256 grid.

    Returns (overlaps int32[F][C] or None, winners int32[F][k], perm float64[C][S]).
    """
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    perm = np.array(perm, dtype=np.float64, order="C", copy=True)
    frames = np.ascontiguousarray(frames, dtype=np.uint32)
    F = frames.shape[0] if frames.ndim == 2 else (0 if frames.size == 0 else 1)
    frames = frames.reshape(F, _words(cfg)) if F else frames.reshape(0, _words(cfg))
    C, k = int(cfg["num_columns"]), int(cfg["winners"])
    ov = np.zeros((F, C), dtype=np.int32) if want_overlaps else None
    win = np.zeros((F, k), dtype=np.int32)
    c = _cfg(cfg)
    rc = _load().spo_run(ctypes.byref(c), _ptr(idx), _ptr(perm), _ptr(frames), F, int(bool(learn)),
                         _ptr(ov) if ov is not None else None, _ptr(win))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return ov, win, perm


def run_threads(cfg: dict, idx: np.ndarray, perm: np.ndarray, frames: np.ndarray,
                threads: int, learn: bool = True, want_overlaps: bool = True):
    """``run`` on `threads` host threads (same results): per frame the
    overlap and the learning split by column ranges, the inhibition on one
    thread."""
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    perm = np.array(perm, dtype=np.float64, order="C", copy=True)
    frames = np.ascontiguousarray(frames, dtype=np.uint32)
    F = frames.shape[0] if frames.ndim == 2 else (0 if frames.size == 0 else 1)
    frames = frames.reshape(F, _words(cfg)) if F else frames.reshape(0, _words(cfg))
    C, k = int(cfg["num_columns"]), int(cfg["winners"])
    ov = np.zeros((F, C), dtype=np.int32) if want_overlaps else None
    win = np.zeros((F, k), dtype=np.int32)
    c = _cfg(cfg)
    rc = _load().spo_run_threads(ctypes.byref(c), _ptr(idx), _ptr(perm), _ptr(frames), F,
                                 int(bool(learn)), _ptr(ov) if ov is not None else None,
                                 _ptr(win), int(threads))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return ov, win, perm


def histogram(winners: np.ndarray, num_columns: int, hist: np.ndarray | None = None) -> np.ndarray:
    """Adds every frame's winners (int32 [F][k], -1 padded) to a per-column
    count (uint32 [C], zeros when not given) and returns it."""
    w = np.ascontiguousarray(winners, dtype=np.int32)
    F, k = (w.shape[0], w.shape[1]) if w.ndim == 2 else (0, 1)
    h = (np.zeros(num_columns, dtype=np.uint32) if hist is None
         else np.array(hist, dtype=np.uint32, copy=True))
    if _load().spo_histogram(_ptr(w), F, k, int(num_columns), _ptr(h)) != 0:
        raise ValueError("winner index out of range")
    return h


def boost_state(num_columns: int):
    """Initial boosting state: duty cycles 0, boosts 1 (256 in 1/256)."""
    C = int(num_columns)
    return (np.zeros(C, dtype=np.uint32), np.zeros(C, dtype=np.uint32),
            np.full(C, 256, dtype=np.uint32))


def run_boost(cfg: dict, bcfg: dict, idx: np.ndarray, perm: np.ndarray, frames: np.ndarray,
              learn: bool = True, state=None, want_overlaps: bool = True):
    """F frames with boosting (readings B1-B7).  bcfg: period_log2,
    min_pct_q16, max_boost_q8, bump_q8.  state: (adc, odc, boost) uint32 [C]
    or None for the initial state.  Returns (boosted overlaps int32 [F][C] or
    None, winners int32 [F][k], perm float64, (adc, odc, boost))."""
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    perm = np.array(perm, dtype=np.float64, order="C", copy=True)
    frames = np.ascontiguousarray(frames, dtype=np.uint32)
    F = frames.shape[0] if frames.ndim == 2 else (0 if frames.size == 0 else 1)
    frames = frames.reshape(F, _words(cfg))
    C, k = int(cfg["num_columns"]), int(cfg["winners"])
    adc, odc, boost = (boost_state(C) if state is None
                       else tuple(np.array(a, dtype=np.uint32, copy=True) for a in state))
    ov = np.zeros((F, C), dtype=np.int32) if want_overlaps else None
    win = np.zeros((F, k), dtype=np.int32)
    b = _Boost(int(bcfg["period_log2"]), int(bcfg["min_pct_q16"]), int(bcfg["max_boost_q8"]),
               int(bcfg["bump_q8"]))
    c = _cfg(cfg)
    rc = _load().spo_run_boost(ctypes.byref(c), ctypes.byref(b), _ptr(idx), _ptr(perm),
                               _ptr(frames), F, int(bool(learn)), _ptr(adc), _ptr(odc),
                               _ptr(boost), _ptr(ov) if ov is not None else None, _ptr(win))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return ov, win, perm, (adc, odc, boost)


def inhibit_local(overlap: np.ndarray, grid_w: int, radius: int, n: int) -> np.ndarray:
    """Algorithm 2 with a neighbourhood (readings L1-L4): uint8 [C] active."""
    ov = np.ascontiguousarray(overlap, dtype=np.int32).reshape(-1)
    act = np.zeros(ov.size, dtype=np.uint8)
    if _load().spo_inhibit_local(_ptr(ov), ov.size, int(grid_w), int(radius), int(n),
                                 _ptr(act)) < 0:
        raise ValueError("bad local inhibition arguments")
    return act


def run_local(cfg: dict, idx: np.ndarray, perm: np.ndarray, frames: np.ndarray, grid_w: int,
              radius: int, n: int, learn: bool = True, want_overlaps: bool = True):
    """F frames with local inhibition.  Returns (overlaps int32 [F][C] or
    None, active uint8 [F][C], perm float64 [C][S])."""
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    perm = np.array(perm, dtype=np.float64, order="C", copy=True)
    frames = np.ascontiguousarray(frames, dtype=np.uint32)
    F = frames.shape[0] if frames.ndim == 2 else (0 if frames.size == 0 else 1)
    frames = frames.reshape(F, _words(cfg))
    C = int(cfg["num_columns"])
    ov = np.zeros((F, C), dtype=np.int32) if want_overlaps else None
    act = np.zeros((F, C), dtype=np.uint8)
    c = _cfg(cfg)
    rc = _load().spo_run_local(ctypes.byref(c), _ptr(idx), _ptr(perm), _ptr(frames), F,
                               int(bool(learn)), int(grid_w), int(radius), int(n),
                               _ptr(ov) if ov is not None else None, _ptr(act))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return ov, act, perm


# ---- adaptive video encoder (Section 3.1.2), readings E1-E6 in enc_oracle.h

def adapt_radius(cfg: dict, idx: np.ndarray, perm: np.ndarray, in_w: int, grid_w: int,
                 radius: int) -> int:
    """The radius after a learning frame from the state it left (reading L5)."""
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    perm = np.ascontiguousarray(perm, dtype=np.float64)
    c = _cfg(cfg)
    return int(_load().spo_adapt_radius(ctypes.byref(c), _ptr(idx), _ptr(perm), int(in_w),
                                        int(grid_w), int(radius)))


def run_local_adaptive(cfg: dict, idx: np.ndarray, perm: np.ndarray, frames: np.ndarray,
                       in_w: int, grid_w: int, radius: int, n: int, learn: bool = True):
    """Local inhibition with the radius adapted after every learning frame.
    Returns (overlaps int32 [F][C], active uint8 [F][C], perm float64,
    radii uint32 [F] (each frame's radius), final radius)."""
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    perm = np.array(perm, dtype=np.float64, order="C", copy=True)
    frames = np.ascontiguousarray(frames, dtype=np.uint32)
    F = frames.shape[0]
    C = int(cfg["num_columns"])
    ov = np.zeros((F, C), dtype=np.int32)
    act = np.zeros((F, C), dtype=np.uint8)
    radii = np.zeros(F, dtype=np.uint32)
    c = _cfg(cfg)
    r = _load().spo_run_local_adaptive(ctypes.byref(c), _ptr(idx), _ptr(perm), _ptr(frames), F,
                                       int(bool(learn)), int(in_w), int(grid_w), int(radius),
                                       int(n), _ptr(ov), _ptr(act), _ptr(radii))
    if r == 0:
        raise ValueError("oracle rejected its arguments")
    return ov, act, perm, radii, int(r)


def enc_reduce(rgb: np.ndarray, factor: int) -> np.ndarray:
    """uint8 [H][W][3] -> uint8 [H/f][W/f][3], block means rounded half up."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    H, W = rgb.shape[:2]
    out = np.zeros((H // factor, W // factor, 3), dtype=np.uint8)
    _load().enc_reduce(_ptr(rgb), W, H, int(factor), _ptr(out))
    return out


def enc_gray(rgb: np.ndarray) -> np.ndarray:
    """uint8 [..., 3] -> uint8 [...] BT.601 luma in 14-bit fixed point."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    out = np.zeros(rgb.shape[:-1], dtype=np.uint8)
    _load().enc_gray(_ptr(rgb), int(out.size), _ptr(out))
    return out


def enc_threshold(gray: np.ndarray, block: int, offset: int) -> np.ndarray:
    """uint8 [h][w] -> uint8 0/1 [h][w]: Y > binomial-window mean - offset."""
    gray = np.ascontiguousarray(gray, dtype=np.uint8)
    h, w = gray.shape
    on = np.zeros((h, w), dtype=np.uint8)
    _load().enc_threshold(_ptr(gray), w, h, int(block), int(offset), _ptr(on))
    return on


def enc_pack(on: np.ndarray) -> np.ndarray:
    on = np.ascontiguousarray(on, dtype=np.uint8).reshape(-1)
    words = np.zeros((on.size + 31) // 32, dtype=np.uint32)
    _load().enc_pack(_ptr(on), int(on.size), _ptr(words))
    return words


def enc_frames(rgb: np.ndarray, factor: int = 1, block: int = 11, offset: int = 2) -> np.ndarray:
    """uint8 [F][H][W][3] -> uint32 [F][ceil(w h / 32)] packed binary frames."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    F, H, W = rgb.shape[:3]
    n = (W // factor) * (H // factor)
    words = np.zeros((F, (n + 31) // 32), dtype=np.uint32)
    c = _EncCfg(W, H, int(factor), int(block), int(offset))
    if _load().enc_frames(ctypes.byref(c), _ptr(rgb), F, _ptr(words)) != 0:
        raise ValueError("encoder oracle rejected its configuration")
    return words
