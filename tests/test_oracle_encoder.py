"""Pins for the adaptive video encoder oracle (Section 3.1.2; readings E1-E6
in oracle/enc_oracle.h): a hand-worked example, closed forms, a library
correlation, brute-force reduction and planted mistakes."""
import json
import os
import subprocess

import numpy as np
import pytest
import scipy.ndimage

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "encoder_5x4.json")


def _binomial(b):
    w = [1]
    for _ in range(b - 1):
        w = [x + y for x, y in zip([0] + w, w + [0])]
    return np.array(w, dtype=np.int64)


def test_handworked_threshold():
    with open(GOLD) as f:
        g = json.load(f)
    gray = np.array(g["gray"], dtype=np.uint8)
    on = oracle.enc_threshold(gray, g["block"], g["offset"])
    assert on.tolist() == g["on"]
    assert oracle.enc_pack(on).tolist() == g["words"]


def test_window_sum_is_a_library_correlation():
    """The window sum equals scipy's correlation with the outer product of
    Pascal's-triangle weights and edge-repeating borders ('nearest'); the
    threshold decisions follow from it."""
    rng = np.random.default_rng(3)
    for b in (3, 5, 7, 9, 11):
        gray = rng.integers(0, 256, size=(23, 37), dtype=np.uint8)
        k = np.outer(_binomial(b), _binomial(b))
        s = scipy.ndimage.correlate(gray.astype(np.int64), k, mode="nearest")
        shift = 2 * (b - 1)
        mean = (s + (1 << (shift - 1))) >> shift
        for off in (-3, 0, 2, 7):
            want = (gray.astype(np.int64) > mean - off).astype(np.uint8)
            assert np.array_equal(oracle.enc_threshold(gray, b, off), want), (b, off)


def test_flat_image():
    """A constant image equals its own mean: all on iff offset > 0."""
    for v in (0, 1, 128, 255):
        gray = np.full((9, 14), v, dtype=np.uint8)
        assert oracle.enc_threshold(gray, 7, 1).min() == 1
        assert oracle.enc_threshold(gray, 7, 0).max() == 0
        assert oracle.enc_threshold(gray, 7, -5).max() == 0


def test_gray_closed_forms():
    """BT.601 luma: pure channels give round-down of 0.299, 0.587, 0.114
    times the level (with the 8192 rounding term), white stays 255, gray
    levels are kept."""
    px = np.array([[255, 0, 0], [0, 255, 0], [0, 0, 255], [255, 255, 255], [0, 0, 0],
                   [77, 77, 77], [200, 100, 50]], dtype=np.uint8)
    got = oracle.enc_gray(px).tolist()
    assert got[:6] == [76, 150, 29, 255, 0, 77]
    assert got[6] == int(0.299 * 200 + 0.587 * 100 + 0.114 * 50 + 0.5)  # 124


def test_reduce_brute_force():
    rng = np.random.default_rng(5)
    rgb = rng.integers(0, 256, size=(13, 22, 3), dtype=np.uint8)
    assert np.array_equal(oracle.enc_reduce(rgb, 1), rgb)
    for f in (2, 3, 4):
        got = oracle.enc_reduce(rgb, f)
        h, w = 13 // f, 22 // f
        assert got.shape == (h, w, 3)
        for y in range(h):
            for x in range(w):
                blk = rgb[y * f:(y + 1) * f, x * f:(x + 1) * f].astype(np.int64)
                want = (blk.sum(axis=(0, 1)) + (f * f) // 2) // (f * f)
                assert got[y, x].tolist() == want.tolist()


def test_pack_layout():
    on = np.zeros(70, dtype=np.uint8)
    on[[0, 31, 32, 69]] = 1
    assert oracle.enc_pack(on).tolist() == [1 | (1 << 31), 1, 1 << 5]


def test_pipeline_composes_the_steps():
    rng = np.random.default_rng(9)
    rgb = rng.integers(0, 256, size=(3, 41, 66, 3), dtype=np.uint8)
    words = oracle.enc_frames(rgb, factor=2, block=5, offset=3)
    for f in range(3):
        on = oracle.enc_threshold(oracle.enc_gray(oracle.enc_reduce(rgb[f], 2)), 5, 3)
        assert words[f].tolist() == oracle.enc_pack(on).tolist()
    with pytest.raises(ValueError):
        oracle.enc_frames(rgb, block=4)
    with pytest.raises(ValueError):
        oracle.enc_frames(rgb, block=13)


MUTANTS = [
    ("x] > mean - offset", "x] >= mean - offset", "threshold comparison made non-strict"),
    ("clampi((int64_t)x + (int64_t)j - r, w)", "clampi((int64_t)x + (int64_t)j - r + 1, w)",
     "window shifted by one column"),
    ("clampi((int64_t)y + (int64_t)i - r, h)", "clampi((int64_t)y + (int64_t)i - r, w)",
     "rows clamped to the width"),
    ("if (v >= (int64_t)n) return n - 1;", "if (v >= (int64_t)n) return 0;",
     "bottom/right border wraps to the first pixel"),
    ("(sum + (1ull << (shift - 1))) >> shift", "sum >> shift", "mean truncated"),
    ("4899u * r + 9617u * g + 1868u * b", "4899u * b + 9617u * g + 1868u * r",
     "red and blue swapped"),
    ("(sum + area / 2) / area", "sum / area", "block mean truncated"),
    ("wt[i] = wt[i - 1] * (block - i) / i", "wt[i] = 1", "box window instead of Gaussian"),
]


@pytest.mark.parametrize("old,new,what", MUTANTS, ids=[m[2] for m in MUTANTS])
def test_planted_mistakes_are_caught(tmp_path, old, new, what):
    """Each single mistake planted in the oracle's C source makes one of the
    pins above fail (checked here with the same pin functions on a copy)."""
    import ctypes
    here = os.path.dirname(oracle.__file__)
    src = open(os.path.join(here, "enc_oracle.c")).read()
    assert old in src
    (tmp_path / "enc_oracle.h").write_text(open(os.path.join(here, "enc_oracle.h")).read())
    (tmp_path / "enc_oracle.c").write_text(src.replace(old, new, 1))
    so = tmp_path / "libenc_mut.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared",
                           str(tmp_path / "enc_oracle.c"), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    saved = oracle._lib
    try:
        # route the wrappers' calls to the mutant for the encoder entry points
        class Mixed:
            def __getattr__(self, name):
                return getattr(lib if name.startswith("enc_") else saved, name)
        P = ctypes.c_void_p
        lib.enc_threshold.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_int32, P]
        lib.enc_gray.argtypes = [P, ctypes.c_uint32, P]
        lib.enc_reduce.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, P]
        lib.enc_pack.argtypes = [P, ctypes.c_uint32, P]
        lib.enc_frames.argtypes = [ctypes.POINTER(oracle._EncCfg), P, ctypes.c_uint32, P]
        oracle._lib = Mixed()
        failed = 0
        for pin in (test_handworked_threshold, test_window_sum_is_a_library_correlation,
                    test_flat_image, test_gray_closed_forms, test_reduce_brute_force):
            try:
                pin()
            except AssertionError:
                failed += 1
        assert failed > 0, f"no pin caught: {what}"
    finally:
        oracle._lib = saved
