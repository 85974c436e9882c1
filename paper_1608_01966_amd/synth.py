"""Seeded synthetic inputs for the spatial pooler: frames, potential pools and
initial permanences.

This module holds none of the spatial pooler's arithmetic (no overlap, no
inhibition, no learning); it only draws random inputs and packs bits, so that
both the GPU library's tests and the oracle's tests can be fed the same data.

The paper's video dataset (rendered "shapes" clips binarised by an adaptive
threshold, Section 4.2 and Section 3.1.2) is not available, so seeded frames
stand in for it: Bernoulli pixels, or random 8x8 blobs that mimic the
clustered foreground an adaptive threshold leaves.

Bit layout: pixel p = y * width + x of a frame is bit (p & 31) of 32-bit word
(p >> 5), least significant bit first; bits past the frame's last pixel are 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

GRID = 256  # permanences live on the 1/256 grid


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    """Independent generator ``stream`` of ``seed``."""
    return np.random.default_rng(np.random.SeedSequence(seed).spawn(stream + 1)[stream])


def words_per_frame(input_bits: int) -> int:
    return (int(input_bits) + 31) // 32


def pack_bits(bits: np.ndarray) -> np.ndarray:
    """bool[..., N] -> uint32[..., ceil(N/32)], LSB-first."""
    bits = np.asarray(bits, dtype=bool)
    n = bits.shape[-1]
    w = words_per_frame(n)
    pad = w * 32 - n
    if pad:
        bits = np.concatenate([bits, np.zeros(bits.shape[:-1] + (pad,), dtype=bool)], axis=-1)
    by = np.packbits(bits, axis=-1, bitorder="little")
    return np.ascontiguousarray(by).view("<u4").astype(np.uint32, copy=False)


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    """uint32[..., W] -> bool[..., n]."""
    words = np.ascontiguousarray(words, dtype="<u4")
    by = words.view(np.uint8)
    return np.unpackbits(by, axis=-1, bitorder="little")[..., :n].astype(bool)


def pools(g: np.random.Generator, input_bits: int, columns: int, synapses: int) -> np.ndarray:
    """Potential pools: per column, ``synapses`` distinct inputs drawn uniformly
    without replacement, sorted ascending.  uint32[C][S]."""
    out = np.empty((columns, synapses), dtype=np.uint32)
    for c in range(columns):
        out[c] = np.sort(g.choice(input_bits, size=synapses, replace=False))
    return out


def permanences_q(g: np.random.Generator, columns: int, synapses: int) -> np.ndarray:
    """Initial permanences in 1/256 units, uniform over {0, ..., 256}.  uint16[C][S]."""
    return g.integers(0, GRID + 1, size=(columns, synapses), dtype=np.uint16)


def q_to_float(q: np.ndarray) -> np.ndarray:
    return (np.asarray(q, dtype=np.float32) / np.float32(GRID)).astype(np.float32)


def bernoulli_frames(g: np.random.Generator, frames: int, input_bits: int, p: float) -> np.ndarray:
    """uint32[F][W]: every pixel on with probability p, independently.  The
    on-pixels are drawn as a Bernoulli process: gaps between successive
    on-pixels are geometric(p), which is the same distribution as drawing
    every pixel and far cheaper for sparse frames."""
    n = int(input_bits)
    out = np.zeros((frames, words_per_frame(n)), dtype=np.uint32)
    if p <= 0.0:
        return out
    if p >= 1.0:
        out[:] = pack_bits(np.ones(n, dtype=bool))
        return out
    chunk = int(n * p * 1.05) + 64
    W = words_per_frame(n)
    for t in range(frames):
        pos = np.cumsum(g.geometric(p, size=chunk)) - 1
        while pos[-1] < n:
            pos = np.concatenate([pos, pos[-1] + np.cumsum(g.geometric(p, size=chunk))])
        pos = pos[pos < n]
        # distinct positions: summing their bit values is OR-ing them
        out[t] = np.bincount(pos >> 5, weights=np.left_shift(1, pos & 31).astype(np.float64),
                             minlength=W).astype(np.uint32)
    return out


def blob_frames(g: np.random.Generator, frames: int, width: int, height: int,
                density: float = 0.05, blob: int = 8) -> np.ndarray:
    """uint32[F][W]: blob x blob squares at uniform top-left corners, added
    until at least ``density`` of the width x height pixels are on."""
    n = width * height
    target = int(np.ceil(density * n))
    out = np.empty((frames, words_per_frame(n)), dtype=np.uint32)
    for t in range(frames):
        img = np.zeros((height, width), dtype=bool)
        on = 0
        while on < target:
            ys = g.integers(0, height - blob + 1, size=32)
            xs = g.integers(0, width - blob + 1, size=32)
            for y, x in zip(ys, xs):
                img[y:y + blob, x:x + blob] = True
            on = int(img.sum())
        out[t] = pack_bits(img.reshape(-1))
    return out


def rgb_frames(g: np.random.Generator, frames: int, width: int, height: int,
               shapes: int = 12) -> np.ndarray:
    """uint8 [F][H][W][3] colour frames standing in for rendered video:
    a smooth illumination gradient whose direction varies per frame, solid
    rectangles and discs of random colour, and uniform noise of +-8 levels."""
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float32)
    out = np.empty((frames, height, width, 3), dtype=np.uint8)
    for t in range(frames):
        ang = g.uniform(0, 2 * np.pi)
        base = g.uniform(40, 120, size=3).astype(np.float32)
        ramp = (np.cos(ang) * xx / max(width, 1) + np.sin(ang) * yy / max(height, 1)) * 90.0
        img = base[None, None, :] + ramp[:, :, None]
        for _ in range(shapes):
            col = g.uniform(0, 255, size=3).astype(np.float32)
            cx, cy = g.uniform(0, width), g.uniform(0, height)
            rx = g.uniform(0.02, 0.15) * width
            ry = g.uniform(0.02, 0.15) * height
            if g.random() < 0.5:
                m = (np.abs(xx - cx) < rx) & (np.abs(yy - cy) < ry)
            else:
                m = ((xx - cx) / rx) ** 2 + ((yy - cy) / ry) ** 2 < 1.0
            img[m] = col
        img += g.uniform(-8, 8, size=img.shape).astype(np.float32)
        out[t] = np.clip(img + 0.5, 0, 255).astype(np.uint8)
    return out


@dataclass
class Workload:
    """One spatial pooler instance plus its input frames."""
    name: str
    cfg: dict
    idx: np.ndarray                 # uint32[C][S]
    perm_q: np.ndarray              # uint16[C][S] (1/256 units)
    frames: np.ndarray              # uint32[F][W]
    learn: bool = True
    meta: dict = field(default_factory=dict)

    @property
    def perm(self) -> np.ndarray:
        return q_to_float(self.perm_q)


def sp_config(input_bits, columns, synapses, min_overlap, winners,
              connected_q8=128, inc_q8=8, dec_q8=4) -> dict:
    return dict(input_bits=int(input_bits), num_columns=int(columns),
                synapses_per_column=int(synapses), min_overlap=int(min_overlap),
                winners=int(winners), connected_q8=int(connected_q8),
                inc_q8=int(inc_q8), dec_q8=int(dec_q8))


def random_instance(seed: int, cfg: dict, frames: int, density: float = 0.1,
                    shape: tuple | None = None, blobs: bool = False) -> Workload:
    """Pools, permanences and frames for ``cfg`` from ``seed`` (three
    independent generator streams)."""
    n, C, S = cfg["input_bits"], cfg["num_columns"], cfg["synapses_per_column"]
    idx = pools(rng(seed, 0), n, C, S)
    q = permanences_q(rng(seed, 1), C, S)
    if blobs:
        w, h = shape
        fr = blob_frames(rng(seed, 2), frames, w, h, density)
    else:
        fr = bernoulli_frames(rng(seed, 2), frames, n, density)
    return Workload(name=f"random_{seed}", cfg=cfg, idx=idx, perm_q=q, frames=fr)


def workload_plain_32x32(frames: int = 100) -> Workload:
    """32x32 input, Bernoulli(0.10) pixels; 256 columns x 64 synapses;
    min_overlap 4, 20 winners, threshold 0.5, inc 8/256, dec 4/256; learning on."""
    cfg = sp_config(32 * 32, 256, 64, 4, 20)
    w = random_instance(1, cfg, frames, density=0.10)
    w.name = "plain_32x32_256c_64s"
    return w


def workload_paper_scale(frames: int = 1000, columns: int = 1024, synapses: int = 256,
                         seed: int = 2) -> Workload:
    """960x540 input, ~5% on as random 8x8 blobs; 1024 columns x 256 synapses
    (sweepable); min_overlap 4, 40 winners, threshold 0.5, inc 8/256,
    dec 4/256; learning on."""
    cfg = sp_config(960 * 540, columns, synapses, 4, 40)
    w = random_instance(seed, cfg, frames, density=0.05, shape=(960, 540), blobs=True)
    w.name = f"paper_960x540_{columns}c_{synapses}s"
    return w


def workload_batched_inference(frames: int = 4096, seed: int = 3) -> Workload:
    """960x540 Bernoulli(0.05) frames through a frozen spatial pooler of 1024
    columns x 256 synapses (min_overlap 4, 40 winners, threshold 0.5);
    learning off."""
    cfg = sp_config(960 * 540, 1024, 256, 4, 40)
    w = random_instance(seed, cfg, frames, density=0.05)
    w.learn = False
    w.name = "infer_960x540_1024c_256s"
    return w


INPUT_SHAPES = [(64, 64), (128, 128), (240, 134), (480, 270), (960, 540)]


def workload_multi(instances: int = 64, frames: int = 500, seed: int = 4) -> list:
    """Independent spatial poolers of uneven size: columns from
    {256, ..., 4096}, synapses from {32, ..., 512}, inputs from 64x64 to
    960x540 at a density drawn uniformly in [0.02, 0.10] (Bernoulli pixels);
    min_overlap 4, 10 winners per 256 columns; learning on."""
    g = rng(seed, 0)
    out = []
    for i in range(instances):
        C = int(g.choice([256, 512, 1024, 2048, 4096]))
        S = int(g.choice([32, 64, 128, 256, 512]))
        wd, ht = INPUT_SHAPES[int(g.integers(0, len(INPUT_SHAPES)))]
        d = float(g.uniform(0.02, 0.10))
        cfg = sp_config(wd * ht, C, S, 4, 10 * C // 256)
        w = random_instance(seed * 1000 + i, cfg, frames, density=d)
        w.name = f"multi_{i}_{wd}x{ht}_{C}c_{S}s"
        w.meta = {"shape": (wd, ht), "density": d}
        out.append(w)
    return out
