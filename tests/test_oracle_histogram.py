"""Pins for the oracle's per-stream SDR histogram (Section 2: every frame's
pooler output is accumulated into a per-video histogram, the video's
feature vector)."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1608_01966_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "handworked_8col.json")


def test_handworked_histogram():
    with open(GOLD) as f:
        g = json.load(f)
    win = np.array(g["winners"], dtype=np.int32)
    assert oracle.histogram(win, g["config"]["num_columns"]).tolist() == g["histogram"]


def test_counts_by_set_membership():
    """hist[c] = number of frames whose winner set contains c, computed by
    membership over sets rather than by adding entries."""
    rng = np.random.default_rng(7)
    F, k, C = 50, 6, 40
    win = np.full((F, k), -1, dtype=np.int32)
    for t in range(F):
        n = int(rng.integers(0, k + 1))
        win[t, :n] = np.sort(rng.choice(C, size=n, replace=False))
    sets = [set(int(x) for x in row if x >= 0) for row in win]
    want = [sum(c in s for s in sets) for c in range(C)]
    assert oracle.histogram(win, C).tolist() == want


def test_accumulates_and_totals():
    w = synth.workload_plain_32x32(frames=30)
    _, win, _ = oracle.run(w.cfg, w.idx, w.perm, w.frames, learn=True, want_overlaps=False)
    h1 = oracle.histogram(win[:10], 256)
    h2 = oracle.histogram(win[10:], 256, h1)
    assert np.array_equal(h2, oracle.histogram(win, 256))
    # every frame adds exactly its number of winners; no column exceeds F
    assert int(h2.sum()) == int((win >= 0).sum())
    assert h2.max() <= 30


def test_rejects_out_of_range():
    with pytest.raises(ValueError):
        oracle.histogram(np.array([[0, 9]], dtype=np.int32), 8)
