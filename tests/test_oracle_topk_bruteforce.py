"""Pin: the oracle's global inhibition against brute force over subsets on
tiny column counts (Section 1.1, Algorithm 2, global form).

Characterisation: among subsets of E = {c : overlap > 0} of size
min(k, |E|), the winners maximise the overlap sum, and among those take the
lexicographically smallest ascending index tuple.  This picks exactly the
highest overlaps with ties to the lower index."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1608_01966_amd import synth


def brute(ov, k):
    E = [c for c in range(len(ov)) if ov[c] > 0]
    n = min(k, len(E))
    best = None
    for sub in itertools.combinations(E, n):
        key = (-sum(ov[c] for c in sub), sub)
        if best is None or key < best:
            best = key
    return list(best[1]) if best else []


@pytest.mark.parametrize("seed", range(300))
def test_inhibit_matches_bruteforce(seed):
    g = np.random.default_rng(seed)
    C = int(g.integers(1, 11))
    k = int(g.integers(1, C + 1))
    hi = int(g.integers(1, 6))
    ov = g.integers(0, hi + 1, size=C).astype(np.int32)
    cfg = synth.sp_config(32, C, 1, 0, k)
    win, active = oracle.inhibit(cfg, ov)
    expect = brute(ov.tolist(), k)
    assert win.tolist() == expect + [-1] * (k - len(expect))
    assert np.flatnonzero(active).tolist() == expect


def test_all_tied():
    cfg = synth.sp_config(32, 10, 1, 0, 4)
    win, _ = oracle.inhibit(cfg, np.full(10, 3, dtype=np.int32))
    assert win.tolist() == [0, 1, 2, 3]


def test_fewer_positive_than_k():
    cfg = synth.sp_config(32, 6, 1, 0, 5)
    win, _ = oracle.inhibit(cfg, np.array([0, 4, 0, 0, 1, 0], dtype=np.int32))
    assert win.tolist() == [1, 4, -1, -1, -1]


def test_k_equals_c():
    cfg = synth.sp_config(32, 5, 1, 0, 5)
    win, _ = oracle.inhibit(cfg, np.array([1, 2, 3, 4, 5], dtype=np.int32))
    assert win.tolist() == [0, 1, 2, 3, 4]
