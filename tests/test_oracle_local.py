"""Pins for the oracle's local inhibition (Algorithm 2 with a neighbourhood,
readings L1-L4) and the local-inhibition run."""
import json
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1608_01966_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "local_inhibition.json")


def test_handworked():
    with open(GOLD) as f:
        g = json.load(f)
    for case in g["cases"]:
        got = oracle.inhibit_local(np.array(case["overlap"]), case["grid_w"], case["radius"],
                                   case["n"])
        assert got.tolist() == case["active"], case["why"]


def _count_form(ov, grid_w, radius, n):
    """active iff overlap >= 2 and fewer than n neighbours have an overlap
    at least as large (equivalent to Algorithm 2's comparison with the n-th
    largest neighbour, floored at 1)."""
    C = ov.size
    out = np.zeros(C, dtype=np.uint8)
    for c in range(C):
        cx, cy = c % grid_w, c // grid_w
        k = 0
        for d in range(C):
            if d != c and abs(d % grid_w - cx) <= radius and abs(d // grid_w - cy) <= radius:
                k += ov[d] >= ov[c]
        out[c] = ov[c] >= 2 and k < n
    return out


@pytest.mark.parametrize("seed", range(6))
def test_count_form_brute_force(seed):
    g = np.random.default_rng(seed)
    for _ in range(25):
        C = int(g.integers(1, 60))
        grid_w = int(g.integers(1, C + 1))
        ov = g.integers(0, 8, size=C).astype(np.int32)
        radius = int(g.integers(0, 6))
        n = int(g.integers(1, 6))
        assert np.array_equal(oracle.inhibit_local(ov, grid_w, radius, n),
                              _count_form(ov, grid_w, radius, n))


def test_global_limit_is_top_n():
    """A radius that covers the grid and distinct overlaps >= 2: the active
    set is the global top-n (the oracle's global inhibition)."""
    g = np.random.default_rng(3)
    for _ in range(20):
        C = int(g.integers(5, 200))
        ov = (g.permutation(C) + 2).astype(np.int32)
        n = int(g.integers(1, C))
        cfg = {"num_columns": C, "winners": n}
        win, _ = oracle.inhibit(dict(synth.sp_config(10, C, 1, 0, n)), ov)
        act = oracle.inhibit_local(ov, int(g.integers(1, C + 1)), C, n)
        assert np.flatnonzero(act).tolist() == win[win >= 0].tolist(), cfg


def test_radius_zero_and_isolated_columns():
    """No neighbours: n_max_overlap is 0, so every overlap >= 2 is active."""
    ov = np.array([0, 1, 2, 9, 3], dtype=np.int32)
    assert oracle.inhibit_local(ov, 5, 0, 1).tolist() == [0, 0, 1, 1, 1]


def test_run_local_composes_the_steps():
    w = synth.workload_plain_32x32(frames=12)
    ov, act, perm = oracle.run_local(w.cfg, w.idx, w.perm, w.frames, 16, 2, 3)
    p = w.perm.astype(np.float64)
    for t in range(12):
        o = oracle.overlap(w.cfg, w.idx, p, w.frames[t])
        a = oracle.inhibit_local(o, 16, 2, 3)
        assert np.array_equal(o, ov[t]) and np.array_equal(a, act[t])
        p = oracle.learn(w.cfg, w.idx, p, w.frames[t], a)
    assert np.array_equal(p, perm)
    _, act2, perm2 = oracle.run_local(w.cfg, w.idx, w.perm, w.frames, 16, 2, 3, learn=False)
    assert np.array_equal(perm2, w.perm.astype(np.float64))
    assert np.array_equal(act2[0], act[0])


MUTANTS = {
    "non_strict": ("active[c] = overlap[c] > max_column ? 1 : 0;",
                   "active[c] = overlap[c] >= max_column ? 1 : 0;"),
    "self_in_neighbourhood": ("      if (d == c) continue;\n", ""),
    "no_floor": ("const int32_t max_column = nth > 1 ? nth : 1;",
                 "const int32_t max_column = nth;"),
    "rows_ignored": ("dy <= (int64_t)radius &&\n          -dy <= (int64_t)radius",
                     "1 &&\n          1"),
    "nth_off_by_one": ("nb[n - 1] : 0;", "nb[n < m ? n : m - 1] : 0;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(name, tmp_path, monkeypatch):
    here = os.path.dirname(oracle.__file__)
    src = open(os.path.join(here, "sp_oracle.c")).read()
    before, after = MUTANTS[name]
    assert before in src, name
    c = tmp_path / "mut.c"
    c.write_text(src.replace(before, after, 1))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-I", here, str(c),
                           os.path.join(here, "sp_oracle_mt.c"),
                           os.path.join(here, "enc_oracle.c"), "-pthread", "-o", str(so)])
    monkeypatch.setattr(oracle, "_LIB_PATH", str(so))
    monkeypatch.setattr(oracle, "_lib", None)
    caught = 0
    for pin in (test_handworked, lambda: test_count_form_brute_force(0),
                test_global_limit_is_top_n, test_radius_zero_and_isolated_columns):
        try:
            pin()
        except AssertionError:
            caught += 1
    oracle._lib = None
    assert caught > 0, f"mutant {name} survived"
