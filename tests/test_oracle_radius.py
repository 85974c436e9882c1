"""Pins of the inhibition-radius adaptation in the oracle (reading L5): a
hand-worked example, a closed form, an independent rational-arithmetic
computation of the same definition on random instances, the sequence of
frames against a loop over the oracle's single-frame functions, and planted
mistakes."""
import json
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1608_01966_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "radius_adapt.json")


def golden_state():
    g = json.load(open(GOLD))
    idx, q = [], []
    for key in ("full", "single", "none"):
        col = g["columns"][key]
        idx += [col["idx"]] * col["count"]
        q += [col["perm_q"]] * col["count"]
    return g, np.array(idx, dtype=np.uint32), np.array(q, dtype=np.float64) / 256.0


def test_handworked():
    g, idx, perm = golden_state()
    assert oracle.adapt_radius(g["config"], idx, perm, g["in_w"], g["grid_w"], 80) == \
        g["radius_after"]
    # nothing connected: the radius stays
    assert oracle.adapt_radius(g["config"], idx, np.zeros_like(perm), g["in_w"], g["grid_w"],
                               80) == 80


def radius_by_definition(cfg, idx, perm, in_w, grid_w, radius):
    """The definition step by step in exact rationals: each connected
    column's extent, their mean, the grid-per-input ratio, the diameter, and
    (d - 1) / 2 rounded half up, at least 1."""
    N, C = cfg["input_bits"], cfg["num_columns"]
    in_h = -(-N // in_w)
    grid_h = -(-C // grid_w)
    conn = perm * 256 >= cfg["connected_q8"]
    spans = []
    for c in range(C):
        px = idx[c][conn[c]].astype(np.int64)
        if px.size == 0:
            continue
        xs, ys = px % in_w, px // in_w
        spans.append(Fraction(int(xs.max() - xs.min() + 1) + int(ys.max() - ys.min() + 1), 2))
    if not spans:
        return radius
    extent = sum(spans) / len(spans)
    ratio = (Fraction(grid_w, in_w) + Fraction(grid_h, in_h)) / 2
    d = extent * ratio
    r = (d - 1) / 2 + Fraction(1, 2)
    return max(1, r.numerator // r.denominator)


@pytest.mark.parametrize("g", [2, 3, 8, 33])
@pytest.mark.parametrize("L", [4, 17, 64])
def test_closed_form_whole_input(g, L):
    """Every column connected to the two far corners of a square L x L input,
    g x g columns: the diameter is the grid's side, the radius floor(g / 2)."""
    C = g * g
    cfg = synth.sp_config(L * L, C, 3, 1, 1)
    rng = np.random.default_rng(g * 100 + L)
    idx = np.stack([np.zeros(C, int), np.full(C, L * L - 1), rng.integers(0, L * L, C)], 1)
    perm = np.ones((C, 3))
    assert oracle.adapt_radius(cfg, idx, perm, L, g, 5) == max(1, g // 2)


@pytest.mark.parametrize("seed", range(60))
def test_random_instances_match_definition(seed):
    rng = np.random.default_rng(seed)
    in_w = int(rng.integers(1, 50))
    N = int(in_w * rng.integers(1, 40) - rng.integers(0, in_w))  # ragged last input row
    C = int(rng.integers(1, 300))
    S = int(rng.integers(1, min(N, 40) + 1))
    grid_w = int(rng.integers(1, C + 1))
    cfg = synth.sp_config(N, C, S, 1, 1, connected_q8=int(rng.integers(0, 257)))
    w = synth.random_instance(seed, cfg, frames=1)
    r0 = int(rng.integers(1, 100))
    got = oracle.adapt_radius(cfg, w.idx, w.perm, in_w, grid_w, r0)
    assert got == radius_by_definition(cfg, w.idx, w.perm, in_w, grid_w, r0)


@pytest.mark.parametrize("learn", [True, False])
def test_sequence_equals_single_frame_functions(learn):
    """Frame t uses the radius frame t - 1 left; learning off keeps it."""
    cfg = synth.sp_config(48 * 30, 300, 40, 2, 4)
    w = synth.random_instance(5, cfg, frames=12, density=0.15)
    in_w, grid_w, r0 = 48, 20, 6
    ov, act, perm, radii, r_end = oracle.run_local_adaptive(cfg, w.idx, w.perm, w.frames, in_w,
                                                            grid_w, r0, 4, learn=learn)
    p = w.perm.astype(np.float64)
    r = r0
    for t in range(w.frames.shape[0]):
        assert radii[t] == r
        o = oracle.overlap(cfg, w.idx, p, w.frames[t])
        a = oracle.inhibit_local(o, grid_w, r, 4)
        assert np.array_equal(o, ov[t]) and np.array_equal(a, act[t])
        if learn:
            p = oracle.learn(cfg, w.idx, p, w.frames[t], a)
            r = radius_by_definition(cfg, w.idx, p, in_w, grid_w, r)
    assert np.array_equal(p, perm) and r == r_end
    if learn:
        assert len(set(radii.tolist())) > 1, "the radius should move on this workload"
    else:
        assert set(radii.tolist()) == {r0}


MUTANTS = {
    "span_without_plus_one": ("A += (uint64_t)(x1 - x0 + 1) + (uint64_t)(y1 - y0 + 1);",
                              "A += (uint64_t)(x1 - x0) + (uint64_t)(y1 - y0 + 1);"),
    # (swapping x and y is no mistake: only span_x + span_y enters)
    "pixels_on_column_grid": ("const uint32_t x = idx[syn] % in_w, y = idx[syn] / in_w;",
                              "const uint32_t x = idx[syn] % grid_w, y = idx[syn] / grid_w;"),
    "no_lower_bound": ("return r < 1 ? 1u :", "return r < 0 ? 1u :"),
    "grid_rows_floor": ("const uint64_t grid_h = ((uint64_t)C + grid_w - 1) / grid_w;",
                        "const uint64_t grid_h = (uint64_t)C / grid_w;"),
    "unconnected_counted": ("      if (!synapse_connected(cfg, perm[syn])) continue;\n      const uint32_t x",
                            "      const uint32_t x"),
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
    pins = [test_handworked, lambda: test_closed_form_whole_input(8, 17)]
    pins += [lambda s=s: test_random_instances_match_definition(s) for s in range(20)]
    for pin in pins:
        try:
            pin()
        except AssertionError:
            caught += 1
    oracle._lib = None
    assert caught > 0, f"mutant {name} passed every pin"
