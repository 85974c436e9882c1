"""Pins for the oracle's boosting and duty cycles (readings B1-B7): a
hand-worked run, the reduction to the unboosted oracle, the real-valued
moving average within its rounding bound, boost invariants and planted
mistakes."""
import json
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1608_01966_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "boost_3col.json")
BC = {"period_log2": 6, "min_pct_q16": 655, "max_boost_q8": 2560, "bump_q8": 13}


def test_handworked():
    with open(GOLD) as f:
        g = json.load(f)
    idx = np.array(g["idx"], dtype=np.uint32)
    perm = np.array(g["perm_q_before"], dtype=np.float64) / 256
    frames = np.array(g["frames"], dtype=np.uint32)
    ov, win, p, (adc, odc, boost) = oracle.run_boost(g["config"], g["boost"], idx, perm, frames)
    assert ov.tolist() == g["boosted_overlaps"]
    assert win.tolist() == g["winners"]
    assert adc.tolist() == g["active_duty_q16"]
    assert odc.tolist() == g["overlap_duty_q16"]
    assert boost.tolist() == g["boost_q8"]
    assert (p * 256).tolist() == g["perm_q_after"]


def test_no_boost_reduces_to_the_plain_step():
    """max boost 1 and no raise: the same winners and permanences as the
    unboosted oracle, overlaps scaled by 256."""
    w = synth.workload_plain_32x32(frames=60)
    bc = dict(BC, max_boost_q8=256, bump_q8=0)
    ov, win, p, _ = oracle.run_boost(w.cfg, bc, w.idx, w.perm, w.frames)
    e_ov, e_win, e_p = oracle.run(w.cfg, w.idx, w.perm, w.frames)
    assert np.array_equal(win, e_win) and np.array_equal(p, e_p)
    assert np.array_equal(ov, 256 * e_ov)


def test_duty_cycles_track_the_real_moving_average():
    """Each step floors once (error < 1 in 1/65536 units) and old error
    decays by (P-1)/P, so the duty cycle stays within P units of the real
    moving average of the same events."""
    w = synth.workload_plain_32x32(frames=150)
    for pl in (0, 3, 6):
        bc = dict(BC, period_log2=pl)
        ov, win, p, (adc, odc, boost) = oracle.run_boost(w.cfg, bc, w.idx, w.perm, w.frames)
        P = 2 ** pl
        da = np.zeros(256)
        do = np.zeros(256)
        for t in range(150):
            act = np.zeros(256)
            act[win[t][win[t] >= 0]] = 1
            da = (da * (P - 1) + 65536 * act) / P
            do = (do * (P - 1) + 65536 * (ov[t] > 0)) / P
        assert np.all(np.abs(da - adc) < P) and np.all(da >= adc)
        assert np.all(np.abs(do - odc) < P) and np.all(do >= odc)


def test_boost_invariants():
    w = synth.workload_paper_scale(frames=40, columns=256, synapses=64)
    ov, win, p, (adc, odc, boost) = oracle.run_boost(w.cfg, BC, w.idx, w.perm, w.frames)
    assert boost.min() >= 256 and boost.max() <= BC["max_boost_q8"]
    order = np.argsort(adc, kind="stable")
    assert np.all(np.diff(boost[order].astype(np.int64)) <= 0)  # nonincreasing in duty
    mn = (int(adc.max()) * BC["min_pct_q16"]) >> 16
    assert np.all(boost[adc >= mn] == 256)
    if mn > 0:
        assert np.all(boost[adc == 0] == BC["max_boost_q8"])
    assert np.all((p * 256) == np.round(p * 256)) and p.min() >= 0 and p.max() <= 1


def test_learning_off_changes_nothing():
    w = synth.workload_plain_32x32(frames=20)
    _, _, _, st = oracle.run_boost(w.cfg, BC, w.idx, w.perm, w.frames[:10])
    _, _, p, st2 = oracle.run_boost(w.cfg, BC, w.idx, w.perm, w.frames[10:], learn=False,
                                    state=st)
    assert np.array_equal(p, w.perm.astype(np.float64))
    assert all(np.array_equal(a, b) for a, b in zip(st, st2))


MUTANTS = {
    "boost_ignored": ("bov[c] = ov[c] * (int32_t)boost[c];", "bov[c] = ov[c] * 256;"),
    "duty_no_decay": ("(uint64_t)adc[c] * (P - 1)", "(uint64_t)adc[c] * P"),
    "overlap_duty_from_active": ("(ov[c] > 0 ? 65536u : 0u)", "(active[c] ? 65536u : 0u)"),
    "min_from_overlap_duty": ("if (adc[c] > max_adc) max_adc = adc[c];",
                              "if (odc[c] > max_adc) max_adc = odc[c];"),
    "boost_slope_halved": ("(uint64_t)(bc->max_boost_q8 - 256) *", "(uint64_t)(bc->max_boost_q8 - 256) / 2 *"),
    "raise_on_active_duty": ("if (odc[c] < min_dc)", "if (adc[c] < min_dc)"),
    "no_clip": ("if (*p > 1.0) *p = 1.0;", ""),
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
    for pin in (test_handworked, test_no_boost_reduces_to_the_plain_step,
                test_duty_cycles_track_the_real_moving_average, test_boost_invariants):
        try:
            pin()
        except AssertionError:
            caught += 1
    oracle._lib = None
    assert caught > 0, f"mutant {name} survived"
