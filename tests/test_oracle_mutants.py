"""The pins are strong enough: plant one plausible mistake at a time in the
oracle's C source (a flipped comparison, a swapped term, a dropped clip, a
wrong bit order), build the mutant on the CPU, and check that the pin suite
(hand-worked example, dense form, brute-force top-k) rejects every one."""
import json
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1608_01966_amd import synth
from tests.dense_reference import dense_run
from tests.test_oracle_topk_bruteforce import brute

SRC = os.path.join(os.path.dirname(oracle.__file__), "sp_oracle.c")
GOLD = os.path.join(os.path.dirname(__file__), "golden", "handworked_8col.json")

MUTANTS = {
    "connected_strict": ("return perm >= cfg->connected_perm;", "return perm > cfg->connected_perm;"),
    "min_overlap_le": ("if (ov < (int32_t)cfg->min_overlap)", "if (ov <= (int32_t)cfg->min_overlap)"),
    "ties_to_higher": ("overlap[c] > best_ov", "overlap[c] >= best_ov"),
    "zero_can_win": ("int32_t best_ov = 0;", "int32_t best_ov = -1;"),
    "inc_dec_swapped": ("p = p + cfg->perm_inc;", "p = p + cfg->perm_dec;"),
    "no_upper_clip": ("if (p > 1.0) p = 1.0;", ""),
    "no_lower_clip": ("if (p < 0.0) p = 0.0;", ""),
    "learn_losers": ("if (!active[c]) continue;", "if (active[c]) continue;"),
    "msb_first_bits": ("(frame[p >> 5] >> (p & 31u))", "(frame[p >> 5] >> (31u - (p & 31u)))"),
    "skip_last_synapse": ("for (uint32_t s = 0; s < S; ++s) {\n      const size_t syn = (size_t)c * S + s;\n      if (synapse",
                          "for (uint32_t s = 0; s + 1 < S; ++s) {\n      const size_t syn = (size_t)c * S + s;\n      if (synapse"),
}


def _pins_pass() -> bool:
    with open(GOLD) as f:
        g = json.load(f)
    idx = np.array(g["idx"], dtype=np.uint32)
    perm = (np.array(g["perm_q_before"], dtype=np.float32) / 256).astype(np.float32)
    ov, win, p = oracle.run(g["config"], idx, perm, np.array(g["frames"], dtype=np.uint32))
    if ov.tolist() != g["overlaps"] or win.tolist() != g["winners"] or \
            (p * 256).tolist() != g["perm_q_after_frame2"]:
        return False
    for seed in range(6):
        cfg = synth.sp_config(300, 40, 24, 2, 8)
        w = synth.random_instance(50 + seed, cfg, frames=10, density=0.3)
        a = oracle.run(cfg, w.idx, w.perm, w.frames)
        b = dense_run(cfg, w.idx, w.perm_q, w.frames)
        if not (np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
                and np.array_equal(a[2] * 256, b[2])):
            return False
    for seed in range(60):
        r = np.random.default_rng(seed)
        C = int(r.integers(1, 9))
        k = int(r.integers(1, C + 1))
        ov = r.integers(0, 4, size=C).astype(np.int32)
        win, _ = oracle.inhibit(synth.sp_config(32, C, 1, 0, k), ov)
        e = brute(ov.tolist(), k)
        if win.tolist() != e + [-1] * (k - len(e)):
            return False
    return True


@pytest.fixture
def swap_lib(monkeypatch, tmp_path):
    def use(src_text):
        c = tmp_path / "mutant.c"
        c.write_text(src_text)
        so = tmp_path / f"mutant_{abs(hash(src_text))}.so"
        # the library also carries the threaded runner and the (unmutated)
        # encoder oracle
        subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-I",
                               os.path.dirname(SRC), str(c),
                               os.path.join(os.path.dirname(SRC), "sp_oracle_mt.c"),
                               os.path.join(os.path.dirname(SRC), "enc_oracle.c"), "-pthread",
                               "-o", str(so)])
        monkeypatch.setattr(oracle, "_LIB_PATH", str(so))
        monkeypatch.setattr(oracle, "_lib", None)
    yield use
    oracle._lib = None


def test_unmutated_passes():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, swap_lib):
    src = open(SRC).read()
    before, after = MUTANTS[name]
    assert before in src, f"mutation site for {name} not found"
    swap_lib(src.replace(before, after, 1))
    assert not _pins_pass(), f"mutant {name} survived the pins"
