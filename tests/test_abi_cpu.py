"""The C ABI without a GPU: the library loads, exports every function that
include/sp.h declares, and its host-only checks behave as documented."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1608_01966_amd as sp
from paper_1608_01966_amd import _native, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            text = open(os.path.join(inc, f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(sp_[a-z_0-9]+)\s*\(", text))
    return names


def test_library_exports_every_declared_function():
    L = _native.lib()
    declared = _declared_functions()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(L, name), name
    assert declared == {n for n, _, _ in _native.SIGNATURES}


def test_config_checks():
    good = synth.sp_config(518400, 1024, 256, 4, 40)
    sp.sp_config_check(good)
    assert sp.sp_frame_words(good) == 16200
    # two exchange slots of 16-bit entries plus an int32 overlap scratch row
    assert sp.sp_workspace_bytes(good) >= 2 * 2 * 1024 + 4 * 1024
    bad = [
        dict(input_bits=0), dict(input_bits=(1 << 23) + 1), dict(num_columns=0),
        dict(num_columns=65537), dict(synapses_per_column=0), dict(synapses_per_column=4097),
        dict(winners=0), dict(winners=1025), dict(connected_q8=257), dict(inc_q8=300),
        dict(dec_q8=257),
    ]
    for b in bad:
        c = dict(good)
        c.update(b)
        with pytest.raises(sp.SpError) as e:
            sp.sp_config_check(c)
        assert e.value.code == sp.SP_EINVAL
        assert sp.sp_frame_words(c) == 0 and sp.sp_workspace_bytes(c) == 0
        assert sp.sp_last_error()


def test_check_state_host():
    cfg = synth.sp_config(100, 4, 8, 1, 2)
    w = synth.random_instance(1, cfg, frames=1)
    sp.sp_check_state_host(cfg, w.idx, w.perm)
    idx = w.idx.copy()
    idx[2, 3] = 100
    with pytest.raises(sp.SpError, match=r"idx\[19\]=100"):
        sp.sp_check_state_host(cfg, idx, w.perm)
    for badp in (0.3, -1 / 256, 257 / 256, np.nan):
        perm = w.perm.copy()
        perm[1, 1] = badp
        with pytest.raises(sp.SpError, match=r"perm\[9\]"):
            sp.sp_check_state_host(cfg, w.idx, perm)


def test_null_handle_and_args_are_rejected_on_host():
    L = _native.lib()
    assert L.sp_step(None, None, 0, 1, None, None, None) == sp.SP_EINVAL
    assert L.sp_step_plain(None, None, 0, 1, None, None, None) == sp.SP_EINVAL
    assert L.sp_sync(None, None) == sp.SP_EINVAL
    assert L.sp_step_is_persistent(None) == sp.SP_EINVAL
    assert L.sp_step_local_kernel(None) == sp.SP_EINVAL
    assert L.sp_step_local_kernel_for(None, 1024, 80) == sp.SP_EINVAL
    assert L.sp_destroy(None) == sp.SP_OK
    out = ctypes.c_void_p()
    cfg = _native.SpConfig.from_dict(synth.sp_config(100, 4, 8, 1, 2))
    assert L.sp_create(ctypes.byref(cfg), None, None, None, ctypes.byref(out)) == sp.SP_EINVAL
    assert L.sp_create(None, None, None, None, ctypes.byref(out)) == sp.SP_EINVAL
    assert out.value is None


def test_state_bytes_and_checkpoint_calls_without_a_handle():
    good = synth.sp_config(518400, 1024, 256, 4, 40)
    assert sp.sp_state_bytes(good) == 8 * 1024 * 256
    bad = dict(good)
    bad["num_columns"] = 0
    assert sp.sp_state_bytes(bad) == 0
    L = _native.lib()
    seen = ctypes.c_uint64()
    u32 = (ctypes.c_uint32 * 4)()
    assert L.sp_get_state(None, None, None, ctypes.byref(seen), None) == sp.SP_EINVAL
    assert L.sp_set_state(None, None, None, 0, None) == sp.SP_EINVAL
    assert L.sp_get_boost_state(None, u32, u32, u32, None) == sp.SP_EINVAL
    assert L.sp_set_boost_state(None, u32, u32, u32, None) == sp.SP_EINVAL
    assert "NULL" in sp.sp_last_error()


def test_inference_modes_are_distinct_constants():
    assert sp.SP_INFER_GATHER == 0 and sp.SP_INFER_MFMA_I8 == 1
    L = _native.lib()
    # mode is checked after the handle: a NULL handle fails first
    assert L.sp_infer(None, None, 0, 7, None, None, None) == sp.SP_EINVAL


def test_adaptive_local_step_and_raw_many_without_a_handle():
    L = _native.lib()
    r = (ctypes.c_uint32 * 1)()
    assert L.sp_step_local_adaptive(None, None, 0, 1, 8, 4, r, None, None, None, None) == \
        sp.SP_EINVAL
    assert "NULL" in sp.sp_last_error()
    # no handles: nothing to step
    # (stream 0: the null stream, named without touching a device)
    sp.sp_step_many_raw(np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0, np.uint32),
                        True, None, np.zeros(0, np.uint64), stream=0)
    with pytest.raises(ValueError):
        sp.sp_step_many_raw(np.zeros(2, np.uint64), np.zeros(1, np.uint64),
                            np.zeros(2, np.uint32), True, None, np.zeros(2, np.uint64), stream=0)
    # a NULL handle in the array is rejected on the host
    with pytest.raises(sp.SpError) as e:
        sp.sp_step_many_raw(np.zeros(1, np.uint64), np.zeros(1, np.uint64),
                            np.ones(1, np.uint32), True, None, np.zeros(1, np.uint64), stream=0)
    assert e.value.code == sp.SP_EINVAL
