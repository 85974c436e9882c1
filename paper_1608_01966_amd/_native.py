"""ctypes declarations of the C ABI in include/sp.h (libhtmsp.so).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

from .build import LIB_PATH

SP_OK, SP_EINVAL, SP_ENOMEM, SP_EDEVICE, SP_EBROKEN = 0, -1, -2, -3, -4
SP_MAX_INPUT_BITS = 1 << 23
SP_MAX_COLUMNS = 65536
SP_MAX_SYNAPSES = 4096
SP_INFER_GATHER = 0
SP_INFER_MFMA_I8 = 1


class SpConfig(ctypes.Structure):
    _fields_ = [
        ("input_bits", ctypes.c_uint32),
        ("num_columns", ctypes.c_uint32),
        ("synapses_per_column", ctypes.c_uint32),
        ("min_overlap", ctypes.c_uint32),
        ("winners", ctypes.c_uint32),
        ("connected_q8", ctypes.c_uint32),
        ("inc_q8", ctypes.c_uint32),
        ("dec_q8", ctypes.c_uint32),
    ]

    @classmethod
    def from_dict(cls, d: dict) -> "SpConfig":
        return cls(*(int(d[name]) for name, _ in cls._fields_))


# (name, restype, argtypes) for every function include/sp.h declares.
class EncCfg(ctypes.Structure):
    """sp_encoder_config of include/sp.h."""
    _fields_ = [
        ("width", ctypes.c_uint32),
        ("height", ctypes.c_uint32),
        ("factor", ctypes.c_uint32),
        ("block", ctypes.c_uint32),
        ("offset", ctypes.c_int32),
    ]


class BoostCfg(ctypes.Structure):
    """sp_boost_config of include/sp.h."""
    _fields_ = [
        ("period_log2", ctypes.c_uint32),
        ("min_pct_q16", ctypes.c_uint32),
        ("max_boost_q8", ctypes.c_uint32),
        ("bump_q8", ctypes.c_uint32),
    ]


P = ctypes.c_void_p
CFG = ctypes.POINTER(SpConfig)
U32 = ctypes.c_uint32
SIGNATURES = [
    ("sp_config_check", ctypes.c_int, [CFG]),
    ("sp_frame_words", ctypes.c_size_t, [CFG]),
    ("sp_workspace_bytes", ctypes.c_size_t, [CFG]),
    ("sp_check_state_host", ctypes.c_int, [CFG, P, P]),
    ("sp_create", ctypes.c_int, [CFG, P, P, P, ctypes.POINTER(P)]),
    ("sp_check_state", ctypes.c_int, [P, P]),
    ("sp_step", ctypes.c_int, [P, P, U32, ctypes.c_int, P, P, P]),
    ("sp_step_plain", ctypes.c_int, [P, P, U32, ctypes.c_int, P, P, P]),
    ("sp_infer", ctypes.c_int, [P, P, U32, ctypes.c_int, P, P, P]),
    ("sp_infer_noalloc_max_bytes", ctypes.c_size_t, []),
    ("sp_infer_noalloc", ctypes.c_int, [P, P, U32, P, P, P]),
    ("sp_step_many", ctypes.c_int, [P, U32, P, P, ctypes.c_int, P, P, P]),
    ("sp_set_histogram", ctypes.c_int, [P, P]),
    ("sp_step_boost", ctypes.c_int, [P, ctypes.POINTER(BoostCfg), P, U32, ctypes.c_int, P, P,
                                     P]),
    ("sp_boost_state", ctypes.c_int, [P, P, P, P, P]),
    ("sp_boost_reset", ctypes.c_int, [P, P]),
    ("sp_inhibit_local", ctypes.c_int, [P, U32, U32, U32, U32, U32, P, P]),
    ("sp_step_local", ctypes.c_int, [P, P, U32, ctypes.c_int, U32, U32, P, P, P]),
    ("sp_step_local_adaptive", ctypes.c_int, [P, P, U32, ctypes.c_int, U32, U32, P, P, P, P, P]),
    ("sp_encoded_bits", ctypes.c_size_t, [ctypes.POINTER(EncCfg)]),
    ("sp_encode", ctypes.c_int, [ctypes.POINTER(EncCfg), P, U32, P, P]),
    ("sp_step_is_persistent", ctypes.c_int, [P]),
    ("sp_step_kernel", ctypes.c_int, [P]),
    ("sp_step_local_kernel", ctypes.c_int, [P]),
    ("sp_step_local_kernel_for", ctypes.c_int, [P, U32, U32]),
    ("sp_step_boost_kernel", ctypes.c_int, [P]),
    ("sp_test_stall", ctypes.c_int, [P, ctypes.c_uint32]),
    ("sp_state_bytes", ctypes.c_size_t, [CFG]),
    ("sp_get_state", ctypes.c_int, [P, P, P, ctypes.POINTER(ctypes.c_uint64), P]),
    ("sp_set_state", ctypes.c_int, [P, P, P, ctypes.c_uint64, P]),
    ("sp_get_boost_state", ctypes.c_int, [P, P, P, P, P]),
    ("sp_set_boost_state", ctypes.c_int, [P, P, P, P, P]),
    ("sp_sync", ctypes.c_int, [P, P]),
    ("sp_destroy", ctypes.c_int, [P]),
    ("sp_last_error", ctypes.c_char_p, []),
]

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library.  torch is imported first so that the library
    binds to the HIP runtime torch already loaded (one runtime per process)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads torch's HIP runtime)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is not built; run `python -m paper_1608_01966_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
