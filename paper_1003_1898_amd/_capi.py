"""ctypes declarations of libprng.so (the C ABI of include/prng.h).

Argument marshalling only: every step of generation runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libprng.so")

SEG_AUTO, SEG_NEVER = 0, 0xFFFFFFFF
PRNG_OK, PRNG_EINVAL, PRNG_ERANGE, PRNG_ENOMEM, PRNG_EHIP, PRNG_ESTATE, PRNG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
ERRORS = {PRNG_EINVAL: "EINVAL", PRNG_ERANGE: "ERANGE", PRNG_ENOMEM: "ENOMEM", PRNG_EHIP: "EHIP",
          PRNG_ESTATE: "ESTATE", PRNG_EUNSUPPORTED: "EUNSUPPORTED"}

_c = ctypes
_vp, _u32, _u64, _sz, _int = _c.c_void_p, _c.c_uint32, _c.c_uint64, _c.c_size_t, _c.c_int
_u64p = _c.POINTER(_c.c_uint64)

# name -> (restype, argtypes); every symbol declared in include/prng.h
SIGNATURES = {
    "prng_last_error": (_c.c_char_p, []),
    "prng_seed_tuple_words": (_int, [_int]),
    "prng_state_words": (_int, [_int]),
    "prng_seed_words": (_int, [_int, _u64, _u64, _u64p]),
    "prng_state_bytes": (_sz, [_int, _u64]),
    "prng_create": (_int, [_c.POINTER(_vp), _int, _u32, _u64, _u64p, _vp, _sz, _vp]),
    "prng_destroy": (None, [_vp]),
    "prng_kind_of": (_int, [_vp]),
    "prng_luxury_of": (_u32, [_vp]),
    "prng_n_streams": (_u64, [_vp]),
    "prng_generate": (_int, [_vp, _u64, _int, _vp, _sz, _vp]),
    "prng_generate_noalloc": (_int, [_vp, _u64, _int, _vp, _sz, _vp]),
    "prng_ranlux_generate_variant": (_int, [_vp, _int, _u64, _int, _vp, _sz, _vp]),
    "prng_generate_packed4": (_int, [_vp, _u64, _int, _vp, _sz, _vp]),
    "prng_fused_sum_hist": (_int, [_vp, _u64, _vp, _vp, _vp]),
    "prng_blob_bytes": (_sz, [_vp]),
    "prng_get_state": (_int, [_vp, _vp, _sz, _vp]),
    "prng_set_state": (_int, [_vp, _vp, _sz, _vp]),
    "prng_table_work_bytes": (_sz, [_c.POINTER(_vp), _int, _vp, _u64, _u32]),
    "prng_table_create": (_int, [_c.POINTER(_vp), _c.POINTER(_vp), _int, _vp, _u64, _u32, _vp, _sz, _vp]),
    "prng_table_work_bytes_ex": (_sz, [_c.POINTER(_vp), _int, _vp, _u64, _vp]),
    "prng_table_create_ex": (_int, [_c.POINTER(_vp), _c.POINTER(_vp), _int, _vp, _u64, _vp, _vp, _sz, _vp]),
    "prng_table_seg_lengths": (_int, [_vp, _vp]),
    "prng_table_tune_work_bytes": (_sz, [_c.POINTER(_vp), _int, _vp, _u64]),
    "prng_table_tune_segments": (_int, [_c.POINTER(_vp), _int, _vp, _u64, _int, _vp, _sz, _vp, _vp,
                                        _c.POINTER(_c.c_float)]),
    "prng_table_run": (_int, [_vp, _int, _vp]),
    "prng_table_autotune": (_int, [_vp, _int, _vp]),
    "prng_table_get_config": (_int, [_vp, _c.POINTER(_int), _c.POINTER(_int), _c.POINTER(_int)]),
    "prng_table_set_config": (_int, [_vp, _int, _int, _int]),
    "prng_table_info": (_int, [_vp, _c.POINTER(_u32), _c.POINTER(_u32), _u64p, _u64p, _u64p]),
    "prng_table_destroy": (None, [_vp]),
    "prng_server_create": (_int, [_c.POINTER(_vp), _c.POINTER(_vp), _int, _vp, _sz, _int, _int, _u32, _u64]),
    "prng_server_submit_many": (_int, [_vp, _u64, _c.POINTER(_u32), _u64p, _u64p, _c.POINTER(_int),
                                       _c.POINTER(_c.c_int64), _int, _u64p]),
    "prng_server_submit": (_int, [_vp, _u32, _u64, _u64, _int, _u64p]),
    "prng_server_result": (_int, [_vp, _u64, _int, _c.POINTER(_vp), _c.POINTER(_sz)]),
    "prng_server_release": (_int, [_vp, _u64]),
    "prng_server_times": (_int, [_vp, _u64, _u64p, _c.POINTER(_c.c_int64), _c.POINTER(_c.c_int64),
                                 _c.POINTER(_c.c_int64)]),
    "prng_server_stats": (_int, [_vp, _u64p, _u64p, _u64p, _c.POINTER(_sz)]),
    "prng_server_timing": (_int, [_vp, _c.POINTER(_c.c_int64), _c.POINTER(_c.c_double)]),
    "prng_server_now_ns": (_c.c_int64, [_vp]),
    "prng_server_destroy": (None, [_vp]),
}


class TableRow(_c.Structure):
    """Mirror of prng_table_row."""
    _fields_ = [("gen", _c.c_uint32), ("dtype", _c.c_uint32), ("stream", _c.c_uint64), ("count", _c.c_uint64),
                ("d_out", _c.c_void_p)]


class SegLengths(_c.Structure):
    """Mirror of prng_seg_lengths."""
    _fields_ = [("lane", _c.c_uint32), ("ranmar", _c.c_uint32), ("mt", _c.c_uint32)]


class PrngError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libprng.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1003_1898_amd.build` "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> int:
    if rc < 0:
        raise PrngError(rc, lib().prng_last_error().decode(errors="replace"))
    return rc
