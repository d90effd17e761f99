"""CPU oracle for the generators of arXiv:1003.1898 (ctypes over prng_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``; the product package never
imports it.  It shares no code with the HIP path.  See ``prng_oracle.c`` for
the definitions, the canonical state layouts and the section citations.
"""
from __future__ import annotations

import ctypes
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .build import LIB_PATH, build

GGL, XOR128, RANECU, RANMAR, RANLUX, MT19937, DRAND48, RANNYU = 1, 2, 3, 4, 5, 6, 7, 8
KINDS = {"ggl": GGL, "xor128": XOR128, "ranecu": RANECU, "ranmar": RANMAR,
         "ranlux": RANLUX, "mt19937": MT19937, "drand48": DRAND48, "rannyu": RANNYU}
U32, F32, F64, F32_PAPER = 1, 2, 3, 4
DTYPES = {"u32": U32, "f32": F32, "f64": F64, "f32_paper": F32_PAPER}
_NP = {U32: np.uint32, F32: np.float32, F64: np.float64, F32_PAPER: np.float32}

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.orc_state_words.argtypes = [ctypes.c_int]
        L.orc_seed_words.argtypes = [ctypes.c_int]
        L.orc_bits.argtypes = [ctypes.c_int]
        L.orc_next.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, u32p]
        L.orc_next.restype = ctypes.c_uint32
        L.orc_init.argtypes = [ctypes.c_int, u64p, u32p]
        L.orc_to_f32.argtypes = [ctypes.c_int, ctypes.c_uint32]
        L.orc_to_f32.restype = ctypes.c_float
        L.orc_to_f32_paper.argtypes = [ctypes.c_int, ctypes.c_uint32]
        L.orc_to_f32_paper.restype = ctypes.c_float
        L.orc_to_f64.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32]
        L.orc_to_f64.restype = ctypes.c_double
        L.orc_generate.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                   u32p, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
        L.orc_fused.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                u32p, ctypes.c_uint64, u64p, u32p]
        L.orc_sum_f32.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, u32p, ctypes.c_uint64]
        L.orc_sum_f32.restype = ctypes.c_double
        L.orc_ggl_period.argtypes = [ctypes.c_uint32]
        L.orc_ggl_period.restype = ctypes.c_uint64
        L.orc_ranmar_c_period.argtypes = [ctypes.c_uint32]
        L.orc_ranmar_c_period.restype = ctypes.c_uint64
        _lib = L
    return _lib


def _kind(k) -> int:
    return KINDS[k] if isinstance(k, str) else int(k)


def _dtype(d) -> int:
    return DTYPES[d] if isinstance(d, str) else int(d)


def _u32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _u64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def state_words(kind) -> int:
    return lib().orc_state_words(_kind(kind))


def seed_words(kind) -> int:
    return lib().orc_seed_words(_kind(kind))


def bits(kind) -> int:
    return lib().orc_bits(_kind(kind))


def init(kind, seeds) -> np.ndarray:
    """Canonical states (n, W) uint32 from mapped seed tuples (n, seed_words) uint64."""
    k = _kind(kind)
    seeds = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64).reshape(-1, seed_words(k)))
    n = seeds.shape[0]
    st = np.zeros((n, state_words(k)), dtype=np.uint32)
    for s in range(n):
        rc = lib().orc_init(k, _u64p(seeds[s]), _u32p(st[s]))
        if rc != 0:
            raise ValueError(f"seed tuple {seeds[s].tolist()} out of range for kind {k}")
    return st


def next_draws(kind, state: np.ndarray, n: int, p: int = 223, r: int = 24) -> np.ndarray:
    """n successive native draws of ONE stream; advances `state` (1-D uint32) in place."""
    k = _kind(kind)
    assert state.dtype == np.uint32 and state.flags.c_contiguous
    out = np.empty(n, dtype=np.uint32)
    ptr = _u32p(state)
    L = lib()
    for i in range(n):
        out[i] = L.orc_next(k, p, r, ptr)
    return out


def generate(kind, states: np.ndarray, count: int, dtype="u32", p: int = 223, r: int = 24,
             threads: int = 1) -> np.ndarray:
    """Next `count` elements of every stream; advances `states` (n, W) in place.

    Returns an (n, count) array (uint32, float32 or float64)."""
    k, d = _kind(kind), _dtype(dtype)
    assert states.dtype == np.uint32 and states.flags.c_contiguous
    n = states.shape[0]
    out = np.empty((n, count), dtype=_NP[d])
    L = lib()

    def run(a, b):
        if b > a:
            L.orc_generate(k, p, r, b - a, _u32p(states[a:b]), count, d,
                           out[a:b].ctypes.data_as(ctypes.c_void_p))

    _split(n, threads, run)
    return out


def fused(kind, states: np.ndarray, draws: int, p: int = 223, r: int = 24, threads: int = 1):
    """Per-stream exact mantissa sum (uint64) and 64-bin histogram (uint32)."""
    k = _kind(kind)
    assert states.dtype == np.uint32 and states.flags.c_contiguous
    n = states.shape[0]
    s = np.zeros(n, dtype=np.uint64)
    h = np.zeros((n, 64), dtype=np.uint32)
    L = lib()

    def run(a, b):
        if b > a:
            L.orc_fused(k, p, r, b - a, _u32p(states[a:b]), draws, _u64p(s[a:b]), _u32p(h[a:b]))

    _split(n, threads, run)
    return s, h


def _split(n, threads, fn):
    threads = max(1, int(threads))
    if threads == 1 or n < 2:
        fn(0, n)
        return
    step = (n + threads - 1) // threads
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda a: fn(a, min(n, a + step)), range(0, n, step)))


def to_f32(kind, u: int) -> float:
    return lib().orc_to_f32(_kind(kind), int(u))


def to_f32_paper(kind, u: int) -> float:
    return lib().orc_to_f32_paper(_kind(kind), int(u))


def to_f64(kind, u1: int, u2: int) -> float:
    return lib().orc_to_f64(_kind(kind), int(u1), int(u2))


def sum_f32(kind, state: np.ndarray, count: int, p: int = 223, r: int = 24) -> float:
    """One stream, one draw per call, single-precision values summed; advances `state` (1-D)."""
    assert state.dtype == np.uint32 and state.flags.c_contiguous
    return lib().orc_sum_f32(_kind(kind), p, r, _u32p(state), count)


def ggl_period(x0: int) -> int:
    return lib().orc_ggl_period(int(x0))


def ranmar_c_period(c0: int) -> int:
    return lib().orc_ranmar_c_period(int(c0))
