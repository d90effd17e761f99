"""Python binding of libprng: a thin wrapper over the C ABI of include/prng.h.

PyTorch provides device memory and streams; the library's HIP kernels do the
work.  Names follow the paper's generators: GGL, XOR128, RANECU, RANMAR, RANLUX
(luxury p) and MT19937.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _capi
from ._capi import check, lib
from .inputs import DTYPE_IDS, KIND_IDS, kind_id

TORCH_DTYPES = {1: torch.uint32, 2: torch.float32, 3: torch.float64, 4: torch.float32}
LAG_VARIANTS = {"registers": 0, "lds": 1, "hbm": 2}
LUXURY_LEVELS = {0: 24, 1: 48, 2: 97, 3: 223, 4: 389}


def dtype_id(dtype) -> int:
    if isinstance(dtype, str):
        return DTYPE_IDS[dtype]
    if isinstance(dtype, torch.dtype):
        return {torch.uint32: 1, torch.float32: 2, torch.float64: 3}[dtype]
    return int(dtype)


def stream_handle(stream=None, device=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return int(stream.cuda_stream)


def seed_words(kind, master: int, n_streams: int) -> np.ndarray:
    """Per-stream seed tuples from a master seed (native prng_seed_words)."""
    k = kind_id(kind)
    w = check(lib().prng_seed_tuple_words(k))
    out = np.zeros((n_streams, w), dtype=np.uint64)
    check(lib().prng_seed_words(k, int(master) & (2**64 - 1), n_streams,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    return out


def state_words(kind) -> int:
    return check(lib().prng_state_words(kind_id(kind)))


class Generator:
    """N independent streams of one generator kind, state resident on the GPU.

    ``Generator("ranlux", 65536, seed=7, p=223)`` seeds stream s from
    SplitMix64(seed) (see ``inputs.py``); ``seed_words=`` passes explicit
    per-stream seed tuples instead.
    """

    def __init__(self, kind, n_streams: int, *, seed: int | None = None, seed_words: np.ndarray | None = None,
                 p: int = 223, device=None, stream=None):
        self.kind = kind_id(kind)
        self.n = int(n_streams)
        self.p = int(p) if self.kind == KIND_IDS["ranlux"] else 0
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if seed_words is None:
            if seed is None:
                raise ValueError("give seed= or seed_words=")
            seed_words = globals()["seed_words"](self.kind, seed, self.n)
        sw = np.ascontiguousarray(np.asarray(seed_words, dtype=np.uint64).reshape(self.n, -1))
        nbytes = lib().prng_state_bytes(self.kind, self.n)
        if nbytes == 0:
            raise ValueError(f"unknown generator kind {kind}")
        self._state = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._handle = ctypes.c_void_p()
        check(lib().prng_create(ctypes.byref(self._handle), self.kind, self.p, self.n,
                                sw.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                self._state.data_ptr(), nbytes, stream_handle(stream, self.device)))

    @property
    def handle(self) -> int:
        return self._handle.value

    def generate(self, count: int, dtype="u32", out: torch.Tensor | None = None, stream=None,
                 lag: str | None = None) -> torch.Tensor:
        """Next `count` elements of every stream as an (n, count) tensor.

        `lag` (RANLUX only) places the lag table: "registers" (the default
        path), "lds" or "hbm" (prng_ranlux_generate_variant)."""
        d = dtype_id(dtype)
        if out is None:
            out = torch.empty((self.n, int(count)), dtype=TORCH_DTYPES[d], device=self.device)
        if out.dtype != TORCH_DTYPES[d] or not out.is_contiguous() or out.device != self.device:
            raise ValueError("out must be a contiguous tensor of the right dtype on the generator's device")
        nbytes = out.numel() * out.element_size()
        if lag is None:
            check(lib().prng_generate(self._handle, int(count), d, out.data_ptr(), nbytes,
                                      stream_handle(stream, self.device)))
        else:
            check(lib().prng_ranlux_generate_variant(self._handle, LAG_VARIANTS[lag], int(count), d, out.data_ptr(),
                                                     nbytes, stream_handle(stream, self.device)))
        return out

    def generate_noalloc(self, count: int, dtype="u32", out: torch.Tensor | None = None,
                         stream=None) -> torch.Tensor:
        """``generate`` through prng_generate_noalloc (RANLUX's scratch in the
        library's static device array instead of the object's buffer)."""
        d = dtype_id(dtype)
        if out is None:
            out = torch.empty((self.n, int(count)), dtype=TORCH_DTYPES[d], device=self.device)
        if out.dtype != TORCH_DTYPES[d] or not out.is_contiguous() or out.device != self.device:
            raise ValueError("out must be a contiguous tensor of the right dtype on the generator's device")
        check(lib().prng_generate_noalloc(self._handle, int(count), d, out.data_ptr(),
                                          out.numel() * out.element_size(), stream_handle(stream, self.device)))
        return out

    def generate_packed4(self, count: int, dtype="f32", out: torch.Tensor | None = None,
                         stream=None) -> torch.Tensor:
        """Next `count` elements of every stream, streams interleaved four by four:
        an (n / 4, count, 4) tensor whose [g, i, k] is element i of stream 4 g + k."""
        d = dtype_id(dtype)
        if out is None:
            out = torch.empty((self.n // 4, int(count), 4), dtype=TORCH_DTYPES[d], device=self.device)
        if out.dtype != TORCH_DTYPES[d] or not out.is_contiguous() or out.device != self.device:
            raise ValueError("out must be a contiguous tensor of the right dtype on the generator's device")
        check(lib().prng_generate_packed4(self._handle, int(count), d, out.data_ptr(),
                                          out.numel() * out.element_size(), stream_handle(stream, self.device)))
        return out

    def fused_sum_hist(self, draws: int, out_sum: torch.Tensor | None = None, out_hist: torch.Tensor | None = None,
                       stream=None):
        """Per-stream exact mantissa sum (uint64, n) and 64-bin histogram (uint32, n x 64)."""
        if out_sum is None:
            out_sum = torch.empty(self.n, dtype=torch.uint64, device=self.device)
        if out_hist is None:
            out_hist = torch.empty((self.n, 64), dtype=torch.uint32, device=self.device)
        check(lib().prng_fused_sum_hist(self._handle, int(draws), out_sum.data_ptr(), out_hist.data_ptr(),
                                        stream_handle(stream, self.device)))
        return out_sum, out_hist

    def get_state(self, stream=None) -> np.ndarray:
        """Canonical state blob (uint8 array): 32-byte header + n x W uint32 words."""
        nb = lib().prng_blob_bytes(self._handle)
        blob = np.zeros(nb, dtype=np.uint8)
        check(lib().prng_get_state(self._handle, blob.ctypes.data, nb, stream_handle(stream, self.device)))
        return blob

    def set_state(self, blob, stream=None) -> None:
        b = np.ascontiguousarray(np.frombuffer(bytes(blob), dtype=np.uint8) if not isinstance(blob, np.ndarray)
                                 else blob.view(np.uint8))
        check(lib().prng_set_state(self._handle, b.ctypes.data, b.nbytes, stream_handle(stream, self.device)))

    def state_words(self) -> np.ndarray:
        """Canonical per-stream state words as an (n, W) uint32 array."""
        blob = self.get_state()
        return blob[32:].view(np.uint32).reshape(self.n, -1).copy()

    @staticmethod
    def blob_from_words(kind, p: int, words: np.ndarray) -> np.ndarray:
        """Canonical blob for (n, W) state words (header layout of include/prng.h)."""
        k = kind_id(kind)
        words = np.ascontiguousarray(words, dtype=np.uint32)
        n, W = words.shape
        hdr = np.zeros(8, dtype=np.uint32)
        hdr[0] = 0x474E5250
        hdr[1] = 1
        hdr[2] = k
        hdr[3] = p if k == KIND_IDS["ranlux"] else 0
        hdr[4] = n & 0xFFFFFFFF
        hdr[5] = n >> 32
        hdr[6] = W
        return np.concatenate([hdr.view(np.uint8), words.reshape(-1).view(np.uint8)])

    def close(self) -> None:
        h = getattr(self, "_handle", None)
        if h is not None and h.value:
            lib().prng_destroy(h)
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


__all__ = ["Generator", "seed_words", "state_words", "dtype_id", "stream_handle", "LUXURY_LEVELS", "_capi"]
