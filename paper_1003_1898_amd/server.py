"""Python binding of the serving loop (prng_server_* in include/prng.h).

Argument marshalling only: admission, batching, planning and the launches run
in libprng's worker thread and HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._capi import SEG_AUTO, check, lib
from .generator import TORCH_DTYPES, Generator, dtype_id

_i64p = ctypes.POINTER(ctypes.c_int64)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class Server:
    """Requests (generator index, stream, count, dtype) answered from resident states.

    ``pool_bytes`` of device memory are the budget for jump tables, in-flight
    outputs and batch workspaces.
    """

    def __init__(self, gens: list[Generator], pool_bytes: int, *, max_inflight: int = 4, max_batch: int = 4096,
                 seg_len: int = SEG_AUTO, max_request_draws: int = 1 << 23, device=None):
        self.gens = list(gens)
        self.device = self.gens[0].device if device is None else torch.device(device)
        self._dtypes: dict[int, int] = {}
        self._pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.device)
        handles = (ctypes.c_void_p * len(self.gens))(*[g.handle for g in self.gens])
        self._h = ctypes.c_void_p()
        torch.cuda.synchronize(self.device)
        check(lib().prng_server_create(ctypes.byref(self._h), handles, len(self.gens), self._pool.data_ptr(),
                                       self._pool.numel(), int(max_inflight), int(max_batch),
                                       int(seg_len) & 0xFFFFFFFF, int(max_request_draws)))

    def submit_many(self, gen, stream, count, dtype, arrive_ns=None, keep: bool = True) -> np.ndarray:
        gen = np.ascontiguousarray(gen, dtype=np.uint32)
        n = len(gen)
        stream = np.ascontiguousarray(stream, dtype=np.uint64)
        count = np.ascontiguousarray(count, dtype=np.uint64)
        dt = np.asarray(dtype)
        dt = np.ascontiguousarray([dtype_id(d) for d in dt] if not np.issubdtype(dt.dtype, np.integer) else dt,
                                  dtype=np.int32)
        arr = None if arrive_ns is None else np.ascontiguousarray(arrive_ns, dtype=np.int64)
        tickets = np.zeros(n, dtype=np.uint64)
        check(lib().prng_server_submit_many(self._h, n, _ptr(gen, ctypes.c_uint32), _ptr(stream, ctypes.c_uint64),
                                            _ptr(count, ctypes.c_uint64), _ptr(dt, ctypes.c_int),
                                            None if arr is None else _ptr(arr, ctypes.c_int64), 1 if keep else 0,
                                            _ptr(tickets, ctypes.c_uint64)))
        for t, d in zip(tickets.tolist(), dt.tolist()):
            self._dtypes[t] = d
        return tickets

    def submit(self, gen: int, stream: int, count: int, dtype) -> int:
        return int(self.submit_many([gen], [stream], [count], [dtype])[0])

    def result(self, ticket: int, timeout_ms: int = -1) -> torch.Tensor | None:
        """A copy of a kept request's output, or None if not done within the timeout."""
        ptr, nbytes = ctypes.c_void_p(), ctypes.c_size_t()
        rc = check(lib().prng_server_result(self._h, int(ticket), int(timeout_ms), ctypes.byref(ptr),
                                            ctypes.byref(nbytes)))
        if rc == 0:
            return None
        off = ptr.value - self._pool.data_ptr()
        return self._pool[off:off + nbytes.value].view(TORCH_DTYPES[self._dtypes[int(ticket)]]).clone()

    def release(self, ticket: int) -> None:
        check(lib().prng_server_release(self._h, int(ticket)))

    def times(self, tickets) -> dict:
        t = np.ascontiguousarray(tickets, dtype=np.uint64)
        a, b, c = (np.zeros(len(t), dtype=np.int64) for _ in range(3))
        check(lib().prng_server_times(self._h, len(t), _ptr(t, ctypes.c_uint64), _ptr(a, ctypes.c_int64),
                                      _ptr(b, ctypes.c_int64), _ptr(c, ctypes.c_int64)))
        return {"arrive_ns": a, "admit_ns": b, "done_ns": c}

    def stats(self) -> dict:
        a, b, c, d = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_size_t()
        check(lib().prng_server_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
        return {"submitted": a.value, "completed": b.value, "batches": c.value, "pool_in_use": d.value}

    def timing(self) -> dict:
        a, b = ctypes.c_int64(), ctypes.c_double()
        check(lib().prng_server_timing(self._h, ctypes.byref(a), ctypes.byref(b)))
        return {"host_plan_ms": a.value / 1e6, "device_ms": b.value}

    def now_ns(self) -> int:
        return int(lib().prng_server_now_ns(self._h))

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().prng_server_destroy(h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
