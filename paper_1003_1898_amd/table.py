"""Python binding of the stream table (batched mixed generation, include/prng.h).

Argument marshalling only: the planning, the persistent kernels, the graph
capture and the autotuner live in libprng.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._capi import TableRow, check, lib
from .generator import TORCH_DTYPES, Generator, dtype_id, stream_handle


class StreamTable:
    """Rows (generator index, stream, count, dtype) over a list of Generator objects.

    Every ``run()`` produces the next `count` elements of each row's stream into
    that row's output view (``outputs[i]``) and advances the stream.
    """

    def __init__(self, gens: list[Generator], gen_idx, streams, counts, dtypes, seg_len: int = 0, device=None,
                 stream=None):
        self.gens = list(gens)
        self.device = self.gens[0].device if device is None else torch.device(device)
        gi = np.asarray(gen_idx, dtype=np.int64)
        si = np.asarray(streams, dtype=np.int64)
        cn = np.asarray(counts, dtype=np.int64)
        dt = np.asarray([dtype_id(d) for d in dtypes] if not np.issubdtype(np.asarray(dtypes).dtype, np.integer)
                        else dtypes, dtype=np.int64)
        n = len(gi)
        self.n_rows = n
        esize = np.where(dt == 3, 8, 4)
        nbytes = (cn * esize + 255) // 256 * 256   # each row 256-byte aligned in one buffer
        offs = np.concatenate([[0], np.cumsum(nbytes)[:-1]]) if n else np.zeros(0, dtype=np.int64)
        total = int(nbytes.sum()) if n else 0
        self._buf = torch.empty(max(total, 256), dtype=torch.uint8, device=self.device)
        base = self._buf.data_ptr()
        rows = (TableRow * max(n, 1))()
        self.outputs = []
        for i in range(n):
            rows[i].gen = int(gi[i])
            rows[i].dtype = int(dt[i])
            rows[i].stream = int(si[i])
            rows[i].count = int(cn[i])
            rows[i].d_out = base + int(offs[i])
            view = self._buf[int(offs[i]):int(offs[i]) + int(cn[i] * esize[i])].view(TORCH_DTYPES[int(dt[i])])
            self.outputs.append(view)
        handles = (ctypes.c_void_p * len(self.gens))(*[g.handle for g in self.gens])
        seg = int(seg_len) & 0xFFFFFFFF
        wb = lib().prng_table_work_bytes(handles, len(self.gens), rows, n, seg)
        if wb == 0:
            check(-1)
        self._work = torch.empty(wb, dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        check(lib().prng_table_create(ctypes.byref(self._h), handles, len(self.gens), rows, n, seg,
                                      self._work.data_ptr(), self._work.numel(), stream_handle(stream, self.device)))

    def run(self, graph: bool = True, stream=None) -> None:
        check(lib().prng_table_run(self._h, 1 if graph else 0, stream_handle(stream, self.device)))

    def autotune(self, repeats: int = 2, stream=None) -> dict:
        check(lib().prng_table_autotune(self._h, int(repeats), stream_handle(stream, self.device)))
        return self.config()

    def config(self) -> dict:
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().prng_table_get_config(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"lane_grid": a.value, "mt_grid": b.value, "concurrent": int(c.value)}

    def set_config(self, lane_grid: int, mt_grid: int, concurrent: int) -> None:
        """concurrent: 0 serial, 1 MT19937 beside the lane classes, 2 every class on a stream of its own,
        3 as 2 with the lane classes started before the MT19937 jumps."""
        check(lib().prng_table_set_config(self._h, int(lane_grid), int(mt_grid), int(concurrent)))

    def info(self) -> dict:
        a, b = ctypes.c_uint32(), ctypes.c_uint32()
        c, d, e = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        check(lib().prng_table_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d),
                                    ctypes.byref(e)))
        return {"lane_tasks": a.value, "mt_tasks": b.value, "total_draws": c.value, "max_draws": d.value,
                "segments": e.value}

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().prng_table_destroy(h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
