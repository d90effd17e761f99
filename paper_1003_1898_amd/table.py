"""Python binding of the stream table (batched mixed generation, include/prng.h).

Argument marshalling only: the planning, the persistent kernels, the graph
capture and the autotuner live in libprng.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._capi import SegLengths, TableRow, check, lib
from .generator import TORCH_DTYPES, Generator, dtype_id, stream_handle


def _rows(gens, device, gen_idx, streams, counts, dtypes):
    """One device buffer holding every row's output (256-byte aligned rows), the
    prng_table_row array pointing into it, and a typed view per row."""
    gi = np.asarray(gen_idx, dtype=np.int64)
    si = np.asarray(streams, dtype=np.int64)
    cn = np.asarray(counts, dtype=np.int64)
    dt = np.asarray([dtype_id(d) for d in dtypes] if not np.issubdtype(np.asarray(dtypes).dtype, np.integer)
                    else dtypes, dtype=np.int64)
    n = len(gi)
    esize = np.where(dt == 3, 8, 4)
    nbytes = (cn * esize + 255) // 256 * 256
    offs = np.concatenate([[0], np.cumsum(nbytes)[:-1]]) if n else np.zeros(0, dtype=np.int64)
    total = int(nbytes.sum()) if n else 0
    buf = torch.empty(max(total, 256), dtype=torch.uint8, device=device)
    base = buf.data_ptr()
    rows = (TableRow * max(n, 1))()
    outputs = []
    for i in range(n):
        rows[i].gen = int(gi[i])
        rows[i].dtype = int(dt[i])
        rows[i].stream = int(si[i])
        rows[i].count = int(cn[i])
        rows[i].d_out = base + int(offs[i])
        outputs.append(buf[int(offs[i]):int(offs[i]) + int(cn[i] * esize[i])].view(TORCH_DTYPES[int(dt[i])]))
    handles = (ctypes.c_void_p * len(gens))(*[g.handle for g in gens])
    return buf, rows, n, outputs, handles


def _seg_struct(seg: dict | None):
    if seg is None:
        return None
    return SegLengths(int(seg.get("lane", 0)) & 0xFFFFFFFF, int(seg.get("ranmar", 0)) & 0xFFFFFFFF,
                      int(seg.get("mt", 0)) & 0xFFFFFFFF)


class StreamTable:
    """Rows (generator index, stream, count, dtype) over a list of Generator objects.

    Every ``run()`` produces the next `count` elements of each row's stream into
    that row's output view (``outputs[i]``) and advances the stream.  Rows are
    cut at ``seg_len`` (one length for every kind) or, when ``seg`` is given, at
    per-class lengths {"lane", "ranmar", "mt"} (0: automatic).
    """

    def __init__(self, gens: list[Generator], gen_idx, streams, counts, dtypes, seg_len: int = 0, device=None,
                 stream=None, seg: dict | None = None):
        self.gens = list(gens)
        self.device = self.gens[0].device if device is None else torch.device(device)
        self._buf, rows, n, self.outputs, handles = _rows(self.gens, self.device, gen_idx, streams, counts, dtypes)
        self.n_rows = n
        sl = _seg_struct(seg)
        if sl is None:
            sv = int(seg_len) & 0xFFFFFFFF
            wb = lib().prng_table_work_bytes(handles, len(self.gens), rows, n, sv)
        else:
            wb = lib().prng_table_work_bytes_ex(handles, len(self.gens), rows, n, ctypes.byref(sl))
        if wb == 0:
            check(-1)
        self._work = torch.empty(wb, dtype=torch.uint8, device=self.device)
        self._h = ctypes.c_void_p()
        sh = stream_handle(stream, self.device)
        if sl is None:
            check(lib().prng_table_create(ctypes.byref(self._h), handles, len(self.gens), rows, n, sv,
                                          self._work.data_ptr(), self._work.numel(), sh))
        else:
            check(lib().prng_table_create_ex(ctypes.byref(self._h), handles, len(self.gens), rows, n,
                                             ctypes.byref(sl), self._work.data_ptr(), self._work.numel(), sh))

    @staticmethod
    def tune_segments(gens: list[Generator], gen_idx, streams, counts, dtypes, repeats: int = 1, device=None,
                      stream=None) -> tuple[dict, float]:
        """Segment lengths (numbers per lane) picked by prng_table_tune_segments for
        these rows, and the time of one tuned run with them; every stream state is
        left where it was."""
        gens = list(gens)
        device = gens[0].device if device is None else torch.device(device)
        buf, rows, n, _, handles = _rows(gens, device, gen_idx, streams, counts, dtypes)
        wb = lib().prng_table_tune_work_bytes(handles, len(gens), rows, n)
        if wb == 0:
            check(-1)
        work = torch.empty(wb, dtype=torch.uint8, device=device)
        best, ms = SegLengths(), ctypes.c_float()
        check(lib().prng_table_tune_segments(handles, len(gens), rows, n, int(repeats), work.data_ptr(), work.numel(),
                                             stream_handle(stream, device), ctypes.byref(best), ctypes.byref(ms)))
        del buf
        return {"lane": best.lane, "ranmar": best.ranmar, "mt": best.mt}, ms.value

    def seg_lengths(self) -> dict:
        sl = SegLengths()
        check(lib().prng_table_seg_lengths(self._h, ctypes.byref(sl)))
        return {"lane": sl.lane, "ranmar": sl.ranmar, "mt": sl.mt}

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
