"""Seeded synthetic inputs: per-stream seed tuples and the mixed workloads.

This module holds none of the generators' arithmetic.  It turns a master seed
into per-stream seed tuples inside each generator's valid seed range, and it
draws the synthetic stream tables (mixed generators, log-uniform lengths) and
request schedules (Poisson arrivals) of the batched and served workloads.  Both
the HIP library and the CPU oracle consume its outputs, so neither side ever
feeds the other.

Seeding rule (the paper only says that seeds are chosen at random and that
distinct RANMAR seed pairs give independent sequences, Sections 3.2 and 3.5):

* ``key_s`` is output ``s`` (0-based) of SplitMix64 started at ``master``;
* ``w_j`` is output ``j`` of SplitMix64 started at ``key_s``;
* attempt ``t`` of stream ``s`` maps the raw words ``w_{tR} .. w_{tR+R-1}``
  (R raw words per attempt) into the generator's range:

  ====== ===== =====================================================
  kind   R     tuple
  ====== ===== =====================================================
  GGL    1     x0 = 1 + w0 mod (2^31 - 2)
  XOR128 2     (lo w0, hi w0, lo w1, hi w1); last word 1 if all zero
  RANECU 2     s1 = 1 + w0 mod 2147483562, s2 = 1 + w1 mod 2147483398
  RANMAR 2     ij = w0 mod 31329, kl = w1 mod 30082
  RANLUX 1     v = 1 + w0 mod 2147483562
  MT     1     s = lo w0
  DRAND48 1    X_0 = w0 mod 2^48
  RANNYU 1     X_0 = (w0 mod 2^48) | 1  (odd: a multiplicative generator)
  ====== ===== =====================================================

* a tuple equal to one already given to an earlier stream of the same call is
  replaced by the next attempt, so every stream of one generator object has a
  distinct seed tuple.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

KIND_IDS = {"ggl": 1, "xor128": 2, "ranecu": 3, "ranmar": 4, "ranlux": 5, "mt19937": 6,
            "drand48": 7, "rannyu": 8}
KIND_NAMES = {v: k for k, v in KIND_IDS.items()}
SEED_TUPLE_WORDS = {1: 1, 2: 4, 3: 2, 4: 2, 5: 1, 6: 1, 7: 1, 8: 1}
RAW_WORDS = {1: 1, 2: 2, 3: 2, 4: 2, 5: 1, 6: 1, 7: 1, 8: 1}
DTYPE_IDS = {"u32": 1, "f32": 2, "f64": 3, "f32_paper": 4}


def kind_id(kind) -> int:
    return KIND_IDS[kind] if isinstance(kind, str) else int(kind)


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(state: int, n: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+n-1 (0-based) of SplitMix64 seeded with `state`."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        z = np.uint64(state) + idx * GAMMA
        return _mix(z)


def _raw(keys: np.ndarray, first: int, count: int) -> np.ndarray:
    """Raw words w_first .. w_{first+count-1} of every stream key -> (n, count)."""
    with np.errstate(over="ignore"):
        idx = np.arange(first + 1, first + count + 1, dtype=np.uint64)
        z = keys[:, None] + idx[None, :] * GAMMA
        return _mix(z)


def _map(kind: int, raw: np.ndarray) -> np.ndarray:
    w0 = raw[:, 0]
    lo = np.uint64(0xFFFFFFFF)
    if kind == 1:
        return (np.uint64(1) + w0 % np.uint64(2147483646))[:, None]
    if kind == 2:
        w1 = raw[:, 1]
        t = np.stack([w0 & lo, w0 >> np.uint64(32), w1 & lo, w1 >> np.uint64(32)], axis=1)
        zero = (t == 0).all(axis=1)
        t[zero, 3] = 1
        return t
    if kind == 3:
        return np.stack([np.uint64(1) + w0 % np.uint64(2147483562),
                         np.uint64(1) + raw[:, 1] % np.uint64(2147483398)], axis=1)
    if kind == 4:
        return np.stack([w0 % np.uint64(31329), raw[:, 1] % np.uint64(30082)], axis=1)
    if kind == 5:
        return (np.uint64(1) + w0 % np.uint64(2147483562))[:, None]
    if kind == 6:
        return (w0 & lo)[:, None]
    if kind in (7, 8):
        x = w0 & np.uint64((1 << 48) - 1)
        return (x | np.uint64(1) if kind == 8 else x)[:, None]
    raise ValueError(f"unknown generator kind {kind}")


def seed_words(kind, master: int, n_streams: int) -> np.ndarray:
    """(n_streams, tuple_words) uint64 seed tuples, distinct within the call."""
    k = kind_id(kind)
    R = RAW_WORDS[k]
    keys = splitmix64(master, n_streams)
    out = _map(k, _raw(keys, 0, R))
    seen = set()
    for s in range(n_streams):
        t = 0
        tup = tuple(out[s].tolist())
        while tup in seen:
            t += 1
            tup = tuple(_map(k, _raw(keys[s:s + 1], t * R, R))[0].tolist())
        seen.add(tup)
        out[s] = tup
    return out


def mixed_table(n_streams: int = 10000, master: int = 4242, len_lo: int = 6, len_hi: int = 20):
    """Synthetic stream table of the batched workload.

    Stream s takes SplitMix64(master) outputs 3s, 3s+1, 3s+2: generator
    kind = 1 + w0 mod 6, length = floor(2^(len_lo + (len_hi-len_lo) U)) with
    U = (w1 >> 11) 2^-53 (log-uniform in [2^len_lo, 2^len_hi]), dtype = 1 + w2 mod 3.
    Returns dict of arrays: kind, count, dtype (all int64)."""
    w = splitmix64(master, 3 * n_streams).reshape(n_streams, 3)
    kind = (w[:, 0] % np.uint64(6)).astype(np.int64) + 1
    u = (w[:, 1] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    count = np.floor(2.0 ** (len_lo + (len_hi - len_lo) * u)).astype(np.int64)
    count = np.clip(count, 2 ** len_lo, 2 ** len_hi)
    dtype = (w[:, 2] % np.uint64(3)).astype(np.int64) + 1
    return {"kind": kind, "count": count, "dtype": dtype}


def request_schedule(n_requests: int, rate_per_s: float, n_states: int = 65536, master: int = 4243,
                     cnt_lo: int = 8, cnt_hi: int = 22):
    """Open-loop Poisson request schedule of the served workload.

    Request i takes SplitMix64(master) outputs 4i..4i+3: inter-arrival
    -ln(1-U0)/rate, stream = w1 mod n_states, count = floor(2^(cnt_lo +
    (cnt_hi-cnt_lo) U2)), dtype = 1 + w3 mod 3.  Returns dict of arrays:
    t_arrival (seconds from start, float64), stream, count, dtype (int64)."""
    w = splitmix64(master, 4 * n_requests).reshape(n_requests, 4)
    u0 = (w[:, 0] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    gaps = -np.log1p(-u0) / float(rate_per_s)
    t = np.cumsum(gaps)
    stream = (w[:, 1] % np.uint64(n_states)).astype(np.int64)
    u2 = (w[:, 2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    count = np.clip(np.floor(2.0 ** (cnt_lo + (cnt_hi - cnt_lo) * u2)).astype(np.int64),
                    2 ** cnt_lo, 2 ** cnt_hi)
    dtype = (w[:, 3] % np.uint64(3)).astype(np.int64) + 1
    return {"t_arrival": t, "stream": stream, "count": count, "dtype": dtype}


SERVED_KINDS = ("ggl", "xor128", "ranecu", "ranmar", "ranlux", "mt19937")


def served_split(stream: np.ndarray, n_states: int = 65536):
    """Resident state s of the served workload belongs to generator object
    s mod 6 (kinds in SERVED_KINDS order, RANLUX at p = 223) as its stream
    s div 6.  Returns (object index, stream within the object, streams per
    object)."""
    stream = np.asarray(stream, dtype=np.int64)
    per = [(n_states - k + 5) // 6 for k in range(6)]
    return stream % 6, stream // 6, per


def expected_log_uniform_mean(lo: int, hi: int) -> float:
    """E[2^(lo + (hi-lo) U)] for U uniform on [0, 1) (before flooring)."""
    a = (hi - lo) * math.log(2.0)
    return 2.0 ** lo * (math.exp(a) - 1.0) / a
