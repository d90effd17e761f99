"""Host-side checks of the product library (no GPU needed).

The shared library loads, exports every entry point declared in include/prng.h,
its native seeding agrees with the seed-tuple generator, and argument checks
that precede any device work return the documented codes.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1003_1898_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KINDS = ["ggl", "xor128", "ranecu", "ranmar", "ranlux", "mt19937", "drand48", "rannyu"]


def _header_functions():
    src = open(os.path.join(ROOT, "include", "prng.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(prng_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(prnglib):
    names = _header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(prnglib, n), f"{n} declared in include/prng.h but not exported"


def test_binding_declares_every_symbol():
    from paper_1003_1898_amd._capi import SIGNATURES
    assert set(_header_functions()) == set(SIGNATURES)


def test_splitmix64_known_answer():
    # published first output of SplitMix64 seeded with 0
    assert int(inputs.splitmix64(0, 1)[0]) == 0xE220A8397B1DCDAF


@pytest.mark.parametrize("kind", KINDS)
def test_native_seed_words_match_input_module(prnglib, kind):
    from paper_1003_1898_amd.generator import seed_words
    a = seed_words(kind, 42, 3000)
    b = inputs.seed_words(kind, 42, 3000)
    assert np.array_equal(a, b)
    assert len({tuple(r) for r in a.tolist()}) == 3000


@pytest.mark.parametrize("kind", KINDS)
def test_seed_tuples_are_accepted_by_the_oracle(oracle, kind):
    w = inputs.seed_words(kind, 7, 2000)
    oracle.init(kind, w)  # raises on any out-of-range tuple


def test_seed_dedup_redraws():
    # GGL tuples come from 1 raw word each; force a collision check on many streams
    w = inputs.seed_words("mt19937", 1, 20000)
    assert len(set(w[:, 0].tolist())) == 20000


def test_enum_values_match_header():
    """The binding's kind, dtype and lag-table numbers are the ones include/prng.h declares."""
    src = open(os.path.join(ROOT, "include", "prng.h")).read()
    from paper_1003_1898_amd.generator import LAG_VARIANTS
    for name, v in inputs.KIND_IDS.items():
        assert re.search(rf"PRNG_{name.upper()}\s*=\s*{v}\b", src), name
    for name, v in inputs.DTYPE_IDS.items():
        assert re.search(rf"PRNG_{name.upper()}\s*=\s*{v}\b", src), name
    for name, v in LAG_VARIANTS.items():
        assert re.search(rf"PRNG_LAG_{name.upper()}\s*=\s*{v}\b", src), name


@pytest.mark.parametrize("kind", KINDS)
def test_word_counts_match_oracle(prnglib, oracle, kind):
    k = inputs.kind_id(kind)
    assert prnglib.prng_state_words(k) == oracle.state_words(kind)
    assert prnglib.prng_seed_tuple_words(k) == oracle.seed_words(kind)
    assert prnglib.prng_state_bytes(k, 1000) >= 1000 * oracle.state_words(kind) * 4
    assert prnglib.prng_state_words(99) < 0 and prnglib.prng_state_bytes(99, 10) == 0


def _create_rc(prnglib, kind, p, seeds):
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    h = ctypes.c_void_p()
    rc = prnglib.prng_create(ctypes.byref(h), inputs.kind_id(kind), p, seeds.shape[0],
                             seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), None, 0, None)
    return rc, prnglib.prng_last_error().decode()


@pytest.mark.parametrize("kind,bad", [("ggl", [[0]]), ("ggl", [[2147483647]]), ("xor128", [[0, 0, 0, 0]]),
                                      ("xor128", [[2**32, 1, 1, 1]]), ("ranecu", [[0, 5]]),
                                      ("ranecu", [[5, 2147483399]]), ("ranmar", [[31329, 5]]),
                                      ("ranmar", [[5, 30082]]), ("ranlux", [[0]]), ("ranlux", [[2147483563]]),
                                      ("mt19937", [[2**32]]), ("drand48", [[2**48]]), ("rannyu", [[2]]),
                                      ("rannyu", [[2**48 + 1]])])
def test_create_rejects_out_of_range_seeds(prnglib, kind, bad):
    rc, msg = _create_rc(prnglib, kind, 223, bad)
    assert rc == -2 and "outside the valid range" in msg


def test_create_rejects_bad_arguments(prnglib):
    assert _create_rc(prnglib, "ranlux", 23, [[5]])[0] == -1      # p below 24
    assert _create_rc(prnglib, "ggl", 0, np.zeros((0, 1)))[0] == -1  # no streams
    rc, msg = _create_rc(prnglib, "ggl", 0, [[5]])                 # valid seeds, no device buffer
    assert rc == -1 and "d_state" in msg
    h = ctypes.c_void_p()
    assert prnglib.prng_create(ctypes.byref(h), 99, 0, 1, None, None, 0, None) == -1  # unknown kind


def test_null_object_calls(prnglib):
    assert prnglib.prng_generate(None, 10, 1, None, 0, None) == -1
    assert prnglib.prng_generate_noalloc(None, 10, 1, None, 0, None) == -1
    assert prnglib.prng_generate_packed4(None, 10, 1, None, 0, None) == -1
    assert prnglib.prng_ranlux_generate_variant(None, 1, 10, 1, None, 0, None) == -1
    assert prnglib.prng_fused_sum_hist(None, 10, None, None, None) == -1
    assert prnglib.prng_get_state(None, None, 0, None) == -1
    assert prnglib.prng_blob_bytes(None) == 0
    prnglib.prng_destroy(None)


def test_table_calls_without_objects(prnglib):
    """The table entry points reject missing objects and arrays on the host."""
    from paper_1003_1898_amd._capi import SegLengths
    sl = SegLengths(0, 0, 0)
    assert prnglib.prng_table_seg_lengths(None, ctypes.byref(sl)) == -1
    assert prnglib.prng_table_work_bytes_ex(None, 0, None, 0, None) == 0
    assert prnglib.prng_table_tune_work_bytes(None, 0, None, 0) == 0
    h = ctypes.c_void_p()
    assert prnglib.prng_table_create_ex(ctypes.byref(h), None, 0, None, 0, ctypes.byref(sl), None, 0, None) == -1
    assert prnglib.prng_table_tune_segments(None, 0, None, 0, 1, None, 0, None, None, None) == -1
    assert prnglib.prng_table_tune_segments(None, 0, None, 0, 1, None, 0, None, ctypes.byref(sl), None) == -1
    assert prnglib.prng_table_set_config(None, 256, 512, 0) == -1


def test_mixed_table_workload_shape():
    t = inputs.mixed_table()
    assert len(t["kind"]) == 10000
    assert t["count"].min() >= 64 and t["count"].max() <= 2**20
    assert set(np.unique(t["kind"])) == set(range(1, 7)) and set(np.unique(t["dtype"])) == {1, 2, 3}
    mean = inputs.expected_log_uniform_mean(6, 20)
    assert abs(t["count"].mean() / mean - 1) < 0.1


def test_request_schedule_shape():
    r = inputs.request_schedule(5000, rate_per_s=1000.0)
    assert np.all(np.diff(r["t_arrival"]) >= 0)
    assert abs(r["t_arrival"][-1] / 5.0 - 1) < 0.1
    assert r["count"].min() >= 256 and r["count"].max() <= 2**22
