"""prng_generate_noalloc, the entry point that allocates nothing (RANLUX's
pre-launch state copy in the library's static device array), called through
the C ABI and compared with prng_generate bit for bit on two calls in a row,
the second smaller, and with the oracle."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1003_1898_amd import inputs
from paper_1003_1898_amd._capi import PrngError, check, lib
from paper_1003_1898_amd.generator import Generator, stream_handle

from mirror import bits

pytestmark = pytest.mark.gpu


def noalloc(g, count, dtype_id, torch_dtype):
    out = torch.empty((g.n, count), dtype=torch_dtype, device=g.device)
    check(lib().prng_generate_noalloc(g.handle, count, dtype_id, out.data_ptr(), out.numel() * out.element_size(),
                                      stream_handle(None, g.device)))
    return out


@pytest.mark.parametrize("kind,n,p", [("ranlux", 1000, 223), ("ranlux", 65536, 24), ("xor128", 1000, 0),
                                      ("ggl", 300, 0), ("mt19937", 64, 0)])
def test_noalloc_equals_generate(oracle, kind, n, p):
    print(f"\n[noalloc] {kind} n={n} p={p}", flush=True)
    seeds = inputs.seed_words(kind, 91, n)
    a = Generator(kind, n, seed_words=seeds, p=p or 223)
    b = Generator(kind, n, seed_words=seeds, p=p or 223)
    st = oracle.init(kind, seeds[:64])
    for count, dt, tdt in [(6000, 2, torch.float32), (1700, 1, torch.uint32)]:  # the second call smaller
        ref = a.generate(count, {1: "u32", 2: "f32"}[dt])
        got = noalloc(b, count, dt, tdt)
        torch.cuda.synchronize()
        assert np.array_equal(bits(got.cpu().numpy()), bits(ref.cpu().numpy())), f"count {count}"
        want = oracle.generate(kind, st, count, {1: "u32", 2: "f32"}[dt], p=p or 223)
        assert np.array_equal(bits(got[:64].cpu().numpy()), bits(want))
    assert np.array_equal(a.state_words(), b.state_words())


def test_noalloc_rejects_objects_beyond_the_scratch():
    g = Generator("ranlux", 81000, seed=5, p=223)  # 81000 x 104 B > 8 MiB
    out = torch.empty((81000, 100), dtype=torch.float32, device=g.device)
    rc = lib().prng_generate_noalloc(g.handle, 100, 2, out.data_ptr(), out.numel() * 4, stream_handle(None, g.device))
    assert rc == -1
    assert b"static scratch" in lib().prng_last_error()
