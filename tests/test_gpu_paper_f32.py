"""The paper-literal single-precision rule (PRNG_F32_PAPER) on the GPU:
bit-exact with the oracle for every generator that has one, through the
full-chunk and ragged emission paths, including outputs that round to 1.0."""
import numpy as np
import pytest
import torch

from paper_1003_1898_amd import inputs
from paper_1003_1898_amd._capi import PrngError
from paper_1003_1898_amd.generator import Generator

from mirror import bits

pytestmark = pytest.mark.gpu

KINDS = ["ggl", "xor128", "ranecu", "ranmar", "ranlux", "mt19937"]


@pytest.mark.parametrize("kind", KINDS)
def test_paper_f32_matches_oracle(oracle, kind):
    print(f"\n[paper f32] {kind}", flush=True)
    for n, sched in ((256, [4096, 4096]), (100, [1, 95, 97, 624, 625, 1000, 4093]), (1, [7, 700])):
        seeds = inputs.seed_words(kind, 77, n)
        g = Generator(kind, n, seed_words=seeds, p=223)
        st = oracle.init(kind, seeds)
        for i, count in enumerate(sched):
            dt = "f32_paper" if i % 2 == 0 else "u32"
            got = bits(g.generate(count, dt).cpu().numpy())
            ref = bits(oracle.generate(kind, st, count, dt, p=223, threads=8))
            assert np.array_equal(got, ref), f"{kind} n={n} count={count} {dt}"
        assert np.array_equal(g.state_words(), st)
        g.close()


def test_paper_f32_reaches_one(oracle):
    """States whose next draw is the largest value: GGL x with 16807 x = 2^31 - 2
    (mod 2^31 - 1), XOR128 with x = 0 and w = 0xFFFFE000 (next w = 2^32 - 1)."""
    m = 2**31 - 1
    x = (2**31 - 2) * pow(16807, m - 2, m) % m
    cases = [("ggl", np.array([[x]], dtype=np.uint32)),
             ("xor128", np.array([[0, 5, 9, 0xFFFFE000]], dtype=np.uint32))]
    for kind, words in cases:
        g = Generator(kind, 1, seed=1)
        g.set_state(Generator.blob_from_words(kind, 0, words))
        out = g.generate(3, "f32_paper").cpu().numpy()
        ref = oracle.generate(kind, words.copy(), 3, "f32_paper")
        assert out[0, 0] == 1.0 and np.array_equal(bits(out), bits(ref)), (kind, out)


@pytest.mark.parametrize("kind", ["drand48", "rannyu"])
def test_paper_f32_unsupported_for_lcg48(kind):
    g = Generator(kind, 4, seed=3)
    with pytest.raises(PrngError, match="EUNSUPPORTED"):
        g.generate(10, "f32_paper")


def test_paper_f32_only_in_plain_generation():
    from paper_1003_1898_amd.table import StreamTable
    g = Generator("ggl", 4, seed=3)
    with pytest.raises(PrngError):
        StreamTable([g], [0], [0], [10], ["f32_paper"])
