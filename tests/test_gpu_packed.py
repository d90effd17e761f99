"""Four-way interleaved output (prng_generate_packed4), the layout of the
paper's four-subthread kernels: element i of stream s at
out[((s / 4) * count + i) * 4 + s % 4], bit-exact with the oracle."""
import numpy as np
import pytest

from paper_1003_1898_amd import inputs
from paper_1003_1898_amd._capi import PrngError
from paper_1003_1898_amd.generator import Generator

from mirror import bits

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["ggl", "ranecu", "ranmar", "xor128", "ranlux", "drand48"])
def test_packed_matches_oracle(oracle, kind):
    print(f"\n[packed] {kind}", flush=True)
    for n, sched in ((256, [(4096, "f32"), (4096, "u32")]), (100, [(1, "u32"), (97, "f32"), (1000, "u32")]),
                     (4, [(5, "f32"), (300, "u32")])):
        seeds = inputs.seed_words(kind, 31, n)
        g = Generator(kind, n, seed_words=seeds, p=223)
        st = oracle.init(kind, seeds)
        for count, dt in sched + ([] if kind == "drand48" else [(333, "f32_paper")]):
            got = g.generate_packed4(count, dt).cpu().numpy()
            assert got.shape == (n // 4, count, 4)
            got = got.transpose(0, 2, 1).reshape(n, count)
            ref = oracle.generate(kind, st, count, dt, p=223, threads=8)
            assert np.array_equal(bits(got), bits(ref)), f"{kind} n={n} count={count} {dt}"
        assert np.array_equal(g.state_words(), st)
        g.close()


def test_packed_rejections():
    with pytest.raises(PrngError, match="EUNSUPPORTED"):
        Generator("mt19937", 4, seed=1).generate_packed4(10, "u32")
    with pytest.raises(PrngError, match="EINVAL"):
        Generator("ggl", 6, seed=1).generate_packed4(10, "u32")     # not a multiple of 4
    with pytest.raises((PrngError, KeyError)):
        Generator("ggl", 8, seed=1).generate_packed4(10, "f64")
    with pytest.raises(PrngError, match="EUNSUPPORTED"):
        Generator("rannyu", 8, seed=1).generate_packed4(10, "f32_paper")
