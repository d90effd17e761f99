"""Plain generation of GGL, RANECU, DRAND48 and RANNYU, where each wavefront
covers one stream and lane l takes positions 4 l .. 4 l + 3 of every block
of 256: counts around block and quad boundaries, rows that are not 16-byte
aligned (odd counts), every dtype, final states; bit-exact with the oracle."""
import numpy as np
import pytest

from paper_1003_1898_amd import inputs
from paper_1003_1898_amd.generator import Generator

from mirror import bits

pytestmark = pytest.mark.gpu

COUNTS = [1, 2, 3, 4, 5, 127, 128, 129, 255, 256, 257, 383, 511, 512, 513, 767, 769, 1021, 4099]


@pytest.mark.parametrize("kind", ["ggl", "ranecu", "drand48", "rannyu"])
def test_leapfrog_boundaries(oracle, kind):
    print(f"\n[leap] {kind}", flush=True)
    n = 37
    seeds = inputs.seed_words(kind, 808, n)
    g = Generator(kind, n, seed_words=seeds)
    st = oracle.init(kind, seeds)
    dts = ["u32", "f32", "f64"] + (["f32_paper"] if kind in ("ggl", "ranecu") else [])
    for i, count in enumerate(COUNTS):
        dt = dts[i % len(dts)]
        got = bits(g.generate(count, dt).cpu().numpy())
        ref = bits(oracle.generate(kind, st, count, dt))
        assert np.array_equal(got, ref), f"{kind} count={count} {dt}"
        assert np.array_equal(g.state_words(), st), f"{kind} state after count={count} {dt}"
