"""Plain generation of GGL, RANECU, DRAND48 and RANNYU, where lane l takes
positions 4 l .. 4 l + 3 of every block of 256: one wavefront per stream for
rows under 4096 positions, four wavefronts on four streams by quarters of
rows from 4096 on.  Counts around quad, block and quarter boundaries, stream
counts that are not a multiple of four, rows that are not 16-byte aligned
(odd counts), every dtype, final states, and rows of 2^26 positions (2^18
leaps per lane); bit-exact with the oracle."""
import numpy as np
import pytest

from paper_1003_1898_amd import inputs
from paper_1003_1898_amd.generator import Generator

from mirror import bits

pytestmark = pytest.mark.gpu

COUNTS = [1, 2, 3, 4, 5, 127, 128, 129, 255, 256, 257, 383, 511, 512, 513, 767, 769, 1021, 1023, 1024, 1025,
          2047, 3073, 4095, 4096, 4097, 4099, 8191, 13313, 16384]


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


@pytest.mark.parametrize("kind,dt", [("ggl", "u32"), ("ranecu", "f32"), ("drand48", "f64"), ("rannyu", "u32")])
def test_leapfrog_long_rows(oracle, kind, dt):
    """Rows of 2^26 + 1003 draws: 2^18 leaps per lane, then a ragged last block."""
    print(f"\n[leap long] {kind} {dt}", flush=True)
    n = 2
    seeds = inputs.seed_words(kind, 909, n)
    g = Generator(kind, n, seed_words=seeds)
    st = oracle.init(kind, seeds)
    per = 2 if dt == "f64" else 1
    count = ((1 << 26) + 1003) // per
    got = g.generate(count, dt).cpu().numpy()
    ref = oracle.generate(kind, st, count, dt)
    for idx in (0, 255, 256 * 64, 256 * 4096 + 17, count - 1000, count - 1):
        assert np.array_equal(bits(got[:, idx]), bits(ref[:, idx])), (kind, idx)
    assert np.array_equal(bits(got), bits(ref))
    assert np.array_equal(g.state_words(), st)
