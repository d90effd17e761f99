"""RANLUX plain generation cut into jumped segments (several wavefronts per
SIMD, chunk grid aligned to the output rows): bit-exact with the oracle for
streams standing at every position of their luxury block, uniform or mixed
across streams, at several luxury levels and segment counts."""
import numpy as np
import pytest

from paper_1003_1898_amd import inputs
from paper_1003_1898_amd.generator import Generator

from mirror import bits

pytestmark = pytest.mark.gpu


def at_positions(oracle, n, p, ks, master):
    """Generator and oracle states with stream s advanced to block position ks[s]."""
    seeds = inputs.seed_words("ranlux", master, n)
    st = oracle.init("ranlux", seeds)
    for s in range(n):
        if ks[s]:
            row = st[s:s + 1].copy()
            oracle.generate("ranlux", row, int(ks[s]), "u32", p=p)
            st[s] = row[0]
    g = Generator("ranlux", n, seed_words=seeds, p=p)
    g.set_state(Generator.blob_from_words("ranlux", p, st))
    return g, st


@pytest.mark.parametrize("k0", [0, 5, 8, 16, 23, 24])
@pytest.mark.parametrize("p", [223, 24, 100])
def test_uniform_block_position(oracle, k0, p):
    print(f"\n[lux plain] k0={k0} p={p}", flush=True)
    n = 200
    g, st = at_positions(oracle, n, p, [k0] * n, 500 + k0)
    for count, dt in [(20001, "u32"), (9999, "f32"), (7777, "f64"), (3072, "f32"), (1, "u32")]:
        got = bits(g.generate(count, dt).cpu().numpy())
        ref = bits(oracle.generate("ranlux", st, count, dt, p=p, threads=8))
        assert np.array_equal(got, ref), f"k0={k0} p={p} count={count} {dt}"
        assert np.array_equal(g.state_words(), st), f"k0={k0} p={p} state after count={count} {dt}"


@pytest.mark.parametrize("n", [1, 63, 130, 1000])
def test_mixed_block_positions(oracle, n):
    print(f"\n[lux plain mixed] n={n}", flush=True)
    p = 389
    g, st = at_positions(oracle, n, p, [s % 25 for s in range(n)], 77 + n)
    for count, dt in [(30000, "f32"), (12345, "f64"), (4097, "u32"), (16384, "f32_paper")]:
        got = bits(g.generate(count, dt).cpu().numpy())
        ref = bits(oracle.generate("ranlux", st, count, dt, p=p, threads=8))
        assert np.array_equal(got, ref), f"n={n} count={count} {dt}"
        assert np.array_equal(g.state_words(), st)
