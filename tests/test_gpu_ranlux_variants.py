"""RANLUX with the lag table in an indexed LDS array or in HBM (the paper's
temporary-array and global-buffer implementations, Section 3.6, Table 3):
bit-exact with the oracle and with the register path, at the classic and the
planar luxury levels, from streams standing anywhere in a luxury block."""
import numpy as np
import pytest

from paper_1003_1898_amd import inputs
from paper_1003_1898_amd._capi import PrngError
from paper_1003_1898_amd.generator import Generator

from mirror import bits

pytestmark = pytest.mark.gpu

LEVELS = [24, 48, 97, 223, 389, 120, 240, 408, 100]


@pytest.mark.parametrize("lag", ["lds", "hbm"])
@pytest.mark.parametrize("p", LEVELS)
def test_variant_matches_oracle(oracle, lag, p):
    print(f"\n[ranlux {lag}] p={p}", flush=True)
    n = 130
    seeds = inputs.seed_words("ranlux", 900 + p, n)
    st = oracle.init("ranlux", seeds)
    for s in range(n):  # streams at every position of a luxury block
        row = st[s:s + 1].copy()
        oracle.generate("ranlux", row, s % 49, "u32", p=p)
        st[s] = row[0]
    g = Generator("ranlux", n, seed_words=seeds, p=p)
    g.set_state(Generator.blob_from_words("ranlux", p, st))
    for count, dt in [(1, "u32"), (95, "f32"), (97, "f64"), (1000, "u32"), (2, "f64"), (4096, "f32")]:
        got = bits(g.generate(count, dt, lag=lag).cpu().numpy())
        ref = bits(oracle.generate("ranlux", st, count, dt, p=p, threads=8))
        assert np.array_equal(got, ref), f"{lag} p={p} count={count} {dt}"
        assert np.array_equal(g.state_words(), st), f"{lag} p={p} state after count={count}"


@pytest.mark.parametrize("p", [24, 223, 408])
def test_three_variants_agree(p):
    n = 300
    seeds = inputs.seed_words("ranlux", 7, n)
    outs, states = [], []
    for lag in ("registers", "lds", "hbm"):
        g = Generator("ranlux", n, seed_words=seeds, p=p)
        a = g.generate(2000, "u32", lag=lag).cpu().numpy()
        b = g.generate(777, "f64", lag=lag).cpu().numpy()
        outs.append((bits(a), bits(b)))
        states.append(g.state_words())
    for o, s in zip(outs[1:], states[1:]):
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
        assert np.array_equal(s, states[0])


def test_variant_rejections():
    g = Generator("ggl", 4, seed=1)
    with pytest.raises(PrngError):
        g.generate(10, "u32", lag="lds")      # not RANLUX
    r = Generator("ranlux", 4, seed=1, p=223)
    with pytest.raises(PrngError):
        r.generate(10, "f32_paper", lag="hbm")
