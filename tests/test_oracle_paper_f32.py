"""Pins of the oracle's paper-literal single-precision conversions.

The paper's kernels scale integers to floats with fp32 constants: x / 2147483647.0
(GGL), w / 4294967295.0 (XOR128), Z * 2^-31 (RANECU), X * 2^-24 (RANMAR, RANLUX)
and (y + 0.5) / 4294967296.0 (MT19937).  The expected values here are worked
out in exact rational arithmetic with an independent round-to-nearest-even to
24 significant bits: the two fp32 constants of GGL and XOR128 round to 2^31
and 2^32, so those divisions are exact and the only rounding is that of the
integer; MT19937 rounds twice (the integer, then the sum with 0.5).
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def rne(q: Fraction, bits: int = 24) -> Fraction:
    """q > 0 rounded to `bits` significant bits, ties to even."""
    if q == 0:
        return q
    e = 0
    while q >= 2 ** (bits - e):   # find e with 2^(bits-1) <= q * 2^e < 2^bits
        e -= 1
    while q * 2 ** e < 2 ** (bits - 1):
        e += 1
    m = q * Fraction(2) ** e
    lo = m.numerator // m.denominator
    rest = m - lo
    if rest > Fraction(1, 2) or (rest == Fraction(1, 2) and lo % 2 == 1):
        lo += 1
    return Fraction(lo) / Fraction(2) ** e


def expected(kind, u):
    u = Fraction(u)
    if kind == "ggl" or kind == "ranecu":
        return rne(u) / 2 ** 31
    if kind == "xor128":
        return rne(u) / 2 ** 32
    if kind in ("ranmar", "ranlux"):
        return u / 2 ** 24
    if kind == "mt19937":
        return rne(rne(u) + Fraction(1, 2)) / 2 ** 32
    raise ValueError(kind)


TOP = {"ggl": 2**31 - 2, "xor128": 2**32 - 1, "ranecu": 2147483562, "ranmar": 2**24 - 1, "ranlux": 2**24 - 1,
       "mt19937": 2**32 - 1}
LOW = {"ggl": 1, "xor128": 0, "ranecu": 1, "ranmar": 0, "ranlux": 0, "mt19937": 0}


def cases(kind):
    top, low = TOP[kind], LOW[kind]
    rng = np.random.default_rng(3)
    us = {low, low + 1, top, top - 1, 2**24 - 1, 2**24, 2**24 + 1, 2**25 + 1, 2**25 + 2, 2**25 + 3,
          2**31 - 64, 2**31 - 65, 2**31 - 63, 2**31 - 128, 2**31 - 192, 2**32 - 128, 2**32 - 129, 2**32 - 256 - 128}
    us |= set(int(v) for v in rng.integers(low, top + 1, 400))
    return sorted(u for u in us if low <= u <= top)


@pytest.mark.parametrize("kind", list(TOP))
def test_paper_f32_exact_values(kind):
    for u in cases(kind):
        got = oracle.to_f32_paper(kind, u)
        assert Fraction(got) == expected(kind, u), (kind, u, got)


def test_paper_f32_endpoints():
    assert oracle.to_f32_paper("ggl", 2**31 - 2) == 1.0       # reaches 1.0
    assert oracle.to_f32_paper("xor128", 2**32 - 1) == 1.0
    assert oracle.to_f32_paper("mt19937", 2**32 - 1) == 1.0
    assert oracle.to_f32_paper("ranecu", 2147483562) < 1.0     # 2^31 - 86 rounds down
    assert oracle.to_f32_paper("mt19937", 0) == 2.0 ** -33      # never 0 for MT19937
    assert oracle.to_f32_paper("xor128", 0) == 0.0
    assert oracle.to_f32_paper("ranlux", 2**24 - 1) == 1 - 2.0 ** -24


@pytest.mark.parametrize("kind", list(TOP))
def test_paper_f32_monotone(kind):
    us = cases(kind)
    vals = [oracle.to_f32_paper(kind, u) for u in us]
    assert all(a <= b for a, b in zip(vals, vals[1:]))


@pytest.mark.parametrize("kind", list(TOP))
def test_generate_uses_paper_rule(kind):
    from paper_1003_1898_amd import inputs
    st = oracle.init(kind, inputs.seed_words(kind, 1, 3))
    u = oracle.generate(kind, st.copy(), 500, "u32")
    f = oracle.generate(kind, st.copy(), 500, "f32_paper")
    ref = np.array([[oracle.to_f32_paper(kind, int(x)) for x in row] for row in u], dtype=np.float32)
    assert np.array_equal(f, ref)


def test_lcg48_has_no_paper_rule():
    assert oracle.to_f32_paper("drand48", 5) == -1.0
