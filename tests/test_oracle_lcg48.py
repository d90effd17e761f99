"""Pins of the oracle's 48-bit linear congruential generators (Appendix A.1).

DRAND48 is checked draw by draw against the C library's own jrand48/erand48
(the same recurrence, implemented independently), RANNYU and DRAND48 against
the closed forms X_n = a^n X_0 (+ c (a^n - 1) / (a - 1)) mod 2^48 evaluated with
Python integers, and both against the periods their low bits must have.
"""
import ctypes
import ctypes.util

import numpy as np
import pytest

import oracle

M48 = 1 << 48
A_DRAND48, C_DRAND48 = 25214903917, 11
A_RANNYU = 31167285


def x_of(state):
    return int(state[0]) | (int(state[1]) << 32)


def closed_form(a, c, x0, n):
    """a^n x0 + c (1 + a + ... + a^(n-1)) mod 2^48, the sum taken exactly."""
    an = pow(a, n, M48)
    geo = (pow(a, n, (a - 1) * M48) - 1) // (a - 1)
    return (an * x0 + c * geo) % M48


@pytest.fixture(scope="module")
def libc():
    name = ctypes.util.find_library("c") or "libc.so.6"
    lib = ctypes.CDLL(name)
    for f in ("jrand48", "nrand48"):
        getattr(lib, f).argtypes = [ctypes.POINTER(ctypes.c_ushort)]
        getattr(lib, f).restype = ctypes.c_long
    lib.erand48.argtypes = [ctypes.POINTER(ctypes.c_ushort)]
    lib.erand48.restype = ctypes.c_double
    return lib


def xsubi(x):
    return (ctypes.c_ushort * 3)(x & 0xFFFF, (x >> 16) & 0xFFFF, (x >> 32) & 0xFFFF)


@pytest.mark.parametrize("x0", [0, 1, 0x330E, (20240607 << 16) | 0x330E, M48 - 1, 0x123456789ABC])
def test_drand48_matches_libc(libc, x0):
    st = oracle.init("drand48", [x0])[0]
    xs = xsubi(x0)
    got = oracle.next_draws("drand48", st, 3000)
    ref = np.array([libc.jrand48(xs) & 0xFFFFFFFF for _ in range(3000)], dtype=np.uint32)
    assert np.array_equal(got, ref)
    # erand48 returns X / 2^48 after one more step; nrand48 the top 31 bits
    u = oracle.next_draws("drand48", st, 1)[0]
    assert libc.erand48(xs) * M48 == x_of(st)
    assert int(u) == x_of(st) >> 16
    assert libc.nrand48(xs) == int(oracle.next_draws("drand48", st, 1)[0]) >> 1


@pytest.mark.parametrize("kind,a,c", [("drand48", A_DRAND48, C_DRAND48), ("rannyu", A_RANNYU, 0)])
def test_closed_form(kind, a, c):
    rng = np.random.default_rng(11)
    for x0 in [1, 3, 0x5DEECE66D | 1, M48 - 1] + [int(v) | 1 for v in rng.integers(0, M48, 4, dtype=np.uint64)]:
        st = oracle.init(kind, [x0])[0]
        done = 0
        for n in (1, 2, 7, 1000, 65537):
            draws = oracle.next_draws(kind, st, n - done)
            done = n
            x = closed_form(a, c, x0, n)
            assert x_of(st) == x, (kind, x0, n)
            assert int(draws[-1]) == x >> 16
            # the draw before it as well: a plausible off-by-one lands here
            if n - 1 >= 1 and len(draws) >= 2:
                assert int(draws[-2]) == closed_form(a, c, x0, n - 1) >> 16


def test_low_bit_periods():
    """The low k bits of an LCG modulo 2^48 are an LCG modulo 2^k: with an odd
    increment and a = 1 mod 4 their period is 2^k (DRAND48); with c = 0,
    a = 5 mod 8 and an odd seed it is 2^(k-2) (RANNYU)."""
    k = 12
    mask = (1 << k) - 1
    for kind, period in (("drand48", 1 << k), ("rannyu", 1 << (k - 2))):
        st = oracle.init(kind, [0x9E3779B97F4B])[0]  # odd
        low0 = int(st[0]) & mask
        seen = []
        for step in range(1, period + 1):
            oracle.next_draws(kind, st, 1)
            if int(st[0]) & mask == low0:
                seen.append(step)
        assert seen == [period], (kind, seen[:4])


def test_seed_ranges():
    oracle.init("drand48", [0])
    oracle.init("drand48", [M48 - 1])
    with pytest.raises(ValueError):
        oracle.init("drand48", [M48])
    with pytest.raises(ValueError):
        oracle.init("rannyu", [2])      # the multiplicative generator needs an odd seed
    with pytest.raises(ValueError):
        oracle.init("rannyu", [M48 + 1])
    st = oracle.init("rannyu", [M48 - 1])[0]
    assert int(st[0]) == 0xFFFFFFFF and int(st[1]) == 0xFFFF


def test_conversions_use_the_top_bits():
    """f32 keeps X's top 24 bits exactly; f64 joins the top 27 and 26 bits of
    two successive draws (the shared rule for 32-bit draws)."""
    for kind in ("drand48", "rannyu"):
        st = oracle.init(kind, [0xABCDEF123457])
        a = st.copy()
        u = oracle.next_draws(kind, a[0], 4)
        f = oracle.generate(kind, st.copy(), 4, "f32")[0]
        assert np.array_equal(f, (u >> 8).astype(np.float64) * 2.0**-24)
        d = oracle.generate(kind, st.copy(), 2, "f64")[0]
        ref = [((int(u[2 * i]) >> 5) * 2**26 + (int(u[2 * i + 1]) >> 6)) * 2.0**-53 for i in range(2)]
        assert list(d) == ref
