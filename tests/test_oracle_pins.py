"""Pins of the CPU oracle against facts fixed outside it (no GPU needed).

* published known-answer values (tests/golden/known_answers.txt, each cited);
* independent engines of the C++ standard library, compiled and run here;
* closed forms and brute force (GGL period and power law, RANMAR C_n period);
* the XOR128 transition matrix of Appendix A.4.2 over GF(2);
* the RANLUX block structure of Appendix A.4.6 (kept r of every p SWB values);
* exactness and range of the conversions, and consistency of the fused sums.
"""
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    rows = []
    with open(os.path.join(HERE, "golden", "known_answers.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split(None, 6)
            kind, seed, p, r, idx, val = parts[:6]
            rows.append((kind, [int(x) for x in seed.split(",")], int(p), int(r), int(idx), int(val)))
    return rows


@pytest.mark.parametrize("kind,seed,p,r,idx,val", _golden())
def test_known_answers(oracle, kind, seed, p, r, idx, val):
    st = oracle.init(kind, [seed])[0]
    draws = oracle.next_draws(kind, st, idx, p=p or 223, r=r or 24)
    assert int(draws[idx - 1]) == val


@pytest.fixture(scope="module")
def stdlib(tmp_path_factory):
    """Sequences of libstdc++'s engines (compiled and run, never read)."""
    d = tmp_path_factory.mktemp("stdlib")
    exe = str(d / "engines")
    subprocess.run(["g++", "-O2", "-std=c++17", os.path.join(HERE, "stdlib_engines.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    seqs = {}
    for line in out.splitlines():
        name, seed, *vals = line.split()
        seqs[(name, int(seed))] = np.array([int(v) for v in vals], dtype=np.uint64)
    return seqs


SEEDS = [1, 12345, 19780503, 2147483562, 987654321]


@pytest.mark.parametrize("seed", SEEDS)
def test_ggl_matches_minstd_rand0(oracle, stdlib, seed):
    ref = stdlib[("minstd_rand0", seed)]
    st = oracle.init("ggl", [seed % 2147483647 or 1])[0]
    assert np.array_equal(oracle.next_draws("ggl", st, len(ref)).astype(np.uint64), ref)


@pytest.mark.parametrize("seed", SEEDS)
def test_mt19937_matches_std(oracle, stdlib, seed):
    ref = stdlib[("mt19937", seed)]
    st = oracle.init("mt19937", [seed])[0]
    assert np.array_equal(oracle.next_draws("mt19937", st, len(ref)).astype(np.uint64), ref)


@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("name,p,r", [("ranlux24_base", 24, 24), ("ranlux_p48", 48, 24), ("ranlux_p97", 97, 24),
                                      ("ranlux_p223", 223, 24), ("ranlux_p389", 389, 24), ("ranlux24", 223, 23)])
def test_ranlux_matches_std(oracle, stdlib, seed, name, p, r):
    """All five luxury levels of Appendix A.4.6 (and the standard's r = 23 variant)."""
    ref = stdlib[(name, seed)]
    st = oracle.init("ranlux", [seed])[0]
    assert np.array_equal(oracle.next_draws("ranlux", st, len(ref), p=p, r=r).astype(np.uint64), ref)


@pytest.mark.parametrize("seed", [(1, 1), (12345, 67890), (2147483562, 2147483398), (40014, 40692)])
def test_ranecu_components(oracle, stdlib, seed):
    """Each RANECU component equals an independent MLCG engine and a big-integer a*x mod m."""
    st = oracle.init("ranecu", [seed])[0]
    s1, s2 = [], []
    for _ in range(500):
        oracle.next_draws("ranecu", st, 1)
        s1.append(int(st[0]))
        s2.append(int(st[1]))
    x1, x2 = seed
    for i in range(500):
        x1 = 40014 * x1 % 2147483563
        x2 = 40692 * x2 % 2147483399
        assert (s1[i], s2[i]) == (x1, x2)
    if seed[0] in SEEDS:
        assert s1 == [int(v) for v in stdlib[("lcg40014", seed[0])][:500]]


def test_ranecu_combination_range(oracle):
    """Combined output lies in [1, m1-1] = [1, 2147483562] and takes both signs of s1 - s2."""
    st = oracle.init("ranecu", [[123, 2147483000]])[0]
    d = oracle.next_draws("ranecu", st, 20000).astype(np.int64)
    assert d.min() >= 1 and d.max() <= 2147483562


M1, M2, A1, A2 = 2147483563, 2147483399, 40014, 40692


def ranecu_prestate(v1: int, v2: int):
    """State (s1, s2) whose next component values are exactly (v1, v2): s_i = v_i * a_i^-1 mod m_i."""
    return [v1 * pow(A1, -1, M1) % M1, v2 * pow(A2, -1, M2) % M2]


def ranecu_combined(v1: int, v2: int) -> int:
    """Appendix A.4.1's combination as a residue: the one z in [1, m1-1] with z = v1 - v2 (mod m1-1)."""
    return (v1 - v2 - 1) % (M1 - 1) + 1


# next component values (v1, v2): equal (z = 0 -> m1-1), v1 < v2 (negative difference), v1 > v2, and the
# extremes of both ranges.  Expected values are written out by hand where the arithmetic is short.
RANECU_CASES = [
    (1, 1, 2147483562), (777, 777, 2147483562), (2147483398, 2147483398, 2147483562),
    (2, 1, 1), (2147483562, 1, 2147483561), (2147483562, 2147483398, 164),
    (1, 2, 2147483561), (1, 2147483398, 165), (1000, 5000, 2147479562),
    (2147483398, 2147483397, 1), (123456789, 987654321, None), (2000000000, 3, None),
]


@pytest.mark.parametrize("v1,v2,want", RANECU_CASES)
def test_ranecu_combination_pinned(oracle, v1, v2, want):
    """Appendix A.4.1: X = (X_1 - X_2) mod (m1 - 1), plus m1 - 1 when X <= 0.

    States are built so the two MLCGs step to (v1, v2); the first draw must be the residue of
    v1 - v2 in [1, m1 - 1].  Equal components give m1 - 1 = 2147483562 (the <= 0 clause; a strict
    < 0 would give 0), and a negative difference is lifted by m1 - 1 (not m1, not m2 - 1)."""
    z = ranecu_combined(v1, v2)
    if want is not None:
        assert z == want
    st = oracle.init("ranecu", [ranecu_prestate(v1, v2)])[0]
    d = oracle.next_draws("ranecu", st, 1)
    assert (int(st[0]), int(st[1])) == (v1, v2)
    assert int(d[0]) == z


def test_ranecu_combination_sequence(oracle):
    """2000 successive draws from three seeds equal the residue definition applied to the closed-form
    components x_n = a^n x_0 mod m, computed in Python integers."""
    for s1, s2 in [(1, 1), (12345, 67890), (2147483562, 2147483398)]:
        st = oracle.init("ranecu", [[s1, s2]])[0]
        d = oracle.next_draws("ranecu", st, 2000)
        for n in (1, 2, 3, 500, 1999, 2000):
            v1, v2 = pow(A1, n, M1) * s1 % M1, pow(A2, n, M2) * s2 % M2
            assert int(d[n - 1]) == ranecu_combined(v1, v2)


@pytest.mark.slow
def test_ggl_period_bruteforce(oracle):
    """Appendix A.1: period of the minimal standard generator is 2^31 - 2."""
    assert oracle.ggl_period(1) == 2147483646


def test_ggl_power_law(oracle):
    rng = np.random.default_rng(1)
    for x0 in rng.integers(1, 2147483647, size=5):
        st = oracle.init("ggl", [int(x0)])[0]
        d = oracle.next_draws("ggl", st, 5000)
        for n in (1, 2, 777, 5000):
            assert int(d[n - 1]) == pow(16807, n, 2147483647) * int(x0) % 2147483647


def test_ranmar_c_period(oracle):
    """Appendix A.4.4: C_n has the full period of its prime modulus M = 2^24 - 3."""
    assert oracle.ranmar_c_period(362436) == 16777213


def _shift_matrix(a: int, left: bool) -> np.ndarray:
    """32x32 GF(2) matrix S with (row bit-vector x) S = x << a (left) or x >> a."""
    S = np.zeros((32, 32), dtype=np.int64)
    for b in range(32):
        t = b + a if left else b - a
        if 0 <= t < 32:
            S[b, t] = 1
    return S


def _xor128_T() -> np.ndarray:
    """128x128 transition matrix of XOR128 from its block form in Appendix A.4.2."""
    I = np.eye(32, dtype=np.int64)
    Z = np.zeros((32, 32), dtype=np.int64)
    A = ((I + _shift_matrix(11, True)) @ (I + _shift_matrix(8, False))) % 2
    B = (I + _shift_matrix(19, False)) % 2
    return np.block([[Z, Z, Z, A], [I, Z, Z, Z], [Z, I, Z, Z], [Z, Z, I, B]]) % 2


def _bits(words) -> np.ndarray:
    return np.array([(int(w) >> b) & 1 for w in words for b in range(32)], dtype=np.int64)


def _words(bits) -> list:
    return [int(sum(int(bits[32 * i + b]) << b for b in range(32))) for i in range(4)]


def test_xor128_is_the_paper_matrix(oracle):
    T = _xor128_T()
    rng = np.random.default_rng(7)
    for _ in range(20):
        s = [int(x) for x in rng.integers(0, 2**32, size=4, dtype=np.uint64)]
        st = oracle.init("xor128", [s])[0]
        oracle.next_draws("xor128", st, 1)
        assert [int(v) for v in st] == _words(_bits(s) @ T % 2)
    # n steps = T^n
    s = [1, 2, 3, 4]
    st = oracle.init("xor128", [s])[0]
    oracle.next_draws("xor128", st, 1000)
    Tn = np.eye(128, dtype=np.int64)
    P, n = T.copy(), 1000
    while n:
        if n & 1:
            Tn = Tn @ P % 2
        P = P @ P % 2
        n >>= 1
    assert [int(v) for v in st] == _words(_bits(s) @ Tn % 2)


def test_xor128_matrix_order_divides_2p128_minus_1():
    """T^(2^128) = T, i.e. the period of every nonzero state divides 2^128 - 1 (Appendix A.4.2)."""
    T = _xor128_T()
    P = T.copy()
    for _ in range(128):
        P = P @ P % 2
    assert np.array_equal(P, T)


def test_xor128_linearity(oracle):
    rng = np.random.default_rng(3)
    a = [int(x) for x in rng.integers(1, 2**32, size=4, dtype=np.uint64)]
    b = [int(x) for x in rng.integers(1, 2**32, size=4, dtype=np.uint64)]
    c = [x ^ y for x, y in zip(a, b)]
    da = oracle.next_draws("xor128", oracle.init("xor128", [a])[0], 300)
    db = oracle.next_draws("xor128", oracle.init("xor128", [b])[0], 300)
    dc = oracle.next_draws("xor128", oracle.init("xor128", [c])[0], 300)
    assert np.array_equal(da ^ db, dc)


@pytest.mark.parametrize("p", [24, 25, 48, 97, 100, 223, 389])
def test_ranlux_keeps_r_of_every_p(oracle, p):
    """Appendix A.4.6: RANLUX(p) output k*24+j equals SWB output k*p+j for j < 24."""
    v = 31337
    swb = oracle.next_draws("ranlux", oracle.init("ranlux", [v])[0], 40 * p, p=24, r=24)
    lux = oracle.next_draws("ranlux", oracle.init("ranlux", [v])[0], 40 * 24, p=p, r=24)
    idx = np.array([k * p + j for k in range(40) for j in range(24)])
    assert np.array_equal(lux, swb[idx])


def test_ranmar_init_ranges(oracle):
    st = oracle.init("ranmar", [[0, 0], [31328, 30081]])
    assert (st[:, :97] < 2**24).all() and (st[:, 97] == 362436).all()
    with pytest.raises(ValueError):
        oracle.init("ranmar", [[31329, 0]])
    with pytest.raises(ValueError):
        oracle.init("ranmar", [[0, 30082]])


@pytest.mark.parametrize("kind", ["ggl", "xor128", "ranecu", "ranmar", "ranlux", "mt19937"])
def test_conversions_exact(oracle, kind):
    b = oracle.bits(kind)
    st = oracle.init(kind, [_seed_for(kind)])
    u = oracle.generate(kind, st.copy(), 3000, "u32")[0]
    f = oracle.generate(kind, st.copy(), 3000, "f32")[0]
    d = oracle.generate(kind, st.copy(), 1500, "f64")[0]
    k = (u.astype(np.uint64) >> np.uint64(b - 24))
    assert np.array_equal(f.astype(np.float64) * 2**24, k.astype(np.float64))
    assert (f >= 0).all() and (f < 1).all()
    for e in range(0, 1500, 97):
        u1, u2 = int(u[2 * e]), int(u[2 * e + 1])
        if b == 24:
            exact = Fraction(u1 * 2**24 + u2, 2**48)
        else:
            exact = Fraction((u1 >> (b - 27)) * 2**26 + (u2 >> (b - 26)), 2**53)
        assert Fraction(float(d[e])) == exact
    assert (d >= 0).all() and (d < 1).all()


def test_conversion_extremes(oracle):
    """Top of the range stays below 1 (the paper's divide-by-modulus forms reach 1.0 in fp32)."""
    assert oracle.to_f32("xor128", 0xFFFFFFFF) == np.float32(1 - 2**-24)
    assert oracle.to_f32("ggl", 2147483646) == np.float32(1 - 2**-24)
    assert oracle.to_f64("mt19937", 0xFFFFFFFF, 0xFFFFFFFF) == 1 - 2**-53
    assert oracle.to_f64("ranlux", 2**24 - 1, 2**24 - 1) == 1 - 2**-48
    assert oracle.to_f32("ranmar", 0) == 0.0


def _seed_for(kind):
    return {"ggl": [12345], "xor128": [1, 2, 3, 4], "ranecu": [12345, 67890], "ranmar": [1802, 9373],
            "ranlux": [314159], "mt19937": [5489]}[kind]


@pytest.mark.parametrize("kind", ["ggl", "xor128", "ranecu", "ranmar", "ranlux", "mt19937"])
@pytest.mark.parametrize("dtype", ["u32", "f32", "f64"])
def test_chunk_invariance(oracle, kind, dtype):
    """generate(a) then generate(b) equals generate(a + b), including mid-block splits."""
    st = oracle.init(kind, [_seed_for(kind), _seed_for(kind)])
    st[1] = st[0]
    whole = oracle.generate(kind, st[:1].copy(), 1500, dtype, p=97)
    part = st[1:].copy()
    a = oracle.generate(kind, part, 311, dtype, p=97)
    b = oracle.generate(kind, part, 1189, dtype, p=97)
    assert np.array_equal(np.concatenate([a, b], axis=1).view(np.uint8), whole.view(np.uint8))


@pytest.mark.parametrize("kind,p", [("ranlux", 24), ("ranlux", 389), ("mt19937", 0), ("ggl", 0)])
def test_fused_consistent_with_generate(oracle, kind, p):
    st = oracle.init(kind, [_seed_for(kind)] * 3)
    f = oracle.generate(kind, st.copy(), 5000, "f32", p=p or 223)
    s, h = oracle.fused(kind, st.copy(), 5000, p=p or 223)
    k = (f.astype(np.float64) * 2**24).astype(np.uint64)
    assert np.array_equal(s, k.sum(axis=1))
    assert (h.sum(axis=1) == 5000).all()
    assert np.array_equal(h[0], np.bincount((k[0] >> np.uint64(18)).astype(np.int64), minlength=64))


def test_sum_f32_is_the_sum_of_generated_values(oracle):
    from paper_1003_1898_amd import inputs
    for kind in ("ggl", "ranlux", "mt19937"):
        st = oracle.init(kind, inputs.seed_words(kind, 3, 1))
        a, b = st[0].copy(), st.copy()
        total = oracle.sum_f32(kind, a, 5000)
        vals = oracle.generate(kind, b, 5000, "f32")[0].astype(np.float64)
        acc = 0.0
        for v in vals:
            acc += v
        assert total == acc and np.array_equal(a, b[0])
