"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Every comparison is element by element on the same seeded inputs: outputs as
raw bits (u32, f32, f64), final canonical states, fused sums and histograms.
Tolerance is zero: the method is integer arithmetic and the conversions are
exact.
"""
import numpy as np
import pytest
import torch

from paper_1003_1898_amd import inputs
from paper_1003_1898_amd.generator import Generator

pytestmark = pytest.mark.gpu

KINDS = ["ggl", "xor128", "ranecu", "ranmar", "ranlux", "mt19937", "drand48", "rannyu"]
NPBITS = {"u32": np.uint32, "f32": np.uint32, "f64": np.uint64}


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint64 if a.dtype.itemsize == 8 else np.uint32)


def gpu_bits(t):
    return bits(t.cpu().numpy())


def check_run(oracle, kind, n, schedule, p=223, master=42):
    """Create n streams on both sides and compare every step of `schedule`."""
    seeds = inputs.seed_words(kind, master, n)
    g = Generator(kind, n, seed_words=seeds, p=p)
    st = oracle.init(kind, seeds)
    assert np.array_equal(g.state_words(), st), "initial state"
    for count, dtype in schedule:
        out = g.generate(count, dtype)
        ref = oracle.generate(kind, st, count, dtype, p=p, threads=8)
        torch.cuda.synchronize()
        got = gpu_bits(out)
        if not np.array_equal(got, bits(ref)):
            bad = np.argwhere(got != bits(ref))
            raise AssertionError(f"{kind} p={p} n={n} count={count} {dtype}: {len(bad)} mismatches, first {bad[:5]}")
        assert np.array_equal(g.state_words(), st), f"final state after count={count} {dtype}"
    return g, st


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("dtype", ["u32", "f32", "f64"])
def test_tiny_config(oracle, kind, dtype):
    """256 streams x 4096 outputs from seeds SplitMix64(42) (RANLUX p = 223)."""
    print(f"\n[tiny] {kind} {dtype}", flush=True)
    check_run(oracle, kind, 256, [(4096, dtype)])


@pytest.mark.parametrize("kind", KINDS)
def test_ragged_sequence(oracle, kind):
    """Stream counts off the wave size, counts off every chunk length, dtypes interleaved."""
    print(f"\n[ragged] {kind}", flush=True)
    sched = [(1, "u32"), (3, "f64"), (95, "f32"), (97, "u32"), (98, "f64"), (193, "u32"), (624, "f32"),
             (625, "f64"), (1000, "u32"), (1249, "f64"), (23, "f32")]
    for n in (1, 63, 100):
        check_run(oracle, kind, n, sched, p=223)


@pytest.mark.parametrize("p", [24, 25, 48, 97, 100, 223, 389, 120, 240, 408])
def test_ranlux_luxury_levels(oracle, p):
    print(f"\n[ranlux p={p}]", flush=True)
    check_run(oracle, "ranlux", 130, [(500, "u32"), (77, "f64"), (1024, "f32")], p=p)


@pytest.mark.parametrize("n,sched", [
    (300, [(10000, "f32"), (4097, "u32")]),          # 5 wavefronts: cut into 8 and 2 segments
    (64, [(2049, "f64"), (9000, "u32"), (1, "f32")]),  # one wavefront: 2 and 4 segments, then uncut
    (1000, [(24581, "u32"), (6000, "f64")]),          # ragged last segments
    (4100, [(16384, "f32"), (30000, "f64")]),
])
def test_xor128_split_segments(oracle, n, sched):
    """XOR128 plain generation cut into jumped segments (powers T^(2^k)), ragged counts and
    every dtype, against the oracle element by element, with final states."""
    print(f"\n[xor128 split] n={n}", flush=True)
    check_run(oracle, "xor128", n, sched)


@pytest.mark.parametrize("kind", KINDS)
def test_heterogeneous_states(oracle, kind):
    """Streams at different positions (RANLUX mid-block, MT mid-block, ring phases)."""
    print(f"\n[hetero] {kind}", flush=True)
    n, p = 150, 97
    seeds = inputs.seed_words(kind, 11, n)
    st = oracle.init(kind, seeds)
    for s in range(n):
        row = st[s:s + 1].copy()
        oracle.generate(kind, row, (s * 37) % 700, "u32", p=p)
        st[s] = row[0]
    g = Generator(kind, n, seed_words=seeds, p=p)
    g.set_state(Generator.blob_from_words(kind, p, st))
    assert np.array_equal(g.state_words(), st)
    for count, dtype in [(333, "u32"), (301, "f64"), (64, "f32"), (1, "f64")]:
        got = gpu_bits(g.generate(count, dtype))
        ref = oracle.generate(kind, st, count, dtype, p=p)
        assert np.array_equal(got, bits(ref)), f"{kind} count={count} {dtype}"
        assert np.array_equal(g.state_words(), st)


@pytest.mark.parametrize("kind", KINDS)
def test_state_roundtrip_and_restart(oracle, kind):
    """get_state -> destroy -> create -> set_state continues exactly (checkpoint/resume)."""
    print(f"\n[restart] {kind}", flush=True)
    n = 70
    seeds = inputs.seed_words(kind, 5, n)
    g = Generator(kind, n, seed_words=seeds)
    first = gpu_bits(g.generate(700, "u32"))
    blob = g.get_state()
    cont = gpu_bits(g.generate(900, "f32"))
    g.close()
    h = Generator(kind, n, seed_words=inputs.seed_words(kind, 6, n))
    h.set_state(blob)
    again = gpu_bits(h.generate(900, "f32"))
    assert np.array_equal(cont, again)
    st = oracle.init(kind, seeds)
    assert np.array_equal(first, bits(oracle.generate(kind, st, 700, "u32")))


def test_set_state_rejects_bad_blobs():
    from paper_1003_1898_amd._capi import PrngError
    g = Generator("ranlux", 10, seed=1, p=223)
    blob = g.get_state()
    bad = blob.copy()
    bad[0] ^= 1
    with pytest.raises(PrngError, match="ESTATE"):
        g.set_state(bad)
    words = g.state_words()
    words[3, 25] = 25          # kept-in-block counter out of range
    with pytest.raises(PrngError, match="ESTATE"):
        g.set_state(Generator.blob_from_words("ranlux", 223, words))
    with pytest.raises(PrngError, match="ESTATE"):
        g.set_state(Generator.blob_from_words("ranlux", 97, g.state_words()))
    other = Generator("mt19937", 10, seed=1)
    with pytest.raises(PrngError, match="ESTATE"):
        g.set_state(other.get_state())
    g.set_state(blob)


def test_generate_argument_errors():
    from paper_1003_1898_amd._capi import PrngError, lib
    g = Generator("ggl", 16, seed=3)
    small = torch.empty(16 * 10 - 1, dtype=torch.uint32, device="cuda")
    with pytest.raises(PrngError, match="EINVAL"):
        from paper_1003_1898_amd._capi import check
        check(lib().prng_generate(g._handle, 10, 1, small.data_ptr(), small.numel() * 4, None))
    before = g.state_words()
    g.generate(0, "u32")
    assert np.array_equal(before, g.state_words())


@pytest.mark.parametrize("kind,p", [("ggl", 0), ("xor128", 0), ("ranecu", 0), ("ranmar", 0), ("ranlux", 24),
                                    ("ranlux", 48), ("ranlux", 97), ("ranlux", 223), ("ranlux", 389),
                                    ("mt19937", 0), ("drand48", 0), ("rannyu", 0)])
def test_fused_sum_hist(oracle, kind, p):
    print(f"\n[fused] {kind} p={p}", flush=True)
    n = 200
    seeds = inputs.seed_words(kind, 42, n)
    g = Generator(kind, n, seed_words=seeds, p=p or 223)
    st = oracle.init(kind, seeds)
    s, h = g.fused_sum_hist(5003)
    rs, rh = oracle.fused(kind, st, 5003, p=p or 223)
    assert np.array_equal(s.cpu().numpy(), rs)
    assert np.array_equal(h.cpu().numpy(), rh)
    assert np.array_equal(g.state_words(), st)
    s0, h0 = g.fused_sum_hist(0)
    assert not s0.cpu().numpy().any() and not h0.cpu().numpy().any()
    got = gpu_bits(g.generate(300, "u32"))
    assert np.array_equal(got, bits(oracle.generate(kind, st, 300, "u32", p=p or 223)))


@pytest.mark.parametrize("p", [24, 97, 100, 223, 389, 120, 408])
def test_fused_ranlux_split(oracle, p):
    """Long fused runs cut each RANLUX stream into jumped segments (one
    wavefront per stream): sums, histograms and final states as one pass."""
    print(f"\n[fused split] p={p}", flush=True)
    n = 37
    seeds = inputs.seed_words("ranlux", 4000 + p, n)
    g = Generator("ranlux", n, seed_words=seeds, p=p)
    st = oracle.init("ranlux", seeds)
    got = gpu_bits(g.generate(7, "u32"))  # streams stop inside a luxury block
    assert np.array_equal(got, bits(oracle.generate("ranlux", st, 7, "u32", p=p)))
    for draws in (65549, 5760, 200000):
        s, h = g.fused_sum_hist(draws)
        rs, rh = oracle.fused("ranlux", st, draws, p=p)
        assert np.array_equal(s.cpu().numpy(), rs), f"draws {draws}"
        assert np.array_equal(h.cpu().numpy(), rh), f"draws {draws}"
        assert np.array_equal(g.state_words(), st), f"draws {draws}"
    got = gpu_bits(g.generate(300, "u32"))
    assert np.array_equal(got, bits(oracle.generate("ranlux", st, 300, "u32", p=p)))


@pytest.mark.parametrize("kind,p", [("ranlux", 24), ("ranlux", 48), ("ranlux", 97), ("ranlux", 223),
                                    ("ranlux", 389), ("mt19937", 0)])
def test_fused_workload_sampled(oracle, kind, p):
    """The fused workload at full size as the benchmark runs it (4096 streams,
    a 1024-draw warm-up call, then 2^20 draws; seeds SplitMix64(42)); sampled
    streams against the oracle, sums, histograms and final states."""
    print(f"\n[fused full] {kind} p={p}", flush=True)
    n, draws = 4096, 1 << 20
    seeds = inputs.seed_words(kind, 42, n)
    g = Generator(kind, n, seed_words=seeds, p=p or 223)
    g.fused_sum_hist(1024)
    s, h = g.fused_sum_hist(draws)
    s, h = s.cpu().numpy(), h.cpu().numpy()
    assert np.all(h.sum(axis=1) == draws)
    words = g.state_words()
    idx = [0, 1, 63, 64, 2047, 4095, 1234, 3001]
    st = oracle.init(kind, seeds[idx])
    oracle.fused(kind, st, 1024, p=p or 223, threads=8)
    rs, rh = oracle.fused(kind, st, draws, p=p or 223, threads=8)
    for j, i in enumerate(idx):
        assert s[i] == rs[j] and np.array_equal(h[i], rh[j]), f"stream {i}"
        assert np.array_equal(words[i], st[j])


@pytest.mark.parametrize("kind", KINDS)
def test_full_scale_sampled(oracle, kind):
    """65536 streams x 16384 numbers (2^30), u32 then f32, seeds SplitMix64(7): the
    benchmark's launch configuration; sampled streams compared in full."""
    print(f"\n[full] {kind}", flush=True)
    n, count, p = 65536, 16384, 223
    seeds = inputs.seed_words(kind, 7, n)
    rng = np.random.default_rng(123)
    idx = np.unique(np.concatenate([[0, 1, 63, 64, 255, 256, n - 1], rng.integers(0, n, 41)]))
    st = oracle.init(kind, seeds[idx])
    g = Generator(kind, n, seed_words=seeds, p=p)
    out = torch.empty((n, count), dtype=torch.uint32, device="cuda")
    sel = torch.as_tensor(idx, device="cuda")
    for dtype in ("u32", "f32"):
        o = out if dtype == "u32" else out.view(torch.float32)
        g.generate(count, dtype, out=o)
        got = gpu_bits(o.index_select(0, sel))
        ref = oracle.generate(kind, st, count, dtype, p=p, threads=8)
        assert np.array_equal(got, bits(ref)), f"{kind} {dtype}"
    words = g.state_words()
    assert np.array_equal(words[idx], st)


@pytest.mark.parametrize("kind", ["ggl", "xor128", "ranecu", "ranmar", "ranlux", "mt19937"])
def test_full_scale_every_stream(oracle, kind):
    """The benchmark's configuration (65536 streams x 16384 u32, seeds
    SplitMix64(7), RANLUX p=223): launch 1 compared for every stream in chunks
    of 4096 streams, then launch 20 and the final states for 256 sampled
    streams."""
    print(f"\n[full every stream] {kind}", flush=True)
    n, count, p, chunk = 65536, 16384, 223, 4096
    seeds = inputs.seed_words(kind, 7, n)
    g = Generator(kind, n, seed_words=seeds, p=p)
    out = torch.empty((n, count), dtype=torch.uint32, device="cuda")
    g.generate(count, "u32", out=out)
    torch.cuda.synchronize()
    for c0 in range(0, n, chunk):
        st = oracle.init(kind, seeds[c0:c0 + chunk])
        ref = oracle.generate(kind, st, count, "u32", p=p, threads=16)
        got = out[c0:c0 + chunk].cpu().numpy()
        bad = np.flatnonzero((got != ref).any(axis=1))
        assert bad.size == 0, f"{kind}: launch 1 differs in stream {c0 + int(bad[0])}"
    for _ in range(19):
        g.generate(count, "u32", out=out)
    rng = np.random.default_rng(20)
    idx = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, 254)]))
    st = oracle.init(kind, seeds[idx])
    oracle.generate(kind, st, 19 * count, "u32", p=p, threads=16)
    ref = oracle.generate(kind, st, count, "u32", p=p, threads=16)
    got = out.index_select(0, torch.as_tensor(idx, device="cuda")).cpu().numpy()
    assert np.array_equal(got, ref), f"{kind}: launch 20"
    assert np.array_equal(g.state_words()[idx], st)
