"""Stream table (batched mixed generation): bit-exact parity with the oracle.

Each run of a table must produce, for every row, exactly the next `count`
elements of that row's stream (as a lone plain generation would), with every
stream state advanced accordingly - through graph replays, eager runs and
autotuning (which must leave the states where they were).
"""
import numpy as np
import pytest
import torch

from paper_1003_1898_amd import inputs
from paper_1003_1898_amd._capi import PrngError
from paper_1003_1898_amd.generator import Generator
from paper_1003_1898_amd.table import StreamTable

from mirror import Mirror, bits

pytestmark = pytest.mark.gpu

OBJS = [("ggl", 0), ("xor128", 0), ("ranecu", 0), ("ranmar", 0), ("ranlux", 223), ("ranlux", 97), ("mt19937", 0),
        ("drand48", 0), ("rannyu", 0)]


def random_rows(rng, n_objs, n, frac=0.6, max_count=3000):
    rows = []
    for gi in range(n_objs):
        for s in np.flatnonzero(rng.random(n) < frac):
            c = int(rng.choice([1, 2, 3, 63, 64, 97, 120, 128, 129, 623, 625, 1000, max_count, rng.integers(1, max_count)]))
            rows.append((gi, int(s), c, ["u32", "f32", "f64"][rng.integers(0, 3)]))
    return rows


def check_table_run(mirror, table, rows):
    torch.cuda.synchronize()
    for i, (gi, s, c, dt) in enumerate(rows):
        got = bits(table.outputs[i].cpu().numpy())
        ref = bits(mirror.expect(gi, s, c, dt))
        assert np.array_equal(got, ref), f"row {i}: {mirror.objs[gi]} stream {s} count {c} {dt}"


def g_kind(g):
    return ["", "ggl", "xor128", "ranecu", "ranmar", "ranlux", "mt19937", "drand48", "rannyu"][g.kind]


def make_table(mirror, rows):
    gi, s, c, d = zip(*rows)
    return StreamTable(mirror.gens, gi, s, c, d)


def test_table_graph_replays_and_eager(oracle):
    rng = np.random.default_rng(2024)
    mirror = Mirror(oracle, OBJS, 150, 42)
    rows = random_rows(rng, len(OBJS), 150)
    t = make_table(mirror, rows)
    print(f"\n[table] rows={len(rows)} info={t.info()}", flush=True)
    for rep, graph in enumerate([True, True, False, True]):
        print(f"[table] run {rep} graph={graph}", flush=True)
        t.run(graph=graph)
        check_table_run(mirror, t, rows)
        mirror.check_states()


def test_table_autotune_keeps_states(oracle):
    rng = np.random.default_rng(7)
    mirror = Mirror(oracle, OBJS, 120, 9)
    rows = random_rows(rng, len(OBJS), 120, frac=0.8)
    t = make_table(mirror, rows)
    cfg = t.autotune(repeats=1)
    print(f"\n[table] tuned {cfg}", flush=True)
    mirror.check_states()            # tuning restored every state
    t.run(graph=True)
    check_table_run(mirror, t, rows)
    mirror.check_states()
    t.set_config(32, 64, 0)
    t.run(graph=True)
    check_table_run(mirror, t, rows)
    mirror.check_states()


def test_table_concurrency_modes(oracle):
    """Every placement of the class kernels on streams (serial, MT19937 beside,
    every class on its own stream), captured and replayed several times with
    eager runs in between, and enqueued directly; each run checked."""
    rng = np.random.default_rng(17)
    mirror = Mirror(oracle, OBJS, 90, 13)
    rows = random_rows(rng, len(OBJS), 90, frac=0.8)
    t = make_table(mirror, rows)
    for mode, lg, mg in ((0, 256, 512), (1, 128, 256), (2, 256, 512), (2, 192, 128), (3, 256, 128), (3, 128, 1024)):
        t.set_config(lg, mg, mode)
        assert t.config() == {"lane_grid": lg, "mt_grid": mg, "concurrent": mode}
        for graph in (True, False, True, True):
            print(f"\n[table] concurrency {mode} grids {lg}/{mg} graph {graph}", flush=True)
            t.run(graph=graph)
            check_table_run(mirror, t, rows)
        mirror.check_states()
    with pytest.raises(PrngError, match="concurrent"):
        t.set_config(256, 512, 4)


@pytest.mark.parametrize("which", ["lane_only", "mt_only"])
def test_table_single_class(oracle, which):
    objs = [("ranlux", 389), ("ranmar", 0)] if which == "lane_only" else [("mt19937", 0)]
    mirror = Mirror(oracle, objs, 100, 3)
    rng = np.random.default_rng(11)
    rows = random_rows(rng, len(objs), 100, frac=0.9)
    t = make_table(mirror, rows)
    for graph in (True, True):
        t.run(graph=graph)
        check_table_run(mirror, t, rows)
    mirror.check_states()


def test_table_equals_plain_generate(oracle):
    """A table over all streams of one object with one count equals prng_generate."""
    n, count = 200, 777
    seeds = inputs.seed_words("xor128", 5, n)
    a = Generator("xor128", n, seed_words=seeds)
    b = Generator("xor128", n, seed_words=seeds)
    t = StreamTable([a], [0] * n, list(range(n)), [count] * n, ["f32"] * n)
    t.run()
    plain = b.generate(count, "f32")
    torch.cuda.synchronize()
    got = np.stack([o.cpu().numpy() for o in t.outputs])
    assert np.array_equal(bits(got), bits(plain.cpu().numpy()))
    assert np.array_equal(a.state_words(), b.state_words())


def test_table_rejects_bad_rows():
    g = Generator("ggl", 10, seed=1)
    with pytest.raises(PrngError, match="twice"):
        StreamTable([g], [0, 0], [3, 3], [5, 6], ["u32", "u32"])
    with pytest.raises(PrngError, match="out of range"):
        StreamTable([g], [1], [0], [5], ["u32"])
    with pytest.raises(PrngError, match="out of range"):
        StreamTable([g], [0], [10], [5], ["u32"])
    with pytest.raises(PrngError, match="too large"):
        StreamTable([g], [0], [0], [2**30 + 1], ["u32"])
    with pytest.raises(PrngError, match="unknown dtype"):
        StreamTable([g], [0], [0], [5], ["f32_paper"])   # a plain-generation output only
    empty = StreamTable([g], [], [], [], [])
    before = g.state_words()
    empty.run()
    empty.run(graph=False)
    assert np.array_equal(before, g.state_words())


SEG_OBJS = [("ggl", 0), ("xor128", 0), ("ranecu", 0), ("ranmar", 0), ("ranlux", 223), ("ranlux", 24),
            ("ranlux", 389), ("ranlux", 100), ("mt19937", 0), ("drand48", 0), ("rannyu", 0)]


@pytest.mark.parametrize("seg", [384, 1152])
def test_table_segments_jump_ahead(oracle, seg):
    """Rows cut into segments started from jumped-ahead states give the same
    bytes and final states; streams first moved to uneven positions (RANLUX
    mid-block with odd offsets, so f64 pairs straddle segment boundaries)."""
    rng = np.random.default_rng(seg)
    mirror = Mirror(oracle, SEG_OBJS, 90, 77)
    warm = random_rows(rng, len(SEG_OBJS), 90, frac=0.7, max_count=700)
    tw = make_table(mirror, warm)
    tw.run(graph=False)
    check_table_run(mirror, tw, warm)
    rows = []
    for gi in range(len(SEG_OBJS)):
        for s in range(90):
            if rng.random() < 0.6:
                c = int(rng.choice([1, 383, 384, 385, 767, 1151, 1152, 2305, int(rng.integers(2000, 6000))]))
                rows.append((gi, s, c, ["u32", "f32", "f64"][rng.integers(0, 3)]))
    gi, s, c, d = zip(*rows)
    t = StreamTable(mirror.gens, gi, s, c, d, seg_len=seg)
    info = t.info()
    print(f"\n[segments] seg={seg} rows={len(rows)} info={info}", flush=True)
    assert info["segments"] > len(rows)
    for graph in (True, True, False):
        t.run(graph=graph)
        check_table_run(mirror, t, rows)
        mirror.check_states()
    for mode in (2, 3):   # every class on its own stream; lane classes before the MT19937 jumps
        t.set_config(256, 512, mode)
        for graph in (True, True, False):
            t.run(graph=graph)
            check_table_run(mirror, t, rows)
            mirror.check_states()


def test_table_segments_long_rows_auto(oracle):
    """Automatic segment length on long rows (the work of a few lanes spread over many)."""
    objs = [("ggl", 0), ("xor128", 0), ("ranecu", 0), ("ranmar", 0), ("ranlux", 223), ("mt19937", 0),
            ("drand48", 0), ("rannyu", 0)]
    mirror = Mirror(oracle, objs, 12, 5)
    rng = np.random.default_rng(3)
    rows = [(gi, s, int(rng.integers(60000, 140000)), ["u32", "f32", "f64"][(gi + s) % 3])
            for gi in range(len(objs)) for s in range(0, 12, 2)]
    gi, s, c, d = zip(*rows)
    t = StreamTable(mirror.gens, gi, s, c, d)
    info = t.info()
    print(f"\n[segments auto] {info}", flush=True)
    assert info["segments"] > len(rows)
    t.run(graph=True)
    check_table_run(mirror, t, rows)
    mirror.check_states()


def test_table_split_equals_unsplit():
    """The same rows with and without cutting produce identical bytes and states."""
    n = 64
    rows_c = [3000 + 17 * s for s in range(n)]
    outs = []
    for seg in (0xFFFFFFFF, 384):
        gens = [Generator(k, n, seed=99, p=223) for k in ("ranlux", "ranmar", "xor128")]
        gi = [g for g in range(3) for _ in range(n)]
        st = [s for _ in range(3) for s in range(n)]
        t = StreamTable(gens, gi, st, rows_c * 3, ["f64", "u32", "f32"] * n, seg_len=seg)
        t.run()
        torch.cuda.synchronize()
        outs.append(([o.cpu().numpy().copy() for o in t.outputs], [g.state_words() for g in gens]))
    for a, b in zip(outs[0][0], outs[1][0]):
        assert np.array_equal(bits(a), bits(b))
    for a, b in zip(outs[0][1], outs[1][1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("seg", [1248, 2496])
def test_table_mt_segments(oracle, seg):
    """MT19937 rows cut into segments whose starting windows come from the
    jump kernel: streams first moved to every kind of block position (0, odd,
    623, 624), then rows around the segment boundaries in all three dtypes
    (fp64 pairs straddle boundaries when the start position is odd)."""
    n = 48
    mirror = Mirror(oracle, [("mt19937", 0)], n, 1234)
    warm = [(0, s, [0, 1, 2, 311, 623, 624, 625, 1247, 1248][s % 9] or 624, "u32") for s in range(n)]
    tw = make_table(mirror, warm)
    tw.run(graph=False)
    check_table_run(mirror, tw, warm)
    counts = [1, 623, 624, 625, seg - 1, seg, seg + 1, 2 * seg - 1, 2 * seg + 3, 3 * seg + 100, 9000, 20001]
    rows = [(0, s, counts[s % len(counts)], ["u32", "f32", "f64"][(s // len(counts)) % 3]) for s in range(n)]
    gi, s, c, d = zip(*rows)
    t = StreamTable(mirror.gens, gi, s, c, d, seg_len=seg)
    info = t.info()
    print(f"\n[mt segments] seg={seg} info={info}", flush=True)
    assert info["segments"] > len(rows)
    for graph in (True, False, True):
        t.run(graph=graph)
        check_table_run(mirror, t, rows)
        mirror.check_states()


def test_table_mt_long_rows_auto(oracle):
    """Automatic MT19937 cutting of rows far longer than the table's share."""
    mirror = Mirror(oracle, [("mt19937", 0), ("ggl", 0)], 8, 9)
    rows = [(0, 0, 1 << 20, "f64"), (0, 1, 700001, "u32"), (0, 2, 300000, "f32"), (0, 3, 5, "u32")]
    rows += [(1, s, 4000, "u32") for s in range(8)]
    gi, s, c, d = zip(*rows)
    t = StreamTable(mirror.gens, gi, s, c, d)
    info = t.info()
    print(f"\n[mt auto] {info}", flush=True)
    assert info["mt_tasks"] > 4
    t.run(graph=True)
    check_table_run(mirror, t, rows)
    mirror.check_states()


def test_table_per_class_segment_lengths(oracle):
    """Lengths given per class (lane kinds, RANMAR, MT19937) cut the rows there
    and leave bytes and final states as without cutting."""
    objs = [("ggl", 0), ("xor128", 0), ("ranmar", 0), ("ranlux", 223), ("mt19937", 0), ("rannyu", 0)]
    mirror = Mirror(oracle, objs, 10, 21)
    rng = np.random.default_rng(5)
    rows = [(gi, s, int(rng.integers(3000, 9000)), ["u32", "f32", "f64"][(gi + s) % 3])
            for gi in range(len(objs)) for s in range(0, 10, 2)]
    gi, s, c, d = zip(*rows)
    t = StreamTable(mirror.gens, gi, s, c, d, seg={"lane": 700, "ranmar": 1500, "mt": 2000})
    assert t.seg_lengths() == {"lane": 768, "ranmar": 1536, "mt": 2496}   # rounded to 384 and to 624
    info = t.info()
    print(f"\n[segments per class] {info}", flush=True)
    assert info["segments"] > 2 * len(rows)
    for graph in (True, False, True):
        t.run(graph=graph)
        check_table_run(mirror, t, rows)
        mirror.check_states()
    never = StreamTable(mirror.gens, gi, s, c, d, seg={"lane": 0xFFFFFFFF, "ranmar": 0xFFFFFFFF, "mt": 0xFFFFFFFF})
    assert never.seg_lengths() == {"lane": 0, "ranmar": 0, "mt": 0}
    assert never.info()["segments"] == len(rows)
    never.run(graph=False)
    check_table_run(mirror, never, rows)
    mirror.check_states()


def test_table_tune_segments_keeps_states(oracle):
    """The segment-length tuner leaves every stream where it was and returns
    lengths whose table reproduces the streams."""
    objs = [("ggl", 0), ("ranecu", 0), ("ranmar", 0), ("ranlux", 97), ("mt19937", 0)]
    mirror = Mirror(oracle, objs, 16, 8)
    rng = np.random.default_rng(9)
    rows = [(gi, s, int(rng.integers(2000, 12000)), ["u32", "f32", "f64"][(gi * 7 + s) % 3])
            for gi in range(len(objs)) for s in range(16) if rng.random() < 0.7]
    gi, s, c, d = zip(*rows)
    best, ms = StreamTable.tune_segments(mirror.gens, gi, s, c, d, repeats=1)
    print(f"\n[tune segments] {best} {ms:.3f} ms", flush=True)
    assert ms > 0 and best["lane"] % 384 == 0 and best["ranmar"] % 384 == 0 and best["mt"] % 624 == 0
    mirror.check_states()
    t = StreamTable(mirror.gens, gi, s, c, d, seg=best)
    assert t.seg_lengths() == best
    for graph in (True, True):
        t.run(graph=graph)
        check_table_run(mirror, t, rows)
    mirror.check_states()


@pytest.mark.parametrize("tuned_lengths", [False, True])
def test_table_full_batched_workload(oracle, tuned_lengths):
    """The benchmark's batched workload (10000 streams over the six generators,
    RANLUX p=223, lengths log-uniform in [2^6, 2^20], dtypes mixed): one graph
    run of the autotuned table, every row and every final state against the
    oracle.  tuned_lengths: the table is built as the benchmark times it, with
    the segment lengths the segment-length tuner picks, then autotuned."""
    from concurrent.futures import ThreadPoolExecutor
    t = inputs.mixed_table()
    kinds = ["ggl", "xor128", "ranecu", "ranmar", "ranlux", "mt19937"]
    gens, seeds, local = [], [], np.zeros(len(t["kind"]), dtype=np.int64)
    for ki, kind in enumerate(kinds):
        sel = np.flatnonzero(t["kind"] == ki + 1)
        local[sel] = np.arange(len(sel))
        sw = inputs.seed_words(kind, 42, max(len(sel), 1))
        seeds.append(sw)
        gens.append(Generator(kind, max(len(sel), 1), seed_words=sw, p=223))
    gi = t["kind"] - 1
    seg = None
    if tuned_lengths:
        seg, _ = StreamTable.tune_segments(gens, gi, local, t["count"], t["dtype"], repeats=1)
        for g, sw in zip(gens, seeds):   # the tuner restores the streams; check that too
            assert np.array_equal(g.state_words(), oracle.init(g_kind(g), sw)), "tuner moved a stream"
    table = StreamTable(gens, gi, local, t["count"], t["dtype"], seg=seg)
    cfg = table.autotune(repeats=1)
    print(f"\n[table full] tuned_lengths={tuned_lengths} seg={table.seg_lengths()} {table.info()} {cfg}", flush=True)
    table.run(graph=True)
    torch.cuda.synchronize()
    names = {1: "u32", 2: "f32", 3: "f64"}

    def expect(i):
        k = kinds[gi[i]]
        st = oracle.init(k, seeds[gi[i]][local[i]:local[i] + 1])
        ref = oracle.generate(k, st, int(t["count"][i]), names[int(t["dtype"][i])], p=223)[0]
        return bits(ref), st[0]

    finals = [gens[k].state_words() for k in range(len(kinds))]
    with ThreadPoolExecutor(16) as pool:
        for i0 in range(0, len(gi), 500):
            rows = range(i0, min(i0 + 500, len(gi)))
            refs = list(pool.map(expect, rows))
            for i, (ref, st) in zip(rows, refs):
                got = bits(table.outputs[i].cpu().numpy())
                assert np.array_equal(got, ref), f"row {i}: {kinds[gi[i]]} count {t['count'][i]} dtype {t['dtype'][i]}"
                assert np.array_equal(finals[gi[i]][local[i]], st), f"row {i}: final state"
