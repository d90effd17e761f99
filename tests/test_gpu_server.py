"""Serving loop: every request's elements equal the oracle's next `count`
elements of its stream (per-stream arrival order), the same whether it was
served in a mix of concurrent batches or alone, under a memory budget smaller
than the work in flight, and the generator states end where the oracle's do.
"""
import time

import numpy as np
import pytest
import torch

from paper_1003_1898_amd import inputs
from paper_1003_1898_amd._capi import SEG_NEVER, PrngError
from paper_1003_1898_amd.server import Server

from mirror import Mirror, bits

pytestmark = pytest.mark.gpu

OBJS = [("ggl", 0), ("xor128", 0), ("ranecu", 0), ("ranmar", 0), ("ranlux", 223), ("ranlux", 24), ("mt19937", 0),
        ("drand48", 0), ("rannyu", 0)]
DT = ["u32", "f32", "f64"]


def random_requests(rng, n_req, n_objs, n_streams, hot=12, max_count=20000):
    """Requests over a few hot streams (so that streams repeat and per-stream
    order matters) plus random ones; counts span one element to many segments."""
    reqs = []
    for _ in range(n_req):
        gi = int(rng.integers(0, n_objs))
        s = int(rng.integers(0, hot)) if rng.random() < 0.5 else int(rng.integers(0, n_streams))
        c = int(rng.choice([1, 2, 63, 64, 65, 120, 128, 383, 384, 385, 1000, 4095, max_count,
                            rng.integers(1, max_count)]))
        reqs.append((gi, s, c, DT[int(rng.integers(0, 3))]))
    return reqs


def submit(server, reqs, arrive_ns=None, keep=True):
    gi, s, c, d = zip(*reqs)
    return server.submit_many(gi, s, c, d, arrive_ns=arrive_ns, keep=keep)


def wait_all(server, n, timeout_s=60.0):
    t0 = time.time()
    while server.stats()["completed"] < n:
        assert time.time() - t0 < timeout_s, f"server stuck: {server.stats()}"
        time.sleep(0.002)


def test_served_mix_matches_oracle_and_final_states(oracle):
    rng = np.random.default_rng(77)
    mirror = Mirror(oracle, OBJS, 160, 500)
    reqs = random_requests(rng, 400, len(OBJS), 160)
    srv = Server(mirror.gens, 64 << 20, max_inflight=4, max_batch=32, seg_len=384, max_request_draws=1 << 16)
    print(f"\n[server] {len(reqs)} requests, seg 384, batch 32, inflight 4", flush=True)
    tickets = submit(srv, reqs)
    for i, (t, (gi, s, c, dt)) in enumerate(zip(tickets, reqs)):
        got = srv.result(int(t), timeout_ms=60000)
        assert got is not None, f"request {i} not done"
        ref = mirror.expect(gi, s, c, dt)
        assert np.array_equal(bits(got.cpu().numpy()), bits(ref)), f"request {i}: {mirror.objs[gi]} stream {s} count {c} {dt}"
        srv.release(int(t))
    st = srv.stats()
    print(f"[server] stats {st}", flush=True)
    assert st["completed"] == len(reqs) and st["batches"] > 1
    tm = srv.times(tickets)
    assert np.all(tm["arrive_ns"] <= tm["admit_ns"]) and np.all(tm["admit_ns"] <= tm["done_ns"])
    srv.close()
    mirror.check_states()


def test_served_equals_solo_replay(oracle):
    """Scheduled arrivals served concurrently give the same bytes as each
    request served alone, one after another."""
    rng = np.random.default_rng(78)
    reqs = random_requests(rng, 160, len(OBJS), 64, hot=6, max_count=6000)
    mix_m = Mirror(oracle, OBJS, 64, 900)
    solo_m = Mirror(oracle, OBJS, 64, 900)
    mix = Server(mix_m.gens, 64 << 20, max_inflight=3, max_batch=16, seg_len=768, max_request_draws=1 << 14)
    now = mix.now_ns()
    arrive = now + np.cumsum(rng.exponential(40_000, len(reqs))).astype(np.int64)  # ~25k requests/s
    print(f"\n[server] mix of {len(reqs)} with scheduled arrivals", flush=True)
    t_mix = submit(mix, reqs, arrive_ns=arrive)
    got_mix = [mix.result(int(t), timeout_ms=60000) for t in t_mix]
    assert all(g is not None for g in got_mix)
    assert mix.stats()["batches"] > 1
    mix.close()
    solo = Server(solo_m.gens, 64 << 20, max_inflight=1, max_batch=1, seg_len=768, max_request_draws=1 << 14)
    print("[server] solo replay", flush=True)
    for i, (r, g) in enumerate(zip(reqs, got_mix)):
        t = solo.submit(*r)
        alone = solo.result(t, timeout_ms=60000)
        assert alone is not None
        assert np.array_equal(bits(alone.cpu().numpy()), bits(g.cpu().numpy())), f"request {i}: {r}"
        solo.release(t)
    assert solo.stats()["batches"] == len(reqs)
    solo.close()
    for a, b in zip(mix_m.gens, solo_m.gens):
        assert np.array_equal(a.state_words(), b.state_words())


def test_budget_smaller_than_the_work(oracle):
    """Outputs of 16 requests need 4x the pool: requests wait for memory, are
    admitted in arrival order within each class of kinds (each object here is
    of its own class) as earlier ones are released, and stay exact."""
    mirror = Mirror(oracle, [("xor128", 0), ("ranlux", 97), ("mt19937", 0)], 8, 31)
    reqs = [(i % 3, (i // 3) % 8, 1 << 18, "f32") for i in range(16)]  # 1 MiB each
    srv = Server(mirror.gens, (4 << 20) + (2 << 20), max_inflight=4, max_batch=8, seg_len=6144,
                 max_request_draws=1 << 18)
    pool_room = srv._pool.numel()
    tickets = submit(srv, reqs)
    peak = 0
    for i, (t, (gi, s, c, dt)) in enumerate(zip(tickets, reqs)):
        got = srv.result(int(t), timeout_ms=60000)
        peak = max(peak, srv.stats()["pool_in_use"])
        assert got is not None, f"request {i} never admitted: {srv.stats()}"
        assert np.array_equal(bits(got.cpu().numpy()), bits(mirror.expect(gi, s, c, dt))), f"request {i}"
        srv.release(int(t))
    assert peak <= pool_room
    tm = srv.times(tickets)
    for gi in range(3):
        sel = [i for i, r in enumerate(reqs) if r[0] == gi]
        assert np.all(np.diff(tm["admit_ns"][sel]) >= 0), f"admission out of arrival order in class of object {gi}"
    srv.close()
    mirror.check_states()


def test_plain_fifo_mode(oracle):
    """Unsegmented, one request per batch, one batch at a time."""
    rng = np.random.default_rng(79)
    mirror = Mirror(oracle, OBJS, 32, 61)
    reqs = random_requests(rng, 40, len(OBJS), 32, hot=4, max_count=3000)
    srv = Server(mirror.gens, 16 << 20, max_inflight=1, max_batch=1, seg_len=SEG_NEVER, max_request_draws=1 << 13)
    tickets = submit(srv, reqs)
    for i, (t, (gi, s, c, dt)) in enumerate(zip(tickets, reqs)):
        got = srv.result(int(t), timeout_ms=60000)
        assert np.array_equal(bits(got.cpu().numpy()), bits(mirror.expect(gi, s, c, dt))), f"request {i}"
        srv.release(int(t))
    srv.close()
    mirror.check_states()


def test_unkept_requests_and_times(oracle):
    mirror = Mirror(oracle, OBJS[:3], 16, 5)
    srv = Server(mirror.gens, 16 << 20, max_inflight=2, max_batch=4)
    reqs = [(i % 3, i % 16, 5000, "u32") for i in range(30)]
    now = srv.now_ns()
    arrive = now + 1_000_000 + 100_000 * np.arange(30, dtype=np.int64)
    t = submit(srv, reqs, arrive_ns=arrive, keep=False)
    wait_all(srv, 30)
    tm = srv.times(t)
    assert np.array_equal(tm["arrive_ns"], arrive)
    assert np.all(tm["admit_ns"] >= arrive) and np.all(tm["done_ns"] >= tm["admit_ns"])
    assert srv.stats()["pool_in_use"] == 0
    with pytest.raises(PrngError):
        srv.release(int(t[0]))  # freed at completion
    srv.close()
    for gi, s, c, dt in reqs:
        mirror.expect(gi, s, c, dt)
    mirror.check_states()


def test_rejected_requests():
    from paper_1003_1898_amd.generator import Generator
    g = Generator("ggl", 4, seed=3)
    srv = Server([g], 4 << 20, max_request_draws=4096)
    with pytest.raises(PrngError):
        srv.submit(0, 4, 10, "u32")        # stream out of range
    with pytest.raises(PrngError):
        srv.submit(1, 0, 10, "u32")        # generator index out of range
    with pytest.raises(PrngError):
        srv.submit(0, 0, 4097, "u32")      # above max_request_draws
    with pytest.raises(PrngError):
        srv.submit(0, 0, 2049, "f64")      # two draws per element
    with pytest.raises(PrngError):
        srv.submit(0, 0, 0, "u32")
    with pytest.raises(PrngError):
        srv.submit(0, 0, 1 << 63, "f64")   # count * 2 draws would wrap to 0 in 64 bits
    with pytest.raises(PrngError):
        srv.submit(0, 0, (1 << 64) - 1, "u32")
    with pytest.raises(PrngError):
        srv.submit(0, 0, 10, "f32_paper")  # the paper's scalings are a plain-generation output
    with pytest.raises(PrngError):
        srv.release(12345)
    t = srv.submit(0, 0, 4096, "u32")
    assert srv.result(t, timeout_ms=30000) is not None
    srv.close()


def test_served_workload_sampled(oracle):
    """The served workload at full size (65536 states, counts up to 2^22) in
    the configuration the benchmark runs; a sample of requests is checked
    against the oracle from the stream's start."""
    n_states = 65536
    sched = inputs.request_schedule(600, 2000.0, n_states=n_states)
    obj, idx, per = inputs.served_split(sched["stream"], n_states)
    gens = []
    from paper_1003_1898_amd.generator import Generator
    for k, kind in enumerate(inputs.SERVED_KINDS):
        gens.append(Generator(kind, per[k], seed_words=inputs.seed_words(kind, 42 + k, per[k]), p=223))
    srv = Server(gens, 1 << 30, max_inflight=4, max_batch=1024)
    reqs = list(zip(obj.tolist(), idx.tolist(), sched["count"].tolist(), sched["dtype"].tolist()))
    print(f"\n[server] served workload: {len(reqs)} requests", flush=True)
    t = submit(srv, reqs)
    rng = np.random.default_rng(5)
    sample = sorted(rng.choice(len(reqs), 24, replace=False).tolist())
    got = {}
    for i, tk in enumerate(t):
        r = srv.result(int(tk), timeout_ms=120000)
        assert r is not None, f"request {i} not done"
        if i in sample:
            got[i] = bits(r.cpu().numpy())
        srv.release(int(tk))
    srv.close()
    for i in sample:
        gi, s, c, dt = reqs[i]
        kind = inputs.SERVED_KINDS[gi]
        st = oracle.init(kind, inputs.seed_words(kind, 42 + gi, per[gi])[s:s + 1])
        for j in range(i):  # earlier requests on the same stream come first
            if reqs[j][0] == gi and reqs[j][1] == s:
                oracle.generate(kind, st, reqs[j][2], DT[reqs[j][3] - 1], p=223)
        ref = oracle.generate(kind, st, c, DT[dt - 1], p=223)[0]
        assert np.array_equal(got[i], bits(ref)), f"request {i}: {kind} stream {s} count {c} dtype {dt}"
