"""RANLUX plain generation and the split in-kernel consumer captured into a
HIP graph (through torch.cuda.graph) and replayed: both calls are
asynchronous and take their jumps from tables written at creation, so a
replay is valid whatever other calls ran on the object in between.  Every
replay is checked against the oracle, with eager calls of other lengths on
the same object between the replays."""
import numpy as np
import pytest
import torch

from paper_1003_1898_amd import inputs
from paper_1003_1898_amd.generator import Generator

from mirror import bits

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("p", [223, 24])
def test_ranlux_generate_graph_replays(oracle, p):
    n, count = 1000, 6000  # 16 wavefronts: every stream cut into 3 jumped segments
    print(f"\n[graph] ranlux p={p} generate", flush=True)
    seeds = inputs.seed_words("ranlux", 77, n)
    g = Generator("ranlux", n, seed_words=seeds, p=p)
    st = oracle.init("ranlux", seeds)
    out = torch.empty((n, count), dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        g.generate(count, "f32", out=out)          # eager, on the capture stream's device
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert np.array_equal(bits(out.cpu().numpy()), bits(oracle.generate("ranlux", st, count, "f32", p=p)))
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.generate(count, "f32", out=out)
    torch.cuda.synchronize()
    assert np.array_equal(g.state_words(), st), "capture must not run the work"
    for rep, other in enumerate([777, 20000, 5]):
        graph.replay()
        torch.cuda.synchronize()
        ref = oracle.generate("ranlux", st, count, "f32", p=p)
        assert np.array_equal(bits(out.cpu().numpy()), bits(ref)), f"replay {rep}"
        # an eager call of another length between replays (other segment lengths)
        x = g.generate(other, "u32")
        torch.cuda.synchronize()
        assert np.array_equal(bits(x.cpu().numpy()), bits(oracle.generate("ranlux", st, other, "u32", p=p)))
    assert np.array_equal(g.state_words(), st)


def test_ranlux_fused_graph_replays(oracle):
    n, draws, p = 200, 30000, 97  # cut into 20 jumped segments per stream
    print(f"\n[graph] ranlux p={p} fused", flush=True)
    seeds = inputs.seed_words("ranlux", 78, n)
    g = Generator("ranlux", n, seed_words=seeds, p=p)
    st = oracle.init("ranlux", seeds)
    s_, h_ = g.fused_sum_hist(draws)
    torch.cuda.synchronize()
    rs, rh = oracle.fused("ranlux", st, draws, p=p)
    assert np.array_equal(s_.cpu().numpy(), rs) and np.array_equal(h_.cpu().numpy(), rh)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.fused_sum_hist(draws, s_, h_)
    torch.cuda.synchronize()
    for rep, other in enumerate([9000, 100000]):
        graph.replay()
        torch.cuda.synchronize()
        rs, rh = oracle.fused("ranlux", st, draws, p=p)
        assert np.array_equal(s_.cpu().numpy(), rs) and np.array_equal(h_.cpu().numpy(), rh), f"replay {rep}"
        a, b = g.fused_sum_hist(other)
        torch.cuda.synchronize()
        rs, rh = oracle.fused("ranlux", st, other, p=p)
        assert np.array_equal(a.cpu().numpy(), rs) and np.array_equal(b.cpu().numpy(), rh)
    assert np.array_equal(g.state_words(), st)
