"""RANECU's combination step (Appendix A.4.1) on the GPU, from states built so
that the two MLCGs reach chosen values at chosen positions.

For target component values (v1, v2) at draw position t of a stream, the state
is s_i = v_i * a_i^-(t+1) mod m_i.  The draw at t must then be the residue of
v1 - v2 in [1, m1 - 1]: m1 - 1 = 2147483562 when v1 = v2, v1 - v2 + m1 - 1 when
v1 < v2.  Positions cover every code path of the HIP side: the first position
of a lane's four, inside a four, the leap between blocks of 256, the
quarter boundaries of long rows, the stream table and the interleaved layout.
Every output is also compared in full with the oracle.
"""
import numpy as np
import pytest

from paper_1003_1898_amd.generator import Generator
from paper_1003_1898_amd.table import StreamTable

from mirror import bits

pytestmark = pytest.mark.gpu

M1, M2, A1, A2 = 2147483563, 2147483399, 40014, 40692
PAIRS = [(1, 1), (777, 777), (2147483398, 2147483398), (2, 1), (2147483562, 1), (1, 2), (1, 2147483398),
         (1000, 5000), (2147483398, 2147483397)]
POSITIONS = [0, 1, 2, 3, 4, 5, 255, 256, 257, 1023, 4095, 4096, 5000, 8191, 12287, 16383]


def combined(v1, v2):
    return (v1 - v2 - 1) % (M1 - 1) + 1


def pinned_states():
    """(n, 2) canonical words and the (stream, position, expected draw) triples they pin."""
    words, pins = [], []
    for t in POSITIONS:
        for v1, v2 in PAIRS:
            s1 = v1 * pow(A1, -(t + 1), M1) % M1
            s2 = v2 * pow(A2, -(t + 1), M2) % M2
            pins.append((len(words), t, combined(v1, v2)))
            words.append((s1, s2))
    while len(words) % 4:
        words.append((12345, 67890))
    return np.array(words, dtype=np.uint32), pins


def make(oracle):
    words, pins = pinned_states()
    g = Generator("ranecu", len(words), seed_words=words.astype(np.uint64))
    g.set_state(Generator.blob_from_words("ranecu", 0, words))
    return g, words.copy(), pins


@pytest.mark.parametrize("count", [16384, 4096, 700, 17])
def test_ranecu_pins_plain(oracle, count):
    """Leapfrog kernels: 16384 and 4096 go by quarters of rows, 700 and 17 one wavefront per row."""
    print(f"\n[ranecu pin] plain count={count}", flush=True)
    g, st, pins = make(oracle)
    got = bits(g.generate(count, "u32").cpu().numpy())
    for s, t, z in pins:
        if t < count:
            assert int(got[s, t]) == z, f"stream {s} position {t}"
    ref = oracle.generate("ranecu", st, count, "u32")
    assert np.array_equal(got, bits(ref))
    assert np.array_equal(g.state_words(), st)


def test_ranecu_pins_packed_and_table(oracle):
    """The lane-per-stream kernel (interleaved layout) and the stream table's lane class."""
    print("\n[ranecu pin] packed4 + table", flush=True)
    g, st, pins = make(oracle)
    n = st.shape[0]
    count = 6000
    got = g.generate_packed4(count, "u32").cpu().numpy().transpose(0, 2, 1).reshape(n, count)
    for s, t, z in pins:
        if t < count:
            assert int(got[s, t]) == z, f"packed stream {s} position {t}"
    assert np.array_equal(bits(got), bits(oracle.generate("ranecu", st, count, "u32")))

    h, st2, pins = make(oracle)
    rows_s = list(range(n))
    t = StreamTable([h], [0] * n, rows_s, [count] * n, ["u32"] * n, seg_len=384)
    t.run(graph=False)
    ref = oracle.generate("ranecu", st2, count, "u32")
    for s in range(n):
        assert np.array_equal(bits(t.outputs[s].cpu().numpy()), bits(ref[s])), f"table row {s}"
    for s, tt, z in pins:
        if tt < count:
            assert int(t.outputs[s][tt].item()) == z
    assert np.array_equal(h.state_words(), st2)
