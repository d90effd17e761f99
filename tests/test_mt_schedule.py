"""The in-place schedules of the MT19937 block twist used by the kernels
(Appendix A.4.3: word i of the next block from words i and i+1 of the current
one and word i+397 of the sequence), checked on the CPU against the oracle's
next block.

The workgroup kernels update the 624 words in three phases, [0,227),
[227,454) and [454,624); the one-wavefront kernels in groups of three 64-word
rounds.  In both, every word of a phase or group is read before any of them is
written.  These tests replay exactly those read/write orders in numpy and
compare with the oracle, and check that a schedule breaking the order is
caught."""
import numpy as np

import oracle as O
from paper_1003_1898_amd import inputs

UPPER, LOWER, MAG = np.uint32(0x80000000), np.uint32(0x7FFFFFFF), np.uint32(0x9908B0DF)


def _update(mt, idx):
    """Reads the inputs of words idx, then writes them (one phase)."""
    a = mt[idx]
    b = mt[(idx + 1) % 624]
    x = mt[np.where(idx + 397 >= 624, idx - 227, idx + 397)]
    y = (a & UPPER) | (b & LOWER)
    mt[idx] = x ^ (y >> np.uint32(1)) ^ np.where((b & np.uint32(1)) != 0, MAG, np.uint32(0))


def twist_phases(table, phases):
    mt = table.copy()
    for idx in phases:
        _update(mt, np.asarray(idx, dtype=np.int64))
    return mt


WORKGROUP = [np.arange(0, 227), np.arange(227, 454), np.arange(454, 624)]
WAVEFRONT = [np.arange(0, 192), np.arange(192, 384), np.arange(384, 576), np.arange(576, 624)]


def _blocks(n=8):
    st = O.init("mt19937", inputs.seed_words("mt19937", 7, n))
    assert np.all(st[:, 624] == 624)  # a fresh state stands at the end of its block
    cur = st[:, :624].copy()
    O.generate("mt19937", st, 624, "u32")
    return cur, st[:, :624].copy()


def test_workgroup_phases_give_the_next_block():
    cur, nxt = _blocks()
    for s in range(cur.shape[0]):
        assert np.array_equal(twist_phases(cur[s], WORKGROUP), nxt[s])


def test_wavefront_groups_give_the_next_block():
    cur, nxt = _blocks()
    for s in range(cur.shape[0]):
        assert np.array_equal(twist_phases(cur[s], WAVEFRONT), nxt[s])


def test_a_schedule_that_reads_too_late_is_caught():
    # one phase for the whole block: words i >= 227 would read the old word
    # i - 227 instead of the new one
    cur, nxt = _blocks()
    assert not np.array_equal(twist_phases(cur[0], [np.arange(624)]), nxt[0])
    # a first phase longer than 227 words: word 227 + k reads word k before
    # that phase has written it
    bad = [np.arange(0, 300), np.arange(300, 624)]
    assert not np.array_equal(twist_phases(cur[0], bad), nxt[0])
