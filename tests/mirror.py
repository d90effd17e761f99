"""Oracle mirrors of device generator objects, shared by the GPU tests."""
import numpy as np

from paper_1003_1898_amd import inputs
from paper_1003_1898_amd.generator import Generator


def bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint64 if a.dtype.itemsize == 8 else np.uint32)


class Mirror:
    """Oracle copies of every stream of a set of generator objects."""

    def __init__(self, oracle, objs, n, master):
        self.oracle = oracle
        self.objs = objs
        self.gens, self.states = [], []
        for i, (kind, p) in enumerate(objs):
            seeds = inputs.seed_words(kind, master + i, n)
            self.gens.append(Generator(kind, n, seed_words=seeds, p=p or 223))
            self.states.append(oracle.init(kind, seeds))

    def expect(self, gi, s, count, dtype):
        kind, p = self.objs[gi]
        row = self.states[gi][s:s + 1].copy()
        out = self.oracle.generate(kind, row, int(count), dtype, p=p or 223)[0]
        self.states[gi][s] = row[0]
        return out

    def check_states(self):
        for g, st in zip(self.gens, self.states):
            assert np.array_equal(g.state_words(), st)
