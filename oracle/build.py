"""Compiles the CPU oracle (prng_oracle.c) into liboracle.so next to this file."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "prng_oracle.c")
LIB_PATH = os.path.join(HERE, "liboracle.so")


def build() -> str:
    tmp = LIB_PATH + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", SRC, "-o", tmp],
                   check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build())
