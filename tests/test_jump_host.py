"""Host-side jump-ahead data of libprng checked on the CPU.

MT19937: the characteristic polynomial of the state transition comes out of
Berlekamp-Massey with degree 19937 and 135 nonzero coefficients (the weight
Matsumoto and Nishimura's generator is known for), and the window J words
ahead built from x^J mod that polynomial equals the one reached by stepping
the recurrence, and the oracle's state after J draws.  DRAND48 and RANNYU:
the affine map of j L steps takes the oracle's starting state to its state
after j L draws (tests/jump_check.cpp).
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def mt_check_output(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("jump") / "jump_check")
    subprocess.run(["g++", "-O2", "-std=c++20", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I", os.path.join(ROOT, "paper_1003_1898_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "jump_check.cpp"),
                    os.path.join(ROOT, "paper_1003_1898_amd", "csrc", "jump.cpp"),
                    "-x", "c", os.path.join(ROOT, "oracle", "prng_oracle.c"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=120).stdout
    return dict(line.split(None, 1) for line in out.splitlines())


def test_mt_characteristic_polynomial_weight(mt_check_output):
    assert mt_check_output["weight"] == "135"


@pytest.mark.parametrize("J", [1, 2, 3, 623, 624, 625, 1000, 19936, 19937, 19938, 62400, 624 * 255, 624 * 767])
def test_mt_jump_window(mt_check_output, J):
    assert mt_check_output[str(J)] == "ok"


def test_mt_segment_table(mt_check_output):
    assert mt_check_output["table"] == "ok"


@pytest.mark.parametrize("kind", [7, 8])
def test_lcg48_jump_maps(mt_check_output, kind):
    assert mt_check_output[f"lcg{kind}"] == "ok"
