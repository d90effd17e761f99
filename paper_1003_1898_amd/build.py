"""Builds libprng.so (HIP kernels for gfx950 + host runtime) inside the package.

Run ``python -m paper_1003_1898_amd.build`` or call ``build()``; the library
lands next to this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(HERE, "libprng.so")
SOURCES = ["k_lux_plain_b.hip", "k_lux_plain_a.hip", "k_lux_plain_c.hip", "k_lux.hip", "k_plain.hip", "k_table.hip",
           "k_fused.hip", "k_init.hip", "k_static.hip",
           "runtime.cpp", "table.cpp", "server.cpp", "jump.cpp"]
# sources of device code (their hash identifies the kernels a profile measured)
DEVICE_SOURCES = ["device.h", "bigint576.h", "internal.h", "lux_plain.h", "k_plain.hip", "k_lux.hip", "k_lux_plain_a.hip",
                  "k_lux_plain_b.hip", "k_lux_plain_c.hip", "k_table.hip", "k_fused.hip",
                  "k_init.hip", "k_static.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++20",
    "-fPIC",
    "-fvisibility=hidden",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-I", INCLUDE,
    "-I", CSRC,
]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    with tempfile.TemporaryDirectory(prefix="prng_build_") as tmp:
        def compile_one(src):
            obj = os.path.join(tmp, src + ".o")
            cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
            return obj

        jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 1)), 16)
        with ThreadPoolExecutor(jobs) as ex:
            objs = list(ex.map(compile_one, SOURCES))
        out_tmp = LIB_PATH + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out_tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
        os.replace(out_tmp, LIB_PATH)
    return LIB_PATH


CALIB_SRC = os.path.join(HERE, "calib", "valu_rate.hip")
CALIB_LIB = os.path.join(HERE, "calib", "libvalu_rate.so")


def build_calib() -> str:
    """The VALU issue-rate calibration kernels (not part of libprng)."""
    tmp = CALIB_LIB + ".tmp"
    r = subprocess.run([HIPCC, *FLAGS, "-shared", CALIB_SRC, "-o", tmp], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {CALIB_SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, CALIB_LIB)
    return CALIB_LIB


def device_sources_sha256() -> str:
    """Hash of the device-code sources, in DEVICE_SOURCES order."""
    import hashlib
    h = hashlib.sha256()
    for src in DEVICE_SOURCES:
        with open(os.path.join(CSRC, src), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


if __name__ == "__main__":
    print(build(verbose=True))
