"""The host C++ of libprng (seeding, table planner, jump-ahead data, serving
bookkeeping) and the CPU oracle, built for the CPU under AddressSanitizer and
UndefinedBehaviorSanitizer and run over tests/host_checks.cpp.  No GPU: the
device launchers are stubs and no HIP call is made."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1003_1898_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def checks_output(tmp_path_factory):
    d = tmp_path_factory.mktemp("hostsan")
    exe = str(d / "host_checks")
    oracle_obj = str(d / "oracle.o")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", *SAN, "-c", os.path.join(ROOT, "oracle", "prng_oracle.c"),
                    "-o", oracle_obj], check=True)
    srcs = [os.path.join(HERE, "host_checks.cpp")] + [os.path.join(CSRC, f) for f in
                                                      ("runtime.cpp", "table.cpp", "server.cpp", "jump.cpp")]
    cxx = ["g++", "-std=c++20", "-O1", "-g", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", CSRC,
           "-I", os.path.join(ROOT, "include")]
    objs = [str(d / (os.path.basename(s) + ".o")) for s in srcs]
    procs = [subprocess.Popen(cxx + ["-c", s, "-o", o]) for s, o in zip(srcs, objs)]
    assert all(p.wait() == 0 for p in procs), "compile failed"
    subprocess.run(["g++", *SAN, *objs, oracle_obj, "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64",
                    "-lpthread", "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, f"host checks failed (rc {r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r.stdout


@pytest.mark.parametrize("check", ["seeding", "planner", "jumps", "server_book", "arena", "oracle", "all"])
def test_host_code_under_sanitizers(checks_output, check):
    assert any(line.startswith(check + " ok") for line in checks_output.splitlines()), checks_output
