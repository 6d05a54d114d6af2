"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The library's host analysis (partition, block schedules, level-pair substitution), compiled with g++ from
  csrc/analysis.hip together with the emulator tests/sched/check_sched.cpp, on its grid, elasticity and graph
  cases.
* The FP64 oracle (oracle/oracle.c), linked into tests/sanitize/oracle_driver.c, which calls every entry point.
Any sanitizer report makes the run fail (halt on the first error).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1312_1553_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, timeout):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=ENV)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "LeakSanitizer" not in out, out[-4000:]
    return r, out


@pytest.fixture(scope="module")
def sched_asan(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path_factory.mktemp("asan") / "check_sched")
    subprocess.check_call([gxx, *SAN, "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC,
                           "-x", "c++", os.path.join(ROOT, "tests", "sched", "check_sched.cpp"),
                           os.path.join(CSRC, "analysis.hip"), "-o", exe])
    return exe


@pytest.mark.parametrize("case", ["grid", "elasticity", "graph"])
def test_host_analysis_clean_under_sanitizers(sched_asan, case):
    r, out = _run([sched_asan, case], 900)
    assert r.returncode == 0 and "bad 0" in out, out[-3000:]


def test_oracle_clean_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("needs gcc")
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call([gcc, *SAN, "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-D_DEFAULT_SOURCE",
                           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe, "-lm"])
    r, out = _run([exe], 300)
    assert r.returncode == 0 and "bad 0" in out, out[-3000:]
