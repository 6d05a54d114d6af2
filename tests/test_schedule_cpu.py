"""CPU checks of the host analysis behind the block triangular solve (tests/sched/check_sched.cpp).

The partition, block schedules (with and without virtual rows) and level-compressed systems are built by the
library's own analysis code, compiled for the host here, and the block solve is emulated sequentially: every
invariant the GPU kernel relies on is checked, and the solution is compared with plain substitution.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1312_1553_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the ROCm headers")
    exe = str(tmp_path_factory.mktemp("sched") / "check_sched")
    cmd = [gxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC, "-x", "c++",
           os.path.join(ROOT, "tests", "sched", "check_sched.cpp"), os.path.join(CSRC, "analysis.hip"), "-o", exe]
    subprocess.check_call(cmd)
    return exe


@pytest.mark.parametrize("case", ["grid", "elasticity", "graph"])
def test_block_schedules_emulated(checker, case):
    r = subprocess.run([checker, case], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "bad 0" in r.stdout


def test_level_pair_substitution_rule(checker):
    """Grids fit six dependencies per substituted row; the geometric graph's substituted rows are longer but add
    under half the entries (chains of virtual rows take the long ones); 27-point elasticity blocks would double
    them, so they keep the factor's own system."""
    r = subprocess.run([checker, "all"], capture_output=True, text=True, timeout=300)
    out = r.stdout
    assert "7-point 24^3: level-pair substitution applies (levels 70 -> 36, 70 -> 36, entries 53568 -> 71748)" in out
    assert "27-point 8^3 x 3 dof: level-pair substitution rejected" in out
    assert "geometric graph 4000: level-pair substitution applies (levels 338 -> 170, 338 -> 170" in out
    assert "geometric graph 4000 split lps forward" in out
