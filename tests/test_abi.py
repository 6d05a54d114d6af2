"""CPU checks of the C-ABI: the library loads, exports every declared entry
point, and the ctypes structures match the C layout of include/bnx.h."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bnx.h")
LIB = os.path.join(ROOT, "paper_1312_1553_amd", "libbnx.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(bnx_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1312_1553_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_1312_1553_amd import bnx
    assert sorted(bnx.EXPORTS) == declared()
    for n in declared():
        assert callable(getattr(bnx, n)), n


def test_struct_layout_matches_header():
    from paper_1312_1553_amd import bnx
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "bnx.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(bnx_solve_opts), offsetof(bnx_solve_opts, seed),
         offsetof(bnx_solve_opts, x0), offsetof(bnx_solve_opts, keep_bfgs), offsetof(bnx_solve_opts, newton),
         offsetof(bnx_solve_opts, bfgs_full), sizeof(bnx_stats), offsetof(bnx_stats, mvp_dacg),
         offsetof(bnx_stats, t_newton));
  printf("%zu %zu %zu %zu %zu\n", sizeof(bnx_factor_opts), offsetof(bnx_factor_opts, lfil),
         offsetof(bnx_factor_opts, tau_ic), offsetof(bnx_stats, nnz_L), offsetof(bnx_stats, fill));
  printf("%zu %zu\n", offsetof(bnx_solve_opts, jd), offsetof(bnx_solve_opts, jd_mmax));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    got = [int(x) for x in out]
    S, T = bnx.SolveOpts, bnx.Stats
    want = [ctypes.sizeof(S), S.seed.offset, S.x0.offset, S.keep_bfgs.offset, S.newton.offset, S.bfgs_full.offset,
            ctypes.sizeof(T), T.mvp_dacg.offset, T.t_newton.offset, ctypes.sizeof(bnx.FactorOpts),
            bnx.FactorOpts.lfil.offset, bnx.FactorOpts.tau_ic.offset, T.nnz_L.offset, T.fill.offset,
            S.jd.offset, S.jd_mmax.offset]
    assert got == want


def test_defaults_match_paper_table2(lib):
    import json
    from paper_1312_1553_amd import bnx
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "default_params.json")))
    o = bnx.bnx_default_solve_opts()
    assert o.tol == g["tau"] and o.itmax == g["itmax"] and o.tol_dacg == g["tau_dacg"]
    assert o.tol_pcg == g["tau_pcg"] and o.itmax_pcg == g["itmax_pcg"]
    assert o.kmax == 5 and o.precision == 0
    assert o.jd == 0 and o.jd_mmin == 5 and o.jd_mmax == 10  # Sec. 6
    f = bnx.bnx_default_factor_opts()
    assert f.lfil == g["lfil"] and f.tau_ic == g["tau_ic"] and f.ict == 0


def test_create_rejects_null_arguments(lib):
    """Argument checks that return before any device call."""
    from paper_1312_1553_amd import bnx
    L = bnx.load()
    h = ctypes.c_void_p()
    assert L.bnx_create_csr(ctypes.byref(h), 0, 0, None, None, None, 0, None) == -1
    assert L.bnx_create_csr(None, 4, 4, None, None, None, 0, None) == -1
    assert L.bnx_factor(None, None) == -1
    assert L.bnx_set_trsv_mode(None, 0) == -1
