"""ctypes wrapper of the FP64 CPU oracle (``oracle.c``).

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  The HIP library never imports or links it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
MAXP = 32


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (plain -O2, single-threaded)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Opts(C.Structure):
    _fields_ = [("p", C.c_int), ("itmax", C.c_int), ("itmax_dacg", C.c_int), ("itmax_pcg", C.c_int),
                ("kmax", C.c_int), ("exit_rule", C.c_int), ("tol", C.c_double), ("tol_dacg", C.c_double),
                ("tol_pcg", C.c_double), ("exit_xi", C.c_double), ("shift0", C.c_double),
                ("shift_max", C.c_double), ("newton", C.c_int), ("bfgs_full", C.c_int), ("ict", C.c_int),
                ("lfil", C.c_int), ("tau_ic", C.c_double), ("jd", C.c_int), ("jd_mmin", C.c_int),
                ("jd_mmax", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("dacg_its", C.c_int * MAXP), ("outer_its", C.c_int * MAXP), ("pcg_its", C.c_int * MAXP),
                ("converged", C.c_int * MAXP), ("relres", C.c_double * MAXP), ("mvp_dacg", C.c_longlong),
                ("mvp_newton", C.c_longlong), ("bfgs_skipped", C.c_int), ("pcg_breakdowns", C.c_int),
                ("ntrace", C.c_int), ("status", C.c_int), ("shift_used", C.c_double), ("t_factor", C.c_double),
                ("t_dacg", C.c_double), ("t_newton", C.c_double), ("dacg_restarts", C.c_int),
                ("nnz_L", C.c_longlong), ("fill", C.c_double)]

    def as_dict(self, p: int) -> dict:
        return {
            "dacg_its": list(self.dacg_its[:p]), "outer_its": list(self.outer_its[:p]),
            "pcg_its": list(self.pcg_its[:p]), "converged": list(self.converged[:p]),
            "relres": list(self.relres[:p]), "mvp_dacg": self.mvp_dacg, "mvp_newton": self.mvp_newton,
            "bfgs_skipped": self.bfgs_skipped, "pcg_breakdowns": self.pcg_breakdowns,
            "status": self.status, "shift_used": self.shift_used, "t_factor": self.t_factor,
            "t_dacg": self.t_dacg, "t_newton": self.t_newton, "dacg_restarts": self.dacg_restarts,
            "nnz_L": self.nnz_L, "fill": self.fill,
        }


_lib = None
_pd = C.POINTER(C.c_double)
_pi = C.POINTER(C.c_int)


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        L.or_spmv.argtypes = [C.c_int, _pi, _pi, _pd, _pd, _pd]
        L.or_tril_nnz.argtypes = [C.c_int, _pi, _pi]
        L.or_tril_nnz.restype = C.c_int
        L.or_ic0.argtypes = [C.c_int, _pi, _pi, _pd, C.c_double, C.c_double, _pi, _pi, _pd, _pd]
        L.or_ic0.restype = C.c_int
        _ppi = C.POINTER(_pi)
        _ppd = C.POINTER(_pd)
        L.or_ict.argtypes = [C.c_int, _pi, _pi, _pd, C.c_int, C.c_double, C.c_double, C.c_double, _ppi, _ppi,
                             _ppd, _pd]
        L.or_ict.restype = C.c_int
        L.or_symeig.argtypes = [C.c_int, _pd, _pd, _pd]
        L.or_symeig.restype = None
        L.or_free.argtypes = [C.c_void_p]
        L.or_free.restype = None
        L.or_lsolve.argtypes = [C.c_int, _pi, _pi, _pd, _pd, _pd]
        L.or_ltsolve.argtypes = [C.c_int, _pi, _pi, _pd, _pd, _pd]
        L.or_linesearch.argtypes = [C.c_double] * 6
        L.or_linesearch.restype = C.c_double
        L.or_solve.argtypes = [C.c_int, _pi, _pi, _pd, C.POINTER(Opts), _pd, _pd, _pd, C.POINTER(Stats), _pd, C.c_int]
        L.or_solve.restype = C.c_int
        L.or_backward.argtypes = [C.c_int, _pi, _pi, _pd, C.c_int, _pd, _pd, _pd, _pd, C.c_double, C.c_int,
                                  C.c_double, C.c_double, _pd]
        L.or_backward.restype = C.c_int
        L.or_bfgspk_apply.argtypes = [C.c_int, _pi, _pi, _pd, C.c_int, _pd, _pd, C.c_int, _pd, _pd, _pd]
        L.or_pcg_apply.argtypes = [C.c_int, _pi, _pi, _pd, _pi, _pi, _pd, C.c_double, C.c_int, _pd, _pd, _pd, _pd,
                                   C.c_int, _pd, _pd, C.c_double, C.c_int, C.c_double, C.c_int, C.c_double, _pd, _pi]
        L.or_pcg_apply.restype = C.c_int
        L.or_dacg_apply.argtypes = [C.c_int, _pi, _pi, _pd, _pi, _pi, _pd, C.c_int, _pd, _pd, C.c_double, C.c_int,
                                    _pd, _pd, C.c_int]
        L.or_dacg_apply.restype = C.c_int
        L.or_window_apply.argtypes = [C.c_int, _pi, _pi, _pd, C.c_int, C.c_int, _pd, _pd, C.c_int, _pd, _pd, _pd]
        L.or_window_apply.restype = C.c_int
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_pd)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_pi)


NULLD = C.cast(None, _pd)


def default_opts(p: int, **kw) -> Opts:
    """Defaults of the paper's parameter table (tau 1e-8, IMAX 100, tau_DACG 1e-2,
    tau_PCG 1e-2, IMAX_PCG 20) with k_max = 5 and the floor exit rule (xi = 0.1).
    newton=0 runs DACG alone to tau (the DACG rows of Tables 4, 5, 7 and 8); bfgs_full=1 stores the
    pairs of eq. (2.1) with y_k = r_{k+1} - r_k instead of the simplified y_k ~ -r_k of eq. (2.2); ict=1
    preconditions with IC(lfil, tau_ic) (Sec. 2; lfil 30, tau_IC 1e-2 as in Table 2) instead of IC(0); jd=1 runs
    the Jacobi-Davidson outer iteration of Sec. 6 (m_min 5, m_max 10) with the same PCG as correction solver."""
    d = dict(p=p, itmax=100, itmax_dacg=5000, itmax_pcg=20, kmax=5, exit_rule=1, tol=1e-8, tol_dacg=1e-2,
             tol_pcg=1e-2, exit_xi=0.1, shift0=1e-3, shift_max=1.0, newton=1, bfgs_full=0, ict=0, lfil=30,
             tau_ic=1e-2, jd=0, jd_mmin=5, jd_mmax=10)
    d.update(kw)
    return Opts(**d)


def spmv(A, x):
    rp, prp = _i(A.rowptr); ci, pci = _i(A.col); v, pv = _d(A.val); x, px = _d(x)
    y = np.empty(A.n); _, py = _d(y)
    lib().or_spmv(A.n, prp, pci, pv, px, py)
    return y


class Factor:
    """Incomplete Cholesky factor in CSR (rows of L, diagonal last)."""

    def __init__(self, rowptr, col, val, shift):
        self.rowptr, self.col, self.val, self.shift = rowptr, col, val, shift

    @property
    def n(self):
        return len(self.rowptr) - 1

    def dense(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n)).toarray()


def ic0(A, shift0=1e-3, shift_max=1.0) -> Factor:
    rp, prp = _i(A.rowptr); ci, pci = _i(A.col); v, pv = _d(A.val)
    nl = lib().or_tril_nnz(A.n, prp, pci)
    Lrp = np.empty(A.n + 1, np.int32); Lci = np.empty(nl, np.int32); Lv = np.empty(nl)
    sh = C.c_double(0)
    rc = lib().or_ic0(A.n, prp, pci, pv, shift0, shift_max, Lrp.ctypes.data_as(_pi), Lci.ctypes.data_as(_pi),
                      Lv.ctypes.data_as(_pd), C.byref(sh))
    if rc != 0:
        raise RuntimeError(f"IC(0) failed (code {rc})")
    return Factor(Lrp, Lci, Lv, sh.value)


def ict(A, lfil=30, tau=1e-2, shift0=1e-3, shift_max=1.0) -> Factor:
    """IC(lfil, tau_IC) factor of Sec. 2 (dropping rule at or_ict in oracle.c)."""
    rp, prp = _i(A.rowptr); ci, pci = _i(A.col); v, pv = _d(A.val)
    pLrp = _pi(); pLci = _pi(); pLv = _pd()
    sh = C.c_double(0)
    rc = lib().or_ict(A.n, prp, pci, pv, int(lfil), float(tau), shift0, shift_max, C.byref(pLrp), C.byref(pLci),
                      C.byref(pLv), C.byref(sh))
    if rc != 0:
        raise RuntimeError(f"IC(lfil, tau) failed (code {rc})")
    n = A.n
    Lrp = np.ctypeslib.as_array(pLrp, shape=(n + 1,)).copy()
    nl = int(Lrp[n])
    Lci = np.ctypeslib.as_array(pLci, shape=(nl,)).copy()
    Lv = np.ctypeslib.as_array(pLv, shape=(nl,)).copy()
    for q in (pLrp, pLci, pLv):
        lib().or_free(C.cast(q, C.c_void_p))
    return Factor(Lrp, Lci, Lv, sh.value)


def symeig(H):
    """Cyclic Jacobi eigen-decomposition of a small symmetric matrix: (ascending values, vectors as columns)."""
    m = H.shape[0]
    Hw = np.ascontiguousarray(H, dtype=np.float64).copy()
    ev = np.empty(m); Y = np.empty(m * m)
    lib().or_symeig(m, Hw.ctypes.data_as(_pd), ev.ctypes.data_as(_pd), Y.ctypes.data_as(_pd))
    return ev, Y.reshape(m, m).T.copy()


def lsolve(F: Factor, b):
    b, pb = _d(b); x = np.empty(F.n)
    lib().or_lsolve(F.n, F.rowptr.ctypes.data_as(_pi), F.col.ctypes.data_as(_pi), F.val.ctypes.data_as(_pd), pb,
                    x.ctypes.data_as(_pd))
    return x


def ltsolve(F: Factor, b):
    b, pb = _d(b); x = np.empty(F.n)
    lib().or_ltsolve(F.n, F.rowptr.ctypes.data_as(_pi), F.col.ctypes.data_as(_pi), F.val.ctypes.data_as(_pd), pb,
                     x.ctypes.data_as(_pd))
    return x


def bfgspk(F: Factor, S, R, Q, g):
    """Alg. 1 with pairs S, R (k x n, oldest first) and projection rows Q (m x n)."""
    n = F.n
    S = np.zeros((0, n)) if S is None else np.atleast_2d(S)
    R = np.zeros((0, n)) if R is None else np.atleast_2d(R)
    Q = np.zeros((0, n)) if Q is None else np.atleast_2d(Q)
    S, pS = _d(S); R, pR = _d(R); Q, pQ = _d(Q); g, pg = _d(g)
    c = np.empty(n)
    lib().or_bfgspk_apply(n, F.rowptr.ctypes.data_as(_pi), F.col.ctypes.data_as(_pi), F.val.ctypes.data_as(_pd),
                          S.shape[0], pS, pR, Q.shape[0], pQ, pg, c.ctypes.data_as(_pd))
    return c


def window_bfgspk(F: Factor, kmax, S, R, Q, g):
    """Push the pairs (rows of S, R, in production order) through the k_max window, then Alg. 1 with the pairs
    it kept.  Returns (c, number kept)."""
    n = F.n
    Q = np.zeros((0, n)) if Q is None else np.atleast_2d(Q)
    S, pS = _d(np.atleast_2d(S)); R, pR = _d(np.atleast_2d(R)); Q, pQ = _d(Q); g, pg = _d(g)
    c = np.empty(n)
    kept = lib().or_window_apply(n, F.rowptr.ctypes.data_as(_pi), F.col.ctypes.data_as(_pi),
                                 F.val.ctypes.data_as(_pd), int(kmax), S.shape[0], pS, pR, Q.shape[0], pQ, pg,
                                 c.ctypes.data_as(_pd))
    return c, kept


def pcg(A, F: Factor, theta, Q, u, Au, r, S=None, R=None, tol_pcg=1e-2, itmax_pcg=20, tau=1e-8, exit_rule=1,
        xi=0.1):
    """One PCG solve of the correction equation; returns (s, its, reason)."""
    n = A.n
    S = np.zeros((0, n)) if S is None else np.atleast_2d(S)
    R = np.zeros((0, n)) if R is None else np.atleast_2d(R)
    Q = np.atleast_2d(Q)
    rp, prp = _i(A.rowptr); ci, pci = _i(A.col); v, pv = _d(A.val)
    Q, pQ = _d(Q); u, pu = _d(u); Au, pAu = _d(Au); r, pr = _d(r); S, pS = _d(S); R, pR = _d(R)
    s = np.empty(n); its = C.c_int(0)
    why = lib().or_pcg_apply(n, prp, pci, pv, F.rowptr.ctypes.data_as(_pi), F.col.ctypes.data_as(_pi),
                             F.val.ctypes.data_as(_pd), theta, Q.shape[0], pQ, pu, pAu, pr, S.shape[0], pS, pR,
                             tol_pcg, itmax_pcg, tau, exit_rule, xi, s.ctypes.data_as(_pd), C.byref(its))
    return s, its.value, why


def dacg(A, F: Factor, Qt, x0, tol=1e-2, itmax=5000):
    """DACG alone; returns (x, its, q_history)."""
    n = A.n
    Qt = np.zeros((0, n)) if Qt is None else np.atleast_2d(Qt)
    rp, prp = _i(A.rowptr); ci, pci = _i(A.col); v, pv = _d(A.val)
    Qt, pQ = _d(Qt); x0, px0 = _d(x0)
    x = np.empty(n); hist = np.full(itmax, np.nan)
    its = lib().or_dacg_apply(n, prp, pci, pv, F.rowptr.ctypes.data_as(_pi), F.col.ctypes.data_as(_pi),
                              F.val.ctypes.data_as(_pd), Qt.shape[0], pQ, px0, tol, itmax, x.ctypes.data_as(_pd),
                              hist.ctypes.data_as(_pd), itmax)
    return x, its, hist[:its]


def linesearch(xAx, dAx, dAd, xx, xd, dd):
    return lib().or_linesearch(xAx, dAx, dAd, xx, xd, dd)


def solve(A, p, x0=None, trace_cap=0, **kw):
    """DACG-Newton (Alg. 2).  Returns (evals, evecs (p x n), stats dict, trace (ntrace x 8)).  Trace rows are
    outer steps (j, k, theta_k, ||r_k||, s_k^T r_k, ||s_k||^2, theta_{k+1}, PCG its) and, with k = -1, returns to
    DACG from a stalled Newton phase (j, -1, DACG tolerance, DACG its, theta, ||r|| after, theta, ||r|| before)."""
    from paper_1312_1553_amd.workloads import initial_block
    n = A.n
    if x0 is None:
        x0 = initial_block(n, p, 0)
    o = default_opts(p, **kw)
    rp, prp = _i(A.rowptr); ci, pci = _i(A.col); v, pv = _d(A.val); x0, px0 = _d(x0)
    ev = np.empty(p); V = np.empty((p, n)); st = Stats()
    tr = np.zeros((max(trace_cap, 1), 8))
    rc = lib().or_solve(n, prp, pci, pv, C.byref(o), px0, ev.ctypes.data_as(_pd), V.ctypes.data_as(_pd),
                        C.byref(st), tr.ctypes.data_as(_pd) if trace_cap else NULLD, trace_cap)
    if rc < 0:
        raise RuntimeError(f"oracle solve failed ({rc})")
    d = st.as_dict(p)
    return ev, V, d, tr[: st.ntrace]


def backward(A, evals, evecs, g_evals, g_evecs=None, tol=1e-12, itmax=2000, shift0=1e-3, shift_max=1.0):
    """Gradient of a loss of (lambda, V) w.r.t. the CSR values (nnz)."""
    n = A.n
    p = len(evals)
    rp, prp = _i(A.rowptr); ci, pci = _i(A.col); v, pv = _d(A.val)
    ev, pev = _d(evals); V, pV = _d(evecs); ge, pge = _d(g_evals)
    if g_evecs is not None:
        GV, pGV = _d(g_evecs)
    else:
        pGV = NULLD
    out = np.empty(A.nnz)
    rc = lib().or_backward(n, prp, pci, pv, p, pev, pV, pge, pGV, tol, itmax, shift0, shift_max,
                           out.ctypes.data_as(_pd))
    if rc < 0:
        raise RuntimeError("oracle backward failed")
    return out
