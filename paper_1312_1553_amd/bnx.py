"""ctypes binding of the bnx C-ABI (include/bnx.h).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch supplies device memory and the stream.  If ``libbnx.so`` cannot be
loaded the import of this module fails; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.environ.get("BNX_LIBPATH") or os.path.join(HERE, "libbnx.so")
MAX_P = 32
FP64, MIXED = 0, 1

STATUS = {0: "BNX_OK", 1: "BNX_NOT_CONVERGED", -1: "BNX_E_ARG", -2: "BNX_E_NOT_SPD", -3: "BNX_E_BREAKDOWN",
          -4: "BNX_E_HIP", -5: "BNX_E_NOMEM", -6: "BNX_E_STATE"}


class BnxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class SolveOpts(C.Structure):
    _fields_ = [("p", C.c_int), ("tol", C.c_double), ("itmax", C.c_int), ("tol_dacg", C.c_double),
                ("itmax_dacg", C.c_int), ("tol_pcg", C.c_double), ("itmax_pcg", C.c_int), ("kmax", C.c_int),
                ("precision", C.c_int), ("exit_rule", C.c_int), ("exit_xi", C.c_double), ("seed", C.c_uint64),
                ("x0", C.c_void_p), ("keep_bfgs", C.c_int), ("newton", C.c_int), ("bfgs_full", C.c_int),
                ("jd", C.c_int), ("jd_mmin", C.c_int), ("jd_mmax", C.c_int)]


class FactorOpts(C.Structure):
    _fields_ = [("shift0", C.c_double), ("shift_max", C.c_double), ("ict", C.c_int), ("lfil", C.c_int),
                ("tau_ic", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("dacg_its", C.c_int * MAX_P), ("outer_its", C.c_int * MAX_P), ("pcg_its", C.c_int * MAX_P),
                ("converged", C.c_int * MAX_P), ("relres", C.c_double * MAX_P), ("mvp_dacg", C.c_longlong),
                ("mvp_newton", C.c_longlong), ("bfgs_skipped", C.c_int), ("pcg_breakdowns", C.c_int),
                ("status", C.c_int), ("levels_L", C.c_int), ("levels_Lt", C.c_int), ("shift_used", C.c_double),
                ("t_factor", C.c_double), ("t_dacg", C.c_double), ("t_newton", C.c_double),
                ("dacg_restarts", C.c_int), ("nnz_L", C.c_longlong), ("fill", C.c_double)]

    def as_dict(self, p):
        return {"dacg_its": list(self.dacg_its[:p]), "outer_its": list(self.outer_its[:p]),
                "pcg_its": list(self.pcg_its[:p]), "converged": list(self.converged[:p]),
                "relres": list(self.relres[:p]), "mvp_dacg": self.mvp_dacg, "mvp_newton": self.mvp_newton,
                "bfgs_skipped": self.bfgs_skipped, "pcg_breakdowns": self.pcg_breakdowns, "status": self.status,
                "levels_L": self.levels_L, "levels_Lt": self.levels_Lt, "shift_used": self.shift_used,
                "t_factor": self.t_factor, "t_dacg": self.t_dacg, "t_newton": self.t_newton,
                "dacg_restarts": self.dacg_restarts, "nnz_L": self.nnz_L, "fill": self.fill}


EXPORTS = ["bnx_default_solve_opts", "bnx_default_factor_opts", "bnx_create_csr", "bnx_set_values", "bnx_factor",
           "bnx_solve", "bnx_backward", "bnx_set_adjoint_params", "bnx_last_error", "bnx_destroy", "bnx_spmv",
           "bnx_ic_apply", "bnx_ic_apply_noalloc", "bnx_prec_apply", "bnx_correction_solve", "bnx_dacg", "bnx_set_trsv_mode",
           "bnx_set_profiling", "bnx_kernel_time", "bnx_probe_latency", "bnx_factor_info"]

_lib = None
_vp = C.c_void_p


def load(path: str = LIBPATH):
    """Load libbnx.so (building it first only if no library exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    L = C.CDLL(path)
    L.bnx_default_solve_opts.argtypes = [C.POINTER(SolveOpts)]
    L.bnx_default_solve_opts.restype = None
    L.bnx_default_factor_opts.argtypes = [C.POINTER(FactorOpts)]
    L.bnx_default_factor_opts.restype = None
    L.bnx_create_csr.argtypes = [C.POINTER(_vp), C.c_int64, C.c_int64, _vp, _vp, _vp, C.c_int, _vp]
    L.bnx_set_values.argtypes = [_vp, _vp]
    L.bnx_factor.argtypes = [_vp, C.POINTER(FactorOpts)]
    L.bnx_solve.argtypes = [_vp, C.POINTER(SolveOpts), _vp, _vp, C.POINTER(Stats)]
    L.bnx_backward.argtypes = [_vp, _vp, _vp, _vp]
    L.bnx_set_adjoint_params.argtypes = [_vp, C.c_double, C.c_int]
    L.bnx_last_error.argtypes = [_vp]
    L.bnx_last_error.restype = C.c_char_p
    L.bnx_destroy.argtypes = [_vp]
    L.bnx_destroy.restype = None
    L.bnx_spmv.argtypes = [_vp, C.c_int, _vp, _vp]
    L.bnx_ic_apply.argtypes = [_vp, C.c_int, C.c_int, _vp, _vp]
    L.bnx_ic_apply_noalloc.argtypes = [_vp, C.c_int, C.c_int, _vp, _vp]
    L.bnx_prec_apply.argtypes = [_vp, C.c_int, C.c_int, _vp, _vp, C.c_int, _vp, _vp, _vp]
    L.bnx_correction_solve.argtypes = [_vp, C.c_int, C.c_int, _vp, C.c_int, _vp, _vp, C.c_double, C.c_int, C.c_double,
                                       C.c_int, C.c_double, _vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.bnx_dacg.argtypes = [_vp, C.c_int, C.c_int, _vp, _vp, C.c_double, C.c_int, _vp, C.POINTER(C.c_int)]
    L.bnx_set_trsv_mode.argtypes = [_vp, C.c_int]
    L.bnx_set_profiling.argtypes = [_vp, C.c_int]
    L.bnx_kernel_time.argtypes = [_vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_longlong)]
    L.bnx_probe_latency.argtypes = [_vp, C.c_int, C.c_int, C.POINTER(C.c_double)]
    L.bnx_factor_info.argtypes = [_vp, C.POINTER(C.c_longlong), C.POINTER(C.c_double), C.POINTER(C.c_int),
                                  C.POINTER(C.c_int), C.POINTER(C.c_double)]
    for f in EXPORTS:
        if f not in ("bnx_default_solve_opts", "bnx_default_factor_opts", "bnx_last_error", "bnx_destroy"):
            getattr(L, f).restype = C.c_int
    _lib = L
    return L


# ----------------------------------------------------------------------------- raw C-ABI names
def bnx_default_solve_opts() -> SolveOpts:
    o = SolveOpts()
    load().bnx_default_solve_opts(C.byref(o))
    return o


def bnx_default_factor_opts() -> FactorOpts:
    o = FactorOpts()
    load().bnx_default_factor_opts(C.byref(o))
    return o


def _check(handle, rc, allow=(0,)):
    if rc not in allow:
        msg = load().bnx_last_error(handle) if handle else b""
        raise BnxError(rc, (msg or b"").decode())
    return rc


def _ptr(x):
    """data pointer of a torch tensor or numpy array (contiguous)."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        assert x.is_contiguous()
        return x.data_ptr()
    assert x.flags["C_CONTIGUOUS"]
    return x.ctypes.data


def bnx_create_csr(n, nnz, rowptr, col, val, device_ptrs, stream=None):
    h = _vp()
    rc = load().bnx_create_csr(C.byref(h), n, nnz, _ptr(rowptr), _ptr(col), _ptr(val), int(device_ptrs), stream)
    if rc != 0:
        raise BnxError(rc, "bnx_create_csr failed")
    return h


def bnx_set_values(h, val):
    return _check(h, load().bnx_set_values(h, _ptr(val)))


def bnx_factor(h, opts: FactorOpts | None = None):
    return _check(h, load().bnx_factor(h, C.byref(opts) if opts is not None else None))


def bnx_solve(h, opts: SolveOpts, evals, evecs, stats: Stats | None = None):
    return _check(h, load().bnx_solve(h, C.byref(opts), _ptr(evals), _ptr(evecs),
                                       C.byref(stats) if stats is not None else None), allow=(0, 1))


def bnx_backward(h, g_evals, g_evecs, g_vals):
    return _check(h, load().bnx_backward(h, _ptr(g_evals), _ptr(g_evecs), _ptr(g_vals)))


def bnx_set_adjoint_params(h, tol, itmax):
    return _check(h, load().bnx_set_adjoint_params(h, tol, itmax))


def bnx_last_error(h) -> str:
    return (load().bnx_last_error(h) or b"").decode()


def bnx_destroy(h):
    load().bnx_destroy(h)


def bnx_spmv(h, precision, x, y):
    return _check(h, load().bnx_spmv(h, precision, _ptr(x), _ptr(y)))


def bnx_ic_apply(h, precision, which, b, x):
    return _check(h, load().bnx_ic_apply(h, precision, which, _ptr(b), _ptr(x)))


def bnx_ic_apply_noalloc(h, precision, which, b, x):
    return _check(h, load().bnx_ic_apply_noalloc(h, precision, which, _ptr(b), _ptr(x)))


def bnx_prec_apply(h, precision, k, S, R, m, Q, g, c):
    return _check(h, load().bnx_prec_apply(h, precision, k, _ptr(S), _ptr(R), m, _ptr(Q), _ptr(g), _ptr(c)))


def bnx_correction_solve(h, precision, m, Q, k, S, R, tol_pcg, itmax_pcg, tau, exit_rule, exit_xi, s):
    its, why = C.c_int(0), C.c_int(0)
    _check(h, load().bnx_correction_solve(h, precision, m, _ptr(Q), k, _ptr(S), _ptr(R), tol_pcg, itmax_pcg, tau,
                                           exit_rule, exit_xi, _ptr(s), C.byref(its), C.byref(why)))
    return its.value, why.value


def bnx_dacg(h, precision, m, Qt, x0, tol, itmax, x):
    its = C.c_int(0)
    _check(h, load().bnx_dacg(h, precision, m, _ptr(Qt), _ptr(x0), tol, itmax, _ptr(x), C.byref(its)))
    return its.value


def bnx_set_trsv_mode(h, mode):
    return _check(h, load().bnx_set_trsv_mode(h, mode))


def bnx_factor_info(h) -> dict:
    """nnz(L), fill ratio sigma, levels of the two solves and the shift of the installed factor."""
    nz, fill, ll, lt, sh = C.c_longlong(), C.c_double(), C.c_int(), C.c_int(), C.c_double()
    _check(h, load().bnx_factor_info(h, C.byref(nz), C.byref(fill), C.byref(ll), C.byref(lt), C.byref(sh)))
    return {"nnz_L": nz.value, "fill": fill.value, "levels_L": ll.value, "levels_Lt": lt.value,
            "shift_used": sh.value}


def bnx_probe_latency(h, kind, hops):
    """Microseconds per dependent hand-over: kind 0 LDS between waves, 1 global flag between workgroups."""
    us = C.c_double()
    _check(h, load().bnx_probe_latency(h, int(kind), int(hops), C.byref(us)))
    return us.value


def bnx_set_profiling(h, on):
    return _check(h, load().bnx_set_profiling(h, int(on)))


KERNEL_IDS = {"spmv_f64": 0, "spmv_f32": 1, "trsv_L_f64": 2, "trsv_L_f32": 3, "trsv_Lt_f64": 4, "trsv_Lt_f32": 5}


def bnx_kernel_time(h, kernel):
    """(milliseconds summed over timed launches, number of launches)."""
    ms, cnt = C.c_double(0), C.c_longlong(0)
    _check(h, load().bnx_kernel_time(h, kernel, C.byref(ms), C.byref(cnt)))
    return ms.value, cnt.value


# ----------------------------------------------------------------------------- object wrapper
class Solver:
    """One matrix on the current HIP device; inputs/outputs are torch tensors on cuda."""

    def __init__(self, rowptr, col, val):
        import torch
        self.torch = torch
        dev = torch.device("cuda", torch.cuda.current_device())
        self.rowptr = torch.as_tensor(np.asarray(rowptr, np.int32)).to(dev)
        self.col = torch.as_tensor(np.asarray(col, np.int32)).to(dev)
        val = torch.as_tensor(val, dtype=torch.float64).to(dev).contiguous()
        self.n = int(self.rowptr.numel() - 1)
        self.nnz = int(self.col.numel())
        self.stream = torch.cuda.current_stream().cuda_stream
        self.h = bnx_create_csr(self.n, self.nnz, self.rowptr, self.col, val, 1, self.stream)
        self.factored = False
        # bnx_backward differentiates the handle's most recent solve; each solve and each change of values
        # starts a new generation, so a backward for an older one can be refused instead of answered wrongly
        self.generation = 0

    def close(self):
        if getattr(self, "h", None):
            bnx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_values(self, val):
        val = self.torch.as_tensor(val, dtype=self.torch.float64).cuda().contiguous()
        bnx_set_values(self.h, val)
        self.factored = False
        self.generation += 1

    def factor(self, shift0=1e-3, shift_max=1.0, ict=0, lfil=30, tau_ic=1e-2):
        """IC(0) (ict=0) or IC(lfil, tau_ic) (ict=1) initial preconditioner (Sec. 2)."""
        bnx_factor(self.h, FactorOpts(shift0, shift_max, ict, lfil, tau_ic))
        self.factored = True

    def solve(self, p, precision=FP64, x0=None, **kw):
        """Returns (evals float64 cpu tensor [p], evecs float64 cuda tensor [p, n], stats dict)."""
        torch = self.torch
        if not self.factored:
            self.factor()
        o = bnx_default_solve_opts()
        o.p = p
        o.precision = precision
        for k, v in kw.items():
            setattr(o, k, v)
        x0t = None
        if x0 is not None:
            x0t = torch.as_tensor(x0, dtype=torch.float64).cuda().contiguous()
            assert x0t.shape == (p, self.n)
            o.x0 = x0t.data_ptr()
        ev = np.empty(p)
        V = torch.empty((p, self.n), dtype=torch.float64, device="cuda")
        st = Stats()
        self.generation += 1
        bnx_solve(self.h, o, ev, V, st)
        return torch.from_numpy(ev), V, st.as_dict(p)

    def backward(self, g_evals, g_evecs=None):
        torch = self.torch
        ge = np.ascontiguousarray(np.asarray(g_evals, dtype=np.float64))
        gV = None if g_evecs is None else torch.as_tensor(g_evecs, dtype=torch.float64).cuda().contiguous()
        out = torch.empty(self.nnz, dtype=torch.float64, device="cuda")
        bnx_backward(self.h, ge, gV, out)
        return out


def eigsh_autograd():
    """torch.autograd.Function: vals (nnz, cuda float64) -> (evals[p], evecs[p, n])."""
    import torch

    class EigSolve(torch.autograd.Function):
        @staticmethod
        def forward(ctx, vals, solver: Solver, p: int, precision: int, opts: dict):
            solver.set_values(vals.detach())
            solver.factor()
            ev, V, st = solver.solve(p, precision=precision, **(opts or {}))
            ctx.solver = solver
            ctx.p = p
            ctx.generation = solver.generation
            return ev.to(vals.device), V

        @staticmethod
        def backward(ctx, g_ev, g_V):
            if ctx.solver.generation != ctx.generation:
                raise RuntimeError("EigSolve.backward: the Solver has solved again (or changed its values) since this "
                                   "forward; the library keeps only the latest eigenpairs, so use one Solver per "
                                   "forward that is differentiated")
            ge = g_ev.detach().double().cpu().numpy() if g_ev is not None else np.zeros(ctx.p)
            gv = ctx.solver.backward(ge, None if g_V is None else g_V.detach())
            return gv, None, None, None, None

    return EigSolve
