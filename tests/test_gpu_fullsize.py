"""Parity at the full sizes of the benchmark configurations, through the C-ABI, in the launch
configuration bench.py times (default block schedule).

* Kernels (SpMV, both IC(0) triangular solves) on the full 100^3 diffusion (n = 10^6), Q1 elasticity
  (50^3 elements, n = 390,150) and 500k-node geometric graph Laplacian matrices,
  compared element by element with the FP64 oracle, which runs these single steps in well under a
  second.
* The full 100^3 diffusion eigensolve (p = 10) against the oracle's eigenvalues stored in tests/golden (written by
  tests/golden/make_oracle_evals.py, which calls only oracle/), plus residual and orthonormality.
* The differentiation case's backward at 64^3 through properties that hold at any size, and against central finite
  differences of the oracle's own solves at 16^3.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_1312_1553_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1312_1553_amd import bnx  # noqa: E402

FP64, MIXED = bnx.FP64, bnx.MIXED
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    oracle.build()
    return oracle


FULL = {
    "diffusion3d_100": lambda: W.diffusion_3d(100, seed=1),
    "elasticity_50": lambda: W.elasticity_q1(50, seed=2),
    "rgg_500k": lambda: W.rgg_laplacian(500_000, seed=3),
}


@pytest.mark.parametrize("name", list(FULL))
def test_fullsize_spmv_and_ic_solves(oracle_mod, name):
    A = FULL[name]()
    say("case fullsize kernels", name, A.n, A.nnz)
    S = bnx.Solver(A.rowptr, A.col, A.val)
    S.factor()
    F = oracle_mod.ic0(A)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(A.n)
    # a1: SpMV, 16 ulp of sum |a_ij x_j| per row in fp64 (any summation order), fp32 storage of A and x
    ref = oracle_mod.spmv(A, x)
    scale = abs(A.to_scipy()) @ np.abs(x)
    y = torch.empty(A.n, dtype=torch.float64, device="cuda")
    bnx.bnx_spmv(S.h, FP64, dev(x), y)
    assert np.all(np.abs(host(y) - ref) <= 16 * 2.0 ** -52 * scale + 1e-300)
    bnx.bnx_spmv(S.h, MIXED, dev(x), y)
    assert np.all(np.abs(host(y) - ref) <= 1e-6 * scale)
    # a0, a5, a6: the device factor against the oracle's, through L z = b, L^T c = b and both
    refs = [oracle_mod.lsolve(F, x), oracle_mod.ltsolve(F, x), oracle_mod.ltsolve(F, oracle_mod.lsolve(F, x))]
    for which in range(3):
        bnx.bnx_ic_apply(S.h, FP64, which, dev(x), y)
        e64 = np.abs(host(y) - refs[which]).max() / np.abs(refs[which]).max()
        bnx.bnx_ic_apply(S.h, MIXED, which, dev(x), y)
        e32 = np.abs(host(y) - refs[which]).max() / np.abs(refs[which]).max()
        say(f"  solve {which}: fp64 {e64:.2e} fp32 {e32:.2e}")
        assert e64 < 1e-11, (which, e64)  # observed <= 5e-13 (graph), 1e-15 (diffusion, elasticity)
        assert e32 < 1e-5, (which, e32)  # observed <= 3.5e-7 on these three matrices
    # which systems the substitutions run: FP64 the factor's own; FP32 the level-compressed ones on the graph
    # (176 rows per level; its long rows as virtual-row chains), the factor's own on the grid (3356 rows per level)
    # and on elasticity (whose substituted rows would hold 2.5x the entries)
    for prec in (FP64, MIXED):
        _, _, st = S.solve(1, precision=prec, itmax=1, tol_dacg=0.5)
        assert (st["levels_L"], st["levels_Lt"]) == LEVELS[name][prec], (name, prec)
    S.close()


LEVELS = {"diffusion3d_100": {FP64: (298, 298), MIXED: (298, 298)},
          "elasticity_50": {FP64: (1041, 1041), MIXED: (1041, 1041)},
          "rgg_500k": {FP64: (2835, 2835), MIXED: (1418, 1418)}}


def test_fullsize_diffusion100_solve_matches_oracle():
    g = json.load(open(os.path.join(GOLDEN, "oracle_evals_diffusion3d_100_p10.json")))
    p = g["p"]
    A = W.diffusion_3d(100, seed=1)
    S = bnx.Solver(A.rowptr, A.col, A.val)
    S.factor()
    x0 = torch.as_tensor(W.initial_block(A.n, p, 0)).cuda()
    ref = np.array(g["evals"])
    M = A.to_scipy()
    for prec in (FP64, MIXED):
        say("case fullsize diffusion 100^3 solve", prec)
        ev, V, st = S.solve(p, precision=prec, x0=x0)
        ev = ev.numpy()
        assert st["status"] == 0 and all(st["converged"][:p])
        # both precisions substitute with the factor's own systems on this grid (3356 rows per level)
        assert (st["levels_L"], st["levels_Lt"]) == (298, 298)
        # both sides stop at ||r|| <= 1e-8 theta; the eigenvalue error is then O(||r||^2 / gap), far below 1e-10
        rel = np.abs(ev - ref) / ref
        say("  max rel eigenvalue difference vs oracle", rel.max())
        assert rel.max() < 1e-10
        Vh = host(V)
        res = max(np.linalg.norm(M @ Vh[j] - ev[j] * Vh[j]) / ev[j] for j in range(p))
        assert res <= 1.0e-8 * 1.01, res
        G = (V @ V.T).cpu().numpy()
        assert np.abs(G - np.eye(p)).max() < 1e-10
    S.close()


def test_fullsize_rgg500k_solve_closed_form():
    """500k-node geometric graph, L + 1e-4 I, p = 10, the benchmark's configuration (level-compressed fp32
    solves with virtual-row chains): each connected component contributes an eigenvalue of exactly 1e-4
    (its constant vector), and the graph has more than p components, so every eigenvalue found is 1e-4.
    The residuals are checked by scipy on the host; orthonormality to 1e-10."""
    from scipy.sparse.csgraph import connected_components
    A = W.rgg_laplacian(500_000, seed=3)
    p = 10
    M = A.to_scipy()
    assert connected_components(M, directed=False)[0] > p
    S = bnx.Solver(A.rowptr, A.col, A.val)
    S.factor()
    x0 = torch.as_tensor(W.initial_block(A.n, p, 0)).cuda()
    for prec in (FP64, MIXED):
        say("case fullsize rgg 500k solve", prec)
        ev, V, st = S.solve(p, precision=prec, x0=x0)
        ev = ev.numpy()
        assert st["status"] == 0 and all(st["converged"][:p])
        say("  max |lambda - 1e-4| / 1e-4", np.abs(ev - 1e-4).max() / 1e-4)
        # relres <= 1e-8 bounds the eigenvalue error by (1e-8)^2 lambda / gap: far below 1e-10
        assert np.abs(ev - 1e-4).max() <= 1e-10 * 1e-4
        Vh = host(V)
        res = max(np.linalg.norm(M @ Vh[j] - ev[j] * Vh[j]) / ev[j] for j in range(p))
        assert res <= 1.0e-8 * 1.01, res
        assert np.abs(Vh @ Vh.T - np.eye(p)).max() < 1e-10
    S.close()


def test_fullsize_elasticity50_solve_matches_oracle():
    """Q1 elasticity on 50^3 elements, p = 20, the benchmark's configuration (six-slot split schedules): both
    precisions match the oracle's eigenvalues stored in tests/golden (written by make_oracle_evals.py, oracle only)
    to 1e-10 relative, reach the outer tolerance by scipy's residuals on the host and return orthonormal vectors."""
    g = json.load(open(os.path.join(GOLDEN, "oracle_evals_elasticity_50_p20.json")))
    ref = np.array(g["evals"])
    assert all(g["converged"])
    A = W.elasticity_q1(50, seed=2)
    assert (A.n, A.nnz) == (g["n"], g["nnz"])
    p = 20
    M = A.to_scipy()
    S = bnx.Solver(A.rowptr, A.col, A.val)
    S.factor()
    x0 = torch.as_tensor(W.initial_block(A.n, p, 0)).cuda()
    evs = []
    for prec in (FP64, MIXED):
        say("case fullsize elasticity 50 solve", prec)
        ev, V, st = S.solve(p, precision=prec, x0=x0)
        ev = ev.numpy()
        assert st["status"] == 0 and all(st["converged"][:p])
        assert np.all(np.diff(ev) >= 0) and ev[0] > 0
        err = (np.abs(ev - ref) / ref).max()
        say("  max rel eigenvalue error vs oracle", err, "pcg its", sum(st["pcg_its"]), "dacg its",
            sum(st["dacg_its"]))
        assert err <= 1e-10
        Vh = host(V)
        res = max(np.linalg.norm(M @ Vh[j] - ev[j] * Vh[j]) / ev[j] for j in range(p))
        say("  max relres", res)
        assert res <= 1.0e-8 * 1.01, res
        assert np.abs(Vh @ Vh.T - np.eye(p)).max() < 1e-10
        evs.append(ev)
    assert np.abs(evs[0] - evs[1]).max() / evs[0].max() < 1e-10
    S.close()


def test_fullsize_diffusion64_backward_properties():
    """64^3, p = 5, loss = sum(lambda) + sum_j w_j v_1[j]^2.  Scaling A leaves the eigenvectors unchanged and
    scales the eigenvalues, so <dL/dvals, vals> = sum(lambda); the eigenvalue part of the gradient is
    sum_i v_i[a] v_i[b] on every stored entry (checked on a sample); the gradient is symmetric."""
    pat, logk, w = W.diffusion_grad_case(64, seed=4)
    A = pat.csr(logk)
    p = 5
    S = bnx.Solver(A.rowptr, A.col, A.val)
    S.factor()
    x0 = torch.as_tensor(W.initial_block(A.n, p, 0)).cuda()
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    cols = A.col.astype(np.int64)
    # transpose position of every entry
    key = rows.astype(np.int64) * A.n + cols
    tkey = cols * A.n + rows
    tpos = np.searchsorted(key, tkey)
    for prec in (FP64, MIXED):
        say("case fullsize diffusion 64^3 backward", prec)
        ev, V, st = S.solve(p, precision=prec, x0=x0, tol=1e-10)
        assert st["status"] == 0
        ev = ev.numpy().astype(np.float64)
        Vh = host(V)
        GV = np.zeros((p, A.n))
        GV[0] = 2 * w * Vh[0]
        g = host(S.backward(np.ones(p), dev(GV)))
        homog = abs(float(g @ A.val) - ev.sum()) / ev.sum()
        say("  <grad, vals> vs sum(lambda):", homog)
        assert homog < 1e-8
        assert np.abs(g - g[tpos]).max() <= 1e-12 * np.abs(g).max()
        g_lam = host(S.backward(np.ones(p), None))
        smp = np.random.default_rng(7).integers(0, A.nnz, 2000)
        expect = (Vh[:, rows[smp]] * Vh[:, cols[smp]]).sum(axis=0)
        assert np.abs(g_lam[smp] - expect).max() <= 1e-12 * np.abs(expect).max()
    S.close()


def test_diffusion_backward_vs_oracle_finite_differences(oracle_mod):
    """16^3 (n = 4096), p = 5: directional derivatives of the GPU gradient w.r.t. log k along 8 random
    directions and 8 coordinates against central differences (h = 1e-4) of the oracle's solves at tol 1e-12,
    each to 1e-6 of the finite difference itself.  The random directions are non-negative with unit 2-norm:
    a step of h then moves log k by at most h per cell, and no direction cancels the derivative.  Against the
    exact gradient (torch eigh on the dense matrix, CPU) these finite differences are accurate to 2e-9
    (random) and 7e-8 (coordinates) relative, so the gate measures the library's gradient."""
    N, p, h = 16, 5, 1e-4
    pat, logk, w = W.diffusion_grad_case(N, seed=4)
    x0 = W.initial_block(pat.n, p, 0)

    def loss_oracle(lk):
        A = pat.csr(lk)
        ev, V, _, _ = oracle_mod.solve(A, p, x0=x0, tol=1e-12)
        return ev.sum() + (w * V[0] ** 2).sum()  # sign-invariant

    A = pat.csr(logk)
    S = bnx.Solver(A.rowptr, A.col, A.val)
    EigSolve = bnx.eigsh_autograd()
    rng = np.random.default_rng(11)
    dirs = []
    for _ in range(8):
        d = rng.uniform(0.0, 1.0, pat.n)
        dirs.append(d / np.linalg.norm(d))
    for c in rng.choice(pat.n, 8, replace=False):
        e = np.zeros(pat.n)
        e[c] = 1.0
        dirs.append(e)
    fd = [(loss_oracle(logk + h * d) - loss_oracle(logk - h * d)) / (2 * h) for d in dirs]
    for prec in (FP64, MIXED):
        say("case backward FD 16^3", prec)
        lkg = torch.tensor(logk, requires_grad=True, device="cuda")
        ev, Vg = EigSolve.apply(pat.values_torch(lkg), S, p, prec, {"tol": 1e-12, "x0": x0})
        loss = ev.sum() + (torch.tensor(w, device="cuda") * Vg[0] ** 2).sum()
        loss.backward()
        grad = host(lkg.grad)
        for d, f in zip(dirs, fd):
            got = float(grad @ d)
            err = abs(got - f) / abs(f)
            say(f"  d/dh {got:+.10e} fd {f:+.10e} rel err {err:.2e}")
            assert err <= 1e-6, (got, f)
    S.close()


def test_fullsize_diffusion100_ict_solves(oracle_mod):
    """IC(30, 1e-2) (Table 2's lfil and tau_IC) on the full 100^3 diffusion matrix: the host factor installed with its
    own block schedules, L z = b, L^T c = b and both against the oracle's factor."""
    A = W.diffusion_3d(100, seed=1)
    say("case fullsize diffusion 100^3 ict", A.n, A.nnz)
    S = bnx.Solver(A.rowptr, A.col, A.val)
    S.factor(ict=1, lfil=30, tau_ic=1e-2)
    F = oracle_mod.ict(A, 30, 1e-2)
    x = np.random.default_rng(6).standard_normal(A.n)
    y = torch.empty(A.n, dtype=torch.float64, device="cuda")
    refs = [oracle_mod.lsolve(F, x), oracle_mod.ltsolve(F, x), oracle_mod.ltsolve(F, oracle_mod.lsolve(F, x))]
    for which in range(3):
        bnx.bnx_ic_apply(S.h, FP64, which, dev(x), y)
        e64 = np.abs(host(y) - refs[which]).max() / np.abs(refs[which]).max()
        bnx.bnx_ic_apply(S.h, MIXED, which, dev(x), y)
        e32 = np.abs(host(y) - refs[which]).max() / np.abs(refs[which]).max()
        say(f"  solve {which}: fp64 {e64:.2e} fp32 {e32:.2e}")
        assert e64 < 1e-11, (which, e64)
        assert e32 < 1e-5, (which, e32)
    S.close()


@pytest.mark.parametrize("kmax", [0, 5])
def test_fullsize_diffusion100_jd_matches_oracle_evals(kmax):
    """Jacobi-Davidson (Sec. 6) on the full 100^3 diffusion problem, p = 10, fp64 and mixed: the same eigenvalues as the
    oracle's DACG-Newton run stored in tests/golden (the eigenpairs do not depend on the outer method),
    residuals by scipy, orthonormality."""
    g = json.load(open(os.path.join(GOLDEN, "oracle_evals_diffusion3d_100_p10.json")))
    p = g["p"]
    A = W.diffusion_3d(100, seed=1)
    S = bnx.Solver(A.rowptr, A.col, A.val)
    S.factor()
    x0 = torch.as_tensor(W.initial_block(A.n, p, 0)).cuda()
    ref = np.array(g["evals"])
    M = A.to_scipy()
    for prec in (FP64, MIXED):
        say("case fullsize diffusion 100^3 jd", kmax, prec)
        ev, V, st = S.solve(p, precision=prec, x0=x0, jd=1, kmax=kmax)
        ev = ev.numpy()
        assert st["status"] == 0 and all(st["converged"][:p]) and sum(st["dacg_its"]) == 0
        rel = np.abs(ev - ref) / ref
        say("  max rel eigenvalue difference vs oracle", rel.max())
        assert rel.max() < 1e-10
        Vh = host(V)
        for i in range(p):
            assert np.linalg.norm(M @ Vh[i] - ev[i] * Vh[i]) <= 1.01e-8 * ev[i]
        assert np.abs(Vh @ Vh.T - np.eye(p)).max() < 1e-10
    S.close()
