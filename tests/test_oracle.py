"""Pins of the FP64 CPU oracle against facts the paper and the mathematics fix.

None of these tests compares the oracle with itself: each checks it against a
closed form, a dense library routine (numpy/scipy/torch), an identity the
paper states or implies, or brute force on a tiny input.
"""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from paper_1312_1553_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def dense(A):
    return A.to_scipy().toarray()


def small_mats():
    return [W.laplacian_2d(8), W.diffusion_3d(5, seed=1), W.elasticity_q1(2, seed=2), W.rgg_laplacian(300, seed=3)]


# ----------------------------------------------------------------------------- SpMV / IC(0) / solves
def test_spmv_matches_dense(oracle_lib):
    rng = np.random.default_rng(0)
    for A in small_mats():
        x = rng.standard_normal(A.n)
        np.testing.assert_allclose(oracle_lib.spmv(A, x), dense(A) @ x, rtol=1e-13, atol=1e-13)


def test_ic0_reproduces_A_on_its_pattern(oracle_lib):
    """IC(0): (L L^T)_ij = A_ij on pattern(A), L on pattern(tril A), fill ratio sigma = 1 (Sec. 5)."""
    for A in small_mats():
        F = oracle_lib.ic0(A)
        assert F.shift == 0.0
        L = F.dense()
        Ad = dense(A)
        assert np.allclose(L, np.tril(L))
        pat = Ad != 0
        assert np.array_equal(L != 0, np.tril(pat)) or np.all((L != 0) <= np.tril(pat))
        assert len(F.val) == int(np.count_nonzero(np.tril(pat)))  # sigma = 1
        LLt = L @ L.T
        scale = np.abs(Ad).max()
        assert np.abs((LLt - Ad)[pat]).max() <= 1e-13 * scale


def test_ic0_equals_cholesky_without_fill(oracle_lib):
    """For a tridiagonal SPD matrix IC(0) is the exact Cholesky factor (numpy)."""
    n = 50
    rng = np.random.default_rng(1)
    off = -rng.uniform(0.1, 1.0, n - 1)
    d = np.abs(np.r_[off, 0]) + np.abs(np.r_[0, off]) + rng.uniform(0.01, 0.5, n)
    T = sp.diags([off, d, off], [-1, 0, 1]).tocsr()
    A = W._from_scipy(T)
    L = oracle_lib.ic0(A).dense()
    np.testing.assert_allclose(L, np.linalg.cholesky(T.toarray()), rtol=1e-13, atol=1e-15)


def test_ic0_breakdown_and_shift(oracle_lib):
    g = json.load(open(os.path.join(GOLD, "kershaw.json")))
    Ad = np.array(g["A"], float)
    np.testing.assert_allclose(np.linalg.eigvalsh(Ad), g["eigenvalues"], rtol=1e-12)
    A = W._from_scipy(sp.csr_matrix(Ad))
    with pytest.raises(RuntimeError):
        oracle_lib.ic0(A, shift0=0.0, shift_max=0.0)
    F = oracle_lib.ic0(A, shift0=1e-3, shift_max=1.0)
    a = F.shift
    assert a > 0 and np.isclose(a / 1e-3, 2 ** round(np.log2(a / 1e-3)))  # a = shift0 * 2^m
    L = F.dense()
    As = Ad + a * np.diag(np.diag(Ad))
    pat = Ad != 0
    assert np.abs((L @ L.T - As)[pat]).max() < 1e-13
    # the previous shift in the schedule still breaks down
    if a > 1e-3:
        with pytest.raises(RuntimeError):
            oracle_lib.ic0(A, shift0=1e-3, shift_max=a / 2)


def test_triangular_solves_match_scipy(oracle_lib):
    rng = np.random.default_rng(2)
    for A in small_mats():
        F = oracle_lib.ic0(A)
        L = F.dense()
        b = rng.standard_normal(A.n)
        np.testing.assert_allclose(oracle_lib.lsolve(F, b), sla.solve_triangular(L, b, lower=True), rtol=1e-12,
                                   atol=1e-12)
        np.testing.assert_allclose(oracle_lib.ltsolve(F, b), sla.solve_triangular(L.T, b, lower=False),
                                   rtol=1e-12, atol=1e-12)


# ----------------------------------------------------------------------------- BFGS preconditioner (Alg. 1)
def _pairs(Ad, k, rng, n):
    """k pairs (s, r) with s^T r < 0, as produced near convergence (r ~ -J s)."""
    S = rng.standard_normal((k, n))
    R = -(S @ Ad) + 0.05 * rng.standard_normal((k, n))
    for t in range(k):
        assert S[t] @ R[t] < 0
    return S, R


def _dense_bfgs(P0, S, R):
    """eq. (2.2) applied recursively: P_{k+1} = -ss'/s'r + (I - s r'/s'r) P_k (I - r s'/s'r)."""
    n = P0.shape[0]
    P = P0.copy()
    I = np.eye(n)
    for s, r in zip(S, R):
        a = s @ r
        P = -np.outer(s, s) / a + (I - np.outer(s, r) / a) @ P @ (I - np.outer(r, s) / a)
    return P


def test_bfgspk_k0_is_projected_ic(oracle_lib):
    A = W.diffusion_3d(4, seed=1)
    F = oracle_lib.ic0(A)
    L = F.dense()
    rng = np.random.default_rng(3)
    Q = np.linalg.qr(rng.standard_normal((A.n, 3)))[0].T
    g = rng.standard_normal(A.n)
    g -= Q.T @ (Q @ g)
    c = oracle_lib.bfgspk(F, None, None, Q, g)
    P0 = np.linalg.inv(L @ L.T)
    Pr = np.eye(A.n) - Q.T @ Q
    np.testing.assert_allclose(c, Pr @ P0 @ g, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 5])
def test_bfgspk_two_loop_equals_dense_update(oracle_lib, k):
    """Alg. 1 equals (I-QQ')P_k(I-QQ') g with P_k from eq. (2.2) (Sec. 4.2, eq. (4.1))."""
    A = W.diffusion_3d(4, seed=1)
    Ad = dense(A)
    F = oracle_lib.ic0(A)
    L = F.dense()
    rng = np.random.default_rng(4 + k)
    S, R = _pairs(Ad, k, rng, A.n)
    Q = np.linalg.qr(rng.standard_normal((A.n, 2)))[0].T
    g = rng.standard_normal(A.n)
    g -= Q.T @ (Q @ g)
    Pk = _dense_bfgs(np.linalg.inv(L @ L.T), S, R)
    Pr = np.eye(A.n) - Q.T @ Q
    ref = Pr @ Pk @ Pr @ g
    c = oracle_lib.bfgspk(F, S, R, Q, g)
    np.testing.assert_allclose(c, ref, rtol=1e-9, atol=1e-11 * np.abs(ref).max())


def test_bfgs_secant_condition(oracle_lib):
    """The newest pair satisfies P_{k+1}(-r_k) = s_k exactly (eq. (2.2) with y = -r)."""
    A = W.laplacian_2d(6)
    F = oracle_lib.ic0(A)
    rng = np.random.default_rng(5)
    S, R = _pairs(dense(A), 4, rng, A.n)
    c = oracle_lib.bfgspk(F, S, R, None, -R[-1])
    np.testing.assert_allclose(c, S[-1], rtol=1e-10, atol=1e-12)
    # an older pair does not (in general) satisfy it: the order of the loops matters
    c_old = oracle_lib.bfgspk(F, S, R, None, -R[0])
    assert np.abs(c_old - S[0]).max() > 1e-6


def test_bfgs_preconditioner_spd(oracle_lib):
    """Theorem 3.2: with every s^T r < 0 each P_k stays symmetric positive definite."""
    A = W.laplacian_2d(6)
    n = A.n
    F = oracle_lib.ic0(A)
    rng = np.random.default_rng(6)
    S, R = _pairs(dense(A), 3, rng, n)
    P = np.column_stack([oracle_lib.bfgspk(F, S, R, None, e) for e in np.eye(n)])
    assert np.abs(P - P.T).max() < 1e-10 * np.abs(P).max()
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0


# ----------------------------------------------------------------------------- PCG (Sec. 4.3)
def _near_eigvec(Ad, j, eps, seed):
    w, V = np.linalg.eigh(Ad)
    rng = np.random.default_rng(seed)
    u = V[:, j] + eps * rng.standard_normal(len(w))
    u -= V[:, :j] @ (V[:, :j].T @ u)
    return u / np.linalg.norm(u), w, V


def test_pcg_solves_projected_correction_equation(oracle_lib):
    """With tight tolerance the PCG iterate solves J s = -r on Q-perp (eq. (1.2), Sec. 3.2)."""
    A = W.diffusion_3d(5, seed=1)  # simple eigenvalues
    Ad = dense(A)
    F = oracle_lib.ic0(A)
    u, w, V = _near_eigvec(Ad, 1, 1e-2, 7)
    Qt = V[:, :1].T
    Q = np.vstack([Qt, u])
    theta = u @ Ad @ u
    Au = Ad @ u
    r = Au - theta * u
    s, its, why = oracle_lib.pcg(A, F, theta, Q, u, Au, r, tol_pcg=1e-13, itmax_pcg=500, tau=0.0, exit_rule=0)
    Pr = np.eye(A.n) - Q.T @ Q
    J = Pr @ (Ad - theta * np.eye(A.n)) @ Pr
    s_ref = -np.linalg.pinv(J, rcond=1e-12) @ (Pr @ r)
    np.testing.assert_allclose(s, s_ref, rtol=1e-8, atol=1e-10 * np.abs(s_ref).max())
    assert abs(Q @ s).max() < 1e-12 * np.linalg.norm(s)


def test_pcg_galerkin_identity(oracle_lib):
    """PCG from s = 0 keeps s^T r = -s^T J s < 0 at any stopping point (the condition of Theorem 3.2)."""
    A = W.diffusion_3d(5, seed=1)
    Ad = dense(A)
    F = oracle_lib.ic0(A)
    u, w, V = _near_eigvec(Ad, 0, 3e-3, 8)
    theta = u @ Ad @ u
    Au = Ad @ u
    r = Au - theta * u
    Q = u[None, :]
    for itmax in (1, 3, 7):
        s, its, why = oracle_lib.pcg(A, F, theta, Q, u, Au, r, tol_pcg=1e-14, itmax_pcg=itmax, tau=0.0,
                                     exit_rule=0)
        assert its == itmax
        Pr = np.eye(A.n) - np.outer(u, u)
        sJs = s @ Pr @ (Ad - theta * np.eye(A.n)) @ Pr @ s
        assert s @ r < 0
        assert abs(s @ r + sJs) <= 1e-10 * abs(sJs)
        # eq. (3.1): ||u + s|| = sqrt(1 + ||s||^2) because s is orthogonal to u
        assert abs(np.linalg.norm(u + s) - np.sqrt(1 + s @ s)) < 1e-13


def test_pcg_exit_tests(oracle_lib):
    """Exit (i) relative residual and (ii) iteration cap are honoured."""
    A = W.diffusion_3d(5, seed=1)
    Ad = dense(A)
    F = oracle_lib.ic0(A)
    u, w, V = _near_eigvec(Ad, 0, 3e-3, 9)
    theta = u @ Ad @ u
    Au = Ad @ u
    r = Au - theta * u
    s, its, why = oracle_lib.pcg(A, F, theta, u[None], u, Au, r, tol_pcg=1e-2, itmax_pcg=100, tau=0.0, exit_rule=0)
    assert why == 1  # PCG_EXIT_TOL
    Pr = np.eye(A.n) - np.outer(u, u)
    g = -Pr @ r - Pr @ (Ad - theta * np.eye(A.n)) @ Pr @ s
    assert np.linalg.norm(g) <= 1e-2 * np.linalg.norm(Pr @ r) * (1 + 1e-9)
    s, its, why = oracle_lib.pcg(A, F, theta, u[None], u, Au, r, tol_pcg=1e-14, itmax_pcg=2, tau=0.0, exit_rule=0)
    assert why == 0 and its == 2


# ----------------------------------------------------------------------------- DACG (Sec. 4.1)
def test_linesearch_is_the_minimiser(oracle_lib):
    rng = np.random.default_rng(10)
    M = rng.standard_normal((6, 6))
    M = M @ M.T + np.eye(6)
    for _ in range(20):
        x, d = rng.standard_normal(6), rng.standard_normal(6)
        a = oracle_lib.linesearch(x @ M @ x, d @ M @ x, d @ M @ d, x @ x, x @ d, d @ d)
        q = lambda t: (x + t * d) @ M @ (x + t * d) / ((x + t * d) @ (x + t * d))
        grid = np.linspace(-50, 50, 200001)
        qs = np.array([q(t) for t in grid[::50]])
        assert q(a) <= qs.min() + 1e-12
        # and the minimum over span{x, d} is the smaller Ritz value of the 2x2 pencil
        B = np.column_stack([x, d])
        ritz = sla.eigh(B.T @ M @ B, B.T @ B, eigvals_only=True)[0]
        assert abs(q(a) - ritz) <= 1e-10 * abs(ritz)


def test_dacg_monotone_and_deflated(oracle_lib):
    A = W.diffusion_3d(6, seed=1)
    Ad = dense(A)
    F = oracle_lib.ic0(A)
    w, V = np.linalg.eigh(Ad)
    Qt = V[:, :2].T
    x0 = W.initial_block(A.n, 1, 0)[0]
    x, its, hist = oracle_lib.dacg(A, F, Qt, x0, tol=1e-6, itmax=500)
    assert its > 2
    assert np.all(np.diff(hist) <= 1e-14 * abs(hist[0]))
    q = x @ Ad @ x
    assert np.linalg.norm(Ad @ x - q * x) <= 1e-6 * q * (1 + 1e-6)
    assert abs(Qt @ x).max() < 1e-10
    assert abs(q - w[2]) < 1e-9 * w[2]  # converges to the third eigenvalue


# ----------------------------------------------------------------------------- full solver (Alg. 2)
def _check_pairs(A, ev, Vr, tol=1e-8):
    Ad = A.to_scipy()
    for j in range(len(ev)):
        assert np.linalg.norm(Ad @ Vr[j] - ev[j] * Vr[j]) <= tol * ev[j] * (1 + 1e-9)
    assert np.abs(Vr @ Vr.T - np.eye(len(ev))).max() < 1e-12


def test_solve_laplace2d_closed_form(oracle_lib):
    A, p = W.config_small()
    ev, Vr, st, tr = oracle_lib.solve(A, p, x0=W.initial_block(A.n, p, 0), trace_cap=500)
    ref = W.laplacian_2d_eigs(32)[:p]
    # closed form 4 sin^2(i pi/66) + 4 sin^2(j pi/66)
    assert abs(ref[0] - (8 * np.sin(np.pi / 66) ** 2)) < 1e-16
    np.testing.assert_allclose(ev, ref, rtol=1e-10)
    _check_pairs(A, ev, Vr)
    assert st["status"] == 0 and all(st["converged"])
    # the double eigenvalue: the computed pair spans the exact eigenspace
    w, V = np.linalg.eigh(dense(A))
    sv = np.linalg.svd(Vr[1:3] @ V[:, 1:3], compute_uv=False)
    assert sv.min() > 1 - 1e-12
    # sign convention: first entry above 1e-12 ||v||_inf is positive
    for v in Vr:
        i = np.argmax(np.abs(v) > 1e-12 * np.abs(v).max())
        assert v[i] > 0


def test_newton_trace_identities(oracle_lib):
    """theta_{k+1} = theta_k + alpha_k/(1+||s_k||^2) (eq. (3.1) with s^T r = -s^T J s), alpha < 0."""
    A = W.diffusion_3d(6, seed=1)
    ev, Vr, st, tr = oracle_lib.solve(A, 4, trace_cap=1000)
    assert len(tr) > 4
    for j, k, th, rn, al, sn2, th1, its in tr[tr[:, 1] >= 0]:  # outer steps (k < 0 marks a return to DACG)
        assert al < 0
        pred = th + al / (1 + sn2)
        assert abs(th1 - pred) <= 1e-7 * abs(al) + 1e-14 * th
        assert th1 < th


def test_solve_diffusion_unit_closed_form(oracle_lib):
    A = W.diffusion_3d(7, unit=True)
    ev, Vr, st, tr = oracle_lib.solve(A, 4)
    np.testing.assert_allclose(ev, W.laplacian_3d_eigs(7)[:4], rtol=1e-10)
    _check_pairs(A, ev, Vr)


@pytest.mark.parametrize("maker,p", [
    (lambda: W.diffusion_3d(8, seed=1), 6),
    (lambda: W.elasticity_q1(3, seed=2), 5),
    (lambda: W.laplacian_2d(20), 5),
])
def test_solve_matches_dense_eigh(oracle_lib, maker, p):
    A = maker()
    ev, Vr, st, tr = oracle_lib.solve(A, p)
    w, V = np.linalg.eigh(dense(A))
    np.testing.assert_allclose(ev, w[:p], rtol=1e-10)
    _check_pairs(A, ev, Vr)
    for j in range(p):  # each vector lies in the eigenspace of its eigenvalue
        cl = np.abs(w - w[j]) <= 1e-8 * w[j]
        proj = V[:, cl].T @ Vr[j]
        assert np.linalg.norm(proj) > 1 - 1e-10


def test_solve_graph_laplacian_cluster(oracle_lib):
    """L + 1e-4 I of a disconnected graph: the leftmost eigenvalue is 1e-4 with multiplicity = #components."""
    A = W.rgg_laplacian(400, seed=3, mean_degree=4.0)
    ncomp = A.meta["components"]
    p = min(4, ncomp)
    assert p >= 2
    ev, Vr, st, tr = oracle_lib.solve(A, p)
    np.testing.assert_allclose(ev, 1e-4, rtol=1e-10)
    _check_pairs(A, ev, Vr)


def test_kmax_zero_keeps_initial_preconditioner(oracle_lib):
    A = W.diffusion_3d(8, seed=1)
    e0, _, s0, _ = oracle_lib.solve(A, 3, kmax=0)
    e5, _, s5, _ = oracle_lib.solve(A, 3, kmax=5)
    np.testing.assert_allclose(e0, e5, rtol=1e-10)
    assert s0["status"] == 0 and s5["status"] == 0


def test_not_converged_is_reported(oracle_lib):
    A = W.diffusion_3d(8, seed=1)
    ev, Vr, st, tr = oracle_lib.solve(A, 2, itmax=1, tol_dacg=0.5)
    assert st["status"] == 1
    assert any(r > 1e-8 for r in st["relres"][:2])


def test_default_parameters_match_table2():
    g = json.load(open(os.path.join(GOLD, "default_params.json")))
    import oracle
    o = oracle.default_opts(4)
    assert o.tol == g["tau"] and o.itmax == g["itmax"] and o.tol_dacg == g["tau_dacg"]
    assert o.tol_pcg == g["tau_pcg"] and o.itmax_pcg == g["itmax_pcg"]


# ----------------------------------------------------------------------------- backward (extension)
def _loss_grad_dense(Ad, p, w8):
    """Reference gradient of sum(lambda_1..p) + sum_j w_j v_1[j]^2 from a full eigendecomposition."""
    lam, V = np.linalg.eigh(Ad)
    n = len(lam)
    G = np.zeros((n, n))
    for i in range(p):
        G += np.outer(V[:, i], V[:, i])
    v1 = V[:, 0]
    g1 = 2 * w8 * v1
    # dv_1 = sum_{j != 1} v_j v_j^T dA v_1 / (lam_1 - lam_j)
    coef = (V[:, 1:].T @ g1) / (lam[0] - lam[1:])
    G += np.outer(V[:, 1:] @ coef, v1)
    return 0.5 * (G + G.T), lam, V


def test_backward_matches_dense_eigendecomposition(oracle_lib):
    N, p = 6, 4
    pat, logk, w = W.diffusion_grad_case(N, seed=4)
    A = pat.csr(logk)
    Ad = dense(A)
    Gd, lam, V = _loss_grad_dense(Ad, p, w)
    ev, Vr, st, tr = oracle_lib.solve(A, p, tol=1e-12)
    ge = np.ones(p)
    GV = np.zeros((p, A.n))
    GV[0] = 2 * w * Vr[0]
    g = oracle_lib.backward(A, ev, Vr, ge, GV, tol=1e-13)
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    ref = Gd[rows, A.col]
    np.testing.assert_allclose(g, ref, rtol=1e-7, atol=1e-9 * np.abs(ref).max())


def test_backward_matches_torch_eigh_autograd(oracle_lib):
    """Chain through the assembly: d loss / d log k against torch.linalg.eigh autograd (fp64, CPU)."""
    import torch
    N, p = 5, 3
    pat, logk, w = W.diffusion_grad_case(N, seed=4)
    A = pat.csr(logk)
    lk = torch.tensor(logk, requires_grad=True)
    vals = pat.values_torch(lk)
    rows = torch.as_tensor(np.repeat(np.arange(A.n), np.diff(A.rowptr)))
    M = torch.zeros(A.n, A.n, dtype=torch.float64).index_put((rows, torch.as_tensor(A.col).long()), vals)
    lam, V = torch.linalg.eigh(M)
    v1 = V[:, 0]
    loss = lam[:p].sum() + (torch.tensor(w) * v1 ** 2).sum()
    loss.backward()
    ev, Vr, st, tr = oracle_lib.solve(A, p, tol=1e-12)
    GV = np.zeros((p, A.n))
    GV[0] = 2 * w * Vr[0]
    gv = oracle_lib.backward(A, ev, Vr, np.ones(p), GV, tol=1e-13)
    lk2 = torch.tensor(logk, requires_grad=True)
    pat.values_torch(lk2).backward(torch.tensor(gv))
    np.testing.assert_allclose(lk2.grad.numpy(), lk.grad.numpy(), rtol=1e-6, atol=1e-9)


def test_backward_matches_finite_differences(oracle_lib):
    N, p = 4, 3
    pat, logk, w = W.diffusion_grad_case(N, seed=4)

    def loss(lk):
        A = pat.csr(lk)
        ev, Vr, st, tr = oracle_lib.solve(A, p, tol=1e-13, tol_pcg=1e-6, itmax_pcg=100)
        return ev.sum() + (w * Vr[0] ** 2).sum(), A, ev, Vr

    L0, A, ev, Vr = loss(logk)
    GV = np.zeros((p, A.n))
    GV[0] = 2 * w * Vr[0]
    gv = oracle_lib.backward(A, ev, Vr, np.ones(p), GV, tol=1e-13)
    # chain rule to log k through the assembly
    import torch
    lk = torch.tensor(logk, requires_grad=True)
    pat.values_torch(lk).backward(torch.tensor(gv))
    grad = lk.grad.numpy()
    rng = np.random.default_rng(11)
    h = 1e-5
    for _ in range(4):
        d = rng.standard_normal(len(logk))
        fd = (loss(logk + h * d)[0] - loss(logk - h * d)[0]) / (2 * h)
        assert abs(fd - grad @ d) <= 1e-6 * abs(fd) + 1e-9


def test_pure_dacg_closed_form_and_dense(oracle_lib):
    """DACG alone to tau (the DACG rows of Tables 4, 5, 7, 8): closed-form 2-D Laplacian eigenvalues, dense
    eigh on a heterogeneous 8^3 diffusion matrix, no Newton or PCG work, residual <= tau per pair."""
    A, p = W.config_small()
    ev, Vr, st, _ = oracle_lib.solve(A, p, x0=W.initial_block(A.n, p, 0), newton=0)
    np.testing.assert_allclose(ev, W.laplacian_2d_eigs(32)[:p], rtol=1e-10)
    _check_pairs(A, ev, Vr)
    assert st["status"] == 0 and sum(st["pcg_its"]) == 0 and sum(st["outer_its"]) == 0
    assert st["mvp_newton"] == p  # the closing residual evaluation of each pair only
    B = W.diffusion_3d(8, seed=1)
    ev2, V2, st2, _ = oracle_lib.solve(B, 5, newton=0)
    np.testing.assert_allclose(ev2, np.linalg.eigvalsh(dense(B))[:5], rtol=1e-10)
    _check_pairs(B, ev2, V2)
    # same eigenpairs as DACG-Newton; DACG alone needs more DACG steps than the tau_DACG phase of DACG-Newton
    ev3, _, st3, _ = oracle_lib.solve(B, 5)
    np.testing.assert_allclose(ev2, ev3, rtol=1e-10)
    assert sum(st2["dacg_its"]) > sum(st3["dacg_its"])


def test_full_bfgs_pairs(oracle_lib):
    """The full update of eq. (2.1) (y_k = r_{k+1} - r_k): closed-form and dense eigenvalues, the same
    eigenpairs as the simplified update, and a different Newton history once pairs accumulate (small
    IMAX_PCG forces several outer steps per pair)."""
    A, p = W.config_small()
    ev, Vr, st, _ = oracle_lib.solve(A, p, x0=W.initial_block(A.n, p, 0), bfgs_full=1)
    np.testing.assert_allclose(ev, W.laplacian_2d_eigs(32)[:p], rtol=1e-10)
    _check_pairs(A, ev, Vr)
    B = W.diffusion_3d(20, seed=1)
    kw = dict(itmax_pcg=5, tol_pcg=1e-4)
    ev1, V1, st1, _ = oracle_lib.solve(B, 4, bfgs_full=1, **kw)
    ev0, V0, st0, _ = oracle_lib.solve(B, 4, bfgs_full=0, **kw)
    _check_pairs(B, ev1, V1)
    np.testing.assert_allclose(ev1, ev0, rtol=1e-10)
    assert st1["pcg_its"] != st0["pcg_its"]
    assert st1["status"] == 0


# ----------------------------------------------------------------------------- IC(lfil, tau_IC) (Sec. 2)
def _scaled(Ad):
    """As = D^-1/2 A D^-1/2 and tau_i = ||As(i,:)||_2: the scaled matrix and row norms of the drop rule."""
    r = 1.0 / np.sqrt(np.diag(Ad))
    As = Ad * r[:, None] * r[None, :]
    return As, np.linalg.norm(As, axis=1)


def test_ict_limits_are_cholesky_and_jacobi(oracle_lib):
    """tau_IC = 0 with unbounded lfil is the exact Cholesky factor (numpy); dropping everything (a huge tau
    or lfil = 0) leaves L = diag(sqrt(a_ii))."""
    for A in small_mats():
        Ad = dense(A)
        L = oracle_lib.ict(A, lfil=A.n, tau=0.0).dense()
        Lc = np.linalg.cholesky(Ad)
        assert np.abs(L - Lc).max() <= 1e-12 * np.abs(Lc).max()
        for lf, tau in ((A.n, 1e300), (0, 0.0)):
            F = oracle_lib.ict(A, lfil=lf, tau=tau)
            assert len(F.val) == A.n
            np.testing.assert_allclose(F.dense(), np.diag(np.sqrt(np.diag(Ad))), rtol=4e-16, atol=0)


@pytest.mark.parametrize("tau", [1e-3, 1e-2, 1e-1])
def test_ict_threshold_rule_characterisation(oracle_lib, tau):
    """With lfil unbounded the factor is fixed by the threshold rule alone: with Ls = D^-1/2 L,
    kept entries satisfy |Ls_ij| >= tau_i and (Ls Ls^T)_ij = As_ij (and the diagonal always matches);
    every dropped position j < i has |As_ij - (Ls Ls^T)_ij| / Ls_jj < tau_i, which is the value the
    entry would have had."""
    for A in small_mats():
        Ad = dense(A)
        As, nrm = _scaled(Ad)
        ti = tau * nrm
        F = oracle_lib.ict(A, lfil=A.n, tau=tau)
        assert F.shift == 0.0
        L = F.dense()
        Ls = L / np.sqrt(np.diag(Ad))[:, None]
        kept = np.zeros_like(L, dtype=bool)
        for i in range(A.n):
            kept[i, F.col[F.rowptr[i]:F.rowptr[i + 1]]] = True
        M = Ls @ Ls.T
        low = np.tril(np.ones_like(kept), -1).astype(bool)
        I, J = np.nonzero(kept & low)
        assert np.all(np.abs(Ls[I, J]) >= ti[I] * (1 - 1e-12))
        assert np.abs(M[I, J] - As[I, J]).max(initial=0) <= 1e-12
        np.testing.assert_allclose(np.diag(M), np.diag(As), rtol=1e-13)
        I, J = np.nonzero(~kept & low)
        would = np.abs(As[I, J] - M[I, J]) / np.diag(Ls)[J]
        assert np.all(would < ti[I] * (1 + 1e-9) + 1e-14)
        if tau == 1e-3 and A.n > 200:
            assert len(F.val) > (A.nnz + A.n) // 2  # fill beyond the pattern of tril(A)


def _ict_dense(Ad, lfil, tau):
    """The IC(lfil, tau_IC) rule on dense arrays, pure-Python loops (tiny inputs only)."""
    n = len(Ad)
    As, nrm = _scaled(Ad)
    ti = tau * nrm
    Ls = np.zeros((n, n))
    kept = np.zeros((n, n), dtype=bool)
    for i in range(n):
        w = As[i, :i].copy()
        live = w != 0
        cand = []
        for k in range(i):
            if not live[k]:
                continue
            lik = w[k] / Ls[k, k]
            if abs(lik) < ti[i]:
                continue
            cand.append((k, lik))
            for m in range(k + 1, i):
                if kept[m, k]:
                    w[m] -= lik * Ls[m, k]
                    live[m] = True
        sel = sorted(sorted(cand, key=lambda c: (-abs(c[1]), c[0]))[:lfil])
        d = As[i, i]
        for k, lik in sel:
            Ls[i, k] = lik
            kept[i, k] = True
            d -= lik * lik
        assert d > 0
        Ls[i, i] = np.sqrt(d)
        kept[i, i] = True
    return Ls * np.sqrt(np.diag(Ad))[:, None], kept


def _random_spd(n, density, seed, ridge=0.5):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n)) * (rng.random((n, n)) < density)
    Ad = M @ M.T + ridge * np.eye(n)
    return Ad


@pytest.mark.parametrize("lfil,tau", [(1, 0.0), (2, 0.0), (4, 0.05), (3, 0.2), (40, 0.05)])
def test_ict_matches_dense_brute_force(oracle_lib, lfil, tau):
    """The lfil rule (keep the lfil largest candidates, ties to the smaller column) and fill creation
    against a dense pure-Python run of the same rule; no row of L holds more than lfil off-diagonal
    entries."""
    for Ad in (_random_spd(40, 0.1, 7), dense(W.laplacian_2d(6)), _random_spd(30, 0.3, 8, ridge=2.0)):
        A = W._from_scipy(sp.csr_matrix(Ad))
        F = oracle_lib.ict(A, lfil=lfil, tau=tau)
        assert F.shift == 0.0
        Lb, kb = _ict_dense(Ad, lfil, tau)
        L = F.dense()
        k = np.zeros_like(kb)
        for i in range(A.n):
            k[i, F.col[F.rowptr[i]:F.rowptr[i + 1]]] = True
        assert np.array_equal(k, kb)
        assert np.abs(L - Lb).max() <= 1e-12 * np.abs(Lb).max()
        assert np.diff(F.rowptr).max() <= lfil + 1


def test_ict_breakdown_restarts_on_shifted_matrix(oracle_lib):
    """A non-positive pivot restarts the factorisation on A + a diag(A), a = shift0 2^m: the result is
    bit-identical to the unshifted factor of that matrix, and the previous shift of the schedule breaks
    down."""
    found = 0
    for seed in range(200):
        Ad = _random_spd(8, 0.4, seed, ridge=0.05)
        A = W._from_scipy(sp.csr_matrix(Ad))
        try:
            F = oracle_lib.ict(A, lfil=2, tau=0.0, shift0=1e-3, shift_max=1.0)
        except RuntimeError:
            continue
        if F.shift == 0.0:
            continue
        m = np.log2(F.shift / 1e-3)
        assert abs(m - round(m)) < 1e-12
        def shifted(a):
            B = W._from_scipy(sp.csr_matrix(Ad))
            dia = B.col == np.repeat(np.arange(B.n), np.diff(B.rowptr))
            B.val = B.val.copy()
            B.val[dia] = B.val[dia] * (1.0 + a)
            return B
        G = oracle_lib.ict(shifted(F.shift), lfil=2, tau=0.0, shift0=0.0)
        assert np.array_equal(G.rowptr, F.rowptr) and np.array_equal(G.col, F.col)
        assert np.array_equal(G.val, F.val)
        prev = F.shift / 2 if F.shift > 1e-3 else 0.0
        with pytest.raises(RuntimeError):
            oracle_lib.ict(shifted(prev), lfil=2, tau=0.0, shift0=0.0)
        found += 1
        if found == 3:
            break
    assert found == 3


def test_solve_with_ict_preconditioner(oracle_lib):
    """IC(lfil, tau_IC) changes the preconditioner, not the eigenpairs: closed-form Laplacian eigenvalues,
    the IC(0) eigenvalues on a diffusion matrix, and the fill ratio sigma of Sec. 5 reported."""
    A, p = W.config_small()
    ev, Vr, st, _ = oracle_lib.solve(A, p, ict=1, lfil=30, tau_ic=1e-2)
    np.testing.assert_allclose(ev, W.laplacian_2d_eigs(32)[:p], rtol=1e-10)
    _check_pairs(A, ev, Vr)
    assert st["fill"] == pytest.approx(st["nnz_L"] / ((A.nnz + A.n) // 2))
    assert st["fill"] > 1.0
    B = W.diffusion_3d(12, seed=1)
    ev0, _, st0, _ = oracle_lib.solve(B, 4)
    assert st0["fill"] == 1.0
    for lf, tau in ((10, 0.1), (30, 1e-2), (50, 1e-4)):
        ev1, V1, st1, _ = oracle_lib.solve(B, 4, ict=1, lfil=lf, tau_ic=tau)
        np.testing.assert_allclose(ev1, ev0, rtol=1e-10)
        _check_pairs(B, ev1, V1)


# ----------------------------------------------------------------------------- Jacobi-Davidson (Sec. 6)
@pytest.mark.parametrize("m", [1, 2, 3, 7, 10, 16])
def test_symeig_matches_numpy(oracle_lib, m):
    """The Rayleigh-Ritz eigensolver (cyclic Jacobi) against numpy.linalg.eigh, and on a matrix with a
    repeated eigenvalue through H Y = Y diag(ev) and Y^T Y = I."""
    rng = np.random.default_rng(m)
    M = rng.standard_normal((m, m))
    H = M + M.T
    ev, Y = oracle_lib.symeig(H)
    np.testing.assert_allclose(ev, np.linalg.eigh(H)[0], rtol=0, atol=1e-13 * np.abs(H).max())
    assert np.abs(H @ Y - Y * ev).max() <= 1e-13 * np.abs(H).max()
    assert np.abs(Y.T @ Y - np.eye(m)).max() <= 1e-13
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    d = np.repeat([1.0, 2.0, 5.0], m)[:m]
    H2 = Q @ np.diag(d) @ Q.T
    ev2, Y2 = oracle_lib.symeig(H2)
    np.testing.assert_allclose(ev2, np.sort(d), atol=1e-13)
    assert np.abs(H2 @ Y2 - Y2 * ev2).max() <= 1e-13
    assert np.abs(Y2.T @ Y2 - np.eye(m)).max() <= 1e-13


@pytest.mark.parametrize("kmax", [0, 5])
def test_jd_closed_form_and_dense(oracle_lib, kmax):
    """Jacobi-Davidson with the PCG correction solver (kmax = 0: the paper's JD with the fixed projected IC
    preconditioner; kmax = 5: with the BFGS pairs): closed-form Laplacian eigenvalues and dense eigh."""
    A, p = W.config_small()
    ev, Vr, st, _ = oracle_lib.solve(A, p, jd=1, kmax=kmax)
    np.testing.assert_allclose(ev, W.laplacian_2d_eigs(32)[:p], rtol=1e-10)
    _check_pairs(A, ev, Vr)
    assert st["status"] == 0 and sum(st["dacg_its"]) == 0
    for B, q in ((W.diffusion_3d(8, seed=1), 5), (W.elasticity_q1(3, seed=2), 4), (W.laplacian_2d(20), 6)):
        ev, Vr, st, _ = oracle_lib.solve(B, q, jd=1, kmax=kmax)
        np.testing.assert_allclose(ev, np.linalg.eigh(dense(B))[0][:q], rtol=1e-10)
        _check_pairs(B, ev, Vr)


def test_jd_ritz_values_decrease_through_restarts(oracle_lib):
    """Rayleigh-Ritz on nested subspaces: the smallest Ritz value never increases, and a thick restart keeps
    it (m_min = 2, m_max = 4 forces many restarts); the space never exceeds m_max."""
    B = W.diffusion_3d(10, seed=1)
    ev, Vr, st, tr = oracle_lib.solve(B, 3, jd=1, jd_mmin=2, jd_mmax=4, trace_cap=4000)
    np.testing.assert_allclose(ev, np.linalg.eigh(dense(B))[0][:3], rtol=1e-10)
    assert tr[:, 4].max() <= 4 and (tr[:, 4] == 4).sum() > 3
    for j in range(3):
        th = tr[tr[:, 0] == j, 2]
        assert len(th) > 5
        assert np.all(np.diff(th) <= 1e-12 * th[0])
    with pytest.raises(RuntimeError):
        oracle_lib.solve(B, 2, jd=1, jd_mmin=4, jd_mmax=4)
