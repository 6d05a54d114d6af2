"""Pins of the parts of the FP64 oracle that set the iteration counts the GPU is compared against:
the PCG exits (iii) and (iv) of Sec. 4.3, the order of the k_max window (Sec. 4.4), the
Fletcher-Reeves direction of DACG (Sec. 4.1) and the return to DACG from a stalled Newton phase.

Each test recomputes what the rule says from dense linear algebra (numpy/scipy) on the oracle's own
iterates, and finds the step where the rule must fire; a planted mistake in the oracle (an unnormalised
eigen-residual, exit (iv) switched off, the window dropping the newest pair, beta = 0, other restart
constants) moves that step or the result and fails the test.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_1312_1553_amd import workloads as W


def _setup(N=12, j=0, eps=2e-3, seed=10):
    A = W.diffusion_3d(N, seed=1)
    Ad = A.to_scipy().toarray()
    w, V = np.linalg.eigh(Ad)
    rng = np.random.default_rng(seed)
    u = V[:, j] + eps * rng.standard_normal(A.n)
    u -= V[:, :j] @ (V[:, :j].T @ u)
    u /= np.linalg.norm(u)
    Q = np.vstack([V[:, :j].T, u])
    theta = u @ Ad @ u
    Au = Ad @ u
    r = Au - theta * u
    return A, Ad, u, Q, theta, Au, r


def _history(oracle_lib, A, Ad, F, u, Q, theta, Au, r, L):
    """Per PCG step l = 1..L, recomputed densely from the oracle's iterate s_l (itmax_pcg = l, every other exit
    off): the normalised eigen-residual ||A x - q x|| / q with x = (u+s)/||u+s|| (eq. (4.2)), ||u + s||, and the
    true linear residual ||g_0 - J s_l|| with J = (I-QQ')(A - theta I)(I-QQ')."""
    n = A.n
    Pr = np.eye(n) - Q.T @ Q
    J = Pr @ (Ad - theta * np.eye(n)) @ Pr
    g0 = -Pr @ r
    out = []
    for l in range(1, L + 1):
        s, its, why = oracle_lib.pcg(A, F, theta, Q, u, Au, r, tol_pcg=0.0, itmax_pcg=l, tau=0.0, exit_rule=0)
        assert its == l and why == 0
        x = u + s
        nx = np.linalg.norm(x)
        xn = x / nx
        q = xn @ Ad @ xn
        eig = np.linalg.norm(Ad @ xn - q * xn)
        out.append(dict(l=l, eig=eig, q=q, nx=nx, g=np.linalg.norm(g0 - J @ s)))
    return out


@pytest.mark.parametrize("eps,L", [(2e-3, 8), (5e-3, 3)])
def test_pcg_exit_iii_uses_the_normalised_iterate(oracle_lib, eps, L):
    """Exit (iii), eq. (4.2) with x = (u+s)/||u+s||: tau is placed between the normalised eigen-residual of some step
    l* and ||u+s|| times it, below every earlier step's.  The oracle must stop exactly at l* with reason 2; an
    eigen-residual computed without the 1/||u+s|| normalisation stops later."""
    A, Ad, u, Q, theta, Au, r = _setup(eps=eps)
    F = oracle_lib.ic0(A)
    h = _history(oracle_lib, A, Ad, F, u, Q, theta, Au, r, L)
    e = [d["eig"] / d["q"] for d in h]
    found = 0
    for i, d in enumerate(h):
        lo, hi = e[i], min([e[i] * d["nx"]] + e[:i])
        if hi <= lo * (1 + 1e-4):
            continue
        tau = np.sqrt(lo * hi)  # strictly inside the window, far from both ends in rounding terms
        s, its, why = oracle_lib.pcg(A, F, theta, Q, u, Au, r, tol_pcg=0.0, itmax_pcg=L + 5, tau=tau, exit_rule=0)
        assert (its, why) == (d["l"], 2), (d["l"], its, why)
        x = (u + s) / np.linalg.norm(u + s)
        q = x @ Ad @ x
        assert np.linalg.norm(Ad @ x - q * x) < tau * q
        found += 1
    assert found >= 1


def test_pcg_exit_iv_fires_at_the_first_floor_step(oracle_lib):
    """Exit (iv) (reading: stop once ||g_l|| <= xi * eigres_l): for several xi, the oracle stops with reason 3 at the
    first step where the densely recomputed ratio ||g_l|| / ||A x - q x|| falls to xi, and not before."""
    A, Ad, u, Q, theta, Au, r = _setup()
    F = oracle_lib.ic0(A)
    L = 14
    h = _history(oracle_lib, A, Ad, F, u, Q, theta, Au, r, L)
    # eigres_l of the rule is ||A x - q x|| of the normalised x (the same quantity as exit (iii))
    ratio = np.array([d["g"] / d["eig"] for d in h])
    for xi in (0.5, 0.1, 0.01):
        first = int(np.argmax(ratio <= xi))
        assert ratio[first] <= xi and (first == 0 or ratio[:first].min() > xi)
        # the decision is not on a knife edge
        assert ratio[first] < 0.97 * xi and (first == 0 or ratio[first - 1] > 1.03 * xi)
        s, its, why = oracle_lib.pcg(A, F, theta, Q, u, Au, r, tol_pcg=0.0, itmax_pcg=L + 10, tau=0.0, exit_rule=1,
                                     xi=xi)
        assert (its, why) == (first + 1, 3), (xi, its, why, first + 1)
    # with the rule off the same solve runs to the cap
    s, its, why = oracle_lib.pcg(A, F, theta, Q, u, Au, r, tol_pcg=0.0, itmax_pcg=L, tau=0.0, exit_rule=0)
    assert (its, why) == (L, 0)


def _dense_bfgs(P0, S, R):
    """eq. (2.2) applied recursively, oldest pair first."""
    n = P0.shape[0]
    P = P0.copy()
    I = np.eye(n)
    for s, r in zip(S, R):
        a = s @ r
        P = -np.outer(s, s) / a + (I - np.outer(s, r) / a) @ P @ (I - np.outer(r, s) / a)
    return P


@pytest.mark.parametrize("kmax,npush", [(3, 7), (5, 5), (5, 6), (1, 4), (4, 2)])
def test_kmax_window_keeps_the_newest_pairs(oracle_lib, kmax, npush):
    """Sec. 4.4: once k_max pairs are stored, each new pair replaces the oldest.  After npush pairs the
    preconditioner equals eq. (2.2) built from the last min(kmax, npush) pairs in production order, and the
    newest pair's secant condition P(-r) = s holds."""
    A = W.diffusion_3d(4, seed=1)
    Ad = A.to_scipy().toarray()
    n = A.n
    F = oracle_lib.ic0(A)
    L = F.dense()
    rng = np.random.default_rng(40 + kmax + npush)
    S = rng.standard_normal((npush, n))
    R = -(S @ Ad) + 0.05 * rng.standard_normal((npush, n))
    assert np.all(np.einsum("ij,ij->i", S, R) < 0)
    keep = min(kmax, npush)
    Pk = _dense_bfgs(np.linalg.inv(L @ L.T), S[npush - keep:], R[npush - keep:])
    g = rng.standard_normal(n)
    c, kept = oracle_lib.window_bfgspk(F, kmax, S, R, None, g)
    assert kept == keep
    np.testing.assert_allclose(c, Pk @ g, rtol=1e-9, atol=1e-11 * np.abs(Pk @ g).max())
    c, _ = oracle_lib.window_bfgspk(F, kmax, S, R, None, -R[-1])
    np.testing.assert_allclose(c, S[-1], rtol=1e-9, atol=1e-11 * np.abs(S[-1]).max())
    if npush > kmax:
        # the oldest pairs are gone: a window that kept them gives another operator
        P_old = _dense_bfgs(np.linalg.inv(L @ L.T), S[:keep], R[:keep])
        assert np.abs(P_old @ g - Pk @ g).max() > 1e-3 * np.abs(Pk @ g).max()


def _dacg_dense(Ad, P0, Qt, x0, steps, fletcher_reeves=True):
    """DACG as read from Sec. 4.1 (R9), in dense numpy: g = A x - q x, h = (I - Qt'Qt) P0 g, d = -h + beta d with
    beta = g'h / (g'h)_prev, and the exact line search as the smallest Ritz pair of A on span{x, d} (scipy's
    generalized eigensolver on the 2 x 2 pencil).  Returns the unit iterates after each step."""
    x = x0 - Qt.T @ (Qt @ x0)
    x = x - Qt.T @ (Qt @ x)
    x /= np.linalg.norm(x)
    d = np.zeros_like(x)
    gh_prev = None
    xs = []
    for _ in range(steps):
        q = x @ Ad @ x
        g = Ad @ x - q * x
        h = P0 @ g
        h -= Qt.T @ (Qt @ h)
        gh = g @ h
        beta = gh / gh_prev if (fletcher_reeves and gh_prev) else 0.0
        d = -h + beta * d
        B = np.column_stack([x, d])
        lam, Y = sla.eigh(B.T @ Ad @ B, B.T @ B)
        y = Y[:, 0] / Y[0, 0]  # the oracle steps x + a d: coefficient 1 on x
        x = B @ y
        x /= np.linalg.norm(x)
        gh_prev = gh
        xs.append(x.copy())
    return xs


def test_dacg_fletcher_reeves_direction(oracle_lib):
    """DACG iterates after 1..8 steps equal the dense transcription with beta = g'h / g_prev'h_prev; with beta = 0
    (preconditioned steepest descent) the iterates differ visibly from the third step on."""
    A = W.diffusion_3d(5, seed=1)
    Ad = A.to_scipy().toarray()
    F = oracle_lib.ic0(A)
    L = F.dense()
    P0 = np.linalg.inv(L @ L.T)
    w, V = np.linalg.eigh(Ad)
    Qt = V[:, :1].T.copy()
    x0 = W.initial_block(A.n, 1, 3)[0]
    steps = 8
    ref = _dacg_dense(Ad, P0, Qt, x0, steps)
    sd = _dacg_dense(Ad, P0, Qt, x0, steps, fletcher_reeves=False)
    for l in range(1, steps + 1):
        x, its, _ = oracle_lib.dacg(A, F, Qt, x0, tol=0.0, itmax=l)
        assert its == l
        assert np.abs(x - ref[l - 1]).max() < 1e-9, (l, np.abs(x - ref[l - 1]).max())
        if l >= 3:
            assert np.abs(x - sd[l - 1]).max() > 1e-4, l


@pytest.mark.parametrize("sig,kw", [(0.03, {}), (0.03, {"itmax_pcg": 3}), (0.03, {"itmax_pcg": 2}),
                                    (0.03, {"kmax": 1}), (0.03, {"tol_pcg": 0.1}), (0.01, {"itmax_pcg": 2}),
                                    (0.1, {"itmax_pcg": 2})])
def test_stalled_newton_returns_to_dacg_by_the_rule(oracle_lib, sig, kw):
    """The return to DACG (the design's reading for a Newton phase that stalls near a cluster; Alg. 2 has no
    restart): it happens after exactly the outer steps where the PCG took no step or the residual failed to
    drop below 0.9x for the second time in a row (at most 5 per pair, not once converged), and DACG then runs
    to clamp(0.005 ||r||/theta, tol, tol_dacg), which the recomputed residual meets.  The cases are 10^3
    diffusions with log k = sig N(0,1), sig small: eight nearly degenerate eigenvalues in three clusters; short
    or loose inner solves make the outer residual ratios land on both sides of 0.9."""
    pat = W.Diffusion3D(10)
    A = pat.csr(sig * np.random.default_rng(1).standard_normal(pat.n))
    tol, tol_dacg, itmax = 1e-8, 1e-2, 100
    ev, Vr, st, tr = oracle_lib.solve(A, 8, trace_cap=20000, **kw)
    assert st["status"] == 0 and len(tr) < 20000
    n_restart = 0
    for j in range(8):
        rec = tr[tr[:, 0] == j]
        slow, restarts = 0, 0
        for i, t in enumerate(rec):
            if t[1] < 0:
                continue
            k, th, rn, th1, its = int(t[1]), t[2], t[3], t[6], int(t[7])
            nxt = rec[i + 1] if i + 1 < len(rec) else None
            if nxt is None:
                continue  # the pair's last step: it converged (status 0)
            rn1 = nxt[7] if nxt[1] < 0 else nxt[3]
            assert np.isclose(th1, nxt[6] if nxt[1] < 0 else nxt[2], rtol=0, atol=0)
            slow = slow + 1 if (its == 0 or rn1 > 0.9 * rn) else 0
            fire = (its == 0 or slow >= 2) and restarts < 5 and rn1 > tol * th1 and k + 1 < itmax
            assert fire == (nxt[1] < 0), (j, k, its, slow, restarts)
            if fire:
                t2 = min(max(0.005 * rn1 / th1, tol), tol_dacg)
                assert nxt[2] == t2
                # DACG met its tolerance (or used its whole budget); the recomputed residual agrees
                assert nxt[3] == 5000 or nxt[5] <= t2 * nxt[4] * (1 + 1e-6)
                slow, restarts = 0, restarts + 1
                n_restart += 1
    assert n_restart == st["dacg_restarts"] >= 1
