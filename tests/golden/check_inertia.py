"""Pin a stored set of oracle eigenvalues as the p LEFTMOST ones, by Sylvester's law of inertia (Alg. 2 asks for
the p smallest eigenpairs; deflation (Sec. 3.2) could in principle skip one, and residuals alone cannot tell).

For a shift sigma, A - sigma I = L D L^T (symmetric elimination, no row interchanges) has exactly as many
negative pivots in D as A has eigenvalues below sigma.  SciPy's SuperLU is run with diagonal pivoting only, and
the row and column orders are checked to be the same permutation, so diag(U) is D.  With sigma just above
lambda_p the count must be p, and with sigma between lambda_{p-1} and lambda_p it must be p - 1.  The counts are
written into the golden file next to the eigenvalues.  Uses only SciPy and the seeded generators.

    python tests/golden/check_inertia.py elasticity 50 20
"""
import json
import os
import sys
import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

from paper_1312_1553_amd import workloads as W  # noqa: E402


def nested_dissection_q1(ne):
    """Geometric nested dissection of the Q1 elasticity unknowns (nodes m x m x ne above the clamped z = 0
    plane, three dofs per node, node-major): split the node box across its longest side at the middle plane,
    order the two halves first and the plane last, recursively; boxes of at most 64 nodes keep their order.
    Returns a permutation of the dofs.  Orderings only change the elimination order, never the inertia."""
    m = ne + 1
    out = []

    def rec(x0, x1, y0, y1, z0, z1):
        sx, sy, sz = x1 - x0, y1 - y0, z1 - z0
        if sx * sy * sz <= 64 or max(sx, sy, sz) < 3:
            z, y, x = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
            out.append((x + m * y + m * m * (z - 1)).ravel())
            return
        if sx >= sy and sx >= sz:
            c = x0 + sx // 2
            rec(x0, c, y0, y1, z0, z1); rec(c + 1, x1, y0, y1, z0, z1); rec(c, c + 1, y0, y1, z0, z1)
        elif sy >= sz:
            c = y0 + sy // 2
            rec(x0, x1, y0, c, z0, z1); rec(x0, x1, c + 1, y1, z0, z1); rec(x0, x1, c, c + 1, z0, z1)
        else:
            c = z0 + sz // 2
            rec(x0, x1, y0, y1, z0, c); rec(x0, x1, y0, y1, c + 1, z1); rec(x0, x1, y0, y1, c, c + 1)

    rec(0, m, 0, m, 1, m)
    nodes = np.concatenate(out)
    perm = (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()
    assert np.array_equal(np.sort(perm), np.arange(3 * m * m * ne))
    return perm


def negative_pivots(M, sigma, perm=None):
    """Number of eigenvalues of the symmetric sparse matrix M below sigma (LDL^T by symmetric-pivot LU).
    With perm the matrix is eliminated in that order (SuperLU's NATURAL on the permuted matrix), else in
    SuperLU's minimum-degree order."""
    K = (M - sigma * sp.identity(M.shape[0], format="csr")).tocsr()
    if perm is not None:
        K = K[perm][:, perm]
    lu = spl.splu(K.tocsc(), permc_spec="NATURAL" if perm is not None else "MMD_AT_PLUS_A",
                  diag_pivot_thresh=0.0, options={"SymmetricMode": True})
    if not np.array_equal(lu.perm_r, lu.perm_c):
        raise RuntimeError("SuperLU interchanged rows: diag(U) does not give the inertia")
    d = lu.U.diagonal()
    if np.any(d == 0):
        raise RuntimeError("zero pivot")
    return int(np.count_nonzero(d < 0)), int(lu.L.nnz + lu.U.nnz)


def main():
    kind, N, p = sys.argv[1], int(sys.argv[2]), int(sys.argv[3])
    if kind == "elasticity":
        A = W.elasticity_q1(N, seed=2)
        path = os.path.join(HERE, f"oracle_evals_elasticity_{N}_p{p}.json")
    else:
        A = W.diffusion_3d(N, seed=1)
        path = os.path.join(HERE, f"oracle_evals_diffusion3d_{N}_p{p}.json")
    g = json.load(open(path))
    ev = np.array(g["evals"])
    M = A.to_scipy()
    perm = nested_dissection_q1(N) if kind == "elasticity" else None
    hi = ev[-1] * (1 + 1e-3)
    mid = 0.5 * (ev[-2] + ev[-1])
    t0 = time.perf_counter()
    c_hi, fill = negative_pivots(M, hi, perm)
    print("count above", c_hi, "factor entries", fill, round(time.perf_counter() - t0, 1), "s", flush=True)
    c_mid, _ = negative_pivots(M, mid, perm)
    order = "geometric nested dissection" if perm is not None else "minimum degree"
    g["inertia"] = {"method": "negative pivots of A - sigma I, SuperLU with diagonal pivoting (SymmetricMode), "
                              + order + " elimination order",
                    "sigma_above_lambda_p": hi, "count_above": c_hi,
                    "sigma_between_lambda_p-1_and_lambda_p": mid, "count_between": c_mid,
                    "factor_entries": fill, "seconds": round(time.perf_counter() - t0, 1)}
    with open(path, "w") as f:
        json.dump(g, f, indent=1)
    print(path, g["inertia"])


if __name__ == "__main__":
    main()
