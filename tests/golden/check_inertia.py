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


def negative_pivots(M, sigma):
    """Number of eigenvalues of the symmetric sparse matrix M below sigma (LDL^T by symmetric-pivot LU)."""
    K = (M - sigma * sp.identity(M.shape[0], format="csr")).tocsc()
    lu = spl.splu(K, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                  options={"SymmetricMode": True})
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
    hi = ev[-1] * (1 + 1e-3)
    mid = 0.5 * (ev[-2] + ev[-1])
    t0 = time.perf_counter()
    c_hi, fill = negative_pivots(M, hi)
    c_mid, _ = negative_pivots(M, mid)
    g["inertia"] = {"method": "negative pivots of A - sigma I, SuperLU with diagonal pivoting (SymmetricMode)",
                    "sigma_above_lambda_p": hi, "count_above": c_hi,
                    "sigma_between_lambda_p-1_and_lambda_p": mid, "count_between": c_mid,
                    "factor_entries": fill, "seconds": round(time.perf_counter() - t0, 1)}
    with open(path, "w") as f:
        json.dump(g, f, indent=1)
    print(path, g["inertia"])


if __name__ == "__main__":
    main()
