"""Write the FP64 oracle's eigenvalues for a workload into tests/golden (calls only oracle/ and the
seeded generators; nothing here touches the HIP library).

    python tests/golden/make_oracle_evals.py diffusion3d 100 10   # the n = 10^6 headline case (~16 min, 1 core)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import oracle  # noqa: E402
from paper_1312_1553_amd import workloads as W  # noqa: E402


def main():
    kind, N, p = sys.argv[1], int(sys.argv[2]), int(sys.argv[3])
    if kind != "diffusion3d":
        raise SystemExit("only diffusion3d is generated here")
    A = W.diffusion_3d(N, seed=1)
    x0 = W.initial_block(A.n, p, 0)
    oracle.build()
    t0 = time.perf_counter()
    ev, V, st, _ = oracle.solve(A, p, x0=x0)
    dt = time.perf_counter() - t0
    out = {
        "source": "FP64 CPU oracle (oracle/oracle.c), Alg. 2 at Table 2 defaults (kmax 5, exit rule 1, xi 0.1), "
                  "tol 1e-8, starting block default_rng(0).uniform(-1,1,(p,n))",
        "workload": f"diffusion3d {N}^3, log k ~ N(0,1) from default_rng(1), harmonic faces",
        "n": A.n, "p": p, "seconds": round(dt, 1),
        "evals": [float(v) for v in ev],
        "relres": [float(r) for r in st["relres"]],
        "converged": [int(c) for c in st["converged"]],
        "dacg_restarts": int(st["dacg_restarts"]),
    }
    path = os.path.join(HERE, f"oracle_evals_diffusion3d_{N}_p{p}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, f"({dt:.0f} s)")


if __name__ == "__main__":
    main()
