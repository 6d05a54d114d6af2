"""Write the FP64 oracle's eigenvalues for a workload into tests/golden (calls only oracle/ and the
seeded generators; nothing here touches the HIP library).

    python tests/golden/make_oracle_evals.py diffusion3d 100 10 --pair1   # n = 10^6 (~16 min, 1 core)
    python tests/golden/make_oracle_evals.py elasticity 50 20             # n = 390150, 3.0e7 nonzeros

--pair1 also times the oracle on the first eigenpair alone (same matrix, same start vector, measured in
the same process just before the full run), so that a short sample of pair 1 taken on another host can be
scaled to the full p-pair time by the ratio of the two.
"""
import argparse
import json
import os
import platform
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import oracle  # noqa: E402
from paper_1312_1553_amd import workloads as W  # noqa: E402


def host_info() -> dict:
    model, mhz = platform.processor(), None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() == "Model name":
                model = v.strip()
            elif k.strip() in ("CPU max MHz", "CPU MHz") and mhz is None:
                mhz = float(v)
    except OSError:
        pass
    return {"cpu_model": model, "cpu_mhz": mhz, "nproc": os.cpu_count(), "threads_used": 1}


def columns(st: dict, secs: float) -> dict:
    """The columns of the paper's result tables (Tables 4-8) from the oracle's counters."""
    return {"seconds": round(secs, 2), "t_factor": round(st["t_factor"], 2), "t_dacg": round(st["t_dacg"], 2),
            "t_newton": round(st["t_newton"], 2), "dacg_its": int(sum(st["dacg_its"])),
            "outer_its": int(sum(st["outer_its"])), "pcg_its": int(sum(st["pcg_its"])),
            "mvp_dacg": int(st["mvp_dacg"]), "mvp_newton": int(st["mvp_newton"]),
            "dacg_restarts": int(st["dacg_restarts"])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("kind", choices=["diffusion3d", "elasticity"])
    ap.add_argument("N", type=int)
    ap.add_argument("p", type=int)
    ap.add_argument("--pair1", action="store_true")
    a = ap.parse_args()
    if a.kind == "diffusion3d":
        A = W.diffusion_3d(a.N, seed=1)
        wl = f"diffusion3d {a.N}^3, log k ~ N(0,1) from default_rng(1), harmonic faces"
    else:
        A = W.elasticity_q1(a.N, seed=2)
        wl = (f"Q1 elasticity on {a.N}^3 elements, z = 0 clamped and eliminated, E = exp(N(0,1)) from "
              f"default_rng(2), nu = 0.3")
    x0 = W.initial_block(A.n, a.p, 0)
    oracle.build()
    out = {
        "source": "FP64 CPU oracle (oracle/oracle.c), Alg. 2 at Table 2 defaults (kmax 5, exit rule 1, xi 0.1), "
                  "tol 1e-8, starting block default_rng(0).uniform(-1,1,(p,n))",
        "workload": wl, "n": A.n, "nnz": A.nnz, "p": a.p, "host": host_info(),
    }
    if a.pair1:
        t0 = time.perf_counter()
        ev1, _, st1, _ = oracle.solve(A, 1, x0=x0[:1])
        out["pair1"] = columns(st1, time.perf_counter() - t0)
        out["pair1"]["eval"] = float(ev1[0])
        print("pair 1:", out["pair1"], flush=True)
    t0 = time.perf_counter()
    ev, V, st, _ = oracle.solve(A, a.p, x0=x0)
    dt = time.perf_counter() - t0
    out.update({
        "seconds": round(dt, 1), "full": columns(st, dt),
        "evals": [float(v) for v in ev],
        "relres": [float(r) for r in st["relres"]],
        "converged": [int(c) for c in st["converged"]],
        "dacg_restarts": int(st["dacg_restarts"]),
    })
    name = "diffusion3d" if a.kind == "diffusion3d" else "elasticity"
    path = os.path.join(HERE, f"oracle_evals_{name}_{a.N}_p{a.p}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, f"({dt:.0f} s)")


if __name__ == "__main__":
    main()
