#!/usr/bin/env python3
"""Benchmark: eigenpairs/s of DACG-Newton on one MI355X, mixed vs FP64.

Workload: 3-D 7-point log-normal diffusion on 100^3 cells (n = 10^6, 6.94e6
nonzeros, log k ~ N(0,1) from seed 1, harmonic-mean faces), p = 10 leftmost
eigenpairs, relative residual <= 1e-8, starting block uniform[-1,1) seed 0.
A step is one pass of the whole path: IC(0) factorisation (device) plus the
DACG-Newton solve of all p pairs.  The matrix is resident in HBM before the
timed region starts.

Prints one JSON line (the last line of stdout).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def spmv_bytes(n, nnz, vb):
    """Algorithmic bytes of y = A x: values + column indices, row pointers, x read once, y written once."""
    return (vb + 4) * nnz + 4 * (n + 1) + 2 * vb * n


def trsv_bytes(n, nnzL, vb):
    """Algorithmic bytes of one IC(0) triangular solve: factor values + indices, row pointers, rhs, solution."""
    return (vb + 4) * nnzL + 4 * (n + 1) + 2 * vb * n


def counter_traffic(kname, n_grid, levels):
    """HBM bytes per launch of the named kernel from the committed rocprofv3 counter summary, or None when the
    summary is for another workload or another system (level count), or the kernel source has changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_counters_diffusion3d_100.txt")
    src = os.path.join(ROOT, "paper_1312_1553_amd", "csrc", "kernels.hip")
    if n_grid != 100 or not os.path.exists(path):
        return None
    tag = ("trsv_" if kname.startswith("trsv") else "spmv_") + kname.split("_")[-1]
    sha, val, lev = None, None, None
    for ln in open(path):
        if ln.startswith("kernels.hip sha256:"):
            sha = ln.split(":", 1)[1].strip()
        elif ln.startswith(f"traffic_bytes {tag}:"):
            val = int(ln.split(":", 1)[1])
        elif ln.startswith("levels:"):
            lev = int(ln.split(":", 1)[1])
    if val is None or sha != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    if tag.startswith("trsv") and lev != levels:
        return None
    return val


def kernel_probe(args, A, S, nnzL, bnx, torch):
    """Each hot kernel args.reps times on the headline matrix, plus a 256 MiB device copy (the reference
    for scaling the HBM counters).  Prints one line per kernel with the live HIP-event average."""
    b = torch.randn(A.n, dtype=torch.float64, device="cuda")
    x = torch.empty_like(b)
    vb = {0: 8, 1: 4}
    for prec in (bnx.FP64, bnx.MIXED):
        for which in (0, 1):
            bnx.bnx_ic_apply(S.h, prec, which, b, x)
            bnx.bnx_set_profiling(S.h, 1)
            for _ in range(args.reps):
                bnx.bnx_ic_apply(S.h, prec, which, b, x)
            ms, cnt = bnx.bnx_kernel_time(S.h, 2 + 2 * which + prec)
            bnx.bnx_set_profiling(S.h, 0)
            us = 1000 * ms / cnt
            byt = trsv_bytes(A.n, nnzL, vb[prec])
            print(f"[kernels] trsv {'L' if which == 0 else 'Lt'} {'f64' if prec == 0 else 'f32'}: {cnt} launches, "
                  f"avg {us:.1f} us, {byt / us / 1e3:.1f} GB/s algorithmic", flush=True)
        bnx.bnx_spmv(S.h, prec, b, x)
        bnx.bnx_set_profiling(S.h, 1)
        for _ in range(args.reps):
            bnx.bnx_spmv(S.h, prec, b, x)
        ms, cnt = bnx.bnx_kernel_time(S.h, prec)
        bnx.bnx_set_profiling(S.h, 0)
        us = 1000 * ms / cnt
        byt = spmv_bytes(A.n, A.nnz, vb[prec])
        print(f"[kernels] spmv {'f64' if prec == 0 else 'f32'}: {cnt} launches, avg {us:.1f} us, "
              f"{byt / us / 1e3:.1f} GB/s algorithmic", flush=True)
    for kind, hops, what in ((0, 8192, "LDS hand-over between waves"), (1, 4096, "global flag between workgroups")):
        us = bnx.bnx_probe_latency(S.h, kind, hops)
        print(f"[kernels] latency probe, {what}: {us * 1000:.0f} ns per hop ({hops} hops)", flush=True)
    src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    dst.copy_(src)
    ev0.record()
    for _ in range(args.reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    us = 1000 * ev0.elapsed_time(ev1) / args.reps
    print(f"[kernels] copy 256 MiB: avg {us:.1f} us, {2 * src.numel() * 8 / us / 1e3:.1f} GB/s (read + write)",
          flush=True)


def columns(res):
    """One leg's last timed step in the columns of the paper's result tables (Tables 4-8): IC, DACG and Newton
    seconds, DACG iterations, Newton outer iterations and MVPs (one SpMV with A each), total MVPs."""
    st = res["stats"]
    return {"max_relres": res["relres"], "t_factor": round(st["t_factor"], 4), "t_dacg": round(st["t_dacg"], 4),
            "t_newton": round(st["t_newton"], 4), "dacg_its": sum(st["dacg_its"]),
            "outer_its": sum(st["outer_its"]), "pcg_its": sum(st["pcg_its"]), "mvp_dacg": st["mvp_dacg"],
            "mvp_newton": st["mvp_newton"], "mvp_total": st["mvp_dacg"] + st["mvp_newton"],
            "dacg_restarts": st["dacg_restarts"], "bfgs_skipped": st["bfgs_skipped"],
            "profiled_step_s": round(res["profiled_step_s"], 3)}


def host_cpu():
    """CPU model, clock and thread count of this host (lscpu; os.cpu_count)."""
    import subprocess
    model, mhz = None, None
    try:
        for ln in subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() == "Model name":
                model = v.strip()
            elif k.strip() in ("CPU max MHz", "CPU MHz") and mhz is None:
                mhz = float(v)
    except (OSError, ValueError):
        pass
    if mhz is None:  # lscpu of some virtual machines shows no clock: the kernel's current figure instead
        try:
            for ln in open("/proc/cpuinfo"):
                k, _, v = ln.partition(":")
                if k.strip() == "cpu MHz":
                    mhz = float(v)
                    break
        except (OSError, ValueError):
            pass
    return {"model": model, "mhz": mhz, "nproc": os.cpu_count()}


def cpu_baseline(A, p, lam1_gpu):
    """The FP64 oracle on this host's cores, one thread.  Its full p = 10 run takes 10-20 minutes, too long for
    this benchmark, so the first eigenpair is timed here (factor + DACG + Newton, about 15-40 s) and scaled by
    the ratio full-run time / first-pair time that tests/golden records for the same matrix and start block,
    both measured in one process on one host.  The estimate is p / (t_pair1 * ratio)."""
    import oracle
    from paper_1312_1553_amd import workloads as W
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "oracle_evals_diffusion3d_100_p10.json")))
    ratio = g["full"]["seconds"] / g["pair1"]["seconds"]
    oracle.build()
    x0c = W.initial_block(A.n, 1, 0)
    t0 = time.perf_counter()
    ev_o, _, st_o, _ = oracle.solve(A, 1, x0=x0c)
    tc = time.perf_counter() - t0
    full = tc * ratio
    hc = host_cpu()
    print(f"[bench] cpu oracle: pair 1 in {tc:.1f}s, scaled by {ratio:.3f} to {full:.0f}s for p = {p}", flush=True)
    return {"value": round(p / full, 6), "unit": "eigenpairs/s", "cores": 1,
            "kind": "oracle (first-pair sample scaled to the full p = 10 run)",
            "sample": f"FP64 oracle, one thread, on the 100^3 diffusion matrix: the first eigenpair (factor + DACG + "
                      f"Newton) took {tc:.1f} s here; the full p = 10 run takes {ratio:.3f}x the first pair's time "
                      f"({g['full']['seconds']:.0f} s / {g['pair1']['seconds']:.1f} s in one process on "
                      f"{g['host']['cpu_model']}), so the full run is estimated at {full:.0f} s; lambda_1 "
                      f"{ev_o[0]:.15e} (GPU fp64 {lam1_gpu:.15e})",
            "pair1_s": round(tc, 2), "ratio_full_over_pair1": round(ratio, 4), "est_full_s": round(full, 1),
            "host": hc}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=100, help="cells per side (100 = the headline n = 10^6 case)")
    ap.add_argument("--p", type=int, default=0, help="eigenpairs (default: the workload's, 10 for the headline)")
    ap.add_argument("--workload", choices=["diffusion100", "elasticity50", "rgg500k", "diffusion64grad"],
                    default="diffusion100",
                    help="diffusion100: 3-D diffusion on --grid^3 cells, p = 10 (the headline); elasticity50: Q1 "
                         "elasticity on 50^3 elements, p = 20; rgg500k: geometric graph Laplacian, 500k nodes, p = 10; "
                         "diffusion64grad: 64^3 diffusion, p = 5, solve + backward of "
                         "sum(lambda) + sum_j w_j v_1[j]^2")
    ap.add_argument("--trsv-mode", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-grid", type=int, default=100)
    ap.add_argument("--kernels", action="store_true",
                    help="time only the hot kernels at full size (IC solves, SpMV) and a plain copy of known size; "
                         "used under rocprofv3 for the kernel summaries and HBM counters")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--newton", type=int, default=1,
                    help="1: DACG-Newton (the method); 0: DACG alone to the same tolerance (the paper's DACG rows)")
    ap.add_argument("--bfgs-full", type=int, default=0,
                    help="1: store the pairs of the full BFGS update eq. (2.1), y_k = r_{k+1} - r_k; 0: the "
                         "simplified update eq. (2.2) (default)")
    ap.add_argument("--jd", type=int, default=0,
                    help="1: Jacobi-Davidson outer iteration (Sec. 6, m_min 5, m_max 10) with the same PCG as "
                         "correction solver, instead of DACG-Newton")
    ap.add_argument("--kmax", type=int, default=5, help="BFGS window (0: the fixed initial preconditioner)")
    ap.add_argument("--itmax-pcg", type=int, default=20, help="IMAX_PCG, the PCG iteration cap (Table 2 default 20)")
    ap.add_argument("--no-kernel-profile", action="store_true",
                    help="skip the extra instrumented step that gives the per-kernel averages (parameter sweeps)")
    ap.add_argument("--tol-dacg", type=float, default=1e-2,
                    help="DACG tolerance before Newton (Table 2 default 1e-2; the paper uses 0.1 and 0.2 on two matrices)")
    ap.add_argument("--ict", type=str, default="",
                    help="'LFIL,TAU': precondition with IC(lfil, tau_IC) instead of IC(0) (the paper's own initial "
                         "preconditioner; Table 2 defaults are 30,1e-2)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solver is built and measured on a "
              f"single GPU, and sharding it across GPUs is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1312_1553_amd import bnx
    from paper_1312_1553_amd import workloads as W

    N = args.grid
    t0 = time.time()
    wgrad = None
    if args.workload == "elasticity50":
        p, A, wname = args.p or 20, W.elasticity_q1(50, seed=2), "elasticity_q1_50^3_lognormal_seed2"
    elif args.workload == "rgg500k":
        p, A, wname = args.p or 10, W.rgg_laplacian(500_000, seed=3), "rgg_laplacian_500k_seed3_rcm"
    elif args.workload == "diffusion64grad":
        pat, logk, wgrad = W.diffusion_grad_case(64, seed=4)
        p, A, wname = args.p or 5, pat.csr(logk), "diffusion3d_64^3_seed4_solve_and_backward"
    else:
        p, A, wname = args.p or 10, W.diffusion_3d(N, seed=1), f"diffusion3d_{N}^3_lognormal_seed1"
    if args.workload != "diffusion100":
        args.no_cpu_baseline = True  # the oracle sample is defined on the headline workload
    x0 = W.initial_block(A.n, p, 0)
    print(f"[bench] workload {wname} n={A.n} nnz={A.nnz} p={p} built in {time.time() - t0:.1f}s", flush=True)
    torch.cuda.set_device(0)
    S = bnx.Solver(A.rowptr, A.col, A.val)
    bnx.bnx_set_trsv_mode(S.h, args.trsv_mode)
    fkw = {}
    if args.ict:
        lf, tau = args.ict.split(",")
        fkw = dict(ict=1, lfil=int(lf), tau_ic=float(tau))
    t0 = time.time()
    S.factor(**fkw)
    print(f"[bench] factor {'IC(%s)' % args.ict if args.ict else 'IC(0)'}: {time.time() - t0:.2f}s", flush=True)
    x0d = torch.as_tensor(x0).cuda()
    wgrad_d = None if wgrad is None else torch.as_tensor(wgrad).cuda()
    finfo = bnx.bnx_factor_info(S.h)
    nnzL = finfo["nnz_L"]
    print(f"[bench] factor: nnz(L) {nnzL}, sigma {finfo['fill']:.3f}, levels {finfo['levels_L']} / "
          f"{finfo['levels_Lt']}", flush=True)
    if args.kernels:
        kernel_probe(args, A, S, nnzL, bnx, torch)
        return

    # latency roofline of the triangular solves: chained hand-overs measured on this device
    t_lds = bnx.bnx_probe_latency(S.h, 0, 8192)
    t_glb = bnx.bnx_probe_latency(S.h, 1, 4096)
    print(f"[bench] latency probe: {t_lds * 1000:.0f} ns per LDS hand-over, {t_glb * 1000:.0f} ns per global one",
          flush=True)

    results = {}
    for name, prec in (("mixed", bnx.MIXED), ("fp64", bnx.FP64)):
        for w in range(args.warmup):
            S.factor(**fkw)
            ev, V, st = S.solve(p, precision=prec, x0=x0d, newton=args.newton, bfgs_full=args.bfgs_full, jd=args.jd,
                                 kmax=args.kmax, tol_dacg=args.tol_dacg, itmax_pcg=args.itmax_pcg)
            print(f"[bench] warmup {name} {w}: {st['t_dacg'] + st['t_newton']:.3f}s status {st['status']}",
                  flush=True)
        def step():
            S.factor(**fkw)
            ev, V, st = S.solve(p, precision=prec, x0=x0d, newton=args.newton, bfgs_full=args.bfgs_full, jd=args.jd,
                                 kmax=args.kmax, tol_dacg=args.tol_dacg, itmax_pcg=args.itmax_pcg)
            if wgrad is not None:  # the backward of the loss through the same solve
                GV = torch.zeros_like(V)
                GV[0] = 2 * wgrad_d * V[0]
                S.backward(np.ones(p), GV)
            return ev, V, st

        # timed steps: no instrumentation inside the timed region
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for k in range(args.steps):
            ev, V, st = step()
            stats.append(st)
            print(f"[bench] {name} step {k}: status {st['status']} (elapsed {time.perf_counter() - t0:.2f}s)",
                  flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # one more step with HIP events recorded around every hot-kernel launch on the library's stream: the
        # per-kernel averages of the roofline (the same work as a timed step; its wall time shows the cost of
        # the events)
        tp = 0.0
        kt = {kname: (0.0, 0) for kname in bnx.KERNEL_IDS}
        if not args.no_kernel_profile:
            bnx.bnx_set_profiling(S.h, 1)
            tp = time.perf_counter()
            step()
            torch.cuda.synchronize()
            tp = time.perf_counter() - tp
            kt = {kname: bnx.bnx_kernel_time(S.h, kid) for kname, kid in bnx.KERNEL_IDS.items()}
            bnx.bnx_set_profiling(S.h, 0)
            print(f"[bench] {name} profiled step: {tp:.3f}s", flush=True)
        # residual check on the last step (independent of the library: scipy on the host)
        Vh = V.cpu().numpy()
        M = A.to_scipy()
        evn = ev.numpy()
        relres = max(float(np.linalg.norm(M @ Vh[j] - evn[j] * Vh[j]) / evn[j]) for j in range(p))
        results[name] = dict(dt=dt, eps=p * args.steps / dt, ms=1000 * dt / args.steps, stats=stats[-1], kt=kt,
                             relres=relres, evals=evn.tolist(), profiled_step_s=tp)
        print(f"[bench] {name}: {results[name]['eps']:.3f} eigenpairs/s, {results[name]['ms']:.1f} ms/step, "
              f"max relres {relres:.2e}, pcg its {sum(st['pcg_its'])}, dacg its {sum(st['dacg_its'])}, "
              f"outer its {sum(st['outer_its'])}", flush=True)
        print(f"[bench]   per pair: dacg its {list(st['dacg_its'])}, pcg its {list(st['pcg_its'])}, "
              f"dacg restarts {st.get('dacg_restarts')}", flush=True)
        for kname, (ms, cnt) in kt.items():
            if cnt:
                print(f"[bench]   {kname}: {cnt} launches, avg {1000 * ms / cnt:.1f} us, total {ms:.1f} ms",
                      flush=True)

    mixed, fp64 = results["mixed"], results["fp64"]
    # dominant kernel of the mixed path: the largest total measured time
    vb = {"f64": 8, "f32": 4}
    best = None
    for kname, (ms, cnt) in mixed["kt"].items():
        if cnt and (best is None or ms > best[1]):
            best = (kname, ms, cnt)
    if best is None:  # --no-kernel-profile: no per-kernel times, no roofline
        best = ("none_f64", float("nan"), 1)
    kname, ms, cnt = best
    prec = kname.split("_")[-1]
    per_launch = (spmv_bytes(A.n, A.nnz, vb[prec]) if kname.startswith("spmv")
                  else trsv_bytes(A.n, nnzL, vb[prec]))
    avg_s = ms / cnt / 1000.0
    achieved = per_launch / avg_s / 1e9
    kernels = {}
    for name_, res in results.items():
        for kn, (kms, kc) in res["kt"].items():
            if not kc:
                continue
            pr = kn.split("_")[-1]
            b = spmv_bytes(A.n, A.nnz, vb[pr]) if kn.startswith("spmv") else trsv_bytes(A.n, nnzL, vb[pr])
            kernels[kn] = {"launches": kc, "avg_us": round(1000 * kms / kc, 2),
                           "alg_bytes": b, "GBs": round(b / (kms / kc / 1000.0) / 1e9, 1)}

    cpu = None
    if not args.no_cpu_baseline and N == 100 and p == 10:
        cpu = cpu_baseline(A, p, fp64["evals"][0])

    levels = mixed["stats"]["levels_L"]
    line = {
        "metric": "eigenpairs/sec (p=10, rel resid <=1e-8) mixed vs FP64; SpMV+IC-solve HBM GB/s",
        "value": round(mixed["eps"], 4),
        "unit": "eigenpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed["ms"], 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 inner / f64 outer (mixed); fp64 path reported beside it",
        "data": "synthetic",
        "config": {"workload": wname, "n": A.n, "nnz": A.nnz, "p": p, "tol": 1e-8,
                   "parallelism": "single GPU", "trsv_mode": args.trsv_mode,
                   "method": ("Jacobi-Davidson" if args.jd else "DACG-Newton" if args.newton else "DACG alone"),
                   "kmax": args.kmax, "itmax_pcg": args.itmax_pcg, "tol_dacg": args.tol_dacg,
                   "preconditioner": f"IC({args.ict})" if args.ict else "IC(0)",
                   "bfgs_update": "eq. (2.1) full" if args.bfgs_full else "eq. (2.2) simplified",
                   "fill_sigma": round(mixed["stats"]["fill"], 4)},
        "fp64": dict(value=round(fp64["eps"], 4), ms_per_step=round(fp64["ms"], 2), **columns(fp64)),
        "mixed": dict(value=round(mixed["eps"], 4), ms_per_step=round(mixed["ms"], 2), **columns(mixed)),
        "speedup_mixed_vs_fp64": round(mixed["eps"] / fp64["eps"], 3),
        "max_rel_eig_diff_mixed_vs_fp64": float(np.max(np.abs(np.array(mixed["evals"]) - np.array(fp64["evals"]))
                                                       / np.array(fp64["evals"]))),
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                     "traffic": counter_traffic(kname, N, levels) if args.workload == "diffusion100" else None,
                     "alg_bytes_per_launch": per_launch, "avg_launch_us": round(avg_s * 1e6, 2),
                     "levels": levels,
                     "limiter": ("latency: a chain of %d dependent levels" % levels) if kname.startswith("trsv")
                     else "hbm",
                     "latency": {"t_lds_hop_us": round(t_lds, 4), "t_global_hop_us": round(t_glb, 4),
                                 "floor_us": round(levels * t_lds, 2),
                                 "frac": round(levels * t_lds / (avg_s * 1e6), 4)}},
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
