"""Benchmark: FGMRES + two-level GDSW on the 16^3 Q2/Q1 Poiseuille problem.

One step = one FGMRES solve to a 1e-8 relative residual from x = 0 on the
16^3 mesh with 4^3 subdomains (overlap 1, FP64 dense local LU): every
preconditioner apply (gathers, batched triangular solves, coarse restriction,
coarse solve, prolongation, scatter), the block SpMV and the CGS2 Arnoldi
steps.  The right-hand side is resident on the GPU before timing starts.

value = preconditioner applications per second over the timed solves
(iterations / time).  The JSON line also reports the time to tolerance, the
stand-alone apply rate, the roofline of the dominant kernel (the batched
triangular solve, HBM bound) and the CPU oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(w, sample_subdomains=8, repeats=5):
    """Oracle apply on a bounded sample: the local solves of `sample_subdomains`
    of the m^3 subdomains plus the full coarse correction; the local part is
    scaled to all subdomains."""
    from threadpoolctl import threadpool_info

    from inputs import random_vector
    from oracle.decomposition import Decomposition
    from oracle.gdsw import TwoLevelGDSW
    from oracle.stokes import StokesProblem
    import scipy.linalg as sla

    p = StokesProblem(w.n, viscosity=w.viscosity, inflow=w.inflow)
    d = Decomposition(p, w.m, w.overlap)
    M = TwoLevelGDSW(p.A, d, factor_local=False)
    nsub = d.n_sub
    pick = np.linspace(0, nsub - 1, sample_subdomains).astype(int)
    lus = {int(i): sla.lu_factor(M.local_matrix(int(i)), check_finite=False) for i in pick}
    r = random_vector(p.n_free, seed=1)
    t_loc, t_crs = [], []
    for _ in range(repeats):
        t0 = time.perf_counter()
        z = np.zeros_like(r)
        for i in pick:
            S = d.S[i]
            z[S] += sla.lu_solve(lus[int(i)], r[S], check_finite=False)
        t1 = time.perf_counter()
        z += M.apply_coarse(r)
        t2 = time.perf_counter()
        t_loc.append(t1 - t0)
        t_crs.append(t2 - t1)
    t_apply = float(np.median(t_loc)) * nsub / len(pick) + float(np.median(t_crs))
    threads = max([int(x.get("num_threads", 1)) for x in threadpool_info()] or [1])
    return {"value": 1.0 / t_apply, "unit": "applies/s", "cores": threads, "kind": "oracle",
            "sample": f"M^-1 apply on the 16^3 workload: local LU solves of {len(pick)} of {nsub} subdomains "
                      f"(scaled x{nsub / len(pick):g}) + the full coarse correction; median of {repeats}; "
                      f"factorisation untimed"}


def measured_traffic(launches):
    """HBM bytes per launch of the triangular solves from the committed counter
    summary, or None when the kernel source changed since it was measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "trsv_step_kernel_16cubed_traffic.txt")
    src = os.path.join(ROOT, "paper_2508_04356_amd", "csrc", "kernels_factor.hip")
    if not os.path.exists(path):
        return None
    kv = dict(line.split(": ", 1) for line in open(path).read().splitlines() if ": " in line)
    if kv.get("kernel_source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    if int(kv.get("launches_per_apply", -1)) != launches:
        return None
    return (float(kv["fetch_bytes_per_apply"]) + float(kv["write_bytes_per_apply"])) / launches


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--precision", default=None, help="local factor precision (default: the workload's)")
    ap.add_argument("--local-algebraic", type=int, default=None,
                    help="1: algebraic overlap instead of Dirichlet u, p on the artificial boundary")
    ap.add_argument("--applies", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB buffer three times (reference for HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_direction": src.numel() * 4, "copies": 3}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(the multi-GPU sharding is described in DESIGN.md, not built)"}))
        sys.exit(2)

    import torch

    import paper_2508_04356_amd as G
    from inputs import random_vector, workload

    w = workload(args.workload)
    prec = args.precision or (w.precision if args.workload not in ("C2", "C2alg") else "fp64")
    alg = w.local_algebraic if args.local_algebraic is None else args.local_algebraic
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"[bench] setup {w.name}: n={w.n} m={w.m} levels={w.levels} precision={prec}")
    t0 = time.perf_counter()
    s = G.Solver(w.n, w.m, overlap=w.overlap, levels=w.levels, group=w.group, viscosity=w.viscosity,
                 inflow=w.inflow, tile=args.tile, precision=prec, local_algebraic=alg,
                 level2_layer=w.level2_layer)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    sz = s.sizes()
    n = sz.n_free
    log(f"[bench] setup {t_setup:.2f} s; n_free={n} Nc={sz.n_coarse} device bytes={sz.device_bytes / 1e9:.2f} GB")

    b = torch.zeros(n, dtype=torch.float64, device=dev)
    s.rhs(b)
    x = torch.zeros_like(b)

    for _ in range(args.warmup):
        s.fgmres(b, x, rtol=w.rtol, restart=w.restart, max_it=w.max_it)
    torch.cuda.synchronize()
    its = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        info = s.fgmres(b, x, rtol=w.rtol, restart=w.restart, max_it=w.max_it)[0]
        its.append(info.iterations)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    ms_per_step = 1e3 * t_steps / args.steps
    log(f"[bench] {args.steps} solves: {ms_per_step:.2f} ms each, iterations {its}, true rel {info.true_rel_res:.2e}")

    # stand-alone applies and per-phase profile (HIP events on the library's stream)
    r = torch.as_tensor(random_vector(n, seed=1), device=dev)
    z = torch.zeros_like(r)
    for _ in range(3):
        s.apply(r, z)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.applies):
        s.apply(r, z)
    e1.record()
    torch.cuda.synchronize()
    t_apply_ms = e0.elapsed_time(e1) / args.applies
    phases = np.array([s.profile_apply(r, z) for _ in range(10)])
    ph = phases.mean(axis=0)
    t_trsv_ms = float(ph[1] + ph[2])
    solve_bytes = float(sz.solve_bytes)
    achieved = solve_bytes / (t_trsv_ms * 1e-3) / 1e9
    launches = int(sz.solve_launches)
    log(f"[bench] apply {t_apply_ms:.3f} ms; phases ms gather/restrict {ph[0]:.3f} trsv {ph[1]:.3f}+{ph[2]:.3f} "
        f"scatter {ph[3]:.3f}; trsv {achieved:.0f} GB/s over {launches} launches")

    out = {
        "metric": f"M^-1 applies/s inside FGMRES to 1e-8 rel. residual ({w.levels}-level monolithic GDSW, {prec})",
        "value": float(sum(its) / t_steps),
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else f"f64 (local factors {prec}, fp32 accumulation)",
        "data": "synthetic: Poiseuille Stokes problem generated in-library (no dataset)",
        "config": {"workload": f"{w.name}: {w.n}^3 Q2/Q1 hexahedra, {w.m}^3 subdomains, overlap {w.overlap}, "
                               f"{w.levels}-level GDSW, FGMRES rtol {w.rtol:g} restart {w.restart}",
                   "n_free": n, "n_coarse": int(sz.n_coarse), "tile": args.tile or 128,
                   "local_problems": "algebraic overlap (closed box grown by one element)" if alg
                   else "Dirichlet u and p on the artificial boundary of the grown box"},
        "iterations": its[-1],
        "time_to_tol_s": ms_per_step / 1e3,
        "true_rel_res": info.true_rel_res,
        "apply_only_per_s": 1e3 / t_apply_ms,
        "apply_phases_ms": {"gather_restrict": ph[0], "trsv_l1": ph[1], "trsv_coarse": ph[2], "scatter": ph[3]},
        "setup_s": t_setup,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(launches) if args.workload == "C2" and not alg else None,
                     "kernel": "trsv_step_kernel (blocked forward/backward solves of every factor)",
                     "bytes_per_apply": solve_bytes, "launches_per_apply": launches,
                     "bytes_per_launch": solve_bytes / launches,
                     "avg_launch_us": t_trsv_ms * 1e3 / launches},
    }
    if not args.no_cpu_baseline and args.workload == "C2":
        log("[bench] CPU oracle sample ...")
        out["cpu_baseline"] = cpu_baseline(w)
    s.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
