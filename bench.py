"""Benchmark: FGMRES + two-level GDSW on the 16^3 Q2/Q1 Poiseuille problem.

One step = one FGMRES solve to a 1e-8 relative residual from x = 0 on the
16^3 mesh with 4^3 subdomains (overlap 1, FP64 local solves): every
preconditioner apply (gathers, coarse restriction, the batched local and
coarse solves, prolongation, scatter), the SpMV and the CGS2 Arnoldi steps.
The right-hand side is resident on the GPU before timing starts.

value = preconditioner applications per second over the timed solves
(iterations / time).  The JSON line also reports the time to tolerance, the
stand-alone apply rate, the roofline of the dominant kernel (the level-1
local solve: by default the batched product with the explicit inverses,
HBM bound), timed with HIP events around each of its launches during the
timed solves, and the CPU oracle timed on a bounded sample.

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


def cpu_model():
    """The host CPU's model name from /proc/cpuinfo (Linux), else the platform string."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_baseline(w, repeats=3, solve=True):
    """The CPU oracle on the same workload, as it stands: its preconditioner
    apply (all subdomains' LU solves in ascending order, then the coarse
    correction) timed with every host thread the BLAS offers and with one
    thread; the same local solves spread over the subdomains on a thread pool
    of one BLAS thread each (the oracle's own per-subdomain function, only
    scheduled in parallel here); and one oracle FGMRES solve to the workload's
    tolerance.  Factorisations are set-up work and untimed."""
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_info, threadpool_limits

    from inputs import random_vector
    from oracle.decomposition import Decomposition
    from oracle.fgmres import fgmres
    from oracle.gdsw import TwoLevelGDSW
    from oracle.stokes import StokesProblem

    t0 = time.perf_counter()
    p = StokesProblem(w.n, viscosity=w.viscosity, inflow=w.inflow)
    d = Decomposition(p, w.m, w.overlap, local_dirichlet=not w.local_algebraic)
    M = TwoLevelGDSW(p.A, d)
    t_setup = time.perf_counter() - t0
    threads = max([int(x.get("num_threads", 1)) for x in threadpool_info()] or [1])
    r = random_vector(p.n_free, seed=1)

    def timed(f, k):
        f()
        ts = []
        for _ in range(k):
            t = time.perf_counter()
            f()
            ts.append(time.perf_counter() - t)
        return float(np.median(ts))

    t_all = timed(lambda: M(r), repeats)
    with threadpool_limits(limits=1):
        t_one = timed(lambda: M(r), repeats)

        def par_apply():
            parts = list(pool.map(lambda i: M.local_solve(i, r[d.S[i]]), range(d.n_sub)))
            z = np.zeros_like(r)
            for i, y in enumerate(parts):  # ascending subdomain order, as the oracle sums
                z[d.S[i]] += y
            return z + M.apply_coarse(r)

        with ThreadPoolExecutor(max_workers=threads) as pool:
            t_par = timed(par_apply, repeats)
    out = {"value": 1.0 / t_all, "unit": "applies/s", "cores": threads, "kind": "oracle",
           "sample": f"the oracle's whole M^-1 apply on the {w.n}^3 workload ({d.n_sub} subdomain LU solves "
                     f"+ coarse correction), median of {repeats} after one warm-up; LU factorisations untimed",
           "cpu_model": cpu_model(), "nproc": os.cpu_count(),
           "one_thread_applies_per_s": 1.0 / t_one,
           "subdomain_parallel_applies_per_s": 1.0 / t_par,
           "subdomain_parallel_workers": threads,
           "oracle_setup_s": t_setup}
    if solve:
        t = time.perf_counter()
        x, it, rel, trel = fgmres(lambda v: p.A @ v, M, p.b, rtol=w.rtol, restart=w.restart, max_it=w.max_it)
        out["fgmres_time_to_tol_s"] = time.perf_counter() - t
        out["fgmres_iterations"] = int(it)
        out["fgmres_true_rel_res"] = float(trel)
    return out


TRAFFIC = {  # committed counter summaries of the dominant kernel on the 16^3 FP64 workload
    "inverse": ("gemv_part_kernel_16cubed_traffic.txt", "kernels_gemv.hip"),
    "triangular": ("trsv_step_kernel_16cubed_traffic.txt", "kernels_factor.hip"),
    "symmetric": ("symv_part_kernel_16cubed_traffic.txt", "kernels_symv.hip"),
    "block": ("symv_part_kernel_block_16cubed_traffic.txt", "kernels_symv.hip"),
}


def learned_variant(s, b, w, steps, solve):
    """Train the conv-net local solve on method-generated pairs, then time
    FGMRES to the same tolerance with it (with and without the exact
    fallback) beside the exact local solves.  It replaces whole local
    inverses, so a block-solve context gets a symmetric-tile twin here."""
    import torch

    import paper_2508_04356_amd as G

    own = solve == "block"
    if own:
        s = G.Solver(w.n, w.m, overlap=w.overlap, levels=w.levels, group=w.group, viscosity=w.viscosity,
                     inflow=w.inflow, precision="fp64", local_algebraic=w.local_algebraic,
                     level2_layer=w.level2_layer, local_solve="symmetric")
    t0 = time.perf_counter()
    info = s.learned_init(seed=7)
    hist = s.learned_train(solves=4, steps=600, batch=32, lr=2e-3, seed=3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    res = {"interior_subdomains": info.subdomains, "grid": info.grid, "train_s": t_train,
           "loss_first": float(np.mean(hist[:20])), "loss_last": float(np.mean(hist[-20:]))}
    for name, mode, tau in (("exact", "lu", 0.7), ("learned", "learned", 1e30), ("learned_fallback", "learned", 0.7)):
        s.set_local_solver(mode, tau)
        x = torch.zeros_like(b)
        s.fgmres(b, x, rtol=w.rtol, restart=w.restart, max_it=w.max_it, raise_on_noconv=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            inf = s.fgmres(b, x, rtol=w.rtol, restart=w.restart, max_it=w.max_it, raise_on_noconv=False)[0]
        torch.cuda.synchronize()
        res[name] = {"iterations": inf.iterations, "true_rel_res": inf.true_rel_res,
                     "time_to_tol_ms": 1e3 * (time.perf_counter() - t0) / steps}
        log(f"[bench] {name}: {inf.iterations} iterations, {res[name]['time_to_tol_ms']:.1f} ms")
    n_l, n_fb = s.learned_stats()
    res["learned_solves"], res["fallbacks"] = n_l, n_fb
    res["local_solve"] = "symmetric" if own else solve
    s.set_local_solver("lu")
    if own:
        s.close()
    return res


def precision_variants(w, args, b, x64, z64, r, solve):
    """The same workload with FP32 and BF16 level-1 inverses (FP32
    accumulation; coarse levels and FGMRES in FP64): FGMRES time to the same
    tolerance on the same GPU, iterations, and the error of the solution and
    of one apply against the FP64 library results."""
    import torch

    import paper_2508_04356_amd as G

    out = {}
    for prec in ("fp32", "bf16"):
        t0 = time.perf_counter()
        s = G.Solver(w.n, w.m, overlap=w.overlap, levels=w.levels, group=w.group, viscosity=w.viscosity,
                     inflow=w.inflow, precision=prec, local_algebraic=w.local_algebraic,
                     level2_layer=w.level2_layer, local_solve=solve)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        x = torch.zeros_like(b)
        for _ in range(max(args.warmup, 1)):
            s.fgmres(b, x, rtol=w.rtol, restart=w.restart, max_it=w.max_it)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            info = s.fgmres(b, x, rtol=w.rtol, restart=w.restart, max_it=w.max_it)[0]
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / args.steps
        z = torch.zeros_like(r)
        s.apply(r, z)
        torch.cuda.synchronize()
        out[prec] = {"iterations": info.iterations, "time_to_tol_ms": ms, "true_rel_res": info.true_rel_res,
                     "x_rel_err_vs_fp64": float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64)),
                     "apply_rel_err_vs_fp64": float((z - z64).abs().max() / z64.abs().max()),
                     "setup_s": t_setup}
        log(f"[bench] {prec} inverses: {info.iterations} iterations, {ms:.2f} ms to tolerance, "
            f"x err {out[prec]['x_rel_err_vs_fp64']:.1e}, apply err {out[prec]['apply_rel_err_vs_fp64']:.1e}")
        s.close()
    return out


def copy_bandwidth(torch, dev, gib=1, reps=5):
    """HBM bandwidth of a 1 GiB device-to-device copy (bytes read + written
    per second), the practical ceiling the roofline fraction is compared with."""
    n = (gib << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def kernel_source_sha256(srcname):
    """Digest of a kernel's source file followed by the device load helpers
    it includes (vec16.h): a change to either invalidates its counters."""
    import hashlib
    h = hashlib.sha256()
    for f in (srcname, "vec16.h"):
        h.update(open(os.path.join(ROOT, "paper_2508_04356_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(solve, launches):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when the kernel source changed since it was measured."""
    if solve not in TRAFFIC:
        return None
    name, srcname = TRAFFIC[solve]
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = dict(line.split(": ", 1) for line in open(path).read().splitlines() if ": " in line)
    if kv.get("kernel_source_sha256") != kernel_source_sha256(srcname):
        return None
    if int(kv.get("launches_per_apply", -1)) != launches:
        return None
    return (float(kv["fetch_bytes_per_apply"]) + float(kv["write_bytes_per_apply"])) / launches


MFMA_PEAK_TFS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}


def run_multi(args, w, prec, nrhs):
    """Several right-hand sides: b_k = c_k b(1) with c_k ~ U[0.5, 2] (the
    32-RHS workload), FGMRES in lockstep, local solves as MFMA products."""
    import torch

    import paper_2508_04356_amd as G
    from inputs import c3_inflow_amplitudes, random_vector

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    K = min(nrhs, 32)
    log(f"[bench] setup {w.name}: n={w.n} m={w.m} precision={prec} nrhs={nrhs}")
    t0 = time.perf_counter()
    s = G.Solver(w.n, w.m, overlap=w.overlap, levels=w.levels, group=w.group, viscosity=w.viscosity,
                 inflow=w.inflow, precision=prec, local_algebraic=w.local_algebraic, max_rhs=K)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    sz = s.sizes()
    n = sz.n_free
    cs = c3_inflow_amplitudes(nrhs)
    b1 = torch.zeros(n, dtype=torch.float64, device=dev)
    s.rhs(b1)
    B = torch.cat([b1 * float(c) for c in cs])
    X = torch.zeros_like(B)
    for _ in range(args.warmup):
        s.fgmres(B, X, rtol=w.rtol, restart=w.restart, max_it=w.max_it, nrhs=nrhs)
    torch.cuda.synchronize()
    s.kernel_timer(True)
    t0 = time.perf_counter()
    col_its = 0
    for _ in range(args.steps):
        infos = s.fgmres(B, X, rtol=w.rtol, restart=w.restart, max_it=w.max_it, nrhs=nrhs)
        col_its += sum(i.iterations for i in infos)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    s.kernel_timer(False)
    k_ms, k_launches, k_bytes = s.kernel_timer_read()
    its = [i.iterations for i in infos]
    ms_per_step = 1e3 * t_steps / args.steps
    # stand-alone batched applies
    R = torch.as_tensor(np.concatenate([random_vector(n, seed=1 + j) for j in range(nrhs)]), device=dev)
    Z = torch.zeros_like(R)
    for _ in range(3):
        s.apply(R, Z, nrhs=nrhs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.applies):
        s.apply(R, Z, nrhs=nrhs)
    e1.record()
    torch.cuda.synchronize()
    t_apply_ms = e0.elapsed_time(e1) / args.applies
    k_avg_us = 1e3 * k_ms / max(k_launches, 1)
    achieved = k_bytes / (k_avg_us * 1e-6) / 1e9
    elem = {"fp64": 8, "fp32": 4, "bf16": 2}[prec]
    flops = 2.0 * (k_bytes / elem) * K
    tfs = flops / (k_avg_us * 1e-6) / 1e12
    log(f"[bench] {args.steps} lockstep solves: {ms_per_step:.1f} ms each, iterations {its[:4]}...; "
        f"{nrhs}-column apply {t_apply_ms:.3f} ms; MFMA product {k_avg_us:.1f} us avg over {k_launches} launches "
        f"-> {achieved:.0f} GB/s, {tfs:.1f} TFLOP/s")
    out = {
        "metric": f"column applies/s of M^-1 inside lockstep FGMRES to 1e-8 ({nrhs} right-hand sides, {prec} local inverses)",
        "value": float(col_its / t_steps),
        "unit": "column applies/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else f"f64 (local inverses {prec}, matrix-core products, fp32 accumulation)",
        "data": "synthetic: Poiseuille Stokes problem generated in-library; b_k = c_k b(1), c_k ~ U[0.5, 2] (seed 3)",
        "config": {"workload": f"{w.name}: {w.n}^3 Q2/Q1 hexahedra, {w.m}^3 subdomains, overlap {w.overlap}, "
                               f"2-level GDSW, {nrhs} right-hand sides, FGMRES rtol {w.rtol:g} restart {w.restart}",
                   "n_free": n, "n_coarse": int(sz.n_coarse)},
        "iterations": its,
        "time_to_tol_s": ms_per_step / 1e3,
        "apply_columns_per_s": nrhs * 1e3 / t_apply_ms,
        "setup_s": t_setup,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": f"gemm_part_kernel ({prec} level-1 inverses x {K} right-hand sides on the matrix cores)",
                     "bytes_per_launch": k_bytes, "launches_timed": k_launches, "avg_launch_us": k_avg_us,
                     "mfma_tflops": tfs, "mfma_peak_tflops": MFMA_PEAK_TFS[prec],
                     "mfma_frac": tfs / MFMA_PEAK_TFS[prec]},
    }
    s.close()
    print(json.dumps(out))


def run_batch(args, prec):
    """16 uneven problems (n ~ U{8,12,16,20}, mu = 10^U[-1,1], c ~ U[0.5,2],
    subdomains of 4^3 elements) in one batch: FGMRES in lockstep, the
    members' local and coarse products one launch pair per level."""
    import torch

    import paper_2508_04356_amd as G
    from inputs import c5_batch_draws, random_vector

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    draws = c5_batch_draws()
    problems = [dict(n=n, m=n // 4, viscosity=mu, inflow=c) for n, mu, c in draws]
    # the block solve by default; the learned interior solve needs whole
    # local inverses (symmetric tiles)
    solve = args.local_solve if args.local_solve != "auto" else ("symmetric" if args.learned else "block")
    if solve == "triangular":
        raise SystemExit("batches need explicit inverses (inverse or symmetric)")
    log(f"[bench] setup C5 batch: n = {[p['n'] for p in problems]} precision={prec} local solve {solve}")
    t0 = time.perf_counter()
    bt = G.Batch(problems, precision=prec, local_solve=solve)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    bs, xs = [], []
    for m in bt.members:
        b = torch.zeros(m.n_free, dtype=torch.float64, device=dev)
        m.rhs(b)
        bs.append(b)
        xs.append(torch.zeros_like(b))
    for _ in range(args.warmup):
        bt.fgmres(bs, xs, use_graph=args.graph)
    torch.cuda.synchronize()
    bt.kernel_timer(True)
    t0 = time.perf_counter()
    total_its = 0
    for _ in range(args.steps):
        infos = bt.fgmres(bs, xs, use_graph=args.graph)
        total_its += sum(i.iterations for i in infos)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    bt.kernel_timer(False)
    k_ms, k_launches, k_bytes = bt.kernel_timer_read()
    if k_launches == 0:  # graph replays carry no event nodes: time the merged product in eager applies
        rs = [torch.as_tensor(random_vector(m.n_free, seed=9), device=dev) for m in bt.members]
        zs = [torch.zeros_like(r) for r in rs]
        bt.kernel_timer(True)
        for _ in range(10):
            bt.apply(rs, zs)
        torch.cuda.synchronize()
        bt.kernel_timer(False)
        k_ms, k_launches, k_bytes = bt.kernel_timer_read()
    its = [i.iterations for i in infos]
    ms_per_step = 1e3 * t_steps / args.steps
    k_avg_us = 1e3 * k_ms / max(k_launches, 1)
    achieved = k_bytes / (k_avg_us * 1e-6) / 1e9
    fb = sum(m.sizes().factor_bytes for m in bt.members)
    log(f"[bench] {args.steps} batch solves: {ms_per_step:.1f} ms each; iterations {its}; merged product "
        f"{k_avg_us:.1f} us avg over {k_launches} launches -> {achieved:.0f} GB/s")
    out = {
        "metric": "member applies/s of M^-1 inside lockstep FGMRES to 1e-8 (16 uneven problems, one batch)",
        "value": float(total_its / t_steps), "unit": "member applies/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else f"f64 (local inverses {prec})",
        "data": "synthetic: 16 Poiseuille problems, n ~ U{8,12,16,20}, mu = 10^U[-1,1], c ~ U[0.5,2] (seed 5)",
        "config": {"workload": "C5: 16 uneven Q2/Q1 problems, 4^3-element subdomains, overlap 1, 2-level GDSW, "
                               "FGMRES rtol 1e-08 restart 100",
                   "n": [p["n"] for p in problems], "factor_bytes_total": fb},
        "iterations": its, "time_to_tol_s": ms_per_step / 1e3, "setup_s": t_setup, "local_solve": solve,
        "graph": bool(args.graph),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": {"symmetric": "symv_part_kernel over the merged upper tiles of the active members' "
                                             "level-1 inverses",
                                "block": "symv_part_kernel<double, 3> over the merged upper tiles of the active "
                                         "members' velocity-block inverses L_i^-1",
                                "inverse": "gemv_part_kernel over the merged level-1 inverses of the active members"}
                               [solve],
                     "bytes_per_launch": k_bytes, "launches_timed": k_launches, "avg_launch_us": k_avg_us},
    }
    if args.learned:
        out["learned"] = batch_learned_variant(bt, bs, xs, args.steps)
    bt.close()
    print(json.dumps(out))


def batch_learned_variant(bt, bs, xs, steps):
    """One conv net, trained on a unit-viscosity 16^3 problem with the same
    4^3-element subdomains and copied to every member with interior
    subdomains (all share its node grid; each member scales its local
    problems to unit viscosity); lockstep batch FGMRES with the learned
    interior solves (with and without the exact fallback) beside the exact
    ones."""
    import torch

    import paper_2508_04356_amd as G

    t0 = time.perf_counter()
    ref = G.Solver(16, 4, viscosity=1.0, inflow=1.0)
    info = ref.learned_init(seed=7)
    hist = ref.learned_train(solves=4, steps=600, batch=32, lr=2e-3, seed=3)
    learned = []
    for k, m in enumerate(bt.members):
        if m.sizes().n_sub >= 27:
            m.learned_init(seed=1)
            m.learned_copy(ref)
            learned.append(k)
    ref.close()
    torch.cuda.synchronize()
    res = {"trained_on": "16^3, 4^3 subdomains, viscosity 1", "members_with_learned_solve": learned,
           "interior_subdomains": int(sum(bt.members[k].learned.subdomains for k in learned)),
           "grid": info.grid, "train_s": time.perf_counter() - t0,
           "loss_first": float(np.mean(hist[:20])), "loss_last": float(np.mean(hist[-20:]))}
    for name, mode, tau in (("learned", "learned", 1e30), ("learned_fallback", "learned", 0.7)):
        for k in learned:
            bt.members[k].set_local_solver(mode, tau)
        bt.fgmres(bs, xs, raise_on_noconv=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            infos = bt.fgmres(bs, xs, raise_on_noconv=False)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        res[name] = {"iterations": [i.iterations for i in infos], "time_to_tol_ms": ms,
                     "max_true_rel_res": max(i.true_rel_res for i in infos)}
        log(f"[bench] batch {name}: {ms:.1f} ms, iterations {[i.iterations for i in infos]}")
    stats = [bt.members[k].learned_stats() for k in learned]
    res["learned_solves"], res["fallbacks"] = sum(a for a, _ in stats), sum(b for _, b in stats)
    for k in learned:
        bt.members[k].set_local_solver("lu")
    return res


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
    ap.add_argument("--local-solve", default="auto", choices=["auto", "inverse", "triangular", "symmetric", "block"],
                    help="auto (default): symmetric tile storage of the explicit inverses for one right-hand "
                         "side (single problems and batches), full inverses for several right-hand sides; or "
                         "one of inverse, symmetric (explicit inverses) and triangular (LU solves)")
    ap.add_argument("--nrhs", type=int, default=None,
                    help="right-hand sides solved together (default: the workload's; C3 has 32)")
    ap.add_argument("--graph", action="store_true", help="replay each FGMRES iteration as a captured HIP graph")
    ap.add_argument("--learned", action="store_true",
                    help="also train the conv-net local solve (interior subdomains) and time FGMRES with it")
    ap.add_argument("--applies", type=int, default=50)
    ap.add_argument("--autotune", action="store_true",
                    help="run gdsw_autotune on the level-1 product after setup (launch shape picked on this GPU)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="C2: skip the FP32 / BF16 / learned variants timed beside plain FP64")
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
                                   "(sharding over several GPUs is not built)"}))
        sys.exit(2)

    import torch

    import paper_2508_04356_amd as G
    from inputs import random_vector, workload

    if args.workload == "C5":
        run_batch(args, args.precision or "fp64")
        return
    w = workload(args.workload)
    prec = args.precision or (w.precision if args.workload not in ("C2", "C2alg", "P16", "P32") else "fp64")
    nrhs = w.nrhs if args.nrhs is None else args.nrhs
    if nrhs > 1:
        run_multi(args, w, prec, nrhs)
        return
    if args.local_solve == "auto":
        # one right-hand side: the saddle-point block solve (the velocity-block
        # inverse and the pressure Schur complement inverse as upper tiles);
        # the learned interior solve replaces whole local inverses, so it runs
        # on the symmetric tiles of A_i^-1
        args.local_solve = "symmetric" if args.learned else "block"
    alg = w.local_algebraic if args.local_algebraic is None else args.local_algebraic
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"[bench] setup {w.name}: n={w.n} m={w.m} levels={w.levels} precision={prec}")
    t0 = time.perf_counter()
    s = G.Solver(w.n, w.m, overlap=w.overlap, levels=w.levels, group=w.group, viscosity=w.viscosity,
                 inflow=w.inflow, tile=args.tile, precision=prec, local_algebraic=alg,
                 level2_layer=w.level2_layer, local_solve=args.local_solve, pressure=w.pressure,
                 coarse=w.coarse)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    t_sym, t_num = s.setup_times()
    sz = s.sizes()
    n = sz.n_free
    log(f"[bench] setup {t_setup:.2f} s (symbolic {t_sym:.2f} s, numeric {t_num:.2f} s); n_free={n} "
        f"Nc={sz.n_coarse} device bytes={sz.device_bytes / 1e9:.2f} GB")
    tuned = None
    if args.autotune:
        code, ms = s.autotune()
        tuned = {"chosen": code, "ms": ms}
        log(f"[bench] autotune: chosen {code}, candidate ms {['%.4f' % t for t in ms]}")

    b = torch.zeros(n, dtype=torch.float64, device=dev)
    s.rhs(b)
    x = torch.zeros_like(b)

    for _ in range(args.warmup):
        s.fgmres(b, x, rtol=w.rtol, restart=w.restart, max_it=w.max_it, use_graph=args.graph)
    torch.cuda.synchronize()
    its = []
    s.kernel_timer(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        info = s.fgmres(b, x, rtol=w.rtol, restart=w.restart, max_it=w.max_it, use_graph=args.graph)[0]
        its.append(info.iterations)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    s.kernel_timer(False)
    k_ms, k_launches, k_bytes = s.kernel_timer_read()
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
    timed_in = "the timed FGMRES solves"
    if k_launches == 0:  # graph replays carry no event nodes: time the same kernel in eager applies
        s.kernel_timer(True)
        for _ in range(args.applies):
            s.apply(r, z)
        torch.cuda.synchronize()
        s.kernel_timer(False)
        k_ms, k_launches, k_bytes = s.kernel_timer_read()
        timed_in = "eager applies after the graph-replayed solves"
    phases = np.array([s.profile_apply(r, z) for _ in range(10)])
    ph = phases.mean(axis=0)
    solve_bytes = float(sz.solve_bytes)
    launches = int(sz.solve_launches)
    k_avg_us = 1e3 * k_ms / max(k_launches, 1)
    achieved = k_bytes / (k_avg_us * 1e-6) / 1e9
    per_apply = k_launches / max(sum(its), 1) if timed_in.startswith("the timed") else k_launches / args.applies
    kname = {"inverse": "gemv_part_kernel (level-1 explicit inverses times the local vectors)",
             "symmetric": "symv_part_kernel (upper 64x64 tiles of the symmetric level-1 inverses, both products "
                          "per tile)",
             "triangular": "trsv_step_kernel (blocked forward/backward solves of the level-1 factors)",
             "block": f"symv_part_kernel<{ {'fp64': 'double', 'fp32': 'float', 'bf16': 'uint16_t'}[prec]}, 3> "
                      "(upper 64x64 tiles of the velocity-block inverses L_i^-1, three "
                      "component vectors per tile; " +
                      ("one launch per apply: W_i = K_i^-1 B_i^T is kept for the last step)" if round(per_apply) == 1
                       else "two launches per apply)")}[args.local_solve]
    log(f"[bench] apply {t_apply_ms:.3f} ms; phases ms gather/restrict {ph[0]:.3f} solve {ph[1]:.3f}+{ph[2]:.3f} "
        f"scatter {ph[3]:.3f}; dominant kernel {k_launches} launches in the timed solves, {k_avg_us:.1f} us avg, "
        f"{k_bytes:.3e} B each -> {achieved:.0f} GB/s")

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
        "config": {"workload": f"{w.name}: {w.n}^3 Q2/{'P1disc' if w.pressure == 'p1disc' else 'Q1'} hexahedra, "
                               f"{w.m}^3 subdomains, overlap {w.overlap}, {w.levels}-level "
                               f"{'GDSW*' if w.coarse == 'gdsw*' else 'GDSW'}, FGMRES rtol {w.rtol:g} "
                               f"restart {w.restart}",
                   "n_free": n, "n_coarse": int(sz.n_coarse), "tile": args.tile or 128,
                   "local_problems": "algebraic overlap (closed box grown by one element)" if alg
                   else "Dirichlet u and p on the artificial boundary of the grown box"},
        "iterations": its[-1],
        "time_to_tol_s": ms_per_step / 1e3,
        "true_rel_res": info.true_rel_res,
        "apply_only_per_s": 1e3 / t_apply_ms,
        "apply_phases_ms": {"gather_restrict": ph[0], "solve_l1": ph[1], "solve_coarse": ph[2], "scatter": ph[3]},
        "setup_s": t_setup,
        "setup_symbolic_s": t_sym,
        "setup_numeric_s": t_num,
        "local_solve": args.local_solve,
        "graph": bool(args.graph),
        "autotune": tuned,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (measured_traffic(args.local_solve, round(per_apply))
                                 if args.workload == "C2" and not alg and prec == "fp64" and not args.autotune
                                 else None),
                     "kernel": kname,
                     "bytes_per_launch": k_bytes, "launches_timed": k_launches,
                     "launches_per_apply": per_apply, "avg_launch_us": k_avg_us, "timed_in": timed_in,
                     "solve_bytes_per_apply_all_sets": solve_bytes, "solve_launches_per_apply_all_sets": launches},
    }
    if args.workload == "C2" and not args.no_variants:
        # mixed precision and the learned interior solve against plain FP64 on
        # the same GPU, same workload and tolerance
        out["variants"] = {"fp64": {"iterations": its[-1], "time_to_tol_ms": ms_per_step,
                                    "true_rel_res": info.true_rel_res}}
        out["variants"].update(precision_variants(w, args, b, x, z, r, args.local_solve))
        args.learned = True
    if args.learned:
        out["learned"] = learned_variant(s, b, w, args.steps, args.local_solve)
        if "variants" in out:
            out["variants"]["learned_fallback"] = out["learned"]["learned_fallback"]
            out["variants"]["learned"] = out["learned"]["learned"]
    cbw = copy_bandwidth(torch, dev)
    out["roofline"]["measured_copy_gbs"] = cbw
    out["roofline"]["frac_of_copy"] = achieved / cbw
    log(f"[bench] 1 GiB copy: {cbw:.0f} GB/s (read + write); dominant kernel at {achieved / cbw:.3f} of it")
    if not args.no_cpu_baseline and args.workload == "C2":
        log("[bench] CPU oracle sample ...")
        out["cpu_baseline"] = cpu_baseline(w)
    s.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
