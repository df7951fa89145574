"""Writes tests/golden/oracle_<name>.json from the CPU oracle only.

Stored: FGMRES iteration count, residual history and norms in
oracle_<name>.json; the whole solution x and the whole preconditioner output
z = B r for r = random_vector(n, 1) on every free DOF in oracle_<name>.npz.
The GPU tests compare the library against these values.
Usage: python tests/golden/make_oracle_golden.py C2 [spread]
       python tests/golden/make_oracle_golden.py C3 apply   (several columns, sampled)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from inputs import random_vector, workload  # noqa: E402
from oracle.decomposition import Decomposition  # noqa: E402
from oracle.fgmres import fgmres  # noqa: E402
from oracle.gdsw import TwoLevelGDSW  # noqa: E402
from oracle.stokes import StokesProblem  # noqa: E402
from oracle.threelevel import ThreeLevelGDSW  # noqa: E402


def spread(name, k=10, eps=1e-14):
    """Iteration counts of the oracle's FGMRES when the preconditioner output
    and the SpMV output are perturbed entry-wise by relative noise of size eps
    (the size of the rounding differences between two FP64 implementations).
    Stored as oracle_<name>_spread.json."""
    w = workload(name)
    p = StokesProblem(w.n, viscosity=w.viscosity, inflow=w.inflow, manufactured=w.manufactured,
                      pressure=w.pressure)
    d = Decomposition(p, w.m, w.overlap, local_dirichlet=not w.local_algebraic, coarse=w.coarse)
    M = (ThreeLevelGDSW(p.A, d, w.group, level2_layer=bool(w.level2_layer)) if w.levels == 3
         else TwoLevelGDSW(p.A, d))
    counts = []
    for seed in range(k):
        rng = np.random.default_rng(100 + seed)

        def noisy(v):
            return v * (1.0 + eps * rng.standard_normal(v.size))

        x, it, rel, trel = fgmres(lambda v: noisy(p.A @ v), lambda v: noisy(M(v)), p.b, rtol=w.rtol,
                                  restart=w.restart, max_it=w.max_it)
        counts.append(int(it))
        print(f"seed {seed}: {it} iterations", flush=True)
    out = {"workload": name, "eps": eps, "counts": counts, "min": min(counts), "max": max(counts)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_{name}_spread.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


def main(name):
    w = workload(name)
    t0 = time.time()
    p = StokesProblem(w.n, viscosity=w.viscosity, inflow=w.inflow, manufactured=w.manufactured,
                      pressure=w.pressure)
    d = Decomposition(p, w.m, w.overlap, local_dirichlet=not w.local_algebraic, coarse=w.coarse)
    if w.levels == 3:
        M = ThreeLevelGDSW(p.A, d, w.group, level2_layer=bool(w.level2_layer))
    else:
        M = TwoLevelGDSW(p.A, d)
    t1 = time.time()
    print(f"setup {t1 - t0:.1f} s", flush=True)
    r = random_vector(p.n_free, seed=1)
    z = M(r)
    hist = []
    x, it, rel, trel = fgmres(lambda v: p.A @ v, M, p.b, rtol=w.rtol, restart=w.restart, max_it=w.max_it,
                              history=hist)
    t2 = time.time()
    print(f"solve {t2 - t1:.1f} s, {it} iterations, rel {rel:.3e}, true {trel:.3e}", flush=True)
    out = {
        "workload": name, "n": w.n, "m": w.m, "levels": w.levels, "group": w.group,
        "viscosity": w.viscosity, "inflow": w.inflow, "rtol": w.rtol, "restart": w.restart,
        "n_free": int(p.n_free), "n_coarse": int(d.n_coarse),
        "iterations": int(it), "rel": float(rel), "true_rel": float(trel),
        "history": [float(h) for h in hist],
        "x_norm": float(np.linalg.norm(x)), "z_norm": float(np.linalg.norm(z)),
        "oracle_setup_s": t1 - t0, "oracle_solve_s": t2 - t1,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f)
    np.savez(path[:-5] + ".npz", x=x, z=z)
    print("wrote", path)


def multi_apply(name="C3", ncols=4, nsample=16384):
    """The preconditioner applied to the first ncols seeded columns of the
    several-right-hand-side workload (column j: random_vector(n, 1 + j)),
    stored at nsample evenly spaced free DOFs, together with the entry-wise
    scale |M_loc| |r| of the level-1 local terms (the sum over subdomains of
    |A_i^-1| |r_i|, from explicit inverses) at those DOFs and its maximum over
    all DOFs: the rounding of the stored inverses to a precision with unit
    roundoff u perturbs z by at most u |M_loc| |r| entry-wise.  Written to
    oracle_<name>_apply.json / .npz."""
    w = workload(name)
    t0 = time.time()
    p = StokesProblem(w.n, viscosity=w.viscosity, inflow=w.inflow, manufactured=w.manufactured,
                      pressure=w.pressure)
    d = Decomposition(p, w.m, w.overlap, local_dirichlet=not w.local_algebraic, coarse=w.coarse)
    M = TwoLevelGDSW(p.A, d)
    R = np.stack([random_vector(p.n_free, seed=1 + j) for j in range(ncols)], 1)
    Z = M(R)
    print(f"apply {time.time() - t0:.1f} s", flush=True)
    M.local_lu = []  # free the factors before the explicit inverses
    scale = np.zeros_like(R)
    for i in range(d.n_sub):
        Mi = np.abs(np.linalg.inv(M.local_matrix(i)))
        S = d.S[i]
        scale[S] += Mi @ np.abs(R[S])
    print(f"scale {time.time() - t0:.1f} s", flush=True)
    idx = np.unique(np.linspace(0, p.n_free - 1, nsample).astype(np.int64))
    out = {"workload": name, "n_free": int(p.n_free), "ncols": ncols, "seeds": [1 + j for j in range(ncols)],
           "z_max": np.abs(Z).max(0).tolist(), "scale_max": scale.max(0).tolist()}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"oracle_{name}_apply.json")
    with open(path, "w") as f:
        json.dump(out, f)
    np.savez(path[:-5] + ".npz", idx=idx, z=Z[idx], scale=scale[idx])
    print("wrote", path)


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[2] == "apply":
        multi_apply(sys.argv[1])
    elif len(sys.argv) > 2 and sys.argv[2] == "spread":
        spread(sys.argv[1])
    else:
        main(sys.argv[1] if len(sys.argv) > 1 else "C2")
