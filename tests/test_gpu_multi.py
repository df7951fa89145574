"""Several right-hand sides: the batched apply (MFMA products with the stored
inverses) and FGMRES in lockstep, through the C ABI, against the CPU oracle.

Tolerances: FP64 columns follow the single-column bar (1e-10 relative in the
max norm for the apply; identical iteration counts and 1e-10 solutions for
FGMRES).  With FP32 storage the right-hand sides are rounded to FP32 for the
products and accumulated in FP32, so batched and single-column applies agree
to a few FP32 ulps of the result (1e-5 relative).  With BF16 storage the
right-hand sides are rounded to BF16 (8 significant bits) for the matrix-core
products: each product term carries a relative error up to 2^-8, and the
sum of n_i terms with mixed signs can cancel, so the batched BF16 apply is
held to 3e-2 relative against the single-column BF16 apply (which keeps the
right-hand side in FP32) and to the same bound against FP64.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_04356_amd as G  # noqa: E402
from inputs import c3_inflow_amplitudes, random_vector, workload  # noqa: E402
from oracle.decomposition import Decomposition  # noqa: E402
from oracle.fgmres import fgmres as oracle_fgmres  # noqa: E402
from oracle.gdsw import TwoLevelGDSW  # noqa: E402
from oracle.stokes import StokesProblem  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def block(n, k, seed):
    """n x k column-major block of standard normal columns (one seed per column)."""
    return np.stack([random_vector(n, seed=seed + j) for j in range(k)], axis=1)


def dev_cm(a):
    """Column-major device copy: column j at offset j * n."""
    return torch.as_tensor(np.ascontiguousarray(a.T).ravel(), dtype=torch.float64, device=DEV)


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("nrhs,max_rhs", [(5, 8), (40, 16)])
def test_batched_apply_parity_fp64(nrhs, max_rhs):
    w = workload("C1").with_(name="n8m4", n=8, m=4)
    p = StokesProblem(w.n)
    d = Decomposition(p, w.m, w.overlap)
    M = TwoLevelGDSW(p.A, d)
    print(f"[gpu] multi apply n={w.n} m={w.m} nrhs={nrhs} max_rhs={max_rhs}", flush=True)
    s = G.Solver(w.n, w.m, max_rhs=max_rhs)
    n = s.n_free
    R = block(n, nrhs, seed=100)
    Z = torch.zeros(nrhs * n, dtype=torch.float64, device=DEV)
    s.apply(dev_cm(R), Z, nrhs=nrhs)
    Zh = host(Z).reshape(nrhs, n).T
    for j in range(nrhs):
        err = relmax(Zh[:, j], M(R[:, j]))
        assert err < 1e-10, (j, err)
    # bitwise repeatable
    Z2 = torch.zeros_like(Z)
    s.apply(dev_cm(R), Z2, nrhs=nrhs)
    assert torch.equal(Z, Z2)
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 3e-2)])
def test_batched_apply_reduced_precision(prec, tol):
    n_el, m, k = 12, 3, 32
    print(f"[gpu] multi apply {prec} n={n_el} m={m} nrhs={k}", flush=True)
    s = G.Solver(n_el, m, precision=prec, max_rhs=32)
    s64 = G.Solver(n_el, m, precision="fp64")
    n = s.n_free
    R = block(n, k, seed=7)
    Rd = dev_cm(R)
    Z = torch.zeros(k * n, dtype=torch.float64, device=DEV)
    s.apply(Rd, Z, nrhs=k)
    Zb = host(Z).reshape(k, n).T
    for j in range(0, k, 7):
        r = Rd[j * n:(j + 1) * n].clone()
        z1 = torch.zeros(n, dtype=torch.float64, device=DEV)
        z64 = torch.zeros_like(z1)
        s.apply(r, z1)
        s64.apply(r, z64)
        e_single = relmax(Zb[:, j], host(z1))
        e64 = relmax(Zb[:, j], host(z64))
        print(f"[gpu] {prec} column {j}: vs single {e_single:.2e} vs fp64 {e64:.2e}", flush=True)
        assert e_single < tol
        assert e64 < (3e-2 if prec == "bf16" else 1e-4)
    s.close()
    s64.close()


def test_lockstep_fgmres_linearity_and_parity():
    """P8: b(c_k) = c_k b(1), so every column has the same Krylov space:
    identical iteration counts, x(c_k) = c_k x(1), and the oracle's count."""
    w = workload("C1").with_(name="n8m4", n=8, m=4)
    p = StokesProblem(w.n)
    d = Decomposition(p, w.m, w.overlap)
    M = TwoLevelGDSW(p.A, d)
    xo, ito, _, _ = oracle_fgmres(lambda v: p.A @ v, M, p.b, rtol=w.rtol)
    cs = c3_inflow_amplitudes(6)
    s = G.Solver(w.n, w.m, max_rhs=8)
    n = s.n_free
    b1 = torch.zeros(n, dtype=torch.float64, device=DEV)
    s.rhs(b1)
    B = torch.cat([b1 * float(c) for c in cs])
    X = torch.zeros_like(B)
    infos = s.fgmres(B, X, rtol=w.rtol, restart=w.restart, max_it=w.max_it, nrhs=len(cs))
    its = [i.iterations for i in infos]
    print(f"[gpu] lockstep its {its} oracle {ito}", flush=True)
    assert len(set(its)) == 1 and its[0] == ito
    Xh = host(X).reshape(len(cs), n)
    for k, c in enumerate(cs):
        assert infos[k].true_rel_res <= w.rtol
        assert np.linalg.norm(Xh[k] - c * Xh[0] / cs[0]) <= 1e-10 * np.linalg.norm(Xh[k])
        assert np.linalg.norm(Xh[k] - c * xo) <= (1e-10 + 10 * w.rtol) * np.linalg.norm(c * xo)
    s.close()


def test_lockstep_fgmres_independent_columns_and_masking():
    """Different right-hand sides stop at their own iteration; a zero column
    is done at once with x = 0 and does not disturb the others."""
    w = workload("C1").with_(name="n8m4", n=8, m=4)
    p = StokesProblem(w.n)
    d = Decomposition(p, w.m, w.overlap)
    M = TwoLevelGDSW(p.A, d)
    s = G.Solver(w.n, w.m, max_rhs=4)
    n = s.n_free
    cols = [random_vector(n, seed=40), np.zeros(n), p.b.copy(), random_vector(n, seed=41)]
    B = dev_cm(np.stack(cols, axis=1))
    X = torch.zeros_like(B)
    infos = s.fgmres(B, X, rtol=1e-8, restart=100, max_it=1000, nrhs=4)
    Xh = host(X).reshape(4, n)
    assert infos[1].iterations == 0 and not np.any(Xh[1])
    for k in (0, 2, 3):
        xo, ito, _, _ = oracle_fgmres(lambda v: p.A @ v, M, cols[k], rtol=1e-8)
        print(f"[gpu] column {k}: its {infos[k].iterations} oracle {ito}", flush=True)
        assert infos[k].iterations == ito
        assert infos[k].true_rel_res <= 1e-8
        assert np.linalg.norm(Xh[k] - xo) <= (1e-10 + 10 * 1e-8) * np.linalg.norm(xo)
    assert np.all(np.isfinite(Xh))
    s.close()
