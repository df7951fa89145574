"""FGMRES with every iteration captured into a HIP graph (one per basis
index, replayed in later cycles and solves) must reproduce the eager solve
bitwise: same iteration count, same solution, on every replay, with eager
work of the program in between."""
import pytest

torch = pytest.importorskip("torch")

import paper_2508_04356_amd as G  # noqa: E402
from inputs import random_vector  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.mark.parametrize("kw", [dict(n=8, m=4), dict(n=12, m=6, levels=3, group=2),
                                dict(n=8, m=2, precision="bf16")],
                         ids=["two-level", "three-level", "bf16"])
def test_graph_fgmres_matches_eager(kw):
    print(f"[gpu] graph fgmres {kw}", flush=True)
    s = G.Solver(**kw)
    b = torch.zeros(s.n_free, dtype=torch.float64, device=DEV)
    s.rhs(b)
    x0 = torch.zeros_like(b)
    info0 = s.fgmres(b, x0, rtol=1e-8, restart=100, max_it=1000)[0]
    r = torch.as_tensor(random_vector(s.n_free, seed=3), device=DEV)
    z = torch.zeros_like(r)
    for rep in range(3):
        x = torch.zeros_like(b)
        info = s.fgmres(b, x, rtol=1e-8, restart=100, max_it=1000, use_graph=True)[0]
        torch.cuda.synchronize()
        print(f"[gpu] replay {rep}: its {info.iterations} (eager {info0.iterations})", flush=True)
        assert info.iterations == info0.iterations
        assert torch.equal(x, x0)
        s.apply(r, z)  # eager work between replays
        torch.cuda.synchronize()
    s.close()


def test_autotune_keeps_results_valid():
    """The launch-shape autotuner picks one of its three column chunks; the
    apply after tuning still matches the untuned apply to rounding and is
    bitwise repeatable."""
    s = G.Solver(12, 3)
    r = torch.as_tensor(random_vector(s.n_free, seed=8), device=DEV)
    z0 = torch.zeros_like(r)
    s.apply(r, z0)
    chunk, ms = s.autotune()
    print(f"[gpu] autotune chunk {chunk} ms {ms}", flush=True)
    assert chunk in (512, 1024, 2048) and all(t > 0 for t in ms)
    assert chunk == (512, 1024, 2048)[min(range(3), key=lambda q: ms[q])]
    z1 = torch.zeros_like(r)
    z2 = torch.zeros_like(r)
    s.apply(r, z1)
    s.apply(r, z2)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
    assert float((z1 - z0).abs().max() / z0.abs().max()) < 1e-13
    s.close()


def test_graph_solve_after_retune():
    """A re-plan (autotuner) replaces the item arrays and partial buffers the
    captured iterations point at: the next graph solve must re-capture and
    reproduce the eager solve on the new plan bitwise."""
    s = G.Solver(12, 3)
    b = torch.zeros(s.n_free, dtype=torch.float64, device=DEV)
    s.rhs(b)
    x0 = torch.zeros_like(b)
    info0 = s.fgmres(b, x0, rtol=1e-8)[0]
    x1 = torch.zeros_like(b)
    info1 = s.fgmres(b, x1, rtol=1e-8, use_graph=True)[0]
    torch.cuda.synchronize()
    assert info1.iterations == info0.iterations and torch.equal(x1, x0)
    chunk, ms = s.autotune()
    print(f"[gpu] retune chunk {chunk}", flush=True)
    x2 = torch.zeros_like(b)
    info2 = s.fgmres(b, x2, rtol=1e-8)[0]
    x3 = torch.zeros_like(b)
    info3 = s.fgmres(b, x3, rtol=1e-8, use_graph=True)[0]
    torch.cuda.synchronize()
    assert info3.iterations == info2.iterations and torch.equal(x3, x2)
    s.close()


@pytest.mark.parametrize("solve,precision", [("symmetric", "fp64"), ("symmetric", "fp32"), ("block", "fp64")])
def test_autotune_symmetric_tiles(solve, precision):
    """Symmetric tiles (and the block solve's velocity-block tiles): the
    autotuner times runs of 2 and 1 tiles in both work-group orders, keeps
    the argmin, and the apply on the new plan matches the untuned one to
    rounding, repeats bitwise, and a graph solve after the retune reproduces
    the eager solve bitwise."""
    print(f"[gpu] autotune {solve} {precision}", flush=True)
    s = G.Solver(12, 3, local_solve=solve, precision=precision)
    r = torch.as_tensor(random_vector(s.n_free, seed=8), device=DEV)
    z0 = torch.zeros_like(r)
    s.apply(r, z0)
    code, ms = s.autotune()
    print(f"[gpu] autotune {solve} {precision}: chosen {code}, ms {ms}", flush=True)
    cand = (20, 21, 10, 11)
    assert len(ms) == 4 and all(t > 0 for t in ms)
    assert code == cand[min(range(4), key=lambda q: ms[q])]
    z1, z2 = torch.zeros_like(r), torch.zeros_like(r)
    s.apply(r, z1)
    s.apply(r, z2)
    torch.cuda.synchronize()
    assert torch.equal(z1, z2)
    tol = 1e-13 if precision == "fp64" else 1e-6
    assert float((z1 - z0).abs().max() / z0.abs().max()) < tol
    b = torch.zeros_like(r)
    s.rhs(b)
    x0, x1 = torch.zeros_like(b), torch.zeros_like(b)
    info0 = s.fgmres(b, x0, rtol=1e-8)[0]
    info1 = s.fgmres(b, x1, rtol=1e-8, use_graph=True)[0]
    torch.cuda.synchronize()
    assert info1.iterations == info0.iterations and torch.equal(x1, x0)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_autotune_mfma_product(precision):
    """The several-column MFMA product: the autotuner keeps the argmin of its
    candidates, and the several-column apply on the tuned plan matches the
    untuned one to rounding."""
    print(f"[gpu] autotune mfma {precision}", flush=True)
    K = 8
    s = G.Solver(8, 2, precision=precision, max_rhs=K)
    n = s.n_free
    # column-major block: column k at offset k n
    R = torch.cat([torch.as_tensor(random_vector(n, seed=20 + k), device=DEV) for k in range(K)])
    Z0 = torch.zeros_like(R)
    s.apply(R, Z0, nrhs=K)
    best, ms = s.autotune_mfma()
    ncand = 6 if precision == "fp64" else 3
    print(f"[gpu] autotune mfma {precision}: chosen {best}, ms {ms}", flush=True)
    assert all(t > 0 for t in ms[:ncand]) and all(t == 0 for t in ms[ncand:])
    assert best == min(range(ncand), key=lambda q: ms[q])
    Z1 = torch.zeros_like(R)
    s.apply(R, Z1, nrhs=K)
    torch.cuda.synchronize()
    tol = 1e-13 if precision == "fp64" else 1e-5
    assert float((Z1 - Z0).abs().max() / Z0.abs().max()) < tol
    s.close()
