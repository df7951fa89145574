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
