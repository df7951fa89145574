"""A batch of independent, uneven problems (different n, m, viscosity,
inflow) whose local and coarse inverse products share one launch pair per
level (full inverses or symmetric tile storage).  A member must compute exactly what it computes alone: the batched
apply and the lockstep FGMRES are compared bitwise with each member's own
apply and FGMRES, and one member against the CPU oracle (1e-10)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_04356_amd as G  # noqa: E402
from inputs import random_vector  # noqa: E402
from oracle.decomposition import Decomposition  # noqa: E402
from oracle.gdsw import TwoLevelGDSW  # noqa: E402
from oracle.stokes import StokesProblem  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"

PROBLEMS = [
    dict(n=8, m=2, viscosity=1.0, inflow=16.0),
    dict(n=12, m=3, viscosity=0.3, inflow=1.2),
    dict(n=4, m=1, viscosity=2.0, inflow=0.7),   # one subdomain: no coarse level
    dict(n=8, m=4, viscosity=5.0, inflow=1.9),
]


@pytest.fixture(scope="module", params=["inverse", "symmetric", "block"])
def batch(request):
    print(f"[gpu] batch setup {PROBLEMS} {request.param}", flush=True)
    b = G.Batch(PROBLEMS, local_solve=request.param)
    yield b
    b.close()


def test_batched_apply_is_each_members_apply(batch):
    rs = [torch.as_tensor(random_vector(m.n_free, seed=20 + k), device=DEV) for k, m in enumerate(batch.members)]
    zs = [torch.zeros_like(r) for r in rs]
    batch.apply(rs, zs)
    for k, m in enumerate(batch.members):
        z1 = torch.zeros_like(rs[k])
        m.apply(rs[k], z1)
        torch.cuda.synchronize()
        assert torch.equal(zs[k], z1), k
    # member 0 against the oracle
    p = PROBLEMS[0]
    prob = StokesProblem(p["n"], viscosity=p["viscosity"], inflow=p["inflow"])
    M = TwoLevelGDSW(prob.A, Decomposition(prob, p["m"], 1))
    zo = M(random_vector(prob.n_free, seed=20))
    z0 = zs[0].cpu().numpy()
    assert np.abs(z0 - zo).max() <= 1e-10 * np.abs(zo).max()


def test_lockstep_batch_fgmres_is_each_members_fgmres(batch):
    bs, xs = [], []
    for m in batch.members:
        b = torch.zeros(m.n_free, dtype=torch.float64, device=DEV)
        m.rhs(b)
        bs.append(b)
        xs.append(torch.zeros_like(b))
    infos = batch.fgmres(bs, xs, rtol=1e-8)
    its = [i.iterations for i in infos]
    print(f"[gpu] batch iterations {its}", flush=True)
    assert its[2] == 1  # one subdomain: M^-1 = A^-1
    assert len(set(its)) > 1  # the members stop at different iterations
    for k, m in enumerate(batch.members):
        x1 = torch.zeros_like(bs[k])
        info1 = m.fgmres(bs[k], x1, rtol=1e-8)[0]
        torch.cuda.synchronize()
        assert infos[k].iterations == info1.iterations, k
        assert infos[k].true_rel_res <= 1e-8
        assert torch.equal(xs[k], x1), k


def test_lockstep_batch_graph_replays_match_eager(batch):
    """Graph mode: each lockstep iteration (every member's kernels on the
    stream lanes, the merged products, the read-backs) is captured once per
    (basis index, members still in the cycle) and replayed.  Three graph
    solves, with eager work in between, reproduce the eager lockstep solve
    bitwise; members drop out at different iterations, so several member
    sets are captured."""
    bs = []
    for m in batch.members:
        b = torch.zeros(m.n_free, dtype=torch.float64, device=DEV)
        m.rhs(b)
        bs.append(b)
    x0 = [torch.zeros_like(b) for b in bs]
    inf0 = batch.fgmres(bs, x0, rtol=1e-8)
    rs = [torch.as_tensor(random_vector(m.n_free, seed=40 + k), device=DEV) for k, m in enumerate(batch.members)]
    zs = [torch.zeros_like(r) for r in rs]
    for rep in range(3):
        xg = [torch.zeros_like(b) for b in bs]
        infg = batch.fgmres(bs, xg, rtol=1e-8, use_graph=True)
        torch.cuda.synchronize()
        print(f"[gpu] batch graph replay {rep}: its {[i.iterations for i in infg]}", flush=True)
        for k in range(len(bs)):
            assert infg[k].iterations == inf0[k].iterations, k
            assert torch.equal(xg[k], x0[k]), k
        batch.apply(rs, zs)  # eager work between replays
        torch.cuda.synchronize()
