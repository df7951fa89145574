"""The learned local solve inside a batch: one network, trained on one
member, copied to the other members whose interior subdomains share its node
grid (4^3-element subdomains; the members differ in viscosity, which the
solve scales out).  In the batch the merged product skips those members'
interior matrices and the network (with its residual check and exact
fallback) fills them in, so every member must compute exactly what it
computes alone with the same network: the batched apply and the lockstep
FGMRES are compared bitwise with each member's own."""
import pytest

torch = pytest.importorskip("torch")

import paper_2508_04356_amd as G  # noqa: E402
from inputs import random_vector  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"

PROBLEMS = [
    dict(n=16, m=4, viscosity=1.0, inflow=16.0),   # 8 interior subdomains: trains the network
    dict(n=8, m=2, viscosity=0.5, inflow=1.0),     # no interior subdomain: exact solves only
    dict(n=12, m=3, viscosity=3.0, inflow=0.8),    # 1 interior subdomain, other viscosity
]


@pytest.fixture(scope="module", params=["inverse", "symmetric"])
def batch(request):
    print(f"[gpu] learned batch setup {PROBLEMS} {request.param}", flush=True)
    b = G.Batch(PROBLEMS, local_solve=request.param)
    src = b.members[0]
    src.learned_init(seed=7)
    src.learned_train(solves=2, steps=150, batch=16, lr=2e-3, seed=3)
    b.members[2].learned_init(seed=1)
    b.members[2].learned_copy(src)
    for k in (0, 2):
        b.members[k].set_local_solver("learned", 0.7)
    yield b
    b.close()


def test_copied_network_is_identical(batch):
    w0 = batch.members[0].learned_weights(which=1)
    w2 = batch.members[2].learned_weights(which=1)
    assert (w0 == w2).all()


def test_batched_learned_apply_is_each_members_apply(batch):
    rs = [torch.as_tensor(random_vector(m.n_free, seed=40 + k), device=DEV) for k, m in enumerate(batch.members)]
    zs = [torch.zeros_like(r) for r in rs]
    batch.apply(rs, zs)
    for k, m in enumerate(batch.members):
        z1 = torch.zeros_like(rs[k])
        m.apply(rs[k], z1)
        torch.cuda.synchronize()
        assert torch.equal(zs[k], z1), k


def test_batched_learned_fgmres_is_each_members_fgmres(batch):
    bs, xs = [], []
    for m in batch.members:
        b = torch.zeros(m.n_free, dtype=torch.float64, device=DEV)
        m.rhs(b)
        bs.append(b)
        xs.append(torch.zeros_like(b))
    before = [batch.members[k].learned_stats() for k in (0, 2)]
    infos = batch.fgmres(bs, xs, rtol=1e-8)
    after = [batch.members[k].learned_stats() for k in (0, 2)]
    print(f"[gpu] learned batch iterations {[i.iterations for i in infos]}, (learned, fallback) solves "
          f"{[(a[0] - b[0], a[1] - b[1]) for a, b in zip(after, before)]}", flush=True)
    # the network did the interior solves of both learned members
    assert all(a[0] + a[1] > b[0] + b[1] for a, b in zip(after, before))
    for k, m in enumerate(batch.members):
        x1 = torch.zeros_like(bs[k])
        info1 = m.fgmres(bs[k], x1, rtol=1e-8)[0]
        torch.cuda.synchronize()
        assert infos[k].iterations == info1.iterations, k
        assert infos[k].true_rel_res <= 1e-8
        assert torch.equal(xs[k], x1), k


def test_no_interior_correction_mode_in_batch(batch):
    """Mode 2 (no interior correction) batched equals alone as well."""
    for k in (0, 2):
        batch.members[k].set_local_solver("none")
    try:
        rs = [torch.as_tensor(random_vector(m.n_free, seed=60 + k), device=DEV) for k, m in enumerate(batch.members)]
        zs = [torch.zeros_like(r) for r in rs]
        batch.apply(rs, zs)
        for k, m in enumerate(batch.members):
            z1 = torch.zeros_like(rs[k])
            m.apply(rs[k], z1)
            torch.cuda.synchronize()
            assert torch.equal(zs[k], z1), k
    finally:
        for k in (0, 2):
            batch.members[k].set_local_solver("learned", 0.7)
