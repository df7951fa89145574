"""gdsw_apply_precond_noalloc (partial sums in the library's static device
array) against gdsw_apply_precond on the same context: the same kernels and
summation orders, so the outputs must agree bit for bit.  Two calls in a row
on one device, the second on a smaller problem, so the second reuses the
array the first left behind; then the first problem again.  Calls go through
the C ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_04356_amd as G  # noqa: E402
from inputs import random_vector  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _pair(s, seed, nrhs=1):
    r = torch.as_tensor(random_vector(s.n_free, seed=seed, ncols=nrhs), device=DEV)
    r = r.T.contiguous().reshape(-1) if nrhs > 1 else r
    z0 = torch.zeros_like(r)
    z1 = torch.full_like(r, float("nan"))
    s.apply(r, z0, nrhs=nrhs)
    s.apply_noalloc(r, z1, nrhs=nrhs)
    torch.cuda.synchronize()
    return z0, z1


@pytest.mark.parametrize("solve", ["block", "symmetric", "inverse"])
@pytest.mark.parametrize("levels", [2, 3])
def test_noalloc_matches_apply(solve, levels):
    big = dict(n=12, m=3) if levels == 2 else dict(n=12, m=6, levels=3, group=3)
    small = dict(n=6, m=3) if levels == 2 else dict(n=8, m=4, levels=3, group=2)
    print(f"[gpu] noalloc {solve} levels {levels}", flush=True)
    a = G.Solver(**big, local_solve=solve)
    b = G.Solver(**small, local_solve=solve)
    assert b.n_free < a.n_free
    for s, seed in [(a, 1), (b, 2), (a, 3)]:
        z0, z1 = _pair(s, seed)
        assert torch.isfinite(z1).all()
        assert torch.equal(z0, z1), float((z0 - z1).abs().max())
    # several columns, one at a time through the same array
    z0, z1 = _pair(b, 4, nrhs=3)
    assert torch.equal(z0, z1)
    if solve == "block":  # the paper's pressure element: the two-pass block form
        c = G.Solver(6, 3, local_algebraic=1, pressure="p1disc", coarse="gdsw*", local_solve="block")
        for s, seed in [(c, 5), (b, 6)]:
            z0, z1 = _pair(s, seed)
            assert torch.equal(z0, z1), float((z0 - z1).abs().max())
        c.close()
    a.close()
    b.close()


def test_noalloc_rejections():
    """Triangular solves are refused (EUNSUPPORTED); a problem whose partial
    sums exceed the static array (24^3, symmetric tiles: 340 MiB) is refused
    with the bytes it needs (EINVAL), and the output is left untouched."""
    s = G.Solver(6, 3, local_solve="triangular")
    r = torch.zeros(s.n_free, dtype=torch.float64, device=DEV)
    z = torch.zeros_like(r)
    with pytest.raises(G.GdswError) as e:
        s.apply_noalloc(r, z)
    assert e.value.name == "EUNSUPPORTED"
    s.close()
    s = G.Solver(24, 6, local_solve="symmetric")
    r = torch.ones(s.n_free, dtype=torch.float64, device=DEV)
    z = torch.full_like(r, 7.0)
    with pytest.raises(G.GdswError) as e:
        s.apply_noalloc(r, z)
    assert e.value.name == "EINVAL" and "bytes of scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((z == 7.0).all())
    s.close()
