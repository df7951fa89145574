"""Status paths of the C ABI, forced from the host (every kernel runs to its
end; only the status and message are checked), and the network file.

* ESINGULAR: a viscosity of 1e-300 makes every velocity pivot fall below
  the pivot tolerance (1e-14 of the largest matrix entry, set by the
  divergence block) -- the setup refuses the factors and names the block.
* A NaN right-hand side: the Arnoldi norm turns non-finite and the solve
  stops with ENOCONV and a message saying so; the context stays usable.
* max_it = 2: ENOCONV, the info filled in, x the last iterate.
* The learned network written to a file and read back gives bitwise the
  same weights and the same preconditioner; a file for another node grid is
  refused (EINVAL); the per-solve fallback counts add up to the totals.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_04356_amd as G  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_singular_local_block_is_reported():
    print("[gpu] ESINGULAR via viscosity 1e-300", flush=True)
    with pytest.raises(G.GdswError) as e:
        G.Solver(4, 2, viscosity=1e-300)
    assert e.value.name == "ESINGULAR"
    assert "pivot" in str(e.value)


def test_nan_right_hand_side_is_reported_and_context_survives():
    s = G.Solver(6, 3)
    b = torch.zeros(s.n_free, dtype=torch.float64, device=DEV)
    s.rhs(b)
    bad = b.clone()
    bad[5] = float("nan")
    x = torch.zeros_like(b)
    print("[gpu] NaN right-hand side", flush=True)
    with pytest.raises(G.GdswError) as e:
        s.fgmres(bad, x, rtol=1e-8)
    assert e.value.name == "ENOCONV" and "non-finite" in str(e.value)
    info = s.fgmres(b, x, rtol=1e-8)[0]
    assert info.true_rel_res <= 1e-8
    s.close()


def test_max_it_reports_enoconv_with_last_iterate():
    s = G.Solver(6, 3)
    b = torch.zeros(s.n_free, dtype=torch.float64, device=DEV)
    s.rhs(b)
    x = torch.zeros_like(b)
    with pytest.raises(G.GdswError) as e:
        s.fgmres(b, x, rtol=1e-8, max_it=2)
    assert e.value.name == "ENOCONV"
    info = s.fgmres(b, x, rtol=1e-8, max_it=2, raise_on_noconv=False)[0]
    assert info.iterations == 2 and info.true_rel_res > 1e-8
    r = torch.zeros_like(b)
    s.spmv(x, r)
    rel = float(torch.linalg.norm(b - r) / torch.linalg.norm(b))
    assert abs(rel - info.true_rel_res) <= 1e-12 + 1e-9 * rel and rel < 1.0
    s.close()


def test_learned_network_file_roundtrip(tmp_path):
    path = str(tmp_path / "net.bin")
    a = G.Solver(12, 3)
    a.learned_init(seed=5)
    print("[gpu] train_local_net", flush=True)
    a.train_local_net(path, steps=40, seed=2)
    assert os.path.getsize(path) == 8 + 8 + 8 + 16 + 4 * a.learned.n_params
    w_a = a.learned_weights(0)
    b = G.Solver(12, 3, viscosity=2.5)
    b.learned_init(seed=9)
    b.learned_load(path)
    assert np.array_equal(b.learned_weights(0), w_a)
    assert np.array_equal(b.learned_weights(1), a.learned_weights(1))
    # same network on a problem with the same unit-viscosity local grid: the
    # learned apply of a copy and of the loaded file agree bitwise
    c = G.Solver(12, 3, viscosity=2.5)
    c.learned_init(seed=1)
    c.learned_copy(a)
    r = torch.as_tensor(np.random.default_rng(3).standard_normal(b.n_free), device=DEV)
    zb, zc = torch.zeros_like(r), torch.zeros_like(r)
    for s in (b, c):
        s.set_local_solver("learned", 0.7)
    b.apply(r, zb)
    c.apply(r, zc)
    torch.cuda.synchronize()
    assert torch.equal(zb, zc)
    # per-solve counts in the info add up to the context's totals
    rhs = torch.zeros_like(r)
    b.rhs(rhs)
    x = torch.zeros_like(r)
    l0, f0 = b.learned_stats()
    info = b.fgmres(rhs, x, rtol=1e-8, raise_on_noconv=False)[0]
    l1, f1 = b.learned_stats()
    assert info.learned_solves == l1 - l0 > 0 and info.fallbacks == f1 - f0
    # a file for another interior node grid is refused
    d = G.Solver(18, 3)
    d.learned_init(seed=1)
    with pytest.raises(G.GdswError) as e:
        d.learned_load(path)
    assert e.value.name == "EINVAL"
    for s in (a, b, c, d):
        s.close()


def test_setup_times_are_split():
    s = G.Solver(8, 2)
    sym, num = s.setup_times()
    assert sym > 0 and num > 0
    s.close()
