"""The algebraic entry point (gdsw_setup_algebraic) on the GPU against the
oracle's algebraic decomposition: any assembled matrix, any partition.
Cases: the cube's box partition (which must reproduce the structured
algebraic-overlap problem), unstructured Voronoi partitions of the cube with
the Q1 and with the P1disc pressure.  Calls go through the C ABI.

Tolerances as for the structured workloads: Phi and A_0 at 1e-12, the apply
at 1e-10, equal FGMRES counts.  The solutions are compared at 1e-8: with the
algebraic overlap the local problems are nearly singular (their rim velocity
is free), and two FP64 implementations of the iteration drift apart to
about that level (1e-10 on the structured cases of the same reading)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_04356_amd as G  # noqa: E402
from inputs import random_vector, voronoi_partition  # noqa: E402
from oracle.decomposition import AlgebraicDecomposition  # noqa: E402
from oracle.fgmres import fgmres as oracle_fgmres  # noqa: E402
from oracle.gdsw import TwoLevelGDSW  # noqa: E402
from oracle.stokes import StokesProblem  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda"


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def repeated_map(p, elem_part):
    full_to_free = -np.ones(p.n_full, dtype=np.int64)
    full_to_free[p.free] = np.arange(p.n_free)
    subs = [set() for _ in range(p.n_free)]
    for e, dofs in enumerate(p.element_dofs):
        for fd in dofs:
            d = full_to_free[fd]
            if d >= 0:
                subs[d].add(int(elem_part[e]))
    return [sorted(s) for s in subs]


def box_partition(n, m):
    e = np.arange(n ** 3)
    s = n // m
    return (e % n) // s + m * (((e // n) % n) // s + m * ((e // (n * n)) // s))


CASES = [("box q1 6/3", 6, "q1", lambda: box_partition(6, 3)),
         ("voronoi q1 8/10", 8, "q1", lambda: voronoi_partition(8, 10, seed=11)),
         ("voronoi p1disc 6/7", 6, "p1disc", lambda: voronoi_partition(6, 7, seed=4))]


@pytest.mark.parametrize("solve", ["inverse", "symmetric"])
@pytest.mark.parametrize("name,n,pressure,part", CASES, ids=[c[0] for c in CASES])
def test_algebraic_entry_point_parity(name, n, pressure, part, solve):
    p = StokesProblem(n, pressure=pressure)
    A = p.A.tocsr()
    A.sort_indices()
    subs = repeated_map(p, part())
    d = AlgebraicDecomposition(A, p.dof_field, subs, p.dof_null, 1)
    M = TwoLevelGDSW(A, d)
    print(f"[gpu] algebraic {name} {solve}: {d.n_sub} subdomains, {d.n_coarse} coarse DOFs", flush=True)
    s = G.Solver.algebraic(A.indptr, A.indices, A.data, p.dof_field, subs, null=p.dof_null, rhs=p.b,
                           local_solve=solve)
    assert s.n_free == p.n_free and s.n_coarse == d.n_coarse
    assert rel_max(s.coarse_basis(), M.Phi.toarray()) < 1e-12
    assert rel_max(s.coarse_matrix(), M.A0) < 1e-12
    r = random_vector(p.n_free, seed=1)
    z = torch.zeros(p.n_free, dtype=torch.float64, device=DEV)
    s.apply(torch.as_tensor(r, device=DEV), z)
    torch.cuda.synchronize()
    err = rel_max(z.cpu().numpy(), M(r))
    xo, ito, _, _ = oracle_fgmres(lambda v: A @ v, M, p.b, rtol=1e-8)
    b = torch.zeros_like(z)
    s.rhs(b)
    x = torch.zeros_like(z)
    info = s.fgmres(b, x, rtol=1e-8)[0]
    torch.cuda.synchronize()
    xerr = float(np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo))
    print(f"[gpu] algebraic {name} {solve}: apply rel err {err:.2e}; it {info.iterations} (oracle {ito}); "
          f"x rel err {xerr:.2e}", flush=True)
    assert err < 1e-10
    assert info.iterations == ito and info.true_rel_res <= 1e-8
    assert xerr < 1e-8
    s.close()


def test_algebraic_box_partition_is_the_structured_problem():
    """The cube's matrix with its box partition through the algebraic entry
    point gives the structured solver's preconditioner (algebraic-overlap
    reading): same apply to rounding, same FGMRES count."""
    n, m = 6, 3
    p = StokesProblem(n)
    A = p.A.tocsr()
    A.sort_indices()
    s1 = G.Solver.algebraic(A.indptr, A.indices, A.data, p.dof_field, repeated_map(p, box_partition(n, m)),
                            rhs=p.b)
    s2 = G.Solver(n, m, local_algebraic=1)
    r = torch.as_tensor(random_vector(p.n_free, seed=2), device=DEV)
    z1, z2 = torch.zeros_like(r), torch.zeros_like(r)
    s1.apply(r, z1)
    s2.apply(r, z2)
    torch.cuda.synchronize()
    assert float((z1 - z2).abs().max() / z2.abs().max()) < 1e-13
    b = torch.zeros_like(r)
    s2.rhs(b)
    x1, x2 = torch.zeros_like(r), torch.zeros_like(r)
    assert s1.fgmres(b, x1)[0].iterations == s2.fgmres(b, x2)[0].iterations
    s1.close()
    s2.close()


def test_block_solve_needs_node_interleaved_velocity():
    """The block local solve relies on K_i = I_3 (x) L_i with the velocity
    numbered node by node (3 node + component).  An assembled matrix whose
    free DOFs break that numbering (here: Dirichlet rows removed component
    by component) is refused at setup with EINVAL, not solved wrongly."""
    p = StokesProblem(6)
    A = p.A.tocsr()
    A.sort_indices()
    subs = repeated_map(p, box_partition(6, 3))
    with pytest.raises(G.GdswError, match="I_3"):
        G.Solver.algebraic(A.indptr, A.indices, A.data, p.dof_field, subs, null=p.dof_null, rhs=p.b,
                           local_solve="block")
