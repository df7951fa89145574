"""CPU checks of the C ABI: exports, host-side setup against the oracle, errors.

No compute call reaches the device here; contexts are host-only.
"""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import paper_2508_04356_amd as G
from oracle.counts import full_gdsw_closed_form
from oracle.decomposition import Decomposition
from oracle.stokes import StokesProblem, dof_count_q2q1

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "gdsw.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(gdsw_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported_and_bound():
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(G._lib, s), s
        assert s in G.EXPORTED, s


def _check_sorted_rows(rp, col):
    """Every CSR row lists distinct columns in ascending order (the assembly
    emits a row's entries in column order without sorting them)."""
    d = np.diff(col.astype(np.int64))
    row_start = np.zeros(len(col), dtype=bool)
    row_start[rp[:-1][rp[:-1] < len(col)]] = True
    assert np.all(d[~row_start[1:]] > 0)
    assert np.all(np.diff(rp) > 0)


@pytest.mark.parametrize("n,m,mu,c,man", [(4, 2, 1.0, 16.0, 0), (6, 3, 0.7, 3.0, 1), (6, 2, 2.0, 1.0, 0)])
def test_host_assembly_matches_oracle(n, m, mu, c, man):
    s = G.Solver(n, m, host_only=True, viscosity=mu, inflow=c, manufactured=man)
    sz = s.sizes()
    p = StokesProblem(n, viscosity=mu, inflow=c, manufactured=man)
    assert sz.n_free == p.n_free and sz.n_full == p.n_full == dof_count_q2q1(n)
    assert sz.n_u_free == p.n_u and sz.n_p == p.n_p
    rp, col, val = s.host_matrix()
    _check_sorted_rows(rp, col)
    A = sp.csr_matrix((val, col, rp), shape=(sz.n_free, sz.n_free))
    assert abs(A - p.A).max() <= 1e-15 * abs(p.A).max()
    assert np.abs(s.host_rhs() - p.b).max() <= 1e-14 * max(1.0, np.abs(p.b).max())
    field, abc = s.dof_map()
    assert np.array_equal(field, p.dof_field) and np.array_equal(abc, p.dof_node)
    d = Decomposition(p, m, 1)
    assert sz.n_entities == d.n_ent == full_gdsw_closed_form(m)
    assert sz.n_coarse == d.n_coarse
    for i in range(d.n_sub):
        assert np.array_equal(s.local_indices(i), d.S[i])
    s.close()


def test_host_sizes_at_16_cubed():
    s = G.Solver(16, 4, host_only=True, local_algebraic=1)
    sz = s.sizes()
    assert sz.n_free == 97169 and sz.n_sub == 64 and sz.n_coarse == 1116
    assert sz.local_min == 3216 and sz.local_max == 6934
    s.close()
    s = G.Solver(16, 4, host_only=True)
    sz = s.sizes()
    assert sz.local_min == 2312 and sz.local_max == 4118
    s.close()


@pytest.mark.parametrize("kw,status", [
    (dict(n=5, m=2), "EINVAL"),
    (dict(n=4, m=2, overlap=0), "EINVAL"),
    (dict(n=4, m=2, levels=4), "EINVAL"),
    (dict(n=4, m=4, levels=3, group=3), "EINVAL"),
    (dict(n=4, m=2, precision=7), "EINVAL"),
    (dict(n=4, m=2, tile=96), "EINVAL"),
    (dict(n=4, m=2, viscosity=-1.0), "EINVAL"),
    (dict(n=0, m=1), "EINVAL"),
])
def test_setup_argument_errors(kw, status):
    with pytest.raises(G.GdswError) as e:
        G.Solver(host_only=True, **kw)
    assert e.value.name == status
    assert len(str(e.value)) > 10


def test_device_calls_rejected_on_host_context():
    s = G.Solver(4, 2, host_only=True)
    with pytest.raises(G.GdswError) as e:
        s.apply(1, 2)
    assert e.value.name == "EINVAL"
    with pytest.raises(G.GdswError):
        s.spmv(1, 2)
    with pytest.raises(G.GdswError):
        s.local_indices(99)
    s.close()


@pytest.mark.parametrize("alg", [0, 1])
def test_host_local_sets_match_oracle(alg):
    s = G.Solver(8, 4, host_only=True, local_algebraic=alg)
    p = StokesProblem(8)
    d = Decomposition(p, 4, 1, local_dirichlet=not alg)
    for i in range(d.n_sub):
        assert np.array_equal(s.local_indices(i), d.S[i])
    s.close()


@pytest.mark.parametrize("n,m,coarse", [(4, 2, "gdsw*"), (6, 3, "gdsw*"), (6, 3, "gdsw")])
def test_host_p1disc_setup_matches_oracle(n, m, coarse):
    """The paper's pair and coarse spaces in the library's host setup: matrix,
    right-hand side, DOF map, local sets and coarse dimension equal the
    oracle's (which computes them independently in numpy)."""
    s = G.Solver(n, m, host_only=True, pressure="p1disc", coarse=coarse, local_algebraic=1, viscosity=0.7,
                 inflow=3.0)
    sz = s.sizes()
    p = StokesProblem(n, pressure="p1disc", viscosity=0.7, inflow=3.0)
    d = Decomposition(p, m, 1, local_dirichlet=False, coarse=coarse)
    assert sz.n_free == p.n_free and sz.n_p == 4 * n ** 3
    rp, col, val = s.host_matrix()
    _check_sorted_rows(rp, col)
    A = sp.csr_matrix((val, col, rp), shape=(sz.n_free, sz.n_free))
    assert abs(A - p.A).max() <= 1e-15 * abs(p.A).max()
    assert np.abs(s.host_rhs() - p.b).max() <= 1e-14 * max(1.0, np.abs(p.b).max())
    field, abc = s.dof_map()
    assert np.array_equal(field, p.dof_field) and np.array_equal(abc, p.dof_node)
    assert sz.n_entities == d.n_ent and sz.n_coarse == d.n_coarse
    for i in range(d.n_sub):
        assert np.array_equal(s.local_indices(i), d.S[i])
    s.close()


def test_host_p1disc_rejections():
    with pytest.raises(G.GdswError):
        G.Solver(4, 2, host_only=True, pressure="p1disc")          # needs the algebraic overlap
    with pytest.raises(G.GdswError):
        G.Solver(4, 2, host_only=True, pressure="p1disc", local_algebraic=1, levels=3, group=1)


def _repeated_map(p, elem_part):
    """Subdomains holding each free DOF: the parts of the elements whose DOF
    lists contain it (sorted)."""
    full_to_free = -np.ones(p.n_full, dtype=np.int64)
    full_to_free[p.free] = np.arange(p.n_free)
    subs = [set() for _ in range(p.n_free)]
    for e, dofs in enumerate(p.element_dofs):
        for fd in dofs:
            d = full_to_free[fd]
            if d >= 0:
                subs[d].add(int(elem_part[e]))
    return [sorted(s) for s in subs]


def _box_partition(n, m):
    e = np.arange(n ** 3)
    s = n // m
    return (e % n) // s + m * (((e // n) % n) // s + m * ((e // (n * n)) // s))


@pytest.mark.parametrize("pressure", ["q1", "p1disc"])
def test_host_algebraic_setup_matches_structured_and_oracle(pressure):
    """The algebraic entry point fed with the cube's matrix and its box
    partition builds the structured algebraic-overlap problem exactly (local
    sets, interface entities, coarse columns); on an unstructured (Voronoi)
    partition it builds what the oracle's algebraic decomposition builds."""
    from oracle.decomposition import AlgebraicDecomposition
    from inputs import voronoi_partition
    n, m = 6, 3
    p = StokesProblem(n, pressure=pressure)
    A = p.A.tocsr()
    A.sort_indices()
    for part, structured in [(_box_partition(n, m), True), (voronoi_partition(n, 7, seed=4), False)]:
        subs = _repeated_map(p, part)
        s = G.Solver.algebraic(A.indptr, A.indices, A.data, p.dof_field, subs, null=p.dof_null, rhs=p.b,
                               host_only=True)
        sz = s.sizes()
        a = AlgebraicDecomposition(A, p.dof_field, subs, p.dof_null, 1)
        assert sz.n_free == p.n_free and sz.n_sub == a.n_sub
        assert sz.n_entities == a.n_ent and sz.n_coarse == a.n_coarse
        for i in range(a.n_sub):
            assert np.array_equal(s.local_indices(i), a.S[i])
        assert np.array_equal(s.host_rhs(), p.b)
        if structured:
            d = Decomposition(p, m, 1, local_dirichlet=False)
            assert a.n_coarse == d.n_coarse
            for i in range(d.n_sub):
                assert np.array_equal(a.S[i], d.S[i]) and np.array_equal(a.I[i], d.I[i])
        s.close()


def test_host_algebraic_rejections():
    p = StokesProblem(2)
    A = p.A.tocsr()
    A.sort_indices()
    subs = _repeated_map(p, _box_partition(2, 2))
    bad = p.dof_field.copy()
    bad[[0, -1]] = bad[[-1, 0]]                      # a pressure DOF before velocity DOFs
    with pytest.raises(G.GdswError):
        G.Solver.algebraic(A.indptr, A.indices, A.data, bad, subs, host_only=True)
    with pytest.raises(G.GdswError):
        G.Solver.algebraic(A.indptr, A.indices, A.data, p.dof_field, [[]] + subs[1:], host_only=True)


def test_host_algebraic_rejects_entry_across_subdomains():
    """A nonzero whose DOFs share no subdomain is refused at the input check
    (A_0 is assembled from the nonzeros each subdomain owns, which needs a
    subdomain holding both DOFs)."""
    p = StokesProblem(2)
    A = p.A.tocsr()
    A.sort_indices()
    subs = [list(s) for s in _repeated_map(p, _box_partition(2, 2))]
    r = next(d for d in range(p.n_free) if len(subs[d]) == 1)
    c = next(int(k) for k in A.indices[A.indptr[r]:A.indptr[r + 1]] if k != r)
    subs[c] = [next(k for k in range(8) if k not in subs[r])]
    with pytest.raises(G.GdswError, match="share no subdomain"):
        G.Solver.algebraic(A.indptr, A.indices, A.data, p.dof_field, subs, host_only=True)
