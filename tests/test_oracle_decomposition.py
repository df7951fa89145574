"""Pins of the decomposition, overlap and interface entities (Section 2.1)."""
import numpy as np
import pytest

from oracle.counts import (full_gdsw_closed_form, full_gdsw_count,
                           paper_three_level_coarse_dim, paper_two_level_coarse_dim)
from oracle.decomposition import Decomposition
from oracle.stokes import StokesProblem


@pytest.mark.parametrize("m", [2, 3, 4])
def test_entity_counts_closed_form(m):
    p = StokesProblem(2 * m)
    d = Decomposition(p, m, 1)
    assert d.n_ent == full_gdsw_closed_form(m) == full_gdsw_count(m)
    kinds = [d.entity_kind(e) for e in range(d.n_ent)]
    assert kinds.count("face") == 3 * (m - 1) * m * m
    assert kinds.count("edge") == 3 * m * (m - 1) ** 2
    assert kinds.count("vertex") == (m - 1) ** 3
    # Q2/Q1: every entity carries all four fields
    assert d.n_coarse == 4 * d.n_ent
    assert [full_gdsw_closed_form(k) * 4 for k in (2, 4, 6, 8)] == [76, 1116, 4460, 11452]


def test_paper_table_coarse_dimensions():
    """Table 1 (GDSW*, 2nd level) and Table 2 (3rd level) coarse-DOF columns."""
    assert paper_two_level_coarse_dim(8) == 5573
    assert paper_two_level_coarse_dim(16) == 48781
    assert paper_two_level_coarse_dim(32) == 407837
    assert paper_three_level_coarse_dim(8, (2, 2, 2)) == 65
    assert paper_three_level_coarse_dim(16, (4, 4, 4)) == 901
    assert paper_three_level_coarse_dim(32, (8, 8, 4)) == 4213


def test_partition_and_interface():
    p = StokesProblem(6)
    d = Decomposition(p, 3, 1)
    allI = np.concatenate(d.I)
    assert np.unique(allI).size == allI.size                   # I_i disjoint
    assert np.intersect1d(allI, d.gamma).size == 0
    assert allI.size + d.gamma.size == p.n_free                 # I and Gamma cover
    # every Gamma DOF sits in >= 2 closed boxes, every I DOF in exactly one
    cnt = np.zeros(p.n_free, dtype=int)
    for B in d.box:
        cnt[B] += 1
    assert np.all(cnt[d.gamma] >= 2) and np.all(cnt[allI] == 1)


def test_overlap_is_one_graph_layer():
    """Algebraic reading: S_i (closed box grown by one element) = closed box
    plus its neighbours in the sparsity graph of A."""
    p = StokesProblem(6)
    d = Decomposition(p, 3, 1, local_dirichlet=False)
    A = p.A.tocsr()
    for i in (0, 4, 13, 26):
        box = d.box[i]
        nb = np.unique(A[box].indices)
        assert np.array_equal(np.union1d(box, nb), d.S[i])


def test_local_sizes():
    p = StokesProblem(4)
    d = Decomposition(p, 2, 1, local_dirichlet=False)
    sz = d.local_sizes()
    assert sz.min() == 712 and sz.max() == 820
    # 16^3 mesh, 4^3 subdomains: corner box grows inward only, interior by one layer
    p = StokesProblem(16)
    dd = Decomposition(p, 4, 1)                    # Dirichlet reading (default)
    szd = dd.local_sizes()
    assert szd.min() == 3 * 9 ** 3 + 5 ** 3 == 2312 and szd.max() == 4118
    d = Decomposition(p, 4, 1, local_dirichlet=False)
    sz = d.local_sizes()
    assert sz.max() == 3 * 13 ** 3 + 7 ** 3 == 6934
    assert sz.min() == 3 * 10 ** 3 + 6 ** 3 == 3216
    assert int((sz.astype(np.int64) ** 2).sum()) * 8 == 13037206048
    isz = [len(I) for I in d.I]
    assert min(isz) == 1056 and max(isz) == 1240


def test_local_dirichlet_sets_and_conditioning():
    """Dirichlet reading of the local problems: the nodes on the faces of the
    grown box inside the cube are left out for u and p.  Sizes follow from the
    node counts (interior 16^3 subdomain: 11 Q2 and 5 Q1 nodes per axis), and
    the local matrix loses the nearly singular pressure-constant mode of the
    algebraic reading."""
    p = StokesProblem(16)
    d = Decomposition(p, 4, 1, local_dirichlet=True)
    sz = d.local_sizes()
    assert sz.max() == 3 * 11 ** 3 + 5 ** 3 == 4118
    assert int((sz.astype(np.int64) ** 2).sum()) * 8 == 5372506496
    from oracle.gdsw import TwoLevelGDSW
    p8 = StokesProblem(8)
    conds = {}
    for ld in (False, True):
        dd = Decomposition(p8, 4, 1, local_dirichlet=ld)
        i = 21                                    # an interior subdomain
        Ai = p8.A[dd.S[i]][:, dd.S[i]].toarray()
        s = np.linalg.svd(Ai, compute_uv=False)
        conds[ld] = s[0] / s[-1]
    assert conds[True] * 10 < conds[False]


@pytest.mark.parametrize("m", [2, 3, 4])
def test_gdsw_star_counts_brute_force(m):
    """GDSW* (vertices grouped with their adjacent edges) on m^3 subdomains
    with the P1disc pressure: enumerated coarse dimension equals the closed
    form 3 [3 (m-1) m^2 + (m-1)^3] + m^3 behind Tables 1-2; every edge class
    is absorbed, entities stay disjoint and each groups one vertex with at
    most 6 edges (one per direction and side)."""
    n = 2 * m
    p = StokesProblem(n, pressure="p1disc")
    d = Decomposition(p, m, 1, local_dirichlet=False, coarse="gdsw*")
    assert d.n_coarse == 3 * (3 * (m - 1) * m * m + (m - 1) ** 3) + m ** 3
    kinds = [d.entity_kind(e) for e in range(d.n_ent)]
    assert kinds.count("edge") == 0
    assert kinds.count("vertex") == (m - 1) ** 3 and kinds.count("face") == 3 * (m - 1) * m * m
    full = Decomposition(p, m, 1, local_dirichlet=False, coarse="gdsw")
    # the grouped classes are unions of the full space's classes
    for e in range(d.n_ent):
        members = np.unique(d.gamma[d.gamma_entity == e])
        fe = np.unique(full.gamma_entity[np.isin(full.gamma, members)])
        assert np.array_equal(np.unique(full.gamma[np.isin(full.gamma_entity, fe)]), members)
        if kinds[e] == "vertex":
            assert 1 <= fe.size <= 7
