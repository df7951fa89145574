"""Pins of the three-level preconditioner (eq. 2.5)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.decomposition import Decomposition
from oracle.fgmres import fgmres
from oracle.gdsw import TwoLevelGDSW
from oracle.stokes import StokesProblem
from oracle.threelevel import ThreeLevelGDSW


@pytest.fixture(scope="module")
def n8m4():
    p = StokesProblem(8)
    d = Decomposition(p, 4, 1)
    return p, d, ThreeLevelGDSW(p.A, d, 2)


def test_level3_dimensions_and_sets(n8m4):
    p, d, M = n8m4
    assert M.n_subregions == 8
    assert M.n_ent3 == 19 and M.n_coarse3 == 76      # full GDSW on a 2^3 subregion grid
    # interior sets disjoint; level-3 interface = coarse DOFs in >= 2 subregions
    allI = np.concatenate(M.I2)
    assert np.unique(allI).size == allI.size
    n_gam = sum(1 for r in M.coarse_regions if len(r) >= 2)
    assert allI.size + n_gam == d.n_coarse
    for j in range(M.n_subregions):
        assert np.all(np.isin(M.I2[j], M.S2[j]))


def test_level3_basis_properties(n8m4):
    p, d, M = n8m4
    Phi3 = M.Phi3
    gam = np.array([c for c, r in enumerate(M.coarse_regions) if len(r) >= 2])
    # partition of unity per field on the level-3 interface
    for f in range(4):
        cols = [k for k in range(M.n_coarse3) if np.any(Phi3[gam[d.coarse_field[gam] == f], k] == 1)]
        rows = gam[d.coarse_field[gam] == f]
        assert np.array_equal(Phi3[np.ix_(rows, cols)].sum(1), np.ones(rows.size))
    # energy-minimising on every subregion interior
    R = M.A0 @ Phi3
    for Ij in M.I2:
        assert np.abs(R[Ij]).max() < 1e-11 * np.abs(M.A0).max() * max(1, np.abs(Phi3).max())
    assert np.abs(M.A03 - M.A03.T).max() < 1e-11 * np.abs(M.A03).max()


def test_one_subregion_reduces_to_two_level():
    """group = m: one subregion holds every coarse DOF, no level-3 space, and the
    level-2 local matrix is A_0 itself, so eq. (2.5) equals eq. (2.2)."""
    p = StokesProblem(4)
    d = Decomposition(p, 2, 1)
    M3 = ThreeLevelGDSW(p.A, d, 2)
    M2 = TwoLevelGDSW(p.A, d)
    assert M3.n_coarse3 == 0 and M3.S2[0].size == d.n_coarse
    r = np.random.default_rng(4).standard_normal(p.n_free)
    assert np.abs(M3(r) - M2(r)).max() < 1e-11 * np.abs(M2(r)).max()


def test_three_level_fgmres_converges_to_direct(n8m4):
    p, d, M = n8m4
    xs = sla.solve(p.A.toarray(), p.b)
    x, it, rel, trel = fgmres(lambda v: p.A @ v, M, p.b, rtol=1e-12)
    assert trel <= 1e-12
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-9
    r = np.random.default_rng(5).standard_normal(p.n_free)
    s = np.random.default_rng(6).standard_normal(p.n_free)
    assert abs(M(r) @ s - r @ M(s)) < 1e-10 * abs(M(r) @ s)
