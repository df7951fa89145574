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


@pytest.mark.parametrize("layer", [False, True])
def test_dense_three_level_operator(layer):
    """eq. (2.5) written out with dense inverses on n = 4, m = 4, group 2
    (64 subdomains, 8 subregions):

        B3 = sum_i R_i^T A_i^-1 R_i
             + Phi [ sum_j R_j^T (R_j A_0 R_j^T)^-1 R_j
                     + Phi3 (Phi3^T A_0 Phi3)^-1 Phi3^T ] Phi^T,

    with the interior rows of Phi3 recomputed here from eq. (2.4) applied to
    A_0 (the level-3 interface rows are its 0/1 partition of unity).  The
    level-3 term is checked to matter, so dropping or rescaling it fails."""
    p = StokesProblem(4)
    d = Decomposition(p, 4, 1)
    M = ThreeLevelGDSW(p.A, d, 2, level2_layer=layer)
    A = p.A.toarray()
    n = p.n_free
    Phi = M.Phi.toarray()
    A0 = Phi.T @ A @ Phi
    assert np.abs(A0 - M.A0).max() < 1e-12 * np.abs(A0).max()
    gam = np.array([c for c, r in enumerate(M.coarse_regions) if len(r) >= 2])
    P3 = np.zeros_like(M.Phi3)
    P3[gam] = M.Phi3[gam]
    assert set(np.unique(P3[gam])) <= {0.0, 1.0}
    for Ij in M.I2:
        if Ij.size:
            P3[Ij] = -np.linalg.solve(A0[np.ix_(Ij, Ij)], A0[Ij] @ P3)
    assert np.abs(P3 - M.Phi3).max() < 1e-12 * np.abs(P3).max()
    B = np.zeros((n, n))
    for Si in d.S:
        B[np.ix_(Si, Si)] += np.linalg.inv(A[np.ix_(Si, Si)])
    C2 = np.zeros_like(A0)
    for Sj in M.S2:
        C2[np.ix_(Sj, Sj)] += np.linalg.inv(A0[np.ix_(Sj, Sj)])
    C3 = P3 @ np.linalg.inv(P3.T @ A0 @ P3) @ P3.T
    B += Phi @ (C2 + C3) @ Phi.T
    X = np.random.default_rng(8).standard_normal((n, 3))
    Z = M(X)
    ref = B @ X
    scale = np.abs(ref).max()
    assert np.abs(Z - ref).max() < 1e-13 * scale
    lvl3 = Phi @ C3 @ Phi.T @ X
    assert np.abs(lvl3).max() > 1e-3 * scale
