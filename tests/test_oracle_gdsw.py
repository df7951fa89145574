"""Pins of the two-level monolithic GDSW preconditioner (eqs. 2.2-2.4)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle.decomposition import Decomposition
from oracle.fgmres import fgmres
from oracle.gdsw import TwoLevelGDSW
from oracle.stokes import StokesProblem


@pytest.fixture(scope="module")
def n6m3():
    p = StokesProblem(6, viscosity=0.8)
    d = Decomposition(p, 3, 1)
    return p, d, TwoLevelGDSW(p.A, d)


def _touches(d, i, axis, side):
    m = d.m
    ijk = (i % m, (i // m) % m, i // (m * m))
    return ijk[axis] == (0 if side == 0 else m - 1)


def test_phi_gamma_partition_of_unity(n6m3):
    p, d, M = n6m3
    Phi = M.Phi.tocsr()
    for f in range(4):
        cols = np.nonzero(d.coarse_field == f)[0]
        rows = d.gamma[d.gamma_field == f]
        s = np.asarray(Phi[rows][:, cols].sum(axis=1)).ravel()
        assert np.array_equal(s, np.ones(rows.size))          # exact
        other = d.gamma[d.gamma_field != f]
        assert Phi[other][:, cols].count_nonzero() == 0


def test_extension_reproduces_constants(n6m3):
    p, d, M = n6m3
    Phi = M.Phi.tocsr()
    for f in range(4):
        cols = np.nonzero(d.coarse_field == f)[0]
        v = np.asarray(Phi[:, cols].sum(axis=1)).ravel()
        for i in range(d.n_sub):
            Ii = d.I[i]
            target = (p.dof_field[Ii] == f).astype(float)
            if f < 3:
                # velocity translation: subdomain must not touch Dirichlet faces
                ok = not (_touches(d, i, 0, 0) or any(_touches(d, i, a, s) for a in (1, 2) for s in (0, 1)))
            else:
                ok = not _touches(d, i, 0, 1)   # pressure: away from the outflow
            err = np.abs(v[Ii] - target).max()
            if ok:
                assert err < 1e-12, (f, i, err)
    # the centre subdomain reproduces all four null-space vectors; a boundary one
    # does not reproduce u_x (check the test has teeth)
    cols = np.nonzero(d.coarse_field == 0)[0]
    v = np.asarray(Phi[:, cols].sum(axis=1)).ravel()
    I0 = d.I[0]
    assert np.abs(v[I0] - (p.dof_field[I0] == 0)).max() > 1e-3


def test_energy_minimising_extension_and_symmetry(n6m3):
    p, d, M = n6m3
    A = p.A.tocsr()
    R = A @ M.Phi
    for i in range(d.n_sub):
        Ii = d.I[i]
        res = np.abs(R[Ii].toarray()).max()
        scale = np.abs(A[Ii]).max() * np.abs(M.Phi).max()
        assert res < 1e-12 * scale
    assert np.abs(M.A0 - M.A0.T).max() < 1e-12 * np.abs(M.A0).max()
    # off-diagonal blocks Phi_{I,u0,p}, Phi_{I,p0,u} are present (monolithic)
    Phi = M.Phi.tocsr()
    vel_cols = np.nonzero(d.coarse_field < 3)[0]
    p_rows = np.nonzero(p.dof_field == 3)[0]
    assert np.abs(Phi[p_rows][:, vel_cols]).max() > 1e-6


def test_preconditioner_symmetric_and_dense_brute_force():
    p = StokesProblem(4)
    d = Decomposition(p, 2, 1)
    M = TwoLevelGDSW(p.A, d)
    n = p.n_free
    A = p.A.toarray()
    # explicit eq. (2.2) with dense inverses
    Md = np.zeros((n, n))
    for Si in d.S:
        Md[np.ix_(Si, Si)] += np.linalg.inv(A[np.ix_(Si, Si)])
    Phi = M.Phi.toarray()
    Md += Phi @ np.linalg.inv(Phi.T @ A @ Phi) @ Phi.T
    rng = np.random.default_rng(0)
    X = rng.standard_normal((n, 3))
    Z = M(X)
    assert np.abs(Z - Md @ X).max() < 1e-11 * np.abs(Z).max()
    x, y = X[:, 0], X[:, 1]
    assert abs(M(x) @ y - x @ M(y)) < 1e-11 * abs(M(x) @ y)


def test_one_subdomain_is_exact_inverse():
    p = StokesProblem(3)
    d = Decomposition(p, 1, 1)
    M = TwoLevelGDSW(p.A, d)
    assert d.n_coarse == 0 and len(d.S) == 1 and d.S[0].size == p.n_free
    r = np.random.default_rng(1).standard_normal(p.n_free)
    assert np.allclose(M(r), spla.spsolve(p.A.tocsc(), r), rtol=1e-11, atol=1e-12)
    x, it, rel, trel = fgmres(lambda v: p.A @ v, M, p.b, rtol=1e-10)
    assert it == 1 and trel <= 1e-10


def test_full_overlap_closed_form():
    """m = 2 with overlap >= n/2: every S_i is the whole domain, so
    B_GDSW = Phi A_0^{-1} Phi^T + 8 A^{-1}."""
    p = StokesProblem(4)
    d = Decomposition(p, 2, 2)
    assert all(S.size == p.n_free for S in d.S)
    M = TwoLevelGDSW(p.A, d)
    A = p.A.toarray()
    Phi = M.Phi.toarray()
    ref = Phi @ np.linalg.solve(Phi.T @ A @ Phi, Phi.T) + 8 * np.linalg.inv(A)
    r = np.random.default_rng(2).standard_normal(p.n_free)
    assert np.abs(M(r) - ref @ r).max() < 1e-10 * np.abs(ref @ r).max()


def test_fgmres_matches_direct_solution():
    p = StokesProblem(4)
    d = Decomposition(p, 2, 1)
    M = TwoLevelGDSW(p.A, d)
    xs = sla.solve(p.A.toarray(), p.b)
    x, it, rel, trel = fgmres(lambda v: p.A @ v, M, p.b, rtol=1e-13)
    assert trel <= 1e-13
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-10
    # paper tolerance
    x8, it8, rel8, trel8 = fgmres(lambda v: p.A @ v, M, p.b, rtol=1e-8)
    assert rel8 <= 1e-8 and trel8 <= 1e-8 and it8 < it


def test_linearity_in_inflow_and_viscosity_scaling():
    """x(c) = c x(1); for f = 0, u(mu) = u(1) and p(mu) = mu p(1)."""
    res = {}
    for mu, c in [(1.0, 1.0), (1.0, 1.7), (3.0, 1.0)]:
        p = StokesProblem(4, viscosity=mu, inflow=c)
        d = Decomposition(p, 2, 1)
        M = TwoLevelGDSW(p.A, d)
        x, it, _, _ = fgmres(lambda v: p.A @ v, M, p.b, rtol=1e-12)
        res[(mu, c)] = (x, it, p.n_u)
    x1, it1, nu = res[(1.0, 1.0)]
    xc, itc, _ = res[(1.0, 1.7)]
    assert itc == it1
    assert np.abs(xc - 1.7 * x1).max() < 1e-9 * np.abs(x1).max() * 1.7
    xm, _, _ = res[(3.0, 1.0)]
    assert np.abs(xm[:nu] - x1[:nu]).max() < 1e-9 * np.abs(x1[:nu]).max()
    assert np.abs(xm[nu:] - 3.0 * x1[nu:]).max() < 1e-9 * 3 * np.abs(x1[nu:]).max()


def _velocity_first(fields):
    fields = np.asarray(fields)
    return np.concatenate([np.nonzero(fields < 3)[0], np.nonzero(fields == 3)[0]])


def _lu_no_row_exchanges(M):
    """Doolittle elimination without row exchanges; raises on a zero pivot."""
    F = np.array(M, dtype=np.float64)
    n = F.shape[0]
    for k in range(n - 1):
        assert F[k, k] != 0.0, k
        F[k + 1:, k] /= F[k, k]
        F[k + 1:, k + 1:] -= np.outer(F[k + 1:, k], F[k, k + 1:])
    return np.tril(F, -1) + np.eye(n), np.triu(F)


def test_coarse_lu_without_pivoting_is_valid(n6m3):
    """The library factors and inverts without row exchanges.  That is valid
    for these saddle-point matrices: with velocity-type columns first, the
    velocity block of A_0 is SPD and its Schur complement negative definite,
    so every leading pivot block is nonsingular; L U reproduces A_0 and the
    solve agrees with LAPACK's pivoted solve (the oracle's) to cond(A_0) * eps."""
    p, d, M = n6m3
    order = _velocity_first(d.coarse_field)
    A0 = M.A0[np.ix_(order, order)]
    nv = int((d.coarse_field < 3).sum())
    K, Bt, C = A0[:nv, :nv], A0[:nv, nv:], A0[nv:, nv:]
    assert np.linalg.eigvalsh(0.5 * (K + K.T)).min() > 0
    S = C - Bt.T @ np.linalg.solve(K, Bt)
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).max() < 0
    L, U = _lu_no_row_exchanges(A0)
    assert np.abs(L @ U - A0).max() < 1e-12 * np.abs(A0).max()
    b = np.random.default_rng(7).standard_normal(d.n_coarse)
    y = np.empty_like(b)
    y[order] = sla.solve_triangular(U, sla.solve_triangular(L, b[order], lower=True, unit_diagonal=True))
    ref = M.coarse_solve(b)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < np.linalg.cond(M.A0) * 1e-14


# --- the paper's variant: Q2/P1disc, one pressure constant per subdomain, GDSW* ---

@pytest.fixture(scope="module")
def p6m3_disc():
    p = StokesProblem(6, viscosity=0.8, pressure="p1disc")
    d = Decomposition(p, 3, 1, local_dirichlet=False, coarse="gdsw*")
    return p, d, TwoLevelGDSW(p.A, d)


def test_p1disc_coarse_columns(p6m3_disc):
    """Velocity interface: Phi_Gamma is a 0/1 partition of unity per field;
    pressure: one column per subdomain whose sum is the pressure null vector
    (1 on every element's constant function, 0 on the linear ones), exactly;
    the velocity and pressure columns do not mix (off-diagonal blocks zero)."""
    p, d, M = p6m3_disc
    Phi = M.Phi.toarray()
    for f in range(3):
        rows = d.gamma[d.gamma_field == f]
        cols = np.nonzero(d.coarse_field == f)[0]
        assert np.array_equal(Phi[np.ix_(rows, cols)].sum(1), np.ones(rows.size))
    assert not np.any(d.gamma_field == 3)
    pc = np.nonzero(d.coarse_field == 3)[0]
    assert pc.size == d.n_sub
    assert np.array_equal(Phi[p.n_u:][:, pc].sum(1), p.dof_null[p.n_u:])
    assert np.all(Phi[:p.n_u][:, pc] == 0) and np.all(Phi[p.n_u:][:, d.coarse_field < 3] == 0)
    # each pressure column lives on its own subdomain's elements
    for i in range(d.n_sub):
        on = np.nonzero(Phi[:, pc[i]])[0]
        assert np.all(np.isin(on, d.box[i]))


def test_p1disc_velocity_extension_is_harmonic_and_reproduces_constants(p6m3_disc):
    """Velocity columns: K_II Phi_I + K_IGamma Phi_Gamma = 0 on every
    subdomain's interior velocity rows (the velocity block alone), and the
    translations are reproduced on the centre subdomain (no Dirichlet face);
    A_0 is symmetric and nonsingular."""
    p, d, M = p6m3_disc
    A = p.A.tocsr()
    Phi = M.Phi.tocsr()
    vcols = np.nonzero(d.coarse_field < 3)[0]
    R = (A[:p.n_u][:, :p.n_u] @ Phi[:p.n_u][:, vcols]).toarray()
    for i in range(d.n_sub):
        Iu = d.I[i][p.dof_field[d.I[i]] < 3]
        assert np.abs(R[Iu]).max() < 1e-12 * np.abs(A).max()
    Iu = d.I[13][p.dof_field[d.I[13]] < 3]
    for f in range(3):
        v = np.asarray(Phi[:, np.nonzero(d.coarse_field == f)[0]].sum(axis=1)).ravel()
        assert np.abs(v[Iu] - (p.dof_field[Iu] == f)).max() < 1e-12
    assert np.abs(M.A0 - M.A0.T).max() < 1e-12 * np.abs(M.A0).max()
    assert np.linalg.cond(M.A0) < 1e8


def test_p1disc_dense_brute_force():
    """eq. (2.2) written out with dense inverses on 4^3 / 2^3 (Q2/P1disc, GDSW*)."""
    p = StokesProblem(4, pressure="p1disc")
    d = Decomposition(p, 2, 1, local_dirichlet=False, coarse="gdsw*")
    M = TwoLevelGDSW(p.A, d)
    A = p.A.toarray()
    n = p.n_free
    Md = np.zeros((n, n))
    for Si in d.S:
        Md[np.ix_(Si, Si)] += np.linalg.inv(A[np.ix_(Si, Si)])
    Phi = M.Phi.toarray()
    Md += Phi @ np.linalg.inv(Phi.T @ A @ Phi) @ Phi.T
    X = np.random.default_rng(3).standard_normal((n, 3))
    Z = M(X)
    assert np.abs(Z - Md @ X).max() < 1e-11 * np.abs(Z).max()
    x = fgmres(lambda v: p.A @ v, M, p.b, rtol=1e-12)[0]
    xs = sla.solve(A, p.b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-9


def test_p1disc_needs_algebraic_overlap():
    """With Dirichlet velocity on the whole artificial boundary, an interior
    local problem's constant pressure is a null vector: refused."""
    p = StokesProblem(6, pressure="p1disc")
    with pytest.raises(ValueError):
        Decomposition(p, 3, 1, local_dirichlet=True)
    # the refused reading is indeed singular on the centre subdomain
    d = Decomposition(p, 3, 1, local_dirichlet=False)
    n = p.n
    abc = p.dof_node
    lo, hi = 2 * (2 * 1 - 1) + 1, 2 * (2 * 2 + 1) - 1   # grown box of subdomain (1,1,1), faces removed
    S = np.nonzero(np.all((abc >= lo) & (abc <= hi), axis=1))[0]
    Ai = p.A[S][:, S].toarray()
    e = np.zeros(S.size)
    e[(p.dof_field[S] == 3) & (p.dof_null[S] == 1)] = 1.0
    assert np.abs(Ai @ e).max() < 1e-12 * np.abs(Ai).max()
    assert d.n_sub == 27 and n == 6


@pytest.mark.parametrize("pressure", ["q1", "p1disc"])
def test_local_matrix_block_structure_and_block_solve(pressure):
    """The block local solve's premise and identity, on the oracle's own local
    matrices: the velocity block of A_i is I_3 (x) L_i (components uncoupled,
    the same scalar matrix for each), and with S = B K^-1 B^T the solution of
    A_i [u; p] = [f; g] is U1 = L^-1 F, p = S^-1 (B U1 - g), u = U1 - L^-1 B^T p
    (equal to the direct solve to 1e-12)."""
    p = StokesProblem(6, pressure=pressure)
    d = Decomposition(p, 3, 1, local_dirichlet=pressure == "q1")
    for i in (0, 13):
        S = d.S[i]
        Ai = p.A[S][:, S].toarray()
        fld = p.dof_field[S]
        vel = np.nonzero(fld < 3)[0]
        prs = np.nonzero(fld == 3)[0]
        K = Ai[np.ix_(vel, vel)]
        L = K[0::3, 0::3]
        # interleaved numbering 3 node + component; equal up to the assembly's rounding
        assert np.abs(K - np.kron(L, np.eye(3))).max() <= 1e-14 * np.abs(K).max()
        B = Ai[np.ix_(prs, vel)]
        rng = np.random.default_rng(i)
        f, g = rng.standard_normal(vel.size), rng.standard_normal(prs.size)
        Li = np.linalg.inv(L)
        F = f.reshape(-1, 3)                                  # row = node, column = component
        U1 = Li @ F
        Sc = B @ np.kron(Li, np.eye(3)) @ B.T
        pp = np.linalg.solve(Sc, B @ U1.ravel() - g)
        u = U1.ravel() - (Li @ (B.T @ pp).reshape(-1, 3)).ravel()
        ref = np.linalg.solve(Ai, np.concatenate([f, g]))
        got = np.empty_like(ref)
        got[vel], got[prs] = u, pp
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
