"""Pins of the Q2/Q1 Stokes discretisation (Section 2, eq. 2.1)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.stokes import (StokesProblem, dof_count_q2p1disc, dof_count_q2q1,
                           element_matrices)


def test_dof_counts_closed_form():
    for n in (1, 2, 3, 4):
        assert StokesProblem(n).n_full == dof_count_q2q1(n)
    # the four configured meshes
    assert [dof_count_q2q1(n) for n in (4, 16, 24, 32)] == [2312, 112724, 368572, 859812]
    assert dof_count_q2q1(4) - 125 == 2187
    # Tables 1-2, #dof column (Q2 / P1-discontinuous)
    assert [dof_count_q2p1disc(n) for n in (32, 64, 128)] == [954947, 7488643, 59312387]


def test_p1disc_dof_counts_and_structure():
    for n in (1, 2, 3):
        p = StokesProblem(n, pressure="p1disc")
        assert p.n_full == dof_count_q2p1disc(n) and p.n_p == 4 * n ** 3
        assert abs(p.A - p.A.T).max() < 1e-15
    p = StokesProblem(2, pressure="p1disc")
    # each element's four pressure DOFs couple only to the 81 velocity DOFs of that element
    Bp = p.A[p.n_u:, :p.n_u].tocsr()
    rows_e0 = Bp[0:4]
    assert rows_e0.count_nonzero() <= 4 * 81
    assert p.A[p.n_u:, p.n_u:].count_nonzero() == 0
    assert np.array_equal(p.dof_null[p.n_u:], np.tile([1.0, 0, 0, 0], 8))


def test_p1disc_divergence_block_tensor_closed_form():
    """B[q, a, c] = -h^2 int psi_q d(phi_a)/dxi_c with psi = 1, 2x-1, 2y-1,
    2z-1, from hand-computed 1-D integrals: int L_a = (1/6, 2/3, 1/6),
    int L_a' = (-1, 0, 1), int (2x-1) L_a = (-1/6, 0, 1/6),
    int (2x-1) L_a' = (2/3, -4/3, 2/3)."""
    h, mu = 0.5, 1.0
    I = np.array([1 / 6, 2 / 3, 1 / 6])
    D = np.array([-1.0, 0.0, 1.0])
    J = np.array([-1 / 6, 0.0, 1 / 6])
    JD = np.array([2 / 3, -4 / 3, 2 / 3])
    k3 = lambda z, y, x: np.kron(z, np.kron(y, x))
    ref = np.zeros((4, 27, 3))
    ref[0, :, 0], ref[0, :, 1], ref[0, :, 2] = k3(I, I, D), k3(I, D, I), k3(D, I, I)
    ref[1, :, 0], ref[1, :, 1], ref[1, :, 2] = k3(I, I, JD), k3(I, D, J), k3(D, I, J)
    ref[2, :, 0], ref[2, :, 1], ref[2, :, 2] = k3(I, J, D), k3(I, JD, I), k3(D, J, I)
    ref[3, :, 0], ref[3, :, 1], ref[3, :, 2] = k3(J, I, D), k3(J, D, I), k3(JD, I, I)
    ref *= -h * h
    _, B = element_matrices(h, mu, pressure="p1disc")
    assert np.allclose(B, ref, rtol=0, atol=1e-14)


def test_free_dofs_and_symmetry():
    p = StokesProblem(4)
    # Dirichlet nodes: x = 0 face and the four walls; interior: a in 1..8, b, c in 1..7
    assert p.n_u == 3 * 8 * 7 * 7
    assert p.n_free == 1301
    assert abs(p.A - p.A.T).max() < 1e-15
    # velocity block first, pressure block has no diagonal
    assert np.all(p.dof_field[:p.n_u] < 3) and np.all(p.dof_field[p.n_u:] == 3)
    App = p.A[p.n_u:, p.n_u:]
    assert App.count_nonzero() == 0


def _exact_1d():
    """Textbook 1-D Q2/Q1 element integrals on [0, 1] (exact rationals)."""
    M = np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) / 30.0      # int L_a L_b
    S = np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 3.0      # int L_a' L_b'
    G = np.array([[1 / 6, 1 / 3, 0.0], [0.0, 1 / 3, 1 / 6]])        # int N_q L_a
    C = np.array([[-5 / 6, 2 / 3, 1 / 6], [-1 / 6, -2 / 3, 5 / 6]])  # int N_q L_a'
    return M, S, G, C


@pytest.mark.parametrize("h,mu", [(1.0, 1.0), (0.25, 0.37)])
def test_element_matrices_tensor_closed_form(h, mu):
    M, S, G, C = _exact_1d()
    k3 = lambda z, y, x: np.kron(z, np.kron(y, x))  # index a = ax + 3 (ay + 3 az)
    K_ref = mu * h * (k3(M, M, S) + k3(M, S, M) + k3(S, M, M))
    B_ref = np.zeros((8, 27, 3))
    B_ref[:, :, 0] = -h * h * k3(G, G, C)
    B_ref[:, :, 1] = -h * h * k3(G, C, G)
    B_ref[:, :, 2] = -h * h * k3(C, G, G)
    K, B = element_matrices(h, mu)
    assert np.allclose(K, K_ref, rtol=0, atol=1e-14 * np.abs(K_ref).max())
    assert np.allclose(B, B_ref, rtol=0, atol=1e-14 * np.abs(B_ref).max())


@pytest.mark.parametrize("pressure", ["q1", "p1disc"])
@pytest.mark.parametrize("n", [2, 3, 4])
def test_manufactured_poiseuille_is_exact(n, pressure):
    """With f = (2 mu c [y(1-y) + z(1-z)], 0, 0) the quadratic profile and p = 0
    solve the continuous problem and lie in Q2/Q1 (and Q2/P1disc), so the
    discrete solution is their nodal interpolant."""
    p = StokesProblem(n, viscosity=0.7, inflow=16.0, manufactured=1, pressure=pressure)
    x = spla.spsolve(p.A.tocsc(), p.b)
    c = p.c
    ref = p.interpolant(lambda X, Y, Z: np.stack([c * Y * (1 - Y) * Z * (1 - Z), 0 * X, 0 * X]),
                        lambda X, Y, Z: 0 * X)
    assert np.abs(p.expand(x) - ref).max() < 1e-10


@pytest.mark.parametrize("pressure", ["q1", "p1disc"])
@pytest.mark.parametrize("n", [2, 3])
def test_linear_pressure_flow_is_exact(n, pressure):
    """u = (c y(1-y), 0, 0), p = 2 mu c (1 - x) solves Stokes with f = 0 and the
    do-nothing condition at x = 1; Dirichlet data from u on x = 0 and the walls."""
    mu, c = 1.3, 2.0
    u = lambda X, Y, Z: np.stack([c * Y * (1 - Y) + 0 * X, 0 * X, 0 * X])
    pfun = lambda X, Y, Z: 2 * mu * c * (1 - X)
    p = StokesProblem(n, viscosity=mu, inflow=c, dirichlet=u, pressure=pressure)
    x = spla.spsolve(p.A.tocsc(), p.b)
    assert np.abs(p.expand(x) - p.interpolant(u, pfun)).max() < 1e-10


def test_plain_poiseuille_is_not_exact():
    """Without the body force the product profile is not a Stokes solution."""
    p = StokesProblem(3)
    x = spla.spsolve(p.A.tocsc(), p.b)
    c = p.c
    ref = p.interpolant(lambda X, Y, Z: np.stack([c * Y * (1 - Y) * Z * (1 - Z), 0 * X, 0 * X]),
                        lambda X, Y, Z: 0 * X)
    assert np.abs(p.expand(x) - ref).max() > 1e-3
