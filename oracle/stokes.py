"""Q2/Q1 discretisation of the Stokes problem on the unit cube (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows Section 2 of the paper: find u in V_g, p in Q with

    mu * int grad u : grad v  -  int div v p  = int f . v     for all v in V_0
         -  int div u q                      = 0              for all q in Q_0

u = g on the Dirichlet boundary, du/dn - p n = 0 on the outflow.  The
discrete system is eq. (2.1), [[A, B^T], [B, 0]] [u; p] = [F; 0].

Readings where the paper is silent (all pinned by tests):

* Q1 continuous pressure instead of the paper's P1-discontinuous one (the
  configured DOF counts fix Q2/Q1).
* Unit cube, n^3 affine hexahedra, 3-point Gauss rule per axis (exact for
  every integrand here).
* Dirichlet velocity on x = 0 (inflow) and y, z in {0, 1} (walls); outflow
  x = 1 is natural.  Every pressure DOF is free.
* Dirichlet DOFs are eliminated symmetrically; the solve runs on free DOFs:
  all free velocity DOFs first (Q2 nodes lexicographic with x fastest, then
  component), then every pressure DOF (Q1 nodes lexicographic).

The paper's own pair (Section 2 and the last paragraph of Section 3), Q2
velocity with P1-discontinuous pressure, is built with ``pressure="p1disc"``:
four pressure DOFs per hexahedron, the basis 1, 2 xi - 1, 2 eta - 1,
2 zeta - 1 in the element's reference coordinates (any basis of the linear
functions spans the same space; this one holds the constant as its first
function), numbered 4 e + k after the velocity DOFs, each attached to its
element's centre node for the decomposition.

Pins: closed-form DOF counts (both pairs); exact recovery of the quadratic
Poiseuille profile with the manufactured body force, and of a flow with a
linear pressure, for both pairs (``tests/test_oracle_stokes.py``).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# --- 1-D reference shape functions on [0, 1] -------------------------------
# Q2: Lagrange polynomials through 0, 1/2, 1.  Q1: through 0, 1.


def q2_1d(x):
    x = np.asarray(x, dtype=np.float64)
    return np.stack([2.0 * (x - 0.5) * (x - 1.0),
                     4.0 * x * (1.0 - x),
                     2.0 * x * (x - 0.5)])


def dq2_1d(x):
    x = np.asarray(x, dtype=np.float64)
    return np.stack([4.0 * x - 3.0, 4.0 - 8.0 * x, 4.0 * x - 1.0])


def q1_1d(x):
    x = np.asarray(x, dtype=np.float64)
    return np.stack([1.0 - x, x])


def gauss3():
    """3-point Gauss-Legendre rule mapped to [0, 1]."""
    t = np.sqrt(3.0 / 5.0)
    pts = 0.5 + 0.5 * np.array([-t, 0.0, t])
    wts = np.array([5.0, 8.0, 5.0]) / 18.0
    return pts, wts


def reference_element(pressure="q1"):
    """Tabulate the 27 Q2 and the pressure shape functions at the 27
    quadrature points of the reference cube.

    Local node index a = ax + 3*(ay + 3*az) for Q2, q = qx + 2*(qy + 2*qz) for
    Q1; for P1disc the four functions 1, 2x-1, 2y-1, 2z-1.
    Returns (points[27,3], weights[27], phi[27,27], dphi[27,27,3], psi[27,np]),
    rows indexed by quadrature point.
    """
    x, w = gauss3()
    P, W, phi, dphi, psi = [], [], [], [], []
    for kz in range(3):
        for ky in range(3):
            for kx in range(3):
                xi = np.array([x[kx], x[ky], x[kz]])
                P.append(xi)
                W.append(w[kx] * w[ky] * w[kz])
                L = [q2_1d(xi[d]) for d in range(3)]
                dL = [dq2_1d(xi[d]) for d in range(3)]
                N = [q1_1d(xi[d]) for d in range(3)]
                ph, dph = [], []
                for az in range(3):
                    for ay in range(3):
                        for ax in range(3):
                            ph.append(L[0][ax] * L[1][ay] * L[2][az])
                            dph.append([dL[0][ax] * L[1][ay] * L[2][az],
                                        L[0][ax] * dL[1][ay] * L[2][az],
                                        L[0][ax] * L[1][ay] * dL[2][az]])
                ps = []
                if pressure == "p1disc":
                    ps = [1.0, 2.0 * xi[0] - 1.0, 2.0 * xi[1] - 1.0, 2.0 * xi[2] - 1.0]
                else:
                    for qz in range(2):
                        for qy in range(2):
                            for qx in range(2):
                                ps.append(N[0][qx] * N[1][qy] * N[2][qz])
                phi.append(ph)
                dphi.append(dph)
                psi.append(ps)
    return (np.array(P), np.array(W), np.array(phi), np.array(dphi),
            np.array(psi))


def element_matrices(h, mu, pressure="q1"):
    """Element blocks of eq. (2.1) on a cube of edge h.

    K[a, b]       = mu * int grad phi_a . grad phi_b           (27 x 27, per component)
    B[q, a, c]    = - int psi_q d(phi_a)/dx_c                  (np x 27 x 3; np = 8 or 4)
    """
    _, W, _, dphi, psi = reference_element(pressure)
    # grad in physical coordinates = grad_ref / h, dx = h^3 dxi
    K = mu * h * np.einsum("q,qad,qbd->ab", W, dphi, dphi)
    B = -(h * h) * np.einsum("q,qp,qac->pac", W, psi, dphi)
    return K, B


class StokesProblem:
    """Assembled free-DOF saddle-point system of eq. (2.1) for one workload.

    Attributes
    ----------
    A : scipy.sparse.csr_matrix, free x free, symmetric
    b : right-hand side on free DOFs, with the Dirichlet data lifted
    n_u, n_p : numbers of free velocity and pressure DOFs
    dof_node : Q2 node coordinates (a, b, c), in units of h/2, of each free DOF
    dof_field : 0, 1, 2 for u_x, u_y, u_z and 3 for p
    """

    def __init__(self, n, viscosity=1.0, inflow=16.0, manufactured=0,
                 dirichlet=None, force=None, chunk=2048, pressure="q1"):
        if pressure not in ("q1", "p1disc"):
            raise ValueError("pressure must be 'q1' or 'p1disc'")
        self.pressure = pressure
        self.n = n
        self.mu = float(viscosity)
        self.c = float(inflow)
        self.h = 1.0 / n
        N2 = 2 * n + 1
        self.n_q2 = N2 ** 3
        self.n_q1 = (n + 1) ** 3
        disc = pressure == "p1disc"
        self.n_pdof = 4 * n ** 3 if disc else self.n_q1
        self.n_full = 3 * self.n_q2 + self.n_pdof

        if dirichlet is None:
            c = self.c

            def dirichlet(x, y, z):
                ux = np.where(np.isclose(x, 0.0), c * y * (1 - y) * z * (1 - z), 0.0)
                return np.stack([ux, np.zeros_like(x), np.zeros_like(x)])
        if force is None:
            c, mu = self.c, self.mu
            if manufactured:
                def force(x, y, z):
                    fx = 2.0 * mu * c * (y * (1 - y) + z * (1 - z))
                    return np.stack([fx, np.zeros_like(x), np.zeros_like(x)])
            else:
                force = None

        # ---- node bookkeeping ------------------------------------------------
        # Q2 node id = a + N2*(b + N2*c), x fastest
        ids = np.arange(self.n_q2)
        a = ids % N2
        b = (ids // N2) % N2
        cc = ids // (N2 * N2)
        self.q2_abc = np.stack([a, b, cc], 1)
        dir_node = (a == 0) | (b == 0) | (b == 2 * n) | (cc == 0) | (cc == 2 * n)
        self.q2_dirichlet = dir_node

        pid = np.arange(self.n_q1)
        pi = pid % (n + 1)
        pj = (pid // (n + 1)) % (n + 1)
        pk = pid // ((n + 1) ** 2)
        self.q1_ijk = np.stack([pi, pj, pk], 1)

        # full DOF numbering: velocity 3*node + comp, pressure 3*n_q2 + pid
        # (Q1) or 3*n_q2 + 4*e + k (P1disc, element e, basis function k)
        vel_dir = np.repeat(dir_node, 3)
        is_dir = np.concatenate([vel_dir, np.zeros(self.n_pdof, dtype=bool)])
        self.full_is_dirichlet = is_dir
        self.free = np.nonzero(~is_dir)[0]
        self.dir = np.nonzero(is_dir)[0]
        self.n_u = int((~vel_dir).sum())
        self.n_p = self.n_pdof
        self.n_free = self.free.size

        # per free DOF: node coordinates in half-element units and field;
        # a P1disc pressure DOF sits at its element's centre node
        if disc:
            e_all = np.arange(n ** 3)
            cen = np.stack([2 * (e_all % n) + 1, 2 * ((e_all // n) % n) + 1, 2 * (e_all // (n * n)) + 1], 1)
            p_abc = np.repeat(cen, 4, axis=0)
            p_null = np.tile([1.0, 0.0, 0.0, 0.0], n ** 3)
        else:
            p_abc = 2 * self.q1_ijk
            p_null = np.ones(self.n_q1)
        node_abc = np.concatenate([np.repeat(self.q2_abc, 3, axis=0), p_abc])
        field = np.concatenate([np.tile([0, 1, 2], self.n_q2),
                                np.full(self.n_pdof, 3)])
        q2id_of_full = node_abc[:, 0] + N2 * (node_abc[:, 1] + N2 * node_abc[:, 2])
        self.full_node_abc = node_abc
        self.full_field = field
        self.dof_node = node_abc[self.free]
        self.dof_field = field[self.free]
        self.dof_q2id = q2id_of_full[self.free]
        # value of the field's null-space vector (translation or constant
        # pressure) on each free DOF: 1, except the linear P1disc functions
        self.dof_null = np.concatenate([np.ones(3 * self.n_q2), p_null])[self.free]

        # ---- assembly --------------------------------------------------------
        Ke, Be = element_matrices(self.h, self.mu, pressure)
        npe = Be.shape[0]
        ne_dofs = 81 + npe
        # element DOF map: 81 velocity (a, comp) with index 3*a + comp, then the pressure
        Ae = np.zeros((ne_dofs, ne_dofs))
        for comp in range(3):
            Ae[comp:81:3, comp:81:3] = Ke
        Bflat = Be.reshape(npe, 81)  # (q, 3*a + c)
        Ae[81:, :81] = Bflat
        Ae[:81, 81:] = Bflat.T
        self.Ae = Ae

        ne = n ** 3
        e = np.arange(ne)
        ex, ey, ez = e % n, (e // n) % n, e // (n * n)
        loc = np.arange(27)
        lx, ly, lz = loc % 3, (loc // 3) % 3, loc // 9
        q2n = ((2 * ex[:, None] + lx) + N2 * ((2 * ey[:, None] + ly)
                                              + N2 * (2 * ez[:, None] + lz)))
        vdofs = (3 * q2n[:, :, None] + np.arange(3)).reshape(ne, 81)
        if disc:
            pdofs = 3 * self.n_q2 + 4 * e[:, None] + np.arange(4)
        else:
            ql = np.arange(8)
            qx, qy, qz = ql % 2, (ql // 2) % 2, ql // 4
            q1n = ((ex[:, None] + qx) + (n + 1) * ((ey[:, None] + qy)
                                                   + (n + 1) * (ez[:, None] + qz)))
            pdofs = 3 * self.n_q2 + q1n
        edofs = np.concatenate([vdofs, pdofs], 1)  # (ne, 81 + npe)
        self.element_dofs = edofs

        Afull = sp.csr_matrix((self.n_full, self.n_full))
        for s0 in range(0, ne, chunk):
            ed = edofs[s0:s0 + chunk]
            k = ed.shape[0]
            rows = np.repeat(ed, ne_dofs, axis=1).ravel()
            cols = np.tile(ed, (1, ne_dofs)).ravel()
            vals = np.tile(Ae.ravel(), k)
            Afull = Afull + sp.csr_matrix((vals, (rows, cols)),
                                          shape=(self.n_full, self.n_full))
        Afull.sum_duplicates()
        self.A_full = Afull

        # load vector F = int f . phi
        F = np.zeros(self.n_full)
        if force is not None:
            P, W, phi, _, _ = reference_element(pressure)
            h = self.h
            for s0 in range(0, ne, chunk):
                sl = slice(s0, s0 + chunk)
                X = (np.stack([ex[sl], ey[sl], ez[sl]], 1)[:, None, :] + P[None]) * h
                f = force(X[..., 0], X[..., 1], X[..., 2])  # (3, k, 27q)
                # Fe[e, a, c] = h^3 sum_q W_q f_c(x_q) phi_a(x_q)
                Fe = (h ** 3) * np.einsum("q,ckq,qa->kac", W, f, phi)
                np.add.at(F, vdofs[sl].ravel(), Fe.reshape(-1))
        self.F_full = F

        # Dirichlet values on the full vector
        g = np.zeros(self.n_full)
        xyz = self.q2_abc * (self.h / 2.0)
        gv = dirichlet(xyz[:, 0], xyz[:, 1], xyz[:, 2])  # (3, n_q2)
        gvel = gv.T.ravel()
        g[:3 * self.n_q2] = np.where(vel_dir, gvel, 0.0)
        self.g_full = g

        free, dirs = self.free, self.dir
        Acsr = Afull.tocsr()
        self.A = Acsr[free][:, free].tocsr()
        self.A.sort_indices()
        self.b = F[free] - Acsr[free][:, dirs] @ g[dirs]

    # -- helpers ---------------------------------------------------------------
    def expand(self, x_free):
        """Full DOF vector: free values plus the Dirichlet data."""
        x = self.g_full.copy()
        x[self.free] = x_free
        return x

    def interpolant(self, u, p):
        """Nodal interpolant of (u, p) on the full DOF vector.  For P1disc the
        pressure coefficients are those of a function linear in x, y, z:
        the value at the element centre and half the change across the
        element along each axis."""
        xyz = self.q2_abc * (self.h / 2.0)
        uv = u(xyz[:, 0], xyz[:, 1], xyz[:, 2])
        if self.pressure == "p1disc":
            n, h = self.n, self.h
            e = np.arange(n ** 3)
            c = np.stack([e % n, (e // n) % n, e // (n * n)], 1) * h + 0.5 * h
            pc = np.asarray(p(c[:, 0], c[:, 1], c[:, 2]), dtype=float) * np.ones(n ** 3)
            coef = [pc]
            for ax in range(3):
                d = np.zeros(3)
                d[ax] = 0.5 * h
                pp = np.asarray(p(c[:, 0] + d[0], c[:, 1] + d[1], c[:, 2] + d[2]), dtype=float) * np.ones(n ** 3)
                coef.append(pp - pc)
            pv = np.stack(coef, 1).ravel()
        else:
            pq = self.q1_ijk * self.h
            pv = p(pq[:, 0], pq[:, 1], pq[:, 2])
        return np.concatenate([np.asarray(uv).T.ravel(), np.asarray(pv, dtype=float)])


def dof_count_q2q1(n):
    """Closed form 3(2n+1)^3 + (n+1)^3 of the Q2/Q1 full DOF count."""
    return 3 * (2 * n + 1) ** 3 + (n + 1) ** 3


def dof_count_q2p1disc(n):
    """Closed form 3(2n+1)^3 + 4n^3: Q2 velocity with a 4-DOF discontinuous
    P1 pressure per hexahedron (the paper's element pair, Tables 1-2)."""
    return 3 * (2 * n + 1) ** 3 + 4 * n ** 3
