"""Two-level monolithic GDSW preconditioner (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Definitions followed, in the paper's notation:

* eq. (2.2):  B_GDSW = Phi A_0^{-1} Phi^T + sum_i R_i^T A_i^{-1} R_i
* eq. (2.3):  A_0 = Phi^T A Phi;  R_i = blockdiag(R_{i,u}, R_{i,p}) restricts
              to the overlapping subdomain, so A_i = R_i A R_i^T.
* eq. (2.4):  Phi = [Phi_I; Phi_Gamma] with Phi_I = -A_II^{-1} A_IGamma Phi_Gamma,
              the energy-minimising (discrete harmonic) extension computed
              with the monolithic saddle-point block A_II, which produces
              the off-diagonal blocks Phi_{I,u0,p} and Phi_{I,p0,u}.
* Phi_Gamma = blockdiag(Phi_{Gamma,u0}, Phi_{Gamma,p0}): column (e, f) is the
  null-space vector of field f (a velocity translation or the pressure
  constant) restricted to interface entity e, i.e. 1 on e's f-DOFs.

Discontinuous pressure (the paper's Q2/P1disc pair, Section 3, last
paragraph): there is no pressure interface, and the coarse space carries one
pressure column per subdomain, constant over it (the pressure null-space
vector on the subdomain's pressure DOFs).  The monolithic extension is then
singular on interior subdomains (velocity fixed on the whole subdomain
boundary leaves the constant pressure free), so this variant extends the
velocity columns with the velocity block alone, Phi_I = -K_II^{-1} K_IGamma
Phi_Gamma over the interior velocity DOFs, and takes the pressure columns as
they are: the off-diagonal blocks Phi_{I,u0,p} and Phi_{I,p0,u} are zero
(``extension="velocity"``, the default whenever subdomain pressure columns
exist).

Every dense factorisation -- the local matrices A_i, the interior blocks
A_II of the extension and the coarse matrix A_0 -- is LAPACK's LU with partial
pivoting (``scipy.linalg.lu_factor``): the paper names no direct solver, and
this is the textbook general one.  The apply sums the local corrections in
ascending subdomain order and adds the coarse correction last.

Pins (``tests/test_oracle_gdsw.py``): Phi_Gamma is a partition of unity; the
extension reproduces constants on subdomains away from the Dirichlet and
outflow boundaries; A_II Phi_I + A_IGamma Phi_Gamma = 0; symmetry of A_0 and of
the preconditioner; one subdomain gives A^{-1}; full overlap gives the
closed form Phi A_0^{-1} Phi^T + N A^{-1}.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def coarse_basis(A, dec, extension="monolithic"):
    """Phi (free DOFs x coarse DOFs) of eq. (2.4), as a CSR matrix.

    extension="monolithic": Phi_I = -A_II^{-1} A_IGamma Phi_Gamma with the
    saddle-point block; "velocity": the same over the interior velocity DOFs
    with the velocity block only, zero pressure rows, plus the subdomain
    pressure columns (discontinuous pressure)."""
    nf = A.shape[0]
    rows, cols, vals = [], [], []
    # Phi_Gamma: indicator of each (entity, field)
    gcol = dec.coarse_col[dec.gamma_entity, dec.gamma_field]
    rows.append(dec.gamma)
    cols.append(gcol)
    vals.append(np.ones(dec.gamma.size))
    PhiG = sp.csr_matrix((np.ones(dec.gamma.size), (dec.gamma, gcol)),
                         shape=(nf, dec.n_coarse))
    A = A.tocsr()
    for i in range(dec.n_sub):
        Ii = dec.I[i]
        if extension == "velocity":
            if dec.sub_pressure_col is not None:
                Pi = Ii[dec.dof_field[Ii] == 3]
                rows.append(Pi)
                cols.append(np.full(Pi.size, dec.sub_pressure_col[i]))
                vals.append(dec.dof_null[Pi])
            Ii = Ii[dec.dof_field[Ii] < 3]
        if Ii.size == 0:
            continue
        AII = A[Ii][:, Ii].toarray()
        rhs = (A[Ii] @ PhiG).toarray()             # A_IGamma Phi_Gamma (I rows only)
        used = np.nonzero(np.any(rhs != 0.0, axis=0))[0]
        if used.size == 0:
            continue
        fac = sla.lu_factor(AII, check_finite=False)
        PhiI = -sla.lu_solve(fac, rhs[:, used], check_finite=False)
        rr, cc = np.meshgrid(Ii, used, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(PhiI.ravel())
    Phi = sp.csr_matrix((np.concatenate(vals),
                         (np.concatenate(rows), np.concatenate(cols))),
                        shape=(nf, dec.n_coarse))
    return Phi


class TwoLevelGDSW:
    """B_GDSW of eq. (2.2) for an assembled problem and its decomposition."""

    def __init__(self, A, dec, factor_local=True, extension=None):
        self.A = A.tocsr()
        self.dec = dec
        if extension is None:
            extension = "velocity" if getattr(dec, "sub_pressure_col", None) is not None else "monolithic"
        self.extension = extension
        self.S = dec.S
        self.local_lu = []
        if factor_local:
            for Si in self.S:
                Ai = self.A[Si][:, Si].toarray()
                self.local_lu.append(sla.lu_factor(Ai, check_finite=False))
        if dec.n_coarse > 0:
            self.Phi = coarse_basis(self.A, dec, extension)
            self.A0 = (self.Phi.T @ (self.A @ self.Phi)).toarray()
            self.A0_lu = sla.lu_factor(self.A0, check_finite=False)
        else:
            self.Phi = None
            self.A0 = np.zeros((0, 0))
            self.A0_lu = None

    def local_matrix(self, i):
        Si = self.S[i]
        return self.A[Si][:, Si].toarray()

    def local_solve(self, i, ri):
        """A_i^{-1} r_i with the stored LU factors."""
        return sla.lu_solve(self.local_lu[i], ri, check_finite=False)

    def coarse_solve(self, r0):
        """A_0^{-1} r_0 with the stored LU factors of A_0."""
        return sla.lu_solve(self.A0_lu, r0, check_finite=False)

    def apply_local(self, r):
        """sum_i R_i^T A_i^{-1} R_i r, ascending i."""
        z = np.zeros_like(r)
        for i, Si in enumerate(self.S):
            z[Si] += self.local_solve(i, r[Si])
        return z

    def apply_coarse(self, r):
        """Phi A_0^{-1} Phi^T r."""
        if self.Phi is None:
            return np.zeros_like(r)
        return self.Phi @ self.coarse_solve(self.Phi.T @ r)

    def apply(self, r):
        """z = B_GDSW r (eq. 2.2): local sum first, coarse correction last."""
        r = np.asarray(r, dtype=np.float64)
        if r.ndim == 2:
            return np.stack([self.apply(r[:, k]) for k in range(r.shape[1])], 1)
        z = self.apply_local(r)
        z += self.apply_coarse(r)
        return z

    __call__ = apply
