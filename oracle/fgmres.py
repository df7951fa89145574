"""Flexible GMRES with right preconditioning (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper solves with FGMRES to a relative tolerance of 1e-8 (unit cube,
Tables 1-2) or 1e-10 (extrusion die, Tables 3-4) but states no restart
length, orthogonalisation or initial guess.  Reading used on both sides:

* x_0 = 0 (or a given x_0), r_0 = b - A x_0, restart length 100, at most
  1000 inner iterations in total;
* Arnoldi with classical Gram-Schmidt applied twice (CGS2);
* Givens rotations: rho = hypot(h_jj, h_{j+1,j}), c = h_jj / rho,
  s = h_{j+1,j} / rho; g_{j+1} = -s g_j, g_j = c g_j;
* stop the cycle once |g_{j+1}| / ||b||_2 <= rtol; form x = x_0 + Z y with
  Z_j = M^{-1} v_j (flexible variant keeps Z); recompute the true residual
  ||b - A x|| / ||b||; if it is above rtol start a new cycle from x.

The iteration count is the number of preconditioner applications.

Pins (``tests/test_oracle_fgmres.py``): converges to the dense direct
solution; with the exact inverse as preconditioner it stops after one
iteration; without a preconditioner on a small SPD system it matches the
Krylov minimal-residual property.
"""
from __future__ import annotations

import math

import numpy as np


def fgmres(matvec, precond, b, rtol=1e-8, restart=100, max_it=1000, x0=None,
           history=None):
    """Return (x, iterations, implicit relative residual, true relative residual)."""
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return x, 0, 0.0, 0.0
    it = 0
    rel = 1.0
    true_rel = float(np.linalg.norm(b - matvec(x))) / bnorm
    while it < max_it:
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        true_rel = beta / bnorm
        if true_rel <= rtol:
            return x, it, rel, true_rel
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            # CGS2: two passes of classical Gram-Schmidt
            h = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            hn = float(np.linalg.norm(w))
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            if hn != 0.0:
                V[j + 1] = w / hn
            # apply the previous rotations to the new column
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / rho
            sn[j] = H[j + 1, j] / rho
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            rel = abs(g[j + 1]) / bnorm
            if history is not None:
                history.append(rel)
            if rel <= rtol or hn == 0.0 or it >= max_it:
                break
        # back substitution with the triangular H[:k, :k]
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
        true_rel = float(np.linalg.norm(b - matvec(x))) / bnorm
        if true_rel <= rtol:
            break
    return x, it, rel, true_rel
