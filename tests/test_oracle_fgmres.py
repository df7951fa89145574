"""Pins of the FGMRES driver."""
import numpy as np

from oracle.fgmres import fgmres


def test_unpreconditioned_spd_minimal_residual():
    """Without restarts GMRES minimises ||b - A x|| over the Krylov space: on an
    n x n system it terminates within n steps, and each residual is the
    least-squares residual over K_k(A, b)."""
    rng = np.random.default_rng(0)
    n = 12
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = Q @ np.diag(np.linspace(1, 30, n)) @ Q.T
    b = rng.standard_normal(n)
    hist = []
    x, it, rel, trel = fgmres(lambda v: A @ v, lambda v: v, b, rtol=1e-14, history=hist)
    assert it <= n and trel < 1e-12
    for k in (1, 3, 6):
        K = np.stack([np.linalg.matrix_power(A, j) @ b for j in range(k)], 1)
        y = np.linalg.lstsq(A @ K, b, rcond=None)[0]
        ref = np.linalg.norm(b - A @ K @ y) / np.linalg.norm(b)
        assert abs(hist[k - 1] - ref) < 1e-8


def test_restart_and_flexible_preconditioner():
    rng = np.random.default_rng(1)
    n = 40
    A = np.diag(np.linspace(1, 100, n)) + 0.1 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    calls = []

    def prec(v):            # changes every call: flexible GMRES must cope
        calls.append(1)
        return v / np.diag(A) * (1.0 + 0.05 * (len(calls) % 3))

    x, it, rel, trel = fgmres(lambda v: A @ v, prec, b, rtol=1e-10, restart=7)
    assert trel <= 1e-10 and it == len(calls)
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) <= 1e-10


def test_exact_preconditioner_one_iteration():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((9, 9)) + 9 * np.eye(9)
    b = rng.standard_normal(9)
    Ainv = np.linalg.inv(A)
    x, it, rel, trel = fgmres(lambda v: A @ v, lambda v: Ainv @ v, b, rtol=1e-12)
    assert it == 1 and trel < 1e-12
