"""Pins for the GMRES oracle: the minimal-residual property (brute force), exact
preconditioning, restarts and the flexible variant."""
import numpy as np

from oracle import krylov


def _nonsym(n, seed):
    rng = np.random.default_rng(seed)
    return np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n), rng.standard_normal(n)


def test_residual_history_is_krylov_minimum():
    """Unrestarted, unpreconditioned GMRES: the k-th residual estimate equals
    min_{x in K_k(A,b)} ||b - A x|| computed by dense least squares on an orthonormal basis."""
    A, b = _nonsym(30, 0)
    res = krylov.gmres(lambda v: A @ v, lambda v: v, b, rtol=1e-13, restart=30, max_iter=12)
    K = np.empty((30, 0))
    v = b.copy()
    for k in range(1, 13):
        K = np.column_stack([K, v])
        Qk, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(A @ Qk, b, rcond=None)
        rmin = np.linalg.norm(b - A @ Qk @ y) / np.linalg.norm(b)
        np.testing.assert_allclose(res.history[k - 1], rmin, rtol=1e-8, atol=1e-12)
        v = A @ v


def test_exact_preconditioner_one_iteration():
    A, b = _nonsym(40, 1)
    Ai = np.linalg.inv(A)
    res = krylov.gmres(lambda v: A @ v, lambda v: Ai @ v, b, rtol=1e-10)
    assert res.iterations == 1 and res.converged
    np.testing.assert_allclose(res.x, np.linalg.solve(A, b), rtol=1e-10)


def test_restarted_converges_to_true_residual():
    A, b = _nonsym(200, 2)
    res = krylov.gmres(lambda v: A @ v, lambda v: v, b, rtol=1e-10, restart=5, max_iter=2000)
    assert res.converged
    assert np.linalg.norm(b - A @ res.x) <= 1e-10 * np.linalg.norm(b)
    assert res.iterations > 5


def test_flexible_equals_standard_for_fixed_preconditioner():
    A, b = _nonsym(80, 3)
    M = np.diag(1.0 / np.diag(A))
    r1 = krylov.gmres(lambda v: A @ v, lambda v: M @ v, b, rtol=1e-10, restart=10)
    r2 = krylov.gmres(lambda v: A @ v, lambda v: M @ v, b, rtol=1e-10, restart=10, flexible=True)
    assert r1.iterations == r2.iterations
    np.testing.assert_allclose(r1.x, r2.x, rtol=1e-8)
