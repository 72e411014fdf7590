"""Pins for the Krylov oracles.  GMRES: the minimal-residual property (brute force), exact
preconditioning, restarts and the flexible variant.  Bi-CGStab: exact preconditioning, finite
termination, consistency of the recurrence residual, the omega step, agreement with a dense
solve."""
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


def test_bicgstab_exact_preconditioner_one_iteration():
    """With P^-1 = A^-1 the first half step gives p^ = x*, v = r0, alpha = 1 and s = 0."""
    A, b = _nonsym(40, 4)
    Ai = np.linalg.inv(A)
    res = krylov.bicgstab(lambda v: A @ v, lambda v: Ai @ v, b, rtol=1e-10)
    assert res.iterations == 1 and res.converged
    np.testing.assert_allclose(res.x, np.linalg.solve(A, b), rtol=1e-10)


def test_bicgstab_terminates_within_n_iterations():
    """BiCG, and with it the BiCG part of Bi-CGStab, ends by step n on an n x n system in
    exact arithmetic.  A wrong beta (sign, or the omega factor dropped) or a wrong p update
    loses this and needs far more than n iterations at this conditioning."""
    for seed in range(5):
        A, b = _nonsym(8, 10 + seed)
        res = krylov.bicgstab(lambda v: A @ v, lambda v: v, b, rtol=1e-11, max_iter=50)
        assert res.converged and res.iterations <= 8, (seed, res.iterations)


def test_bicgstab_recurrence_residual_and_omega_step():
    """Along the history the recurrence residual equals b - A x_k (a wrong coefficient in
    the x update breaks it), and omega minimises ||s - omega t|| (the new residual is
    orthogonal to t)."""
    A, b = _nonsym(60, 5)
    M = np.diag(1.0 / np.diag(A))
    rec = []
    res = krylov.bicgstab(lambda v: A @ v, lambda v: M @ v, b, rtol=1e-12, record=rec)
    assert res.converged and len(rec) == res.iterations
    for x, r, s, t, om in rec:
        np.testing.assert_allclose(r, b - A @ x, atol=1e-10 * np.linalg.norm(b))
        if t is not None:
            assert abs(r @ t) <= 1e-10 * np.linalg.norm(r) * np.linalg.norm(t) + 1e-300
            # brute force: omega is the minimiser of the 1-D quadratic
            grid = om + np.linspace(-1e-3, 1e-3, 21) * max(abs(om), 1.0)
            vals = [np.linalg.norm(s - w * t) for w in grid]
            assert np.argmin(vals) == 10


def test_bicgstab_matches_dense_solve_and_cap():
    A, b = _nonsym(300, 6)
    res = krylov.bicgstab(lambda v: A @ v, lambda v: v, b, rtol=1e-10, max_iter=2000)
    assert res.converged
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(res.x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert np.linalg.norm(b - A @ res.x) <= 1e-10 * np.linalg.norm(b)
    capped = krylov.bicgstab(lambda v: A @ v, lambda v: v, b, rtol=1e-14, max_iter=3)
    assert not capped.converged and capped.iterations == 3
