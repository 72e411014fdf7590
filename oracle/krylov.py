"""Oracle: restarted right-preconditioned GMRES / FGMRES and right-preconditioned
Bi-CGStab (test infrastructure only).

The paper's outer solver setting (Section 4): zero initial guess and the exit
test ||r_k||_2 / ||r_0||_2 <= tau with tau = 1e-8.  GMRES is named in
Section 3 as the standard alternative to Bi-CGStab for non-symmetric systems.
Right preconditioning makes the Arnoldi residual estimate the unpreconditioned
residual; each restart cycle ends with the true residual recomputed in FP64,
and a cycle whose estimate met the target but whose true residual did not is
followed by another cycle.  Orthogonalisation: modified Gram-Schmidt.

Bi-CGStab is the paper's outer solver (Section 4, after van der Vorst 1992):
x0 = 0, stop when ||r_k|| <= tau ||r_0||, "NC" past an iteration cap.  Right
preconditioning keeps the recurrence residual the unpreconditioned one.  An
iteration applies the preconditioner and the matrix twice; convergence at the
half step (the residual s) ends the iteration there.  Before returning, the
true residual is recomputed in FP64; if it misses the target (drift of the
recurrence) or the recurrence breaks down (rho, (r^, v) or omega zero), the
method restarts from the current iterate with r^ = r = b - A x.

Pins (tests/test_oracle_krylov.py): identity preconditioner against the
minimal-residual property computed by dense least squares on the Krylov
basis; exact inverse preconditioner converges in one iteration; restarts.
Bi-CGStab: one iteration with the exact inverse; termination within n
iterations on an n x n system (exact arithmetic ends BiCG by step n); the
recurrence residual equals b - A x_k along the history; agreement with a
dense solve; omega minimising ||s - omega t||.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Result:
    x: np.ndarray
    iterations: int
    converged: bool
    relres_true: float
    history: list = field(default_factory=list)   # residual estimates / ||b||


def gmres(matvec, prec, b, rtol=1e-8, restart=50, max_iter=5000, flexible=False):
    n = b.size
    bnorm = np.linalg.norm(b)
    x = np.zeros(n)
    if bnorm == 0.0:
        return Result(x, 0, True, 0.0)
    r = b.copy()
    beta = bnorm
    total = 0
    hist = []
    while total < max_iter:
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n)) if flexible else None
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(m):
            z = prec(V[j])
            if flexible:
                Z[j] = z
            w = matvec(z)
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_end = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= rtol * bnorm or total >= max_iter:
                break
        k = j_end
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k]) if k else np.zeros(0)
        if flexible:
            x = x + Z[:k].T @ y
        else:
            x = x + prec(V[:k].T @ y)
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm:
            return Result(x, total, True, beta / bnorm, hist)
    return Result(x, total, False, beta / bnorm, hist)


def bicgstab(matvec, prec, b, rtol=1e-8, max_iter=2000, record=None):
    """Right-preconditioned Bi-CGStab, x0 = 0.  record (a list or None) receives, per
    iteration, (x, r, s, t, omega) for the pins."""
    n = b.size
    bnorm = np.linalg.norm(b)
    x = np.zeros(n)
    if bnorm == 0.0:
        return Result(x, 0, True, 0.0)
    tol = rtol * bnorm
    total = 0
    hist = []
    r = b.copy()
    while True:
        # (re)start: shadow residual = current residual
        rhat = r.copy()
        rho_old = alpha = omega = 1.0
        v = np.zeros(n)
        p = np.zeros(n)
        breakdown = False
        while total < max_iter:
            rho = rhat @ r
            if rho == 0.0:
                breakdown = True
                break
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
            ph = prec(p)
            v = matvec(ph)
            rv = rhat @ v
            if rv == 0.0:
                breakdown = True
                break
            alpha = rho / rv
            s = r - alpha * v
            total += 1
            if np.linalg.norm(s) <= tol:
                x = x + alpha * ph
                r = s
                hist.append(np.linalg.norm(r) / bnorm)
                if record is not None:
                    record.append((x.copy(), r.copy(), s.copy(), None, None))
                break
            sh = prec(s)
            t = matvec(sh)
            tt = t @ t
            omega = (t @ s) / tt if tt > 0.0 else 0.0
            x = x + alpha * ph + omega * sh
            r = s - omega * t
            rho_old = rho
            hist.append(np.linalg.norm(r) / bnorm)
            if record is not None:
                record.append((x.copy(), r.copy(), s.copy(), t.copy(), omega))
            if np.linalg.norm(r) <= tol:
                break
            if omega == 0.0:
                breakdown = True
                break
        r = b - matvec(x)
        rn = np.linalg.norm(r)
        if rn <= tol:
            return Result(x, total, True, rn / bnorm, hist)
        if total >= max_iter:
            return Result(x, total, False, rn / bnorm, hist)
        # recurrence drifted or broke down: restart on the true residual
        del breakdown
