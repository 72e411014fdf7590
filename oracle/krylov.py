"""Oracle: restarted right-preconditioned GMRES / FGMRES (test infrastructure only).

The paper's outer solver setting (Section 4): zero initial guess and the exit
test ||r_k||_2 / ||r_0||_2 <= tau with tau = 1e-8.  GMRES is named in
Section 3 as the standard alternative to Bi-CGStab for non-symmetric systems.
Right preconditioning makes the Arnoldi residual estimate the unpreconditioned
residual; each restart cycle ends with the true residual recomputed in FP64,
and a cycle whose estimate met the target but whose true residual did not is
followed by another cycle.  Orthogonalisation: modified Gram-Schmidt.

Pins (tests/test_oracle_krylov.py): identity preconditioner against the
minimal-residual property computed by dense least squares on the Krylov
basis; exact inverse preconditioner converges in one iteration; restarts.
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
