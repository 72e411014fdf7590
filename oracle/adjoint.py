"""Oracle: adjoint gradient of a pressure-mismatch loss (test infrastructure only).

Not in the paper; derived here from its discretisation.  The system residual is
R(u; theta) = A(theta) u - b(theta) (eq. system), with theta_E the natural log of a
multiplier of the permeability tensor K^E of cell E.  Scaling K^E by exp(theta_E)
scales B^E (eq. B_ij, which integrates K^-1) by exp(-theta_E), hence W^E = (B^E)^-1 by
exp(theta_E).  For a loss L(u) with A^T lambda = dL/du,

    dL/dtheta_E = -lambda^T dR/dtheta_E (u).

Only cell E's element enters dR/dtheta_E:
* face rows (eq. cont_fluxes): the local flux q^E = W^E (p^E 1 - pi^E) of eq.
  fluxes_MHFEM_3 is linear in W^E, so dq^E/dtheta_E = q^E;
* cell rows (eq. discr_bal_FV_2 with the strong flux of eq. fluxes_MHFEM_STRONG):
  on an interior face the strong flux q = (W'_ii Lam^E - W_ii Lam^E') / (W_ii + W'_ii)
  has Lam^E and W_ii proportional to exp(theta_E), so dq/dtheta_E = q W'_ii/(W_ii + W'_ii);
  it enters row E with + and the neighbour's row with -.  A Dirichlet face enters row
  E with the one-sided q_i^E; a Neumann face with its prescribed flux (no dependence).
Dirichlet face pressures take their boundary values.

Pins (tests/test_oracle_adjoint.py): central differences of the residual itself (the
assembly of perturbed problems, at random u and lambda, every cell, bricks, full
tensors and distorted hexahedra), and central differences of the loss through direct
solves of perturbed problems.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .mhfe import System, DIRICHLET, INTERIOR


def loss(p, obs, target):
    """L = sum over observation cells of (p_o - p*_o)^2."""
    d = p[obs] - target
    return float(d @ d)


def dloss_du(sysm: System, p, obs, target):
    """dL/du: zero on the face unknowns, 2 (p_o - p*_o) on the observed cells."""
    g = np.zeros(sysm.n)
    np.add.at(g, sysm.nfu + np.asarray(obs), 2.0 * (p[obs] - target))
    return g


def adjoint_direct(sysm: System, rhs):
    """lambda = A^-T rhs by a sparse LU of A^T."""
    return spla.splu(sysm.matrix().T.tocsc()).solve(rhs)


def face_pressures(sysm: System, prob, u):
    """pi on every face: the unknown where there is one, the boundary value on Dirichlet faces."""
    pi = np.asarray(prob.bc_value, dtype=np.float64).copy()
    known = sysm.uidx >= 0
    pi[known] = u[sysm.uidx[known]]
    return pi


def grad_logk(sysm: System, prob, u, lam):
    """dL/dtheta_E = -lambda^T dR/dtheta_E(u) for every cell (formula in the header)."""
    topo = sysm.topo
    ne, nfu = sysm.ne, sysm.nfu
    cf = topo.cell_faces                     # (Ne,6)
    fc = topo.face_cells                     # (Nf,2)
    W = sysm.W
    p = u[nfu:]
    pi = face_pressures(sysm, prob, u)[cf]   # (Ne,6)
    # local fluxes q^E_a = sum_b W_ab (p^E - pi_b)
    q = np.einsum("eab,eb->ea", W, p[:, None] - pi)
    lam_face = np.where(sysm.uidx[cf] >= 0, lam[np.maximum(sysm.uidx[cf], 0)], 0.0)
    lam_cell = lam[nfu:]
    g = -(lam_face * q).sum(axis=1)          # face rows
    kind = sysm.kind[cf]
    g -= np.where(kind == DIRICHLET, lam_cell[:, None] * q, 0.0).sum(axis=1)
    # interior faces: strong flux through face a, seen from E
    Wd = W[:, np.arange(6), np.arange(6)]
    L = W.sum(axis=2)
    cells = np.arange(ne)
    for a in range(6):
        inter = kind[:, a] == INTERIOR
        E = cells[inter]
        nb = np.where(a % 2 == 1, fc[cf[E, a], 1], fc[cf[E, a], 0])
        ap = a ^ 1
        # Lam^E_a = L_a p^E - sum_{b != a} W_ab pi_b
        lamE = L[E, a] * p[E] - (W[E, a, :] * pi[E]).sum(axis=1) + W[E, a, a] * pi[E, a]
        lamN = L[nb, ap] * p[nb] - (W[nb, ap, :] * pi[nb]).sum(axis=1) + W[nb, ap, ap] * pi[nb, ap]
        w, wn = Wd[E, a], Wd[nb, ap]
        qs = (wn * lamE - w * lamN) / (w + wn)
        g[E] -= (lam_cell[E] - lam_cell[nb]) * qs * wn / (w + wn)
    return g
