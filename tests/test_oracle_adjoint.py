"""Pins of the oracle adjoint gradient (oracle/adjoint.py) against things other than itself:
central differences of the assembled residual, central differences of the loss through
direct solves, and the invariance of steady pressures under a uniform scaling of K."""
import dataclasses

import numpy as np
import pytest

from oracle import adjoint, mhfe
from paper_2009_13916_amd import inputs


def _scaled(prob, cell, h):
    K = prob.K.copy()
    K[cell] *= np.exp(h)
    return dataclasses.replace(prob, K=K)


def _residual(prob, u):
    s = mhfe.assemble(prob)
    return s.matrix() @ u - s.b


def _problems():
    iso = inputs.lognormal_iso_problem(4, sigma=1.0, config_id=101)
    full = inputs.full_tensor_problem(3, sigma=1.0, corr=1.0, config_id=102)
    dist = inputs.channel_problem(4, 3, 3, contrast=1e2, perturb=0.2, config_id=103, dt=1e-3)
    aniso = inputs.anisotropic_problem(4, sigma=1.0, ratio=10.0, config_id=104)
    return {"iso4": iso, "full3": full, "distorted4x3x3": dist, "aniso4": aniso}


@pytest.mark.parametrize("name", ["iso4", "full3", "distorted4x3x3", "aniso4"])
def test_gradient_formula_matches_residual_differences(name):
    """-lambda^T (R(u; theta + h e_E) - R(u; theta - h e_E)) / 2h at random u, lambda, every cell."""
    prob = _problems()[name]
    s = mhfe.assemble(prob)
    rng = np.random.default_rng(7)
    u = rng.standard_normal(s.n)
    lam = rng.standard_normal(s.n)
    g = adjoint.grad_logk(s, prob, u, lam)
    h = 1e-4
    fd = np.empty(s.ne)
    for E in range(s.ne):
        rp = _residual(_scaled(prob, E, h), u)
        rm = _residual(_scaled(prob, E, -h), u)
        fd[E] = -lam @ (rp - rm) / (2 * h)
    assert np.max(np.abs(g - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_gradient_matches_loss_differences_through_direct_solves():
    prob = inputs.anisotropic_problem(5, sigma=1.5, ratio=10.0, config_id=105)
    s = mhfe.assemble(prob)
    rng = np.random.default_rng(11)
    obs = rng.choice(s.ne, size=8, replace=False)
    target = rng.uniform(0, 1, size=8)
    u = mhfe.direct_solve(s)
    p = u[s.nfu:]
    lam = adjoint.adjoint_direct(s, adjoint.dloss_du(s, p, obs, target))
    g = adjoint.grad_logk(s, prob, u, lam)
    cells = rng.choice(s.ne, size=12, replace=False)
    h = 1e-5
    fd = []
    for E in cells:
        Lp = adjoint.loss(mhfe.direct_solve(mhfe.assemble(_scaled(prob, E, h)))[s.nfu:], obs, target)
        Lm = adjoint.loss(mhfe.direct_solve(mhfe.assemble(_scaled(prob, E, -h)))[s.nfu:], obs, target)
        fd.append((Lp - Lm) / (2 * h))
    fd = np.array(fd)
    assert np.linalg.norm(g[cells] - fd) <= 1e-6 * np.linalg.norm(fd)


def test_uniform_scaling_of_K_leaves_the_loss_unchanged():
    """Scaling every K^E by the same factor scales A's flux terms and b alike; with the storage
    term negligible the pressures do not move, so the gradient sums to ~0 over cells."""
    prob = inputs.lognormal_iso_problem(5, sigma=1.0, config_id=106)
    s = mhfe.assemble(prob)
    rng = np.random.default_rng(3)
    obs = rng.choice(s.ne, size=6, replace=False)
    target = rng.uniform(0, 1, size=6)
    u = mhfe.direct_solve(s)
    lam = adjoint.adjoint_direct(s, adjoint.dloss_du(s, u[s.nfu:], obs, target))
    g = adjoint.grad_logk(s, prob, u, lam)
    assert abs(g.sum()) <= 1e-8 * np.abs(g).sum()
    assert np.abs(g).sum() > 0


def test_adjoint_direct_solves_the_transposed_system():
    prob = inputs.full_tensor_problem(3, sigma=1.0, corr=1.0, config_id=107)
    s = mhfe.assemble(prob)
    rhs = np.random.default_rng(5).standard_normal(s.n)
    lam = adjoint.adjoint_direct(s, rhs)
    assert np.linalg.norm(s.matrix().T @ lam - rhs) <= 1e-12 * np.linalg.norm(rhs)
