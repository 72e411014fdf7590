"""GPU parity of the adjoint path: the per-cell gradient kernel against the oracle formula,
the transposed EDFA-GMRES against the oracle's transposed iteration and a direct solve of
A^T, the end-to-end gradient against the oracle chain, finite differences on the 48^3
anisotropic workload, and the torch.autograd.Function."""
import dataclasses

import numpy as np
import pytest
import torch

from oracle import adjoint as oadj, edfa as oedfa, krylov, mhfe
from paper_2009_13916_amd import inputs

pytestmark = pytest.mark.gpu

PROBLEMS = {
    "iso6": lambda: inputs.lognormal_iso_problem(6, config_id=31),
    "full4x5x3": lambda: inputs.full_tensor_problem(4, 5, 3, sigma=2.0, corr=2.0, config_id=32),
    "distorted5x4x3": lambda: inputs.channel_problem(5, 4, 3, contrast=1e4, config_id=33),
    "aniso7": lambda: inputs.anisotropic_problem(7, config_id=34),
}
DYN = dict(variant="dynamic", n_add=1, n_ent=4)


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_grad_kernel_matches_oracle_formula(lib, name):
    """Same (u, lambda), random: GPU dL/dtheta within 1e-12 of the oracle, relative to max |g|."""
    prob = PROBLEMS[name]()
    o = mhfe.assemble(prob)
    rng = np.random.default_rng(17)
    u = rng.standard_normal(o.n)
    lam = rng.standard_normal(o.n)
    ref = oadj.grad_logk(o, prob, u, lam)
    S = lib.System(prob)
    g = lib.grad_logk(S, _dev(u), _dev(lam)).cpu().numpy()
    assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_grad_kernel_batched_equals_per_grid(lib):
    probs = [PROBLEMS["iso6"](), PROBLEMS["aniso7"]()]
    S = lib.System(probs)
    nfu, ne = S.info["nfu"], S.info["ne"]
    rng = np.random.default_rng(19)
    u = rng.standard_normal(nfu + ne)
    lam = rng.standard_normal(nfu + ne)
    g = lib.grad_logk(S, _dev(u), _dev(lam)).cpu().numpy()
    f0 = c0 = 0
    for p in probs:
        o = mhfe.assemble(p)
        uu = np.concatenate([u[f0:f0 + o.nfu], u[nfu + c0:nfu + c0 + o.ne]])
        ll = np.concatenate([lam[f0:f0 + o.nfu], lam[nfu + c0:nfu + c0 + o.ne]])
        ref = oadj.grad_logk(o, p, uu, ll)
        assert np.max(np.abs(g[c0:c0 + o.ne] - ref)) <= 1e-12 * np.max(np.abs(ref))
        f0 += o.nfu
        c0 += o.ne


def _obs_loss(o, seed, count=8):
    rng = np.random.default_rng(seed)
    return inputs.observations(o.ne, count, rng)


@pytest.mark.parametrize("name", ["iso6", "full4x5x3"])
def test_transposed_solve_matches_oracle(lib, name):
    """Transposed EDFA-GMRES (P^-T with the forward factors) against the oracle's GMRES on
    A^T with its transposed EDFA: solution within 1e-8, iterations within +-2."""
    prob = PROBLEMS[name]()
    o = mhfe.assemble(prob)
    E = oedfa.build(o, oedfa.Params(**DYN))
    obs, target = _obs_loss(o, 23)
    u = mhfe.direct_solve(o)
    rhs = oadj.dloss_du(o, u[o.nfu:], obs, target)
    AT = o.matrix().T.tocsr()
    ref = krylov.gmres(lambda v: AT @ v, E.apply_T, rhs, 1e-8, 50)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**DYN))
    lam, info, st = lib.solve(S, P, _dev(rhs), rtol=1e-8, restart=50, transpose=True)
    lg = lam.cpu().numpy()
    assert st == 0
    assert np.linalg.norm(rhs - AT @ lg) <= 1e-8 * np.linalg.norm(rhs)
    assert np.linalg.norm(lg - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
    assert abs(info["iterations"] - ref.iterations) <= 2, (info["iterations"], ref.iterations)


def test_transposed_solve_tight_matches_direct(lib):
    prob = PROBLEMS["aniso7"]()
    o = mhfe.assemble(prob)
    obs, target = _obs_loss(o, 29)
    u = mhfe.direct_solve(o)
    rhs = oadj.dloss_du(o, u[o.nfu:], obs, target)
    lam_ref = oadj.adjoint_direct(o, rhs)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**DYN))
    lam, info, st = lib.solve(S, P, _dev(rhs), rtol=1e-12, restart=50, transpose=True)
    assert st == 0
    assert np.linalg.norm(lam.cpu().numpy() - lam_ref) <= 1e-8 * np.linalg.norm(lam_ref)


@pytest.mark.parametrize("name", ["aniso7", "distorted5x4x3"])
def test_gradient_end_to_end_matches_oracle_chain(lib, name):
    """GPU forward (1e-12), adjoint (1e-12) and gradient against direct oracle solves and
    the oracle formula: within 1e-8 relative."""
    prob = PROBLEMS[name]()
    o = mhfe.assemble(prob)
    obs, target = _obs_loss(o, 31)
    u = mhfe.direct_solve(o)
    lam = oadj.adjoint_direct(o, oadj.dloss_du(o, u[o.nfu:], obs, target))
    ref = oadj.grad_logk(o, prob, u, lam)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**DYN))
    ug, _, st = lib.solve(S, P, S.rhs(), rtol=1e-12)
    assert st == 0
    rhs = torch.zeros_like(ug)
    rhs[o.nfu:][torch.as_tensor(obs, device="cuda")] = 2.0 * (ug[o.nfu:][torch.as_tensor(obs, device="cuda")]
                                                              - _dev(target))
    lg, _, st = lib.solve(S, P, rhs, rtol=1e-12, transpose=True)
    assert st == 0
    g = lib.grad_logk(S, ug, lg).cpu().numpy()
    assert np.linalg.norm(g - ref) <= 1e-8 * np.linalg.norm(ref)


def test_autograd_function_matches_oracle_chain(lib):
    from paper_2009_13916_amd import adjoint
    prob = PROBLEMS["aniso7"]()
    o = mhfe.assemble(prob)
    obs, target = _obs_loss(o, 37)
    u = mhfe.direct_solve(o)
    lam = oadj.adjoint_direct(o, oadj.dloss_du(o, u[o.nfu:], obs, target))
    ref = oadj.grad_logk(o, prob, u, lam)
    theta = torch.zeros(o.ne, dtype=torch.float64, device="cuda", requires_grad=True)
    p = adjoint.pressure(theta, prob, lib.Params(**DYN), rtol=1e-12, rtol_adjoint=1e-12)
    oi = torch.as_tensor(obs, device="cuda")
    L = ((p[oi] - _dev(target)) ** 2).sum()
    L.backward()
    assert abs(L.item() - oadj.loss(u[o.nfu:], obs, target)) <= 1e-9 * oadj.loss(u[o.nfu:], obs, target)
    assert np.linalg.norm(theta.grad.cpu().numpy() - ref) <= 1e-8 * np.linalg.norm(ref)


def test_finite_differences_48cubed(lib):
    """48^3 anisotropic workload (ln k ~ N(0, 1.5^2), K = k diag(1, 1, 0.1)), 64 observation
    cells.  Forward to 1e-12, adjoint to 1e-10; central differences with h = 1e-6 on 32
    random cells.  Each perturbed pressure is obtained as u + du with
    A(theta +- h) du = -(R(u; theta +- h) - R(u; theta)), the residual change being exact zero
    outside the perturbed cell's rows, so the difference quotient is not swamped by solver
    noise.  Relative 2-norm error over the 32 cells <= 1e-5."""
    prob = inputs.anisotropic_problem(48, sigma=1.5, ratio=10.0)
    rngs = inputs.seed_streams(5)
    S = lib.System(prob)
    ne, nfu = S.info["ne"], S.info["nfu"]
    obs, target = inputs.observations(ne, 64, rngs[4])
    oi = torch.as_tensor(obs, device="cuda")
    tg = _dev(target)
    P = lib.Precond(S, lib.Params(**DYN))
    b = S.rhs()
    u, _, st = lib.solve(S, P, b, rtol=1e-12)
    assert st == 0
    rhs = torch.zeros_like(u)
    rhs[nfu:][oi] = 2.0 * (u[nfu:][oi] - tg)
    lam, _, st = lib.solve(S, P, rhs, rtol=1e-10, transpose=True)
    assert st == 0
    g = lib.grad_logk(S, u, lam).cpu().numpy()
    r0 = S.spmv(u) - b
    dev_p = u[nfu:][oi] - tg
    cells = np.random.default_rng(41).choice(ne, size=32, replace=False)
    h = 1e-6
    fd = np.empty(32)
    for t, E in enumerate(cells):
        dL = []
        for sgn in (1.0, -1.0):
            K = prob.K.copy()
            K[E] *= np.exp(sgn * h)
            Sp = lib.System(dataclasses.replace(prob, K=K))
            d = (Sp.spmv(u) - Sp.rhs()) - r0
            Pp = lib.Precond(Sp, lib.Params(**DYN))
            du, _, st = lib.solve(Sp, Pp, -d, rtol=1e-10)
            assert st == 0
            dp = du[nfu:][oi]
            dL.append(float((2.0 * dev_p * dp + dp * dp).sum()))
        fd[t] = (dL[0] - dL[1]) / (2 * h)
        print(f"cell {E}: adjoint {g[E]: .6e}  fd {fd[t]: .6e}", flush=True)
    err = np.linalg.norm(g[cells] - fd) / np.linalg.norm(fd)
    print(f"relative 2-norm error over 32 cells: {err:.3e}", flush=True)
    assert err <= 1e-5
