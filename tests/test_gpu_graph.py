"""Graph-captured GMRES cycles (use_graph = 1): the first cycle runs eagerly, later cycles
replay one captured cycle.  Launch order and every reduction are deterministic, so each
replayed solve must reproduce the eager solve bit for bit; short restarts make a solve
replay the graph many times, with the host's state reads and synchronisations between."""
import numpy as np
import pytest
import torch

from oracle import mhfe
from paper_2009_13916_amd import inputs

pytestmark = pytest.mark.gpu

DYN = dict(variant="dynamic", n_add=1, n_ent=4)


def _pair(lib, S, P, b, **kw):
    x0, i0, s0 = lib.solve(S, P, b, use_graph=False, **kw)
    x1, i1, s1 = lib.solve(S, P, b, use_graph=True, **kw)
    return (x0.cpu().numpy(), i0, s0), (x1.cpu().numpy(), i1, s1)


@pytest.mark.parametrize("restart", [10, 50])
@pytest.mark.parametrize("transpose", [False, True])
def test_graph_solve_equals_eager_single_grid(lib, restart, transpose):
    prob = inputs.full_tensor_problem(6, sigma=2.0, corr=2.0, config_id=61)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**DYN))
    b = torch.tensor(np.random.default_rng(3).standard_normal(S.n), device="cuda")
    (xe, ie, se), (xg, ig, sg) = _pair(lib, S, P, b, rtol=1e-10, restart=restart, transpose=transpose)
    print(f"[graph] restart {restart} transpose {transpose}: {ie['iterations']} iterations, "
          f"{ie['cycles']} cycles", flush=True)
    assert se == sg == 0
    assert ie["iterations"] == ig["iterations"] and ie["cycles"] == ig["cycles"]
    assert np.array_equal(xe, xg)


def test_graph_solve_equals_eager_mixed_precision_batch(lib):
    probs = [inputs.lognormal_iso_problem(n, sigma=s, config_id=4, extra=i)
             for i, (n, s) in enumerate([(5, 0.5), (9, 2.5), (7, 1.0), (6, 3.0)])]
    S = lib.System(probs)
    P = lib.Precond(S, lib.Params(**DYN, precision=1))
    b = S.rhs()
    for rep in range(3):   # repeated graph solves with eager solves in between
        (xe, ie, se), (xg, ig, sg) = _pair(lib, S, P, b, rtol=1e-8, restart=8, flexible=True)
        assert se == sg == 0 and ie["converged"] == ig["converged"] == 4
        assert ie["iterations"] == ig["iterations"]
        assert np.array_equal(xe, xg), rep


def test_graph_solution_matches_direct(lib):
    prob = inputs.lognormal_iso_problem(8, config_id=62)
    o = mhfe.assemble(prob)
    u = mhfe.direct_solve(o)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**DYN))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-12, restart=12, use_graph=True)
    assert st == 0 and info["cycles"] > 2
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg[o.nfu:] - u[o.nfu:]) <= 1e-8 * np.linalg.norm(u[o.nfu:])
