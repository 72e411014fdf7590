"""Edge cases against the oracle: degenerate grids (one cell; a line whose every cell touches
a Dirichlet face; a column; a single-layer slab), a ragged batch that mixes them with a larger
grid, wide static patches (Patch(2): the factor-in-LDS kernel for patterns over 48; Patch(3):
past the compiled capacity, an error), several entries added per sweep, GMRES(1), and a zero
right-hand side."""
import numpy as np
import pytest
import torch

from oracle import edfa as oedfa, krylov, mhfe
from paper_2009_13916_amd import inputs

pytestmark = pytest.mark.gpu

DYN = dict(variant="dynamic", n_add=1, n_ent=4)


def _grid(nx, ny, nz, seed, full=False):
    if full:
        return inputs.full_tensor_problem(nx, ny, nz, sigma=1.0, corr=1.0, config_id=seed)
    rngs = inputs.seed_streams(seed)
    ne = nx * ny * nz
    K = inputs.iso_tensor(np.exp(rngs[0].standard_normal(ne)))
    return inputs._common(nx, ny, nz, inputs.brick_nodes(nx, ny, nz), K, rngs, 1.0,
                          {"workload": f"edge_{nx}x{ny}x{nz}"})


CASES = {
    "one_cell": lambda: _grid(1, 1, 1, 91),
    "line_x5": lambda: _grid(5, 1, 1, 92),
    "column_z6": lambda: _grid(1, 1, 6, 93),
    "slab_4x3x1": lambda: _grid(4, 3, 1, 94),
    "full_2x2x2": lambda: _grid(2, 2, 2, 95, full=True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_degenerate_grids_match_oracle(lib, name):
    prob = CASES[name]()
    o = mhfe.assemble(prob)
    S = lib.System(prob)
    rp, col, val = S.export_block("A")
    import scipy.sparse as sp
    A = sp.csr_matrix((val.cpu().numpy(), col.cpu().numpy(), rp.cpu().numpy()), shape=(o.n, o.n))
    ref = o.matrix()
    assert abs(A - ref).max() <= 1e-12 * abs(ref).max()
    assert np.allclose(S.rhs().cpu().numpy(), o.b, rtol=0, atol=1e-12 * np.abs(o.b).max())
    E = oedfa.build(o, oedfa.Params(**DYN))
    P = lib.Precond(S, lib.Params(**DYN))
    r = np.random.default_rng(1).standard_normal(o.n)
    z = P.apply(torch.tensor(r, device="cuda")).cpu().numpy()
    assert np.linalg.norm(z - E.apply(r)) <= 1e-10 * np.linalg.norm(E.apply(r))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-12)
    u = mhfe.direct_solve(o)
    assert st == 0
    assert np.linalg.norm(x.cpu().numpy() - u) <= 1e-9 * np.linalg.norm(u)


def test_ragged_batch_with_degenerate_members(lib):
    probs = [CASES["one_cell"](), inputs.lognormal_iso_problem(7, sigma=2.0, config_id=96),
             CASES["line_x5"](), CASES["slab_4x3x1"]()]
    S = lib.System(probs)
    P = lib.Precond(S, lib.Params(**DYN))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-12)
    assert st == 0 and info["converged"] == 4
    xg = x.cpu().numpy()
    nfu = S.info["nfu"]
    f0 = c0 = 0
    for p in probs:
        o = mhfe.assemble(p)
        u = mhfe.direct_solve(o)
        xs = np.concatenate([xg[f0:f0 + o.nfu], xg[nfu + c0:nfu + c0 + o.ne]])
        assert np.linalg.norm(xs - u) <= 1e-9 * np.linalg.norm(u)
        f0 += o.nfu
        c0 += o.ne


def test_wide_static_patches(lib):
    """Patch(2) patterns (up to 113 entries) exceed 48: the factor-in-LDS kernel."""
    prob = inputs.lognormal_iso_problem(6, sigma=1.5, config_id=97)
    kw = dict(variant="static", static_level=2)
    o = mhfe.assemble(prob)
    E = oedfa.build(o, oedfa.Params(**kw))
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    assert P.info()["max_pattern"] > 48
    import scipy.sparse as sp
    rp, col, val, _ = P.export("G")
    G = sp.csr_matrix((val.cpu().numpy(), col.cpu().numpy(), rp.cpu().numpy()), shape=(o.ne, o.nfu))
    D = (G - E.st1.Gt).tocsr()
    assert abs(D).max() <= 1e-10 * abs(E.st1.Gt).max()
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-8)
    A = o.matrix()
    ref = krylov.gmres(lambda v: A @ v, E.apply, o.b, 1e-8, 50)
    assert st == 0 and abs(info["iterations"] - ref.iterations) <= 1
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg[o.nfu:] - ref.x[o.nfu:]) <= 1e-8 * np.linalg.norm(ref.x[o.nfu:])


def test_patterns_over_capacity_are_an_error(lib):
    """Patch(3) reaches 243 entries, past the compiled 128: a capacity error, not a result."""
    prob = inputs.lognormal_iso_problem(6, sigma=1.5, config_id=97)
    S = lib.System(prob)
    with pytest.raises(lib.EdfaError) as e:
        lib.Precond(S, lib.Params(variant="static", static_level=3))
    assert e.value.status == -7


def test_several_entries_per_sweep(lib):
    prob = inputs.full_tensor_problem(5, sigma=2.0, corr=2.0, config_id=98)
    kw = dict(variant="dynamic", n_add=3, n_ent=6)
    o = mhfe.assemble(prob)
    E = oedfa.build(o, oedfa.Params(**kw))
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    r = np.random.default_rng(2).standard_normal(o.n)
    z = P.apply(torch.tensor(r, device="cuda")).cpu().numpy()
    assert np.linalg.norm(z - E.apply(r)) <= 1e-10 * np.linalg.norm(E.apply(r))


def test_gmres_restart_one(lib):
    prob = inputs.lognormal_iso_problem(5, sigma=0.5, config_id=99)
    o = mhfe.assemble(prob)
    E = oedfa.build(o, oedfa.Params(**DYN))
    A = o.matrix()
    ref = krylov.gmres(lambda v: A @ v, E.apply, o.b, 1e-8, 1, max_iter=5000)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**DYN))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-8, restart=1, max_iter=5000)
    assert st == 0 and ref.converged
    assert abs(info["iterations"] - ref.iterations) <= 2, (info["iterations"], ref.iterations)
    xg = x.cpu().numpy()
    assert np.linalg.norm(o.b - A @ xg) <= 1e-8 * np.linalg.norm(o.b)


def test_zero_rhs_returns_zero(lib):
    prob = inputs.lognormal_iso_problem(4, config_id=100)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**DYN))
    b = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    x, info, st = lib.solve(S, P, b, rtol=1e-8)
    assert st == 0 and info["iterations"] == 0
    assert bool(torch.all(x == 0))
