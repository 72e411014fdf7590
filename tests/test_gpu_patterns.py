"""The pattern library on the GPU against the oracle: static strips along a fixed axis and
along each cell's axis of largest transmissibility (patterns bit-exact, values to 1e-10,
GMRES pressure to 1e-8), and the parameter tuner (edfa_tune_params): it returns the fastest
converged candidate of those it timed, skips a candidate the system cannot take, and the
chosen setting solves the system."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import edfa as oedfa, krylov, mhfe
from paper_2009_13916_amd import inputs

pytestmark = pytest.mark.gpu


def _to_sp(rp, col, val, shape):
    M = sp.csr_matrix((val.cpu().numpy(), col.cpu().numpy(), rp.cpu().numpy()), shape=shape)
    M.sort_indices()
    return M


@pytest.mark.parametrize("axis,level,full", [(1, 1, True), (3, 2, False), (4, 1, True),
                                             (4, 2, False)])
def test_axis_strips_match_oracle(lib, axis, level, full):
    if full:
        prob = inputs.full_tensor_problem(6, 5, 7, sigma=2.0, corr=2.0, config_id=51)
    else:
        prob = inputs.anisotropic_problem(7, sigma=1.5, ratio=10.0, config_id=52)
    kw = dict(variant="static", static_level=level, static_axis=axis)
    o = mhfe.assemble(prob)
    E = oedfa.build(o, oedfa.Params(**kw))
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    from test_gpu_midsize import _cmp
    ne, nfu = o.ne, o.nfu
    _cmp(_to_sp(*P.export("G")[:3], (ne, nfu)), E.st1.Gt, 1e-10, "G~")
    _cmp(_to_sp(*P.export("FT")[:3], (ne, nfu)), E.st1.Ft.T, 1e-10, "F~^T")
    _cmp(_to_sp(*P.export("H_raw")[:3], (ne, ne)), E.st1.H_raw, 1e-10, "H~ raw")
    _cmp(_to_sp(*P.export("S")[:3], (ne, ne)), E.st2.S, 1e-10, "S~")
    rp, col, val, perm = P.export("L")
    assert np.array_equal(perm.cpu().numpy(), E.st2.perm), "colour permutation differs"
    _cmp(_to_sp(rp, col, val, (ne, ne)), E.st2.L, 1e-9, "L")
    _cmp(_to_sp(*P.export("U")[:3], (ne, ne)), E.st2.U, 1e-9, "U")
    _cmp(_to_sp(*P.export("ML")[:3], (ne, ne)), E.st2.ML, 1e-9, "M_L")
    _cmp(_to_sp(*P.export("MU")[:3], (ne, ne)), E.st2.MU, 1e-9, "M_U")
    _cmp(_to_sp(*P.export("GF")[:3], (nfu, nfu)), E.st1.GF, 1e-12, "G_F")
    r = np.random.default_rng(3).standard_normal(o.n)
    z = P.apply(torch.tensor(r, device="cuda")).cpu().numpy()
    ref = E.apply(r)
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-8)
    A = o.matrix()
    gm = krylov.gmres(lambda v: A @ v, E.apply, o.b, 1e-8, 50)
    xg = x.cpu().numpy()
    assert st == 0
    assert np.linalg.norm(xg[o.nfu:] - gm.x[o.nfu:]) <= 1e-8 * np.linalg.norm(gm.x[o.nfu:])
    assert abs(info["iterations"] - gm.iterations) <= 1


def test_parameter_tuner_picks_the_fastest_converged_candidate(lib):
    prob = inputs.full_tensor_problem(10, sigma=2.0, corr=3.0, config_id=53)
    S = lib.System(prob)
    cands = list(lib.DEFAULT_CANDIDATES) + [lib.Params("static", static_level=3)]  # too wide
    best, rec = lib.tune_params(S, cands, rtol=1e-8)
    times = [r["ms"] for r in rec]
    print("[tune params] " + ", ".join(f"{r['ms']:.1f} ms/{r['iterations']} it" for r in rec),
          flush=True)
    assert rec[-1]["status"] == -7 and math.isinf(rec[-1]["ms"])   # capacity: skipped
    finite = [t for t in times if math.isfinite(t)]
    assert len(finite) >= len(cands) - 1
    assert best == cands[int(np.argmin(times))]
    P = lib.Precond(S, best)
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-8)
    assert st == 0
