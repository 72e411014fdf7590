"""GPU parity of the EDFA setup, application and GMRES against the oracle (FP64).

Sizes span several tiles / wavefront batches and include boundary (ragged) rows.
Tolerances: structural patterns, colourings and permutations bit-exact; FP64 values
within 1e-10 relative to the row scale (different but equally valid summation orders
in the restricted Cholesky solves and the triple product); solutions to the north-star
1e-8 relative pressure tolerance.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import edfa as oedfa, krylov, mhfe
from paper_2009_13916_amd import inputs

pytestmark = pytest.mark.gpu

CASES = {
    "iso8_dyn14": (lambda: inputs.lognormal_iso_problem(8, config_id=21),
                   dict(variant="dynamic", n_add=1, n_ent=4)),
    "iso7_static": (lambda: inputs.lognormal_iso_problem(7, sigma=2.0, config_id=22),
                    dict(variant="static")),
    "full5_dyn16_postH": (lambda: inputs.full_tensor_problem(5, 4, 6, sigma=2.0, corr=2.0, config_id=23),
                          dict(variant="dynamic", n_add=1, n_ent=6, tau=1e-3, filt="post_H")),
    "dist5_dyn26_pre": (lambda: inputs.channel_problem(5, 6, 4, contrast=1e4, config_id=24),
                        dict(variant="dynamic", n_add=2, n_ent=6, tau=1e-3, filt="pre")),
    "iso6_patch1_postS": (lambda: inputs.lognormal_iso_problem(6, config_id=25),
                          dict(variant="static", static_level=1, tau=1e-2, filt="post_S")),
}

_cache = {}


def _build(name):
    if name not in _cache:
        mk, kw = CASES[name]
        prob = mk()
        o = mhfe.assemble(prob)
        E = oedfa.build(o, oedfa.Params(**kw))
        _cache[name] = (prob, o, E, kw)
    return _cache[name]


def _to_sp(rp, col, val, shape):
    return sp.csr_matrix((val.cpu().numpy(), col.cpu().numpy(), rp.cpu().numpy()), shape=shape)


def _cmp(G, O, tol, what):
    G = G.tocsr(); O = O.tocsr()
    G.sort_indices(); O.sort_indices()
    assert G.shape == O.shape, what
    assert np.array_equal(G.indptr, O.indptr), f"{what}: row lengths differ"
    assert np.array_equal(G.indices, O.indices), f"{what}: columns differ"
    scale = np.maximum(abs(O).max(axis=1).toarray().ravel(), 1e-300)
    rows = np.repeat(np.arange(O.shape[0]), np.diff(O.indptr))
    err = np.abs(G.data - O.data) / scale[rows] if O.nnz else np.zeros(0)
    assert err.size == 0 or err.max() <= tol, f"{what}: max rel err {err.max():.3e}"


@pytest.mark.parametrize("name", list(CASES))
def test_stage1_and_stage2_artefacts(lib, name):
    prob, o, E, kw = _build(name)
    print(f"[edfa parity] {name}", flush=True)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    ne, nfu = o.ne, o.nfu
    _cmp(_to_sp(*P.export("G")[:3], (ne, nfu)), E.st1.Gt, 1e-10, "G~")
    _cmp(_to_sp(*P.export("FT")[:3], (ne, nfu)), E.st1.Ft.T, 1e-10, "F~^T")
    _cmp(_to_sp(*P.export("H_raw")[:3], (ne, ne)), E.st1.H_raw, 1e-10, "H~ raw")
    _cmp(_to_sp(*P.export("H")[:3], (ne, ne)), E.st1.H, 1e-10, "H~")
    _cmp(_to_sp(*P.export("GF")[:3], (nfu, nfu)), E.st1.GF, 1e-12, "G_F")
    _cmp(_to_sp(*P.export("S")[:3], (ne, ne)), E.st2.S, 1e-10, "S~")
    rp, col, val, perm = P.export("L")
    assert np.array_equal(perm.cpu().numpy(), E.st2.perm), "colour permutation differs"
    _cmp(_to_sp(rp, col, val, (ne, ne)), E.st2.L, 1e-9, "L")
    _cmp(_to_sp(*P.export("U")[:3], (ne, ne)), E.st2.U, 1e-9, "U")
    _cmp(_to_sp(*P.export("ML")[:3], (ne, ne)), E.st2.ML, 1e-9, "M_L")
    _cmp(_to_sp(*P.export("MU")[:3], (ne, ne)), E.st2.MU, 1e-9, "M_U")
    info = P.info()
    assert info["n_colors"] == E.st2.color.max() + 1
    assert abs(info["mu"] - E.density()) < 1e-12


def _entrywise(z, ref, tol, what):
    """Entry-wise agreement beside the norm-wise one (a few wrong entries in a region of small
    values hide in a norm): every entry above 1e-6 of the largest agrees to `tol` relative,
    the smaller ones to `tol` of 1e-6 of the largest."""
    big = np.abs(ref).max()
    err = np.abs(z - ref) / np.maximum(np.abs(ref), 1e-6 * big)
    assert err.max() <= tol, f"{what}: entry {err.argmax()} rel err {err.max():.3e}"


@pytest.mark.parametrize("name", ["iso8_dyn14", "full5_dyn16_postH", "dist5_dyn26_pre"])
@pytest.mark.parametrize("transpose", [False, True])
def test_apply_matches_oracle(lib, name, transpose):
    import torch
    prob, o, E, kw = _build(name)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    r = np.random.default_rng(5).standard_normal(o.n)
    z = P.apply(torch.tensor(r, device="cuda"), transpose=transpose).cpu().numpy()
    ref = E.apply_T(r) if transpose else E.apply(r)
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)
    _entrywise(z, ref, 1e-8, "apply")


@pytest.mark.parametrize("steps", [2, 3])
def test_isai_refinement_steps(lib, steps):
    import torch
    prob = inputs.full_tensor_problem(4, 5, 4, sigma=1.5, corr=2.0, config_id=26)
    o = mhfe.assemble(prob)
    kw = dict(variant="dynamic", n_add=1, n_ent=4, isai_steps=steps)
    E = oedfa.build(o, oedfa.Params(**kw))
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    r = np.random.default_rng(6).standard_normal(o.n)
    for tr in (False, True):
        z = P.apply(torch.tensor(r, device="cuda"), transpose=tr).cpu().numpy()
        ref = E.apply_T(r) if tr else E.apply(r)
        assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)


def test_exact_substitution_variant(lib):
    import torch
    prob = inputs.lognormal_iso_problem(6, sigma=1.5, config_id=27)
    o = mhfe.assemble(prob)
    kw = dict(variant="dynamic", n_add=1, n_ent=4, schur="exact")
    E = oedfa.build(o, oedfa.Params(**kw))
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    r = np.random.default_rng(7).standard_normal(o.n)
    for tr in (False, True):
        z = P.apply(torch.tensor(r, device="cuda"), transpose=tr).cpu().numpy()
        ref = E.apply_T(r) if tr else E.apply(r)
        assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", ["iso8_dyn14", "iso7_static", "full5_dyn16_postH", "dist5_dyn26_pre"])
def test_gmres_matches_oracle(lib, name):
    """P1: same parameters, x0 = 0, same pattern -> pressures within 1e-8 relative and
    iteration counts within +-1 (static) / +-2 (dynamic); P2: true residual <= 1e-8."""
    prob, o, E, kw = _build(name)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    b = S.rhs()
    x, info, st = lib.solve(S, P, b, rtol=1e-8, restart=50)
    A = o.matrix()
    ref = krylov.gmres(lambda v: A @ v, E.apply, o.b, 1e-8, 50)
    xg = x.cpu().numpy()
    assert st == 0 and info["converged"] == 1
    assert np.linalg.norm(o.b - A @ xg) <= 1e-8 * np.linalg.norm(o.b)
    p_rel = np.linalg.norm(xg[o.nfu:] - ref.x[o.nfu:]) / np.linalg.norm(ref.x[o.nfu:])
    assert p_rel <= 1e-8, p_rel
    _entrywise(xg[o.nfu:], ref.x[o.nfu:], 1e-6, "pressure")
    tol = 1 if kw["variant"] == "static" else 2
    assert abs(info["iterations"] - ref.iterations) <= tol, (info["iterations"], ref.iterations)


def test_gmres_tight_tolerance_reaches_direct_solution(lib):
    """P2 at 1e-12: the GPU solution is within 1e-8 of the direct solve u*."""
    prob, o, E, kw = _build("iso8_dyn14")
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-12, restart=50)
    u = mhfe.direct_solve(o)
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg[o.nfu:] - u[o.nfu:]) <= 1e-8 * np.linalg.norm(u[o.nfu:])


def test_not_converged_status(lib):
    prob, o, E, kw = _build("iso8_dyn14")
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-12, restart=5, max_iter=3)
    assert st == lib.NOT_CONVERGED and info["converged"] == 0 and info["iterations"] == 3


def test_batched_solve_matches_individual(lib):
    """A batch of uneven grids: every grid converges on its own residual, and the batch solution
    equals the per-grid oracle solutions to 1e-8."""
    probs = [inputs.lognormal_iso_problem(n, sigma=s, config_id=4, extra=i)
             for i, (n, s) in enumerate([(5, 0.5), (7, 2.5), (6, 1.0)])]
    kw = dict(variant="dynamic", n_add=1, n_ent=4)
    S = lib.System(probs)
    P = lib.Precond(S, lib.Params(**kw))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-8, restart=50)
    assert st == 0 and info["converged"] == 3
    xg = x.cpu().numpy()
    nfu_tot = S.info["nfu"]
    fo = co = 0
    for p in probs:
        o = mhfe.assemble(p)
        E = oedfa.build(o, oedfa.Params(**kw))
        A = o.matrix()
        ref = krylov.gmres(lambda v: A @ v, E.apply, o.b, 1e-8, 50)
        pg = xg[nfu_tot + co: nfu_tot + co + o.ne]
        assert np.linalg.norm(pg - ref.x[o.nfu:]) <= 1e-8 * np.linalg.norm(ref.x[o.nfu:])
        fo += o.nfu
        co += o.ne
