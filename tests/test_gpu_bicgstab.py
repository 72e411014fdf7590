"""GPU Bi-CGStab (the paper's outer solver, Section 4) against the oracle Bi-CGStab with the same
EDFA (FP64): pressures within 1e-8 relative and iteration counts within +-2 at the same 1e-8
target, the true residual at the target, the direct solution at a tight target, the "NC" status
at an iteration cap, a batch equal to its grids solved one by one, the transposed system, and
the FP32 preconditioner."""
import numpy as np
import pytest
import torch

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
}


def _ref(prob, kw, rtol, transpose=False):
    o = mhfe.assemble(prob)
    E = oedfa.build(o, oedfa.Params(**kw))
    A = o.matrix()
    if transpose:
        At = A.T.tocsr()
        return o, krylov.bicgstab(lambda v: At @ v, E.apply_T, o.b, rtol, 2000)
    return o, krylov.bicgstab(lambda v: A @ v, E.apply, o.b, rtol, 2000)


@pytest.mark.parametrize("name", list(CASES))
def test_bicgstab_matches_oracle(lib, name):
    mk, kw = CASES[name]
    prob = mk()
    print(f"[bicgstab parity] {name}", flush=True)
    o, ref = _ref(prob, kw, 1e-8)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-8, max_iter=2000, method="bicgstab")
    xg = x.cpu().numpy()
    A = o.matrix()
    assert st == 0 and info["converged"] == 1
    assert np.linalg.norm(o.b - A @ xg) <= 1e-8 * np.linalg.norm(o.b)
    assert info["relres_true"] <= 1e-8
    assert abs(info["iterations"] - ref.iterations) <= 2, (info["iterations"], ref.iterations)
    p_rel = np.linalg.norm(xg[o.nfu:] - ref.x[o.nfu:]) / np.linalg.norm(ref.x[o.nfu:])
    assert p_rel <= 1e-8, p_rel
    # entry-wise beside the norm: entries above 1e-6 of the largest to 1e-6 relative
    p, q = xg[o.nfu:], ref.x[o.nfu:]
    err = np.abs(p - q) / np.maximum(np.abs(q), 1e-6 * np.abs(q).max())
    print(f"[bicgstab parity] {name}: pressure entry-wise max rel err {err.max():.2e}", flush=True)
    assert err.max() <= 1e-6, err.max()


def test_bicgstab_tight_target_reaches_direct_solution(lib):
    mk, kw = CASES["iso8_dyn14"]
    prob = mk()
    o = mhfe.assemble(prob)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-12, max_iter=2000, method="bicgstab")
    u = mhfe.direct_solve(o)
    xg = x.cpu().numpy()
    assert st == 0
    assert np.linalg.norm(xg[o.nfu:] - u[o.nfu:]) <= 1e-8 * np.linalg.norm(u[o.nfu:])


def test_bicgstab_not_converged_at_cap(lib):
    mk, kw = CASES["iso8_dyn14"]
    S = lib.System(mk())
    P = lib.Precond(S, lib.Params(**kw))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-14, max_iter=3, method="bicgstab")
    assert st == lib.NOT_CONVERGED and info["converged"] == 0 and info["iterations"] == 3
    assert torch.isfinite(x).all()


def test_bicgstab_transposed_matches_oracle(lib):
    mk, kw = CASES["full5_dyn16_postH"]
    prob = mk()
    o, ref = _ref(prob, kw, 1e-8, transpose=True)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-8, max_iter=2000, transpose=True,
                            method="bicgstab")
    xg = x.cpu().numpy()
    At = o.matrix().T.tocsr()
    assert st == 0
    assert np.linalg.norm(o.b - At @ xg) <= 1e-8 * np.linalg.norm(o.b)
    assert abs(info["iterations"] - ref.iterations) <= 2
    p_rel = np.linalg.norm(xg[o.nfu:] - ref.x[o.nfu:]) / np.linalg.norm(ref.x[o.nfu:])
    assert p_rel <= 1e-8, p_rel


def test_bicgstab_batch_equals_individual(lib):
    probs = [inputs.lognormal_iso_problem(n, sigma=s, config_id=4, extra=i)
             for i, (n, s) in enumerate([(5, 0.5), (7, 2.5), (6, 1.0)])]
    kw = dict(variant="dynamic", n_add=1, n_ent=4)
    S = lib.System(probs)
    P = lib.Precond(S, lib.Params(**kw))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-8, max_iter=2000, method="bicgstab")
    assert st == 0 and info["converged"] == 3
    xg = x.cpu().numpy()
    nfu_tot = S.info["nfu"]
    co = 0
    its = []
    for p in probs:
        S1 = lib.System(p)
        P1 = lib.Precond(S1, lib.Params(**kw))
        x1, i1, st1 = lib.solve(S1, P1, S1.rhs(), rtol=1e-8, max_iter=2000, method="bicgstab")
        ne, nfu = S1.info["ne"], S1.info["nfu"]
        p1 = x1.cpu().numpy()[nfu:]
        pg = xg[nfu_tot + co: nfu_tot + co + ne]
        # the batch is the grids side by side (summation orders of the products may differ
        # with the launch shapes chosen for the batch)
        assert np.linalg.norm(pg - p1) <= 1e-8 * np.linalg.norm(p1)
        its.append(i1["iterations"])
        co += ne
    assert abs(info["iterations"] - max(its)) <= 2


def test_bicgstab_fp32_preconditioner(lib):
    mk, kw = CASES["full5_dyn16_postH"]
    prob = mk()
    o = mhfe.assemble(prob)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**kw, precision=1))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-8, max_iter=2000, method="bicgstab")
    xg = x.cpu().numpy()
    assert st == 0
    assert np.linalg.norm(o.b - o.matrix() @ xg) <= 1e-8 * np.linalg.norm(o.b)
    with pytest.raises(lib.EdfaError):
        lib.solve(S, P, S.rhs(), method="bicgstab", use_graph=True)
