"""The launch-shape autotuner: it changes only which kernel (and therefore the rounding order)
computes each sparse product, so tuned solves must agree with untuned ones to the solver
tolerance, and the choice must survive a re-setup."""
import numpy as np
import pytest

from oracle import mhfe
from paper_2009_13916_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
def test_autotuned_solve_matches_untuned(lib, precision):
    prob = inputs.full_tensor_problem(8, sigma=2.0, corr=2.0, config_id=71)
    o = mhfe.assemble(prob)
    u = mhfe.direct_solve(o)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params("dynamic", n_add=1, n_ent=6, precision=precision))
    flex = precision == 1
    b = S.rhs()
    x0, i0, s0 = lib.solve(S, P, b, rtol=1e-12, flexible=flex)
    rep = P.autotune(report=True)
    # without refinement steps the application needs no copies of L and U themselves
    assert {"A", "G_F", "G_F^T", "M_L", "M_U", "A_ppi", "A_pip"} <= set(rep)
    assert "L" not in rep and "U" not in rep
    for name, r in rep.items():
        vb = 8 if name in ("A", "A^T") or not flex else 4   # the operator stays FP64
        assert r["value_bytes"] == vb and len(r["us"]) == len(lib.TUNE_VARIANTS)
        assert all(t > 0 for t in r["us"].values())
        # the default kernel stays unless another is at least 3% faster
        assert r["us"][r["variant"]] * 0.97 <= min(r["us"].values()) * (1 + 1e-6)
    assert rep["A"]["rows"] == rep["A"]["cols"] == S.n and rep["A"]["nnz"] == S.info["nnz"]
    x1, i1, s1 = lib.solve(S, P, b, rtol=1e-12, flexible=flex)
    lam, il, sl = lib.solve(S, P, b, rtol=1e-12, flexible=flex, transpose=True)
    P.resetup()
    x2, i2, s2 = lib.solve(S, P, b, rtol=1e-12, flexible=flex)
    assert s0 == s1 == s2 == sl == 0
    for x in (x0, x1, x2):
        xg = x.cpu().numpy()
        assert np.linalg.norm(xg[o.nfu:] - u[o.nfu:]) <= 1e-8 * np.linalg.norm(u[o.nfu:])
    assert abs(i1["iterations"] - i0["iterations"]) <= 2
    lam_ref = mhfe.spla.splu(o.matrix().T.tocsc()).solve(b.cpu().numpy())
    assert np.linalg.norm(lam.cpu().numpy() - lam_ref) <= 1e-8 * np.linalg.norm(lam_ref)


def test_setup_buckets_and_tuner(lib):
    """A batch of an isotropic grid (patterns of up to 16 entries) and a full-tensor grid (up
    to 44, fewer next to the boundary) fills several capacity buckets, each one launch of its
    own kernel; the application matches the per-grid oracle.  The setup tuner times every
    bucket, keeps a capacity no smaller than the bucket's own, and a re-setup with its
    choice still matches."""
    import torch
    from oracle import edfa as oedfa
    probs = [inputs.lognormal_iso_problem(6, sigma=1.0, config_id=72),
             inputs.full_tensor_problem(6, 5, 7, sigma=2.0, corr=2.0, config_id=73)]
    kw = dict(variant="dynamic", n_add=1, n_ent=6)
    S = lib.System(probs)
    P = lib.Precond(S, lib.Params(**kw))
    rep = P.autotune_setup()
    print("[setup tuner] " + "; ".join(f"cap {b['capacity']}: {b['cells']} cells -> {b['chosen']} "
                                       f"{b['us']}" for b in rep), flush=True)
    assert len(rep) >= 3
    assert sum(b["cells"] for b in rep) == S.info["ne"]
    for b in rep:
        assert b["chosen"] >= b["capacity"] and b["capacity"] in b["us"]
    P.resetup()
    r = np.random.default_rng(11).standard_normal(S.info["n"])
    z = P.apply(torch.tensor(r, device="cuda")).cpu().numpy()
    nfu_tot = S.info["nfu"]
    f0 = c0 = 0
    for p in probs:
        o = mhfe.assemble(p)
        E = oedfa.build(o, oedfa.Params(**kw))
        rg = np.concatenate([r[f0:f0 + o.nfu], r[nfu_tot + c0:nfu_tot + c0 + o.ne]])
        zg = np.concatenate([z[f0:f0 + o.nfu], z[nfu_tot + c0:nfu_tot + c0 + o.ne]])
        ref = E.apply(rg)
        assert np.linalg.norm(zg - ref) <= 1e-10 * np.linalg.norm(ref)
        f0 += o.nfu
        c0 += o.ne


def test_cgs2_width_is_tuned(lib):
    prob = inputs.full_tensor_problem(12, sigma=2.0, corr=2.0, config_id=74)
    o = mhfe.assemble(prob)
    u = mhfe.direct_solve(o)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params("dynamic", n_add=1, n_ent=6))
    assert P.info()["cgs2_width"] == 4
    P.autotune()
    w = P.info()["cgs2_width"]
    assert w in (2, 4, 8)
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-12)
    assert st == 0
    assert np.linalg.norm(x.cpu().numpy() - u) <= 1e-9 * np.linalg.norm(u)
