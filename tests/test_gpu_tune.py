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
