"""Every sparse-product kernel variant (SELL with 4 or 8 entries in flight, on the plain or the
length-sorted layout; CSR with 2..32 lanes per row and 2 or 4 entries in flight; the chunk
kernel on matrices with long rows) computes the same products: pinned on every matrix, the
EDFA application, its transpose and a GMRES solve match the oracle, for one grid and for a
batch whose converged grids are masked."""
import numpy as np
import pytest
import torch

from oracle import edfa as oedfa, mhfe
from paper_2009_13916_amd import inputs
from paper_2009_13916_amd.edfa import TUNE_VARIANTS

pytestmark = pytest.mark.gpu

PRM = dict(variant="dynamic", n_add=1, n_ent=6, tau=1e-3, filt="post_H")


@pytest.fixture(scope="module")
def case():
    prob = inputs.full_tensor_problem(9, 8, 7, sigma=2.0, corr=2.0, config_id=73)
    o = mhfe.assemble(prob)
    E = oedfa.build(o, oedfa.Params(**PRM))
    return prob, o, E, mhfe.direct_solve(o)


@pytest.mark.parametrize("v", range(len(TUNE_VARIANTS)))
def test_pinned_variant_matches_oracle(lib, case, v):
    prob, o, E, u = case
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**PRM))
    rep = P.autotune(report=True)
    # rows of very different lengths (the ISAI factors): the SELL copies are sorted, and the
    # chunk kernel (their default) runs on them
    assert rep["M_L"]["sell_sorted"] and rep["M_U"]["sell_sorted"]
    assert np.isfinite(rep["M_L"]["us"]["chunk/12"]) and np.isfinite(rep["M_U"]["us"]["chunk/12"])
    assert not np.isfinite(rep["G_F"]["us"]["chunk/12"])
    P.set_variant(v)
    r = np.random.default_rng(v).standard_normal(o.n)
    rt = torch.tensor(r, device="cuda")
    z = P.apply(rt).cpu().numpy()
    zr = E.apply(r)
    assert np.linalg.norm(z - zr) <= 1e-10 * np.linalg.norm(zr), lib.variant_name(v)
    zt = P.apply(rt, transpose=True).cpu().numpy()
    ztr = E.apply_T(r)
    assert np.linalg.norm(zt - ztr) <= 1e-10 * np.linalg.norm(ztr), lib.variant_name(v)
    y = S.spmv(rt).cpu().numpy()
    assert np.linalg.norm(y - o.matrix() @ r) <= 1e-13 * np.linalg.norm(o.matrix() @ r)
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-12)
    assert st == 0
    assert np.linalg.norm(x.cpu().numpy() - u) <= 1e-9 * np.linalg.norm(u)


@pytest.mark.parametrize("name", ["sell/4", "sell/8", "csr8/4"])
def test_pinned_variant_batch_with_masks(lib, name):
    """Grids of very different difficulty: the easy ones converge first and their rows are
    masked in every product while the others iterate."""
    probs = [inputs.lognormal_iso_problem(4, sigma=0.3, config_id=74),
             inputs.full_tensor_problem(7, sigma=2.5, corr=2.0, config_id=75),
             inputs.lognormal_iso_problem(5, sigma=0.5, config_id=76)]
    kw = dict(variant="dynamic", n_add=1, n_ent=4)
    S = lib.System(probs)
    P = lib.Precond(S, lib.Params(**kw))
    P.set_variant(name)
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-10)
    assert st == 0 and info["converged"] == 3
    xg = x.cpu().numpy()
    nfu = S.info["nfu"]
    f0 = c0 = 0
    for p in probs:
        o = mhfe.assemble(p)
        u = mhfe.direct_solve(o)
        xs = np.concatenate([xg[f0:f0 + o.nfu], xg[nfu + c0:nfu + c0 + o.ne]])
        assert np.linalg.norm(xs - u) <= 1e-8 * np.linalg.norm(u)
        f0 += o.nfu
        c0 += o.ne


def test_chunk_kernel_batch_with_masks(lib):
    """The chunk kernel on the long rows of a full-tensor batch whose easy grids converge
    first: chunks of whole rows can straddle two grids, and the masked rows are skipped."""
    probs = [inputs.full_tensor_problem(4, sigma=0.3, corr=1.0, config_id=78),
             inputs.full_tensor_problem(7, sigma=2.5, corr=2.0, config_id=75),
             inputs.full_tensor_problem(5, sigma=0.5, corr=1.0, config_id=79)]
    kw = dict(variant="dynamic", n_add=1, n_ent=6)
    S = lib.System(probs)
    P = lib.Precond(S, lib.Params(**kw))
    rep = P.autotune(report=True)
    assert np.isfinite(rep["M_L"]["us"]["chunk/12"])
    P.set_variant("chunk/12")
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-10)
    assert st == 0 and info["converged"] == 3
    xg = x.cpu().numpy()
    nfu = S.info["nfu"]
    f0 = c0 = 0
    for p in probs:
        o = mhfe.assemble(p)
        u = mhfe.direct_solve(o)
        xs = np.concatenate([xg[f0:f0 + o.nfu], xg[nfu + c0:nfu + c0 + o.ne]])
        assert np.linalg.norm(xs - u) <= 1e-8 * np.linalg.norm(u)
        f0 += o.nfu
        c0 += o.ne


def test_set_variant_rejects_out_of_range(lib):
    prob = inputs.lognormal_iso_problem(4, config_id=77)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(variant="dynamic", n_add=1, n_ent=4))
    with pytest.raises(lib.EdfaError):
        P.set_variant(len(lib.TUNE_VARIANTS))
    with pytest.raises(lib.EdfaError):
        P.set_variant(0, slot=16)
    P.set_variant(None)   # back to the defaults


def _greedy_chunks(rp, cap):
    """Row-aligned greedy cut: close the chunk before the first row that would take it past
    `cap` entries (a longer row alone)."""
    n, r0 = 1, 0
    for r in range(len(rp) - 1):
        if r > r0 and rp[r + 1] - rp[r0] > cap:
            n, r0 = n + 1, r
    return n


def test_chunk_descriptors_match_the_greedy_cut(lib):
    """The chunk kernel's descriptors, computed on the device by pointer doubling, hold as
    many chunks as the sequential greedy cut of the natural-order rows of M_L and M_U."""
    prob = inputs.full_tensor_problem(16, 14, 12, sigma=2.0, corr=3.0, config_id=77)
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**PRM))
    info = P.info()
    for name, key in (("ML", "chunks_ML"), ("MU", "chunks_MU")):
        rp, col, val, perm = P.export(name)
        lens = torch.diff(rp).cpu().numpy()
        nat = np.zeros_like(lens)
        nat[perm.cpu().numpy()] = lens
        rpn = np.concatenate([[0], np.cumsum(nat)])
        assert info[key] == _greedy_chunks(rpn, 768) > 8, (name, info[key])
