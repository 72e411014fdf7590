"""GPU parity at the full 64^3 full-tensor workload, in the configuration the benchmark times
(dynamic patterns with n_add = 1 and n_ent = 6, post-filtration of H~ at 1e-3), on outputs
the oracle computes one at a time: the restricted solves of a seeded sample of cells
(Algorithm 1: the final pattern Q, g~ and f~ of each sampled cell, eq. prol_res for the
growth of Q), and the true residual of the GMRES solution with the oracle's own matrix."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import edfa as oedfa
from oracle import mhfe
from paper_2009_13916_amd import inputs

pytestmark = pytest.mark.gpu

KW = dict(variant="dynamic", n_add=1, n_ent=6, tau=1e-3, filt="post_H")


@pytest.fixture(scope="module")
def full64():
    prob = inputs.full_tensor_problem(64)
    print("[full size] oracle assembly of the 64^3 workload", flush=True)
    o = mhfe.assemble(prob)
    # the restricted solves read column m of A_pip as a row of its transpose
    o.ApcT = o.Apc.T.tocsr()
    o.ApcT.sort_indices()
    return prob, o


def _rows(P, name, shape):
    rp, col, val = (t.cpu().numpy() for t in P.export(name)[:3])
    M = sp.csr_matrix((val, col, rp), shape=shape)
    M.sort_indices()
    return M


def test_sampled_restricted_solves_at_full_size(lib, full64):
    """48 seeded cells of the 1,052,672-unknown system: the GPU's final pattern of each is
    the oracle's (bit-exact), g~ and f~ agree to 1e-10 of the row's largest entry.  A wrong
    candidate rule, a dropped residual term or a transposed block changes the pattern or
    the values of most cells."""
    prob, o = full64
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**KW))
    G = _rows(P, "G", (o.ne, o.nfu))
    F = _rows(P, "FT", (o.ne, o.nfu))
    prm = oedfa.Params(**KW)
    cells = np.random.default_rng(2009).choice(o.ne, 48, replace=False)
    print(f"[full size] oracle restricted solves of {cells.size} cells", flush=True)
    for m in cells.tolist():
        cr = oedfa.local_cell(o, m, prm)
        order = np.argsort(cr.Q)
        for M, ref, what in ((G, cr.g, "g~"), (F, cr.f, "f~")):
            a, e = M.indptr[m], M.indptr[m + 1]
            assert np.array_equal(M.indices[a:e], cr.Q[order]), f"cell {m}: pattern of {what}"
            scale = np.abs(ref).max()
            err = np.abs(M.data[a:e] - ref[order]).max() / scale
            assert err <= 1e-10, f"cell {m}: {what} rel err {err:.2e}"


def test_full_size_solution_against_oracle_matrix(lib, full64):
    """The benchmark's solve (GMRES(50) to 1e-8) checked with the oracle's assembly: its
    true residual with the oracle's matrix.  The solver stops on its own product, whose
    entries agree with the oracle's to 1e-12 of each row's largest, so the bound carries a
    1% margin."""
    prob, o = full64
    S = lib.System(prob)
    P = lib.Precond(S, lib.Params(**KW))
    x, info, st = lib.solve(S, P, S.rhs(), rtol=1e-8, restart=50)
    xg = x.cpu().numpy()
    assert st == 0 and info["converged"] == 1
    rel = np.linalg.norm(o.b - o.matrix() @ xg) / np.linalg.norm(o.b)
    print(f"[full size] {info['iterations']} iterations, true residual with the oracle's "
          f"matrix {rel:.3e}", flush=True)
    assert rel <= 1.01e-8, rel
