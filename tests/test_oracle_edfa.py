"""Pins for the EDFA oracle (Section 3, Algorithms 1-2, Proposition 1, Remarks 1-5)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import edfa, krylov, mhfe
from oracle.edfa import unit_lower as oedfa_unit
from paper_2009_13916_amd import inputs


@pytest.fixture(scope="module")
def small_full():
    prob = inputs.full_tensor_problem(4, 3, 3, sigma=1.5, corr=2.0, config_id=81)
    return mhfe.assemble(prob)


@pytest.fixture(scope="module")
def small_iso():
    prob = inputs.lognormal_iso_problem(5, sigma=1.0, config_id=82)
    return mhfe.assemble(prob)


def _own_faces(s, m):
    u = s.uidx[s.topo.cell_faces[m]]
    return u[u >= 0]


def _cvec(s, m):
    """Row m of C: C[m, i] = W_ii/(W_ii + W'_ii) (interior), 1 (Neumann) on own faces."""
    out = {}
    for a in range(6):
        u = s.uidx[s.topo.cell_faces[m, a]]
        if u >= 0:
            out[int(u)] = s.Dcoef[m, a]
    return out


@pytest.mark.parametrize("variant", ["static", "dynamic"])
def test_g_equals_cQ_minus_f(small_full, variant):
    """With the own faces in Q, R a_ppi = -R a_pip - R A_pipi c_m gives g~ = c_Q - f~
    (from A_ppi = -A_pip^T - C A_pipi, the exact row-combination identity)."""
    s = small_full
    edfa._ensure_apct(s)
    prm = edfa.Params(variant, n_add=2, n_ent=4)
    for m in range(0, s.ne, 5):
        cr = edfa.local_cell(s, m, prm)
        c = _cvec(s, m)
        cQ = np.array([c.get(int(q), 0.0) for q in cr.Q])
        np.testing.assert_allclose(cr.g, cQ - cr.f, atol=1e-12 * max(1, np.abs(cr.g).max()))


def test_proposition_1_energy_minimality(small_full):
    """The restricted solution minimises the A-energy norm of the error among all vectors
    supported on Q (Proposition 1): random perturbations on Q never lower it."""
    s = small_full
    edfa._ensure_apct(s)
    A = -s.App.toarray()
    rng = np.random.default_rng(0)
    for m in (0, 7, 20):
        cr = edfa.local_cell(s, m, edfa.Params("dynamic", n_add=1, n_ent=3))
        b = s.Acp[m].toarray().ravel()
        xstar = np.linalg.solve(A, b)

        def energy(xq):
            e = xstar.copy()
            e[cr.Q] -= xq
            return e @ A @ e

        e0 = energy(cr.g)
        for _ in range(20):
            d = rng.standard_normal(len(cr.Q)) * 1e-3 * np.abs(cr.g).max()
            assert energy(cr.g + d) >= e0 - 1e-14 * abs(e0)


def test_prolonged_residual_vanishes_on_Q_and_support_remark_3(small_full):
    """r = a + A R^T g~ is zero on Q (restricted system solved) and supported on the faces of
    the cells sharing a face with Q (Remark 3)."""
    s = small_full
    edfa._ensure_apct(s)
    topo = s.topo
    for m in range(0, s.ne, 3):
        cr = edfa.local_cell(s, m, edfa.Params("static"))
        a_idx, a_val = s.Acp.indices[s.Acp.indptr[m]:s.Acp.indptr[m + 1]], s.Acp.data[s.Acp.indptr[m]:s.Acp.indptr[m + 1]]
        idx, r = edfa.prolonged_residual(s, a_idx, a_val, cr.Q, cr.g)
        onq = np.isin(idx, cr.Q)
        assert np.abs(r[onq]).max() <= 1e-12 * np.abs(r).max()
        allowed = set()
        for q in cr.Q:
            f = s.ufaces[q]
            for e in topo.face_cells[f]:
                if e >= 0:
                    allowed.update(int(u) for u in s.uidx[topo.cell_faces[e]] if u >= 0)
        assert set(idx[r != 0].tolist()) <= allowed


def test_exact_factor_identities(small_full):
    """G = -A_ppi A_pipi^-1 = C - F^T and S = A_pp - G A_pipi F is symmetric positive definite
    (it equals the Schur complement of the classical hybridised system)."""
    s = small_full
    App = s.App.toarray()
    G = -s.Acp.toarray() @ np.linalg.inv(App)
    F = -np.linalg.solve(App, s.Apc.toarray())
    C = np.zeros((s.ne, s.nfu))
    for m in range(s.ne):
        for k, v in _cvec(s, m).items():
            C[m, k] = v
    np.testing.assert_allclose(G, C - F.T, atol=1e-12)
    S = s.Acc.toarray() - G @ App @ F
    np.testing.assert_allclose(S, S.T, atol=1e-12 * abs(S).max())
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() > 0


def test_full_pattern_gives_exact_factors_and_one_step_solve():
    """Q = all faces: G~ = G, F~ = F, S~ = S (eqs. dec_fac, schur_compl); with exact inner
    solves P^-1 = A^-1 (eq. inv_A_fac) and GMRES converges in one iteration."""
    prob = inputs.full_tensor_problem(2, 2, 2, sigma=1.0, corr=1.0, config_id=83)
    s = mhfe.assemble(prob)
    prm = edfa.Params("static", static_level=4)
    st1 = edfa.stage1(s, prm)
    App = s.App.toarray()
    G = -s.Acp.toarray() @ np.linalg.inv(App)
    F = -np.linalg.solve(App, s.Apc.toarray())
    np.testing.assert_allclose(st1.Gt.toarray(), G, atol=1e-11)
    np.testing.assert_allclose(st1.Ft.toarray(), F, atol=1e-11)
    S = s.Acc.toarray() - s.Acp.toarray() @ np.linalg.solve(App, s.Apc.toarray())
    st2 = edfa.stage2(s, st1, prm)
    np.testing.assert_allclose(st2.S.toarray(), S, atol=1e-11 * abs(S).max())
    E = edfa.Edfa(s, prm, st1, st2)
    E.apply_App_inv = lambda v: np.linalg.solve(App, v)
    Sinv = np.linalg.inv(st2.S.toarray())
    E.apply_S_inv = lambda y: Sinv @ y
    A = s.matrix()
    res = krylov.gmres(lambda v: A @ v, E.apply, s.b, 1e-10, 50)
    assert res.iterations == 1 and res.converged


def test_ilu0_defining_property(small_full):
    """ILU(0): (L U)_ij = B_ij on the pattern of B, L unit lower and U upper on that pattern."""
    s = small_full
    prm = edfa.Params("static")
    st1 = edfa.stage1(s, prm)
    st2 = edfa.stage2(s, st1, prm)
    B = st2.S[st2.perm][:, st2.perm].toarray()
    n = B.shape[0]
    Lf = st2.L.toarray() + np.eye(n)
    U = st2.U.toarray()
    P = st2.S[st2.perm][:, st2.perm].tocsr()
    mask = np.zeros((n, n), bool)
    for i in range(n):
        mask[i, P.indices[P.indptr[i]:P.indptr[i + 1]]] = True
    LU = Lf @ U
    np.testing.assert_allclose(LU[mask], B[mask], atol=1e-12 * abs(B).max())
    assert not np.any(np.tril(st2.L.toarray() != 0) & ~mask)
    assert not np.any((U != 0) & ~mask)
    assert np.allclose(np.triu(st2.L.toarray()), 0) and np.allclose(np.tril(U, -1), 0)


def test_fsai_defining_property(small_full):
    """FSAI of M = -A_pipi: (G_F M)_ij = 0 for j in P_i, j != i, and (G_F M G_F^T)_ii = 1."""
    s = small_full
    GF = edfa.fsai(s).toarray()
    M = -s.App.toarray()
    GM = GF @ M
    pat = GF != 0
    off = pat & ~np.eye(len(M), dtype=bool)
    assert np.abs(GM[off]).max() < 1e-12 * np.abs(M).max()
    np.testing.assert_allclose(np.diag(GF @ M @ GF.T), 1.0, rtol=1e-12)
    assert np.allclose(np.triu(GF, 1), 0)


def test_coloring_is_valid_greedy(small_full):
    """Adjacent rows of S~ + S~^T never share a colour, and every vertex of colour c has, for
    each c' < c, a higher-priority neighbour of colour c' (first fit in priority order)."""
    s = small_full
    prm = edfa.Params("dynamic", n_add=1, n_ent=3)
    st1 = edfa.stage1(s, prm)
    S = edfa.structural_sub(s.Acc, st1.H)
    col = edfa.greedy_coloring(S)
    _check_structural_greedy(S, col)


def _check_structural_greedy(S, col):
    """Every stored entry (i, j) of S, explicit zeros included, is an edge of the graph."""
    S = S.tocsr()
    n = S.shape[0]
    nbrs = [set() for _ in range(n)]
    for i in range(n):
        for j in S.indices[S.indptr[i]:S.indptr[i + 1]]:
            if j != i:
                nbrs[i].add(int(j))
                nbrs[int(j)].add(i)
    pri = edfa.fmix32(np.arange(n)).astype(np.int64)
    for v in range(n):
        nb = np.array(sorted(nbrs[v]), dtype=np.int64)
        assert np.all(col[nb] != col[v])
        higher = nb[pri[nb] > pri[v]]
        assert set(range(col[v])) <= set(col[higher].tolist())


def test_coloring_counts_explicit_zeros_as_edges():
    """A pattern entry whose value is an exact zero (structural patterns keep them) is an edge:
    the two vertices get different colours.  A value-based graph would drop it."""
    n = 6
    rows = [0, 1, 2, 3, 4, 5, 0, 3, 1, 4]
    cols = [0, 1, 2, 3, 4, 5, 3, 0, 4, 1]
    vals = [4.0, 4.0, 4.0, 4.0, 4.0, 4.0, 0.0, 0.0, -1.0, -1.0]
    S = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    assert S.nnz == 10                           # the zeros are stored
    col = edfa.greedy_coloring(S)
    assert col[0] != col[3] and col[1] != col[4]
    _check_structural_greedy(S, col)


def test_filtration_keeps_diagonal_and_drops_small(small_full):
    s = small_full
    prm = edfa.Params("static", tau=0.05, filt="post_H")
    st1 = edfa.stage1(s, prm)
    Hr, H = st1.H_raw.tocsr(), st1.H.tocsr()
    for m in range(s.ne):
        rc, rv = Hr.indices[Hr.indptr[m]:Hr.indptr[m + 1]], Hr.data[Hr.indptr[m]:Hr.indptr[m + 1]]
        kc = set(H.indices[H.indptr[m]:H.indptr[m + 1]].tolist())
        nrm = np.linalg.norm(rv)
        for c, v in zip(rc, rv):
            assert (c in kc) == (abs(v) >= 0.05 * nrm or c == m)


def test_uniform_dynamic_patterns_in_homogeneous_media():
    """Homogeneous isotropic K: interior cells pick translation-equivalent dynamic patterns
    (Test 1 discussion of the dynamic (1,4) and (2,6) patterns)."""
    n = 8
    prob = inputs.lognormal_iso_problem(n, sigma=0.0, config_id=84)
    s = mhfe.assemble(prob)
    edfa._ensure_apct(s)
    topo = s.topo
    fcen = None
    shapes = set()
    for (na, ne_) in ((1, 4), (2, 6)):
        shapes = set()
        for k in range(3, n - 3):
            for j in range(3, n - 3):
                for i in range(3, n - 3):
                    m = i + n * (j + n * k)
                    cr = edfa.local_cell(s, m, edfa.Params("dynamic", n_add=na, n_ent=ne_))
                    # express the added faces relative to the cell: (face, cell offset)
                    rel = []
                    for q in cr.Q[len(edfa.base_pattern(s, m)):]:
                        f = s.ufaces[q]
                        e = topo.face_cells[f][topo.face_cells[f] >= 0].min()
                        ei, ej, ek = e % n, (e // n) % n, e // (n * n)
                        a = int(np.nonzero(topo.cell_faces[e] == f)[0][0])
                        rel.append((ei - i, ej - j, ek - k, a))
                    shapes.add(tuple(sorted(rel)))
        assert len(shapes) == 1, shapes


def test_transposed_edfa_is_transpose_of_forward(small_full):
    """EDFA built on the transposed blocks (A_pipi, A_ppi^T, A_pip^T, A_pp^T) with the same initial
    pattern has G~' = F~^T, F~' = G~^T, H~' = H~^T, and its ILU(0) product is (LU)^T."""
    s = small_full
    prm = edfa.Params("dynamic", n_add=1, n_ent=3, schur="exact")
    fwd = edfa.build(s, prm)
    import copy
    st = copy.copy(s)
    st.Apc, st.Acp, st.Acc = s.Acp.T.tocsr(), s.Apc.T.tocsr(), s.Acc.T.tocsr()
    st.ApcT = None
    for m_ in (st.Apc, st.Acp, st.Acc):
        m_.sort_indices()
    st1t = edfa.stage1(st, prm, base_rows=s.Acp)
    np.testing.assert_allclose(st1t.Gt.toarray(), fwd.st1.Ft.toarray().T, atol=1e-12)
    np.testing.assert_allclose(st1t.Ft.toarray(), fwd.st1.Gt.toarray().T, atol=1e-12)
    np.testing.assert_allclose(st1t.H.toarray(), fwd.st1.H.toarray().T, atol=1e-12)
    st2t = edfa.stage2(st, st1t, prm)
    assert np.array_equal(st2t.perm, fwd.st2.perm)
    n = s.ne
    LUf = (fwd.st2.L.toarray() + np.eye(n)) @ fwd.st2.U.toarray()
    LUt = (st2t.L.toarray() + np.eye(n)) @ st2t.U.toarray()
    np.testing.assert_allclose(LUt, LUf.T, atol=1e-11 * abs(LUf).max())
    # and the transposed application equals the transpose of the forward one
    N = s.n
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal(N), rng.standard_normal(N)
    assert abs(y @ fwd.apply(x) - x @ fwd.apply_T(y)) < 1e-11 * np.linalg.norm(x) * np.linalg.norm(y) * 1e3


@pytest.mark.parametrize("steps", [1, 2, 3])
def test_isai_transposed_application(small_full, steps):
    """y . P^-1 x = x . P^-T y for the ISAI variant with refinement steps."""
    s = small_full
    E = edfa.build(s, edfa.Params("dynamic", n_add=1, n_ent=3, isai_steps=steps))
    rng = np.random.default_rng(steps)
    x, y = rng.standard_normal(s.n), rng.standard_normal(s.n)
    lhs, rhs = y @ E.apply(x), x @ E.apply_T(y)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs) + 1e-12


def test_isai_defining_property(small_full):
    """ISAI M of a triangular T: (M T)_ij = delta_ij for j in the pattern of row i of T."""
    s = small_full
    E = edfa.build(s, edfa.Params("static"))
    n = s.ne
    for T, M in ((oedfa_unit(E.st2.L), E.st2.ML), (E.st2.U.tocsr(), E.st2.MU)):
        MT = (M @ T).toarray()
        Td = T.toarray()
        mask = Td != 0
        np.testing.assert_allclose(MT[mask], np.eye(n)[mask], atol=1e-12)
        assert not np.any((M.toarray() != 0) & ~mask)


def test_isai_refinement_approaches_exact_triangular_solves(small_full):
    """ISAI with refinement steps converges to the exact ILU(0) triangular solves."""
    s = small_full
    Ex = edfa.build(s, edfa.Params("static", schur="exact"))
    y = np.random.default_rng(9).standard_normal(s.ne)
    ref = Ex.apply_S_inv(y)
    errs = []
    for k in (1, 2, 4, 8):
        Ek = edfa.Edfa(s, edfa.Params("static", isai_steps=k), Ex.st1,
                       edfa.stage2(s, Ex.st1, edfa.Params("static", isai_steps=k)))
        errs.append(np.linalg.norm(Ek.apply_S_inv(y) - ref) / np.linalg.norm(ref))
    assert errs[-1] < 1e-6 and all(b < a for a, b in zip(errs, errs[1:]))


@pytest.mark.parametrize("schur,filt,bound", [("exact", "none", 1e-12), ("isai", "none", 1e-2),
                                               ("exact", "post_H", 1e-1), ("isai", "post_H", 1e-1)])
def test_transposed_application_vs_edfa_of_transposed_blocks(small_full, schur, filt, bound):
    """P^-T (the transpose of the forward EDFA, used by the adjoint solve) equals the EDFA
    built on the transposed blocks only without post-filtration on H~ and with exact
    substitution: the filter on H~ uses the row norms of H~ where the transposed EDFA would
    use those of H~^T, and the row-wise ISAI of U^T is not the transpose of the row-wise ISAI
    of U.  Elsewhere P^-T is still a preconditioner of A^T (the transposed solve stops on its
    true residual); this measures how far it is from EDFA(A^T): 3e-4 with the approximate
    inverses, 3e-2 with post-filtration at 1e-2 on this grid."""
    import copy
    s = small_full
    prm = edfa.Params("dynamic", n_add=1, n_ent=3, schur=schur, filt=filt, tau=1e-2)
    fwd = edfa.build(s, prm)
    st = copy.copy(s)
    st.Apc, st.Acp, st.Acc = s.Acp.T.tocsr(), s.Apc.T.tocsr(), s.Acc.T.tocsr()
    st.ApcT = None
    for m_ in (st.Apc, st.Acp, st.Acc):
        m_.sort_indices()
    st1t = edfa.stage1(st, prm, base_rows=s.Acp)
    Et = edfa.Edfa(st, prm, st1t, edfa.stage2(st, st1t, prm))
    rng = np.random.default_rng(4)
    d = 0.0
    for _ in range(4):
        y = rng.standard_normal(s.n)
        a, b = fwd.apply_T(y), Et.apply(y)
        d = max(d, np.linalg.norm(a - b) / np.linalg.norm(b))
    assert d <= bound
    if bound > 1e-12:
        assert d > 1e-8     # the two really differ in this setting
