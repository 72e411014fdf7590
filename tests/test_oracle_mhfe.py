"""Pins for the oracle's discretisation and assembly (Section 2, Appendix A).

Each test checks the oracle against something other than itself: closed
forms, a classical textbook system related by an exact identity, the flux
equations evaluated directly, exact solutions, and structural statements of
the paper.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import mhfe
from paper_2009_13916_amd import inputs


def _single_cell(hx, hy, hz, K6):
    nodes = inputs.brick_nodes(1, 1, 1, hx, hy, hz)
    topo = mhfe.topology(1, 1, 1)
    return nodes[topo.cell_nodes], np.asarray(K6, dtype=float)[None]


def _random_spd6(rng):
    M = rng.standard_normal((3, 3))
    K = M @ M.T + 0.5 * np.eye(3)
    return [K[0, 0], K[1, 1], K[2, 2], K[0, 1], K[0, 2], K[1, 2]], K


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brick_element_matrix_closed_form(seed):
    """RT0 on a brick: B_{d+-,d+-} = g Kinv_dd h_d/(3A_d), B_{d+,d-} = -g Kinv_dd h_d/(6A_d),
    B_{d s, e s'} = s s' g Kinv_de / (4 h_f) (f the third direction).  Derived from the basis
    properties (eqs. MFE_property_1/2) and eq. B_ij by hand, not by the quadrature code."""
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.3, 2.0, 3)
    K6, K = _random_spd6(rng)
    gamma = rng.uniform(0.5, 2.0)
    X8, K6a = _single_cell(*h, K6)
    B, vol = mhfe.element_matrices(X8, K6a, gamma)
    Ki = np.linalg.inv(K)
    area = [h[1] * h[2], h[0] * h[2], h[0] * h[1]]
    ref = np.zeros((6, 6))
    sgn = [-1, 1]
    for d in range(3):
        for e in range(3):
            for s in range(2):
                for t in range(2):
                    a, b = 2 * d + s, 2 * e + t
                    if d == e:
                        ref[a, b] = gamma * Ki[d, d] * h[d] / area[d] * (1 / 3 if s == t else -1 / 6)
                    else:
                        f = 3 - d - e
                        ref[a, b] = sgn[s] * sgn[t] * gamma * Ki[d, e] / (4 * h[f])
    np.testing.assert_allclose(B[0], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    assert abs(vol[0] - np.prod(h)) < 1e-14


def test_diag_brick_W_block_form():
    """Diagonal K on a brick: W = blockdiag_d (K_dd A_d/(g h_d)) [[4,2],[2,4]]."""
    h = (0.3, 0.5, 0.7)
    kd = (2.0, 0.5, 3.0)
    gamma = 1.3
    X8, K6 = _single_cell(*h, [kd[0], kd[1], kd[2], 0, 0, 0])
    B, _ = mhfe.element_matrices(X8, K6, gamma)
    W = np.linalg.inv(B[0])
    area = [h[1] * h[2], h[0] * h[2], h[0] * h[1]]
    ref = np.zeros((6, 6))
    for d in range(3):
        t = kd[d] * area[d] / (gamma * h[d])
        ref[2 * d:2 * d + 2, 2 * d:2 * d + 2] = t * np.array([[4, 2], [2, 4]])
    np.testing.assert_allclose(W, ref, rtol=1e-12, atol=1e-12)


def test_element_matrix_rotation_invariance():
    """Rigidly rotating a distorted cell and its tensor leaves B unchanged (frame invariance)."""
    rng = np.random.default_rng(5)
    nodes = inputs.brick_nodes(1, 1, 1)
    nodes = nodes + rng.uniform(-0.15, 0.15, nodes.shape)
    topo = mhfe.topology(1, 1, 1)
    K6, K = _random_spd6(rng)
    R = inputs.haar_rotations(1, rng)[0]
    X8 = nodes[topo.cell_nodes]
    B1, v1 = mhfe.element_matrices(X8, np.array([K6]), 1.0)
    KR = R @ K @ R.T
    X8r = X8 @ R.T
    B2, v2 = mhfe.element_matrices(X8r, inputs.pack_sym(KR[None]), 1.0)
    np.testing.assert_allclose(B1, B2, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(v1, v2, rtol=1e-13)


def _classical_cell_rows(s: mhfe.System, prob):
    """Classical hybridised MHFE cell rows: sum_a q_a^E + Omega c p/dt = Omega (s + c p_n/dt).

    Columns over unknown faces and cells; Dirichlet faces moved to the RHS.
    """
    topo = s.topo
    ne = topo.ne
    W = s.W
    L = W.sum(axis=2)
    rows, cols, vals = [], [], []
    rhs = s.vol * prob.source + s.vol * prob.c * prob.p_prev / prob.dt
    cells = np.arange(ne)
    for b in range(6):
        fb = topo.cell_faces[:, b]
        u = s.uidx[fb]
        coef = -L[:, b]              # d(sum_a q_a)/d pi_b = -sum_a W_ab
        m = u >= 0
        rows.append(cells[m]); cols.append(u[m]); vals.append(coef[m])
        rhs = rhs - np.where(m, 0.0, coef * prob.bc_value[fb])
    Acp = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                        shape=(ne, s.nfu))
    Acc = sp.diags(W.sum(axis=(1, 2)) + s.vol * prob.c / prob.dt)
    return Acp, Acc, rhs


def _cmat(s: mhfe.System):
    topo = s.topo
    rows, cols, vals = [], [], []
    for a in range(6):
        u = s.uidx[topo.cell_faces[:, a]]
        m = u >= 0
        rows.append(np.nonzero(m)[0]); cols.append(u[m]); vals.append(s.Dcoef[m, a])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(s.ne, s.nfu))


@pytest.mark.parametrize("maker", ["iso", "full", "distorted"])
def test_assembly_equals_row_combination_of_classical_system(maker):
    """Strong-flux cell rows = classical cell rows - sum_i D_i (face row i), i.e.
    A_ppi = A_ppi^std - C A_pipi, A_pp = A_pp^std - C A_pip, b_p = b_p^std - C b_pi,
    with C[E,i] = W_ii/(W_ii + W'_ii) (interior), 1 (Neumann).  Exact algebra of
    eqs. fluxes_MHFEM_STRONG and cont_fluxes; the classical rows are the textbook
    hybridised mass balance, not the Appendix A formulas."""
    if maker == "iso":
        prob = inputs.lognormal_iso_problem(4, sigma=1.0, config_id=91)
    elif maker == "full":
        prob = inputs.full_tensor_problem(4, 3, 5, sigma=1.0, corr=2.0, config_id=92)
    else:
        prob = inputs.channel_problem(5, 4, 3, contrast=1e3, config_id=93)
    prob.source = np.random.default_rng(1).standard_normal(prob.n_cells)
    s = mhfe.assemble(prob)
    Acp_std, Acc_std, bp_std = _classical_cell_rows(s, prob)
    C = _cmat(s)
    scale = abs(s.App).max()
    np.testing.assert_allclose((Acp_std - C @ s.App - s.Acp).toarray(), 0, atol=1e-12 * scale)
    np.testing.assert_allclose((Acc_std - C @ s.Apc - s.Acc).toarray(), 0, atol=1e-12 * scale)
    np.testing.assert_allclose(bp_std - C @ s.b[:s.nfu], s.b[s.nfu:], atol=1e-12 * scale)


def test_assembly_matches_flux_equations():
    """A u - b equals the discrete equations evaluated from the fluxes of eq. fluxes_MHFEM_3
    and eq. fluxes_MHFEM_STRONG for random u (random Neumann fluxes and sources too)."""
    rng = np.random.default_rng(3)
    prob = inputs.full_tensor_problem(3, 4, 3, sigma=1.0, corr=2.0, config_id=94)
    topo = mhfe.topology(prob.nx, prob.ny, prob.nz)
    kind = mhfe.face_kinds(topo, prob.bc_type)
    prob.bc_value = np.where(kind == mhfe.NEUMANN, rng.standard_normal(topo.nf), prob.bc_value)
    prob.source = rng.standard_normal(topo.ne)
    s = mhfe.assemble(prob)
    u = rng.standard_normal(s.n)
    pi_full = prob.bc_value.copy()
    pi_full[s.ufaces] = u[:s.nfu]
    p = u[s.nfu:]
    W, cf = s.W, topo.cell_faces
    q = np.einsum("eab,eb->ea", W, p[:, None] - pi_full[cf])           # local fluxes
    res_face = np.zeros(topo.nf)
    np.add.at(res_face, cf.ravel(), q.ravel())
    res_face[kind == mhfe.NEUMANN] -= prob.bc_value[kind == mhfe.NEUMANN]
    Lam = lambda e, a: (W[e, a].sum() * p[e]
                        - sum(W[e, a, j] * pi_full[cf[e, j]] for j in range(6) if j != a))
    res_cell = s.vol * prob.c * (p - prob.p_prev) / prob.dt - s.vol * prob.source
    for e in range(topo.ne):
        for a in range(6):
            f = cf[e, a]
            if kind[f] == mhfe.NEUMANN:
                res_cell[e] += prob.bc_value[f]
            elif kind[f] == mhfe.DIRICHLET:
                res_cell[e] += q[e, a]
            else:
                e2 = topo.face_cells[f, 1] if topo.face_cells[f, 0] == e else topo.face_cells[f, 0]
                a2 = a ^ 1
                w1, w2 = W[e, a, a], W[e2, a2, a2]
                res_cell[e] += (w2 * Lam(e, a) - w1 * Lam(e2, a2)) / (w1 + w2)
    r_ref = np.concatenate([res_face[s.ufaces], res_cell])
    r = s.matrix() @ u - s.b
    np.testing.assert_allclose(r, r_ref, atol=1e-11 * np.abs(r_ref).max())


def test_linear_pressure_exact_on_bricks():
    """Homogeneous K, Dirichlet 1/0 on x, no flow elsewhere: p^E = 1 - x_E, pi = 1 - x_face."""
    prob = inputs.lognormal_iso_problem(5, sigma=0.0, config_id=95)
    topo = mhfe.topology(5, 5, 5)
    X8 = prob.nodes[topo.cell_nodes]
    xc = X8[:, :, 0].mean(axis=1)
    prob.p_prev = 1.0 - xc
    s = mhfe.assemble(prob)
    u = mhfe.direct_solve(s)
    np.testing.assert_allclose(u[s.nfu:], 1.0 - xc, atol=1e-13)
    # face centroids of unknown faces
    fx = np.zeros(topo.nf)
    cnt = np.zeros(topo.nf)
    cen = {0: [0, 2, 4, 6], 1: [1, 3, 5, 7], 2: [0, 1, 4, 5], 3: [2, 3, 6, 7], 4: [0, 1, 2, 3], 5: [4, 5, 6, 7]}
    for a, nn in cen.items():
        np.add.at(fx, topo.cell_faces[:, a], X8[:, nn, 0].mean(axis=1))
        np.add.at(cnt, topo.cell_faces[:, a], 1)
    fx /= cnt
    np.testing.assert_allclose(u[:s.nfu], 1.0 - fx[s.ufaces], atol=1e-13)


def test_linear_pressure_exact_on_parallelepipeds_full_tensor():
    """Affine grid, constant full tensor, Dirichlet on all boundary faces with a linear p:
    the lowest-order mixed-hybrid method reproduces linear pressures exactly."""
    n = 4
    rng = np.random.default_rng(7)
    A = np.eye(3) + 0.25 * rng.standard_normal((3, 3))
    nodes = inputs.brick_nodes(n, n, n) @ A.T
    K6, _ = _random_spd6(rng)
    topo = mhfe.topology(n, n, n)
    gvec = np.array([0.7, -1.1, 0.4])
    plin = lambda X: 2.0 + X @ gvec
    X8 = nodes[topo.cell_nodes]
    cen = {0: [0, 2, 4, 6], 1: [1, 3, 5, 7], 2: [0, 1, 4, 5], 3: [2, 3, 6, 7], 4: [0, 1, 2, 3], 5: [4, 5, 6, 7]}
    fcen = np.zeros((topo.nf, 3))
    cnt = np.zeros(topo.nf)
    for a, nn in cen.items():
        np.add.at(fcen, topo.cell_faces[:, a], X8[:, nn, :].mean(axis=1))
        np.add.at(cnt, topo.cell_faces[:, a], 1)
    fcen /= cnt[:, None]
    boundary = (topo.face_cells < 0).any(axis=1)
    prob = inputs.Problem(n, n, n, nodes, np.tile(K6, (n ** 3, 1)), np.full(n ** 3, 0.3), 0.5, 1.0,
                          boundary.astype(np.int8), np.where(boundary, plin(fcen), 0.0),
                          plin(X8.mean(axis=1)), np.zeros(n ** 3))
    s = mhfe.assemble(prob)
    assert not s.axis
    u = mhfe.direct_solve(s)
    np.testing.assert_allclose(u[s.nfu:], plin(X8.mean(axis=1)), atol=1e-12)
    np.testing.assert_allclose(u[:s.nfu], plin(fcen)[s.ufaces], atol=1e-12)


def test_constant_pressure_null_test():
    """All no-flow, p_n = c0, no source: A [1;1] = [0; Omega c/dt] and the solve returns c0."""
    prob = inputs.full_tensor_problem(4, sigma=1.0, corr=2.0, config_id=96)
    prob.bc_type[:] = 0
    prob.bc_value[:] = 0.0
    prob.c[:] = 1.0
    prob.p_prev[:] = 3.5
    s = mhfe.assemble(prob)
    ones = np.ones(s.n)
    r = s.matrix() @ ones
    np.testing.assert_allclose(r[:s.nfu], 0.0, atol=1e-12)
    np.testing.assert_allclose(r[s.nfu:], s.vol * prob.c / prob.dt, rtol=1e-12)
    u = mhfe.direct_solve(s)
    np.testing.assert_allclose(u, 3.5, rtol=1e-11)


def test_block_properties_section_2_3():
    """A_pipi symmetric negative definite; A_pp structurally symmetric but not symmetric;
    A_pip != +-A_ppi^T (Section 2.3)."""
    prob = inputs.full_tensor_problem(4, sigma=2.0, corr=2.0, config_id=97)
    s = mhfe.assemble(prob)
    App = s.App.toarray()
    np.testing.assert_allclose(App, App.T, atol=1e-14 * abs(App).max())
    assert np.linalg.eigvalsh(App).max() < 0
    pat = (s.Acc != 0).astype(int) + 0 * s.Acc
    P = s.Acc.copy(); P.data[:] = 1
    assert (P - P.T).count_nonzero() == 0
    assert abs(s.Acc - s.Acc.T).max() > 1e-6 * abs(s.Acc).max()
    assert abs(s.Apc - s.Acp.T).max() > 1e-3 and abs(s.Apc + s.Acp.T).max() > 1e-3


@pytest.mark.parametrize("full", [False, True])
def test_interior_row_counts(full):
    """Interior rows hold 3/2/12/7 (axis structure) or 11/2/36/7 (full W) entries in
    A_pipi / A_pip / A_ppi / A_pp."""
    if full:
        prob = inputs.full_tensor_problem(5, sigma=1.0, corr=2.0, config_id=98)
    else:
        prob = inputs.lognormal_iso_problem(5, config_id=98)
    s = mhfe.assemble(prob)
    want = (11, 2, 36, 7) if full else (3, 2, 12, 7)
    for m, w in zip((s.App, s.Apc, s.Acp, s.Acc), want):
        assert np.diff(m.indptr).max() == w


def test_paper_table_test_setup_ratios():
    """Per-row non-zero ratios of the paper's structured 4-layer grid (Table test_setup:
    nnz/N_f = 2.815 / 1.815 for A_pipi / A_pip, nnz/N_e = 11.39 / 6.39 for A_ppi / A_pp)
    are reproduced within 1.5% by a structured 4-layer grid of similar size."""
    nx, ny, nz = 60, 220, 4
    ne = nx * ny * nz
    prob = inputs.Problem(nx, ny, nz, inputs.brick_nodes(nx, ny, nz, 1200, 2200, 8),
                          inputs.iso_tensor(np.ones(ne)), np.zeros(ne), 1.0, 1.0,
                          np.zeros(0, np.int8), np.zeros(0), np.zeros(ne), np.zeros(ne))
    nf = prob.n_faces
    prob.bc_type = np.zeros(nf, np.int8)
    prob.bc_value = np.zeros(nf)
    s = mhfe.assemble(prob)
    got = (s.App.nnz / s.nfu, s.Apc.nnz / s.nfu, s.Acp.nnz / s.ne, s.Acc.nnz / s.ne)
    paper = (481636 / 171070, 310446 / 171070, 589299 / 51741, 330533 / 51741)
    for g, p in zip(got, paper):
        assert abs(g - p) / p < 0.015, (got, paper)
