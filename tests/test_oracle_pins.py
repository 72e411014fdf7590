"""Independent pins for oracle pieces that other tests cover only indirectly.

Each test names the plausible mistake it would catch.

* Dynamic selection (Section 3, eq. prol_res; Algorithm 1, "largest components"): the
  prolonged residual is recomputed densely by brute force, r = a_ppi + A_pipi[:, Q] g~, with
  g~ from a dense solve, and every sweep of the oracle must append exactly the top-n |r_j|
  with j outside Q.  Exact ties go to the smaller index.
* Pre-filtration (Section 3, implementation details): entries below tau times the Euclidean
  norm of their own vector are dropped, entries at or above it are kept.
* Static Patch(k) (Section 3, static technique): the faces of the cells within k
  face-neighbour steps, counted by hand on a brick lattice and by a breadth-first search over
  the face graph written here.
* Density mu (Section 4): on a one-cell grid every count is known by hand.
"""
import numpy as np
import pytest

from oracle import edfa, mhfe
from paper_2009_13916_amd import inputs


# ---------------------------------------------------------------------------------------------
# dynamic selection
# ---------------------------------------------------------------------------------------------
def _dense_trace(s, m, cr, base_len, n_add, n_ent):
    """Replay the sweeps of cell m with dense linear algebra; yields (Q_k, added_k, r, n)."""
    App = s.App.toarray()
    a = s.Acp[m].toarray().ravel()          # a_ppi^(m) over all face unknowns
    pos = base_len
    n_prog = 0
    for cnt in cr.added:
        Q = cr.Q[:pos]
        g = np.linalg.solve(-App[np.ix_(Q, Q)], a[Q])
        r = a + App[:, Q] @ g                # brute-force prolonged residual
        n = min(n_add, n_ent - n_prog)
        yield Q, cr.Q[pos:pos + cnt], r, n
        pos += cnt
        n_prog += cnt
    assert pos == len(cr.Q)


def _top_n_outside(Q, r, n):
    """Indices outside Q with |r| > 0, by decreasing |r|, ties to the smaller index."""
    cand = np.setdiff1d(np.nonzero(r)[0], Q)
    order = np.lexsort((cand, -np.abs(r[cand])))
    return cand[order[:n]], cand[order]


@pytest.mark.parametrize("kind", ["full", "iso"])
@pytest.mark.parametrize("n_add,n_ent", [(1, 4), (3, 7)])
def test_dynamic_sweeps_append_largest_residual_entries(kind, n_add, n_ent):
    """Mistakes caught: choosing the smallest |r|, using signed r, re-adding indices of Q,
    dropping the a_ppi term of the residual, a wrong tie order or a wrong count per sweep."""
    if kind == "full":
        prob = inputs.full_tensor_problem(4, 4, 3, sigma=1.5, corr=2.0, config_id=91)
    else:
        prob = inputs.lognormal_iso_problem(5, sigma=1.0, config_id=92)
    s = mhfe.assemble(prob)
    edfa._ensure_apct(s)
    prm = edfa.Params("dynamic", n_add=n_add, n_ent=n_ent)
    checked = 0
    for m in range(0, s.ne, 3):
        cr = edfa.local_cell(s, m, prm)
        base_len = len(edfa.base_pattern(s, m))
        assert len(cr.Q) == len(set(cr.Q.tolist()))
        sweeps = 0
        for Q, added, r, n in _dense_trace(s, m, cr, base_len, n_add, n_ent):
            top, ranked = _top_n_outside(Q, r, n)
            mags = np.abs(r[ranked])
            # entries that cancel exactly in one summation order are rounding noise in another:
            # those past the clearly non-zero candidates are only checked to be noise
            clear = ranked[mags > 1e-12 * mags[0]]
            k = min(len(added), len(clear))
            assert len(added) == n or len(added) >= len(clear), (m, added, clear)
            assert np.all(np.abs(r[added[k:]]) <= 1e-12 * mags[0])
            # compare exactly where the k-th and (k+1)-th magnitudes are well separated
            if k < len(ranked) and k > 0 and mags[k - 1] - mags[k] <= 1e-9 * mags[0]:
                continue
            assert np.array_equal(np.sort(added[:k]), np.sort(ranked[:k])), (m, added, ranked[:k])
            # and appended in decreasing |r|
            assert np.all(np.diff(np.abs(r[added[:k]])) <= 1e-12 * mags[0])
            sweeps += 1
            checked += 1
        assert sweeps >= 1
    assert checked > 10


def test_select_new_tie_and_rounding_rules():
    """Mistakes caught: ties to the larger index, ties broken by position instead of index,
    zero entries taken as candidates, members of Q re-selected, keys that keep more or fewer
    than 40 significant bits."""
    Q = np.array([2, 4])
    idx = np.array([9, 7, 5, 3, 4, 11, 13])
    val = np.array([1.0, -1.0, 0.5, 1.0, 50.0, 0.0, -0.75])
    # |1.0| appears at 9, 7 and 3: smallest index first; 4 is in Q; 11 is zero
    assert edfa.select_new(Q, idx, val, 2).tolist() == [3, 7]
    assert edfa.select_new(Q, idx, val, 4).tolist() == [3, 7, 9, 13]
    assert edfa.select_new(Q, idx, val, 10).tolist() == [3, 7, 9, 13, 5]
    # values equal to 40 significant bits tie (smaller index wins) ...
    x = 1.0 + 2.0 ** -45
    assert edfa.select_new(np.array([], dtype=int), np.array([8, 6]), np.array([x, 1.0]), 1).tolist() == [6]
    assert edfa.select_new(np.array([], dtype=int), np.array([6, 8]), np.array([1.0, x]), 1).tolist() == [6]
    # ... while a difference in the 30th bit orders them
    y = 1.0 + 2.0 ** -30
    assert edfa.select_new(np.array([], dtype=int), np.array([6, 8]), np.array([1.0, y]), 1).tolist() == [8]
    # the key of a value rounds to nearest at 40 significant bits (a 53-bit mantissa keeps 39
    # fraction bits): 1 + 2^-40 rounds up to 1 + 2^-39, 1 + 2^-41 rounds down to 1
    k = edfa.key40(np.array([1.0, 1.0 + 2.0 ** -41, 1.0 + 2.0 ** -40, 1.0 + 2.0 ** -39]))
    assert k[0] == k[1] and k[2] == k[3] and k[2] > k[1]


# ---------------------------------------------------------------------------------------------
# pre-filtration
# ---------------------------------------------------------------------------------------------
def test_filter_keep_threshold_is_relative_to_own_euclidean_norm():
    """Mistakes caught: the 1- or inf-norm instead of the 2-norm, dropping entries equal to the
    threshold, comparing signed values."""
    x = np.array([3.0, -4.0, 0.0])            # ||x||_2 = 5 (||x||_1 = 7, ||x||_inf = 4)
    assert edfa.filter_keep(x, 0.8).tolist() == [False, True, False]     # threshold 4: -4 kept
    assert edfa.filter_keep(x, 0.6).tolist() == [True, True, False]      # threshold 3: 3 kept
    assert edfa.filter_keep(x, 0.6 + 1e-12).tolist() == [False, True, False]
    assert edfa.filter_keep(x, 0.6 - 1e-12).tolist() == [True, True, False]
    assert edfa.filter_keep(x, 0.0).tolist() == [True, True, True]
    # with tau = 0.7: 2-norm threshold 3.5 keeps only -4; the 1-norm (4.9) would keep none
    # and the inf-norm (2.8) would keep 3 as well
    assert edfa.filter_keep(x, 0.7).tolist() == [False, True, False]


def test_prefiltration_in_stage1_uses_each_vector_norm():
    """G~ row m keeps |g_i| >= tau ||g~^(m)||_2, F~ column m keeps |f_i| >= tau ||f~^(m)||_2.
    Mistake caught: one norm shared by g~ and f~, or the norm of the filtered vector."""
    prob = inputs.full_tensor_problem(3, 3, 3, sigma=1.5, corr=2.0, config_id=93)
    s = mhfe.assemble(prob)
    tau = 0.05
    st = edfa.stage1(s, edfa.Params("static", tau=tau, filt="pre"))
    G, F = st.Gt.tocsr(), st.Ft.tocsc()
    dropped = 0
    for m, cr in enumerate(st.cells):
        keep_g = {int(q) for q, v in zip(cr.Q, cr.g) if abs(v) >= tau * np.sqrt(np.sum(cr.g ** 2))}
        keep_f = {int(q) for q, v in zip(cr.Q, cr.f) if abs(v) >= tau * np.sqrt(np.sum(cr.f ** 2))}
        assert set(G.indices[G.indptr[m]:G.indptr[m + 1]].tolist()) == keep_g
        assert set(F.indices[F.indptr[m]:F.indptr[m + 1]].tolist()) == keep_f
        dropped += 2 * len(cr.Q) - len(keep_g) - len(keep_f)
    assert dropped > 0


# ---------------------------------------------------------------------------------------------
# static Patch(k)
# ---------------------------------------------------------------------------------------------
def _bfs_faces(s, m, level):
    """Unknown faces of the cells within `level` steps of m over shared faces (written here)."""
    topo = s.topo
    face_cells = topo.face_cells
    dist = {m: 0}
    frontier = [m]
    for d in range(1, level + 1):
        nxt = []
        for e in frontier:
            for f in topo.cell_faces[e]:
                for e2 in face_cells[f]:
                    if e2 >= 0 and e2 not in dist:
                        dist[e2] = d
                        nxt.append(int(e2))
        frontier = nxt
    faces = set()
    for e in dist:
        for f in topo.cell_faces[e]:
            if s.uidx[f] >= 0:
                faces.add(int(s.uidx[f]))
    return faces


@pytest.mark.parametrize("kind", ["iso", "full"])
def test_patch_levels_interior_counts(kind):
    """Interior cell of a brick lattice: the cells within k face steps form the L1 ball of
    radius k (7 and 25 cells); its faces are 6 * cells - adjacent pairs inside the ball:
    level 1: 6*7 - 6 = 36; level 2: 6*25 - 36 = 114 (12 adjacent pairs per direction).
    Level 0 is the base pattern: 12 faces for a block-diagonal W^E (own faces and the face
    of each neighbour opposite the shared one), 36 for a full W^E.
    Mistakes caught: 26-neighbour instead of face adjacency, a missed ring, the base pattern
    left out of the union."""
    n = 7
    if kind == "iso":
        prob = inputs.lognormal_iso_problem(n, sigma=0.5, config_id=94)
    else:
        prob = inputs.full_tensor_problem(n, n, n, sigma=1.0, corr=2.0, config_id=95)
    s = mhfe.assemble(prob)
    m = 3 + n * (3 + n * 3)
    base = edfa.base_pattern(s, m)
    assert len(base) == (12 if kind == "iso" else 36)
    assert len(edfa.patch_pattern(s, m, 1)) == 36
    assert len(edfa.patch_pattern(s, m, 2)) == 114
    for lev in (1, 2):
        assert set(edfa.patch_pattern(s, m, lev).tolist()) == _bfs_faces(s, m, lev) | set(base.tolist())


def test_patch_levels_near_boundaries():
    """Cells next to a no-flow face and next to a Dirichlet face, against the face-graph BFS.
    At level 1 a cell with one missing neighbour touches 6 cells: 6*6 - 5 = 31 faces; next to
    x = 0 the five x- faces on the Dirichlet boundary are not unknowns: 26."""
    n = 6
    prob = inputs.lognormal_iso_problem(n, sigma=0.5, config_id=96)
    s = mhfe.assemble(prob)
    m_noflow = 2 + n * (0 + n * 2)      # j = 0: no-flow y- face
    m_dir = 0 + n * (2 + n * 2)         # i = 0: Dirichlet x- face
    assert len(edfa.patch_pattern(s, m_noflow, 1)) == 31
    assert len(edfa.patch_pattern(s, m_dir, 1)) == 26
    for m in (m_noflow, m_dir, 0, s.ne - 1):
        for lev in (1, 2, 3):
            got = set(edfa.patch_pattern(s, m, lev).tolist())
            assert got == _bfs_faces(s, m, lev) | set(edfa.base_pattern(s, m).tolist())


@pytest.mark.parametrize("kind", ["iso", "full"])
def test_axis_strip_counts(kind):
    """Strip patterns along one axis, interior cell: the cells within k steps along the axis
    are a line of 2k + 1 cells with 2k shared faces, so 6(2k + 1) - 2k faces (16 at k = 1,
    26 at k = 2), in union with the base pattern.  Iso bricks: the base adds the far face of
    each of the four side neighbours (12 - 6 - 2 = 4 faces outside the strip): 20 and 30.
    Full W: the base already holds every face of the six face neighbours (6 + 6 * 5 = 36),
    so level 1 stays at 36 and level 2 adds the five new faces of each of the two far cells:
    46.  A strip along the wrong axis, or a level-k ball instead of a line, changes the
    count."""
    n = 7
    if kind == "iso":
        prob = inputs.lognormal_iso_problem(n, sigma=0.5, config_id=94)
    else:
        prob = inputs.full_tensor_problem(n, n, n, sigma=1.0, corr=2.0, config_id=95)
    s = mhfe.assemble(prob)
    m = 3 + n * (3 + n * 3)
    want = {"iso": {1: 20, 2: 30}, "full": {1: 36, 2: 46}}[kind]
    for axis in (1, 2, 3):
        for lev in (1, 2):
            Q = edfa.patch_pattern(s, m, lev, axis=axis)
            assert len(Q) == want[lev], (axis, lev, len(Q))
            # the strip's own faces: the cells m + t e_d, |t| <= lev, all their faces
            d = axis - 1
            step = (1, n, n * n)[d]
            cells = [m + t * step for t in range(-lev, lev + 1)]
            strip = {int(s.uidx[f]) for c in cells for f in s.topo.cell_faces[c] if s.uidx[f] >= 0}
            assert strip <= set(Q.tolist())
            assert set(Q.tolist()) == strip | set(edfa.base_pattern(s, m).tolist())


def test_flow_axis_follows_the_largest_transmissibility():
    """K = diag(kx, ky, kz) on cubes: the transmissibility of axis d is proportional to
    K_dd, so the strip of axis 4 runs along the largest diagonal entry (ties to x)."""
    n = 5
    prob = inputs.lognormal_iso_problem(n, sigma=0.0, config_id=98)
    ne = n ** 3
    K = np.zeros((ne, 6))
    rng = np.random.default_rng(0)
    diag = rng.uniform(0.1, 10.0, (ne, 3))
    diag[0] = [2.0, 2.0, 1.0]                    # a tie: x wins
    K[:, :3] = diag
    import dataclasses
    s = mhfe.assemble(dataclasses.replace(prob, K=K))
    for m in range(ne):
        want = int(np.argmax(diag[m]))
        assert edfa.flow_axis(s, m) == want
        assert np.array_equal(edfa.patch_pattern(s, m, 1, axis=4),
                              edfa.patch_pattern(s, m, 1, axis=want + 1))


# ---------------------------------------------------------------------------------------------
# density mu
# ---------------------------------------------------------------------------------------------
def test_density_on_one_cell_by_hand():
    """One brick cell, isotropic K, Dirichlet on both x faces: 4 face unknowns (y-, y+, z-, z+)
    and 1 cell.  W^E is block-diagonal per direction, so nnz(A_pipi) = 8, nnz(A_pip) =
    nnz(A_ppi) = 4, nnz(A_pp) = 1: denominator 17.  The FSAI factor holds the lower pattern of
    A_pipi, 6 entries, stored with its transpose: 12.  S~ is 1 x 1: its ILU(0) has no strict
    lower entry and U = 1 entry; the ISAI factors hold 1 entry each.
    mu = (12 + 4 + 4 + [M_L + M_U = 2]) / 17 with sparse approximate inverses (one step),
    (12 + 4 + 4 + [L + M_L + U + M_U = 3]) / 17 with refinement steps (the factors are read
    too), and (12 + 4 + 4 + [L + U = 1]) / 17 with exact substitution."""
    prob = inputs.lognormal_iso_problem(1, sigma=0.0, config_id=97)
    s = mhfe.assemble(prob)
    assert (s.nfu, s.ne) == (4, 1)
    assert (s.App.nnz, s.Apc.nnz, s.Acp.nnz, s.Acc.nnz) == (8, 4, 4, 1)
    E = edfa.build(s, edfa.Params("static"))
    assert E.density() == pytest.approx(22 / 17, rel=1e-15)
    E2 = edfa.build(s, edfa.Params("static", isai_steps=2))
    assert E2.density() == pytest.approx(23 / 17, rel=1e-15)
    Ex = edfa.build(s, edfa.Params("static", schur="exact"))
    assert Ex.density() == pytest.approx(21 / 17, rel=1e-15)
