"""Oracle: MHFE-FV discretisation and assembly (test infrastructure only).

Follows Section 2.2-2.3 of the paper and its Appendix A.

* Element matrix (eq. B_ij): B_ij = gamma * int_E eta_i^T K^-1 eta_j, with the
  lowest-order Raviart-Thomas basis mapped from the unit cube by the
  contravariant Piola transform, integrated with the 3x3x3 Gauss-Legendre
  rule.  W = B^-1 (every "B^{-1}_ij" of the paper is an entry of W).
* Local flux law (eq. fluxes_MHFEM_3): q^E = W (p^E 1 - pi^E).
* Face rows: flux continuity / Neumann (eq. cont_fluxes).
* Cell rows: FV mass balance with backward Euler (eq. discr_bal_FV_2) and the
  strong inter-element flux (eq. fluxes_MHFEM_STRONG)
      q_i = (W'_ii Lam^E - W_ii Lam^E') / (W_ii + W'_ii),
      Lam^E = L_i p^E - sum_{j != i} W_ij pi_j,  L_i = sum_j W_ij.
  Boundary faces: a Neumann face contributes its prescribed flux (a ghost
  neighbour with W' = 0); a Dirichlet face contributes the one-sided local
  flux q_i^E evaluated with pi_i = p_bar (W' -> infinity).
* Dirichlet face pressures are eliminated (not unknowns).

Unknown order: u = [pi over non-Dirichlet faces, ascending face index; p over
cells].  Face numbering: x-faces (i + (nx+1)(j + ny k)), then y-faces
(i + nx(j + (ny+1)k)), then z-faces (i + nx(j + ny k)).  Local faces of a
cell: 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+.  Local nodes: a + 2b + 4c for node
(i+a, j+b, k+c).

Pins (tests/test_oracle_mhfe.py): closed-form brick matrices; assembly
against the classical hybridised system via the exact row-combination
identity; direct evaluation of the flux equations; exact linear pressure;
constant-pressure null test; block properties stated in Section 2.3; the
interior non-zero counts implied by the paper's Table test_setup.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# 3-point Gauss-Legendre rule on [0, 1]
_G = np.sqrt(3.0 / 5.0)
GAUSS_X = np.array([0.5 * (1 - _G), 0.5, 0.5 * (1 + _G)])
GAUSS_W = np.array([5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0])

INTERIOR, NEUMANN, DIRICHLET = 0, 1, 2


# ----------------------------------------------------------------------------
# Topology
# ----------------------------------------------------------------------------
@dataclass
class Topology:
    nx: int
    ny: int
    nz: int
    cell_faces: np.ndarray   # (Ne, 6) global face of each local face
    face_cells: np.ndarray   # (Nf, 2) [cell on minus side, cell on plus side], -1 if none
    cell_nodes: np.ndarray   # (Ne, 8)

    @property
    def ne(self):
        return self.cell_faces.shape[0]

    @property
    def nf(self):
        return self.face_cells.shape[0]


def topology(nx, ny, nz) -> Topology:
    ne = nx * ny * nz
    nfx = (nx + 1) * ny * nz
    nfy = nx * (ny + 1) * nz
    nfz = nx * ny * (nz + 1)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    fx = lambda ii, jj, kk: ii + (nx + 1) * (jj + ny * kk)
    fy = lambda ii, jj, kk: nfx + ii + nx * (jj + (ny + 1) * kk)
    fz = lambda ii, jj, kk: nfx + nfy + ii + nx * (jj + ny * kk)
    cf = np.stack([fx(i, j, k), fx(i + 1, j, k), fy(i, j, k), fy(i, j + 1, k),
                   fz(i, j, k), fz(i, j, k + 1)], axis=1).astype(np.int64)
    face_cells = -np.ones((nfx + nfy + nfz, 2), dtype=np.int64)
    cells = np.arange(ne)
    for a in range(6):
        # a face is the "plus" face (odd local index) of the cell on its minus side
        side = 0 if a % 2 == 1 else 1
        face_cells[cf[:, a], side] = cells
    nid = lambda ii, jj, kk: ii + (nx + 1) * (jj + (ny + 1) * kk)
    cn = np.stack([nid(i + a, j + b, k + c) for c in (0, 1) for b in (0, 1) for a in (0, 1)],
                  axis=1).astype(np.int64)
    return Topology(nx, ny, nz, cf, face_cells, cn)


def face_kinds(topo: Topology, bc_type: np.ndarray) -> np.ndarray:
    kind = np.full(topo.nf, INTERIOR, dtype=np.int64)
    boundary = (topo.face_cells < 0).any(axis=1)
    kind[boundary] = NEUMANN
    kind[boundary & (np.asarray(bc_type) == 1)] = DIRICHLET
    return kind


# ----------------------------------------------------------------------------
# Element matrices (eq. B_ij with the Piola map)
# ----------------------------------------------------------------------------
def _ref_basis(xh):
    """Reference RT0 fields at reference point xh (3,): rows = local faces."""
    x, y, z = xh
    e = np.zeros((6, 3))
    e[0, 0], e[1, 0] = x - 1.0, x
    e[2, 1], e[3, 1] = y - 1.0, y
    e[4, 2], e[5, 2] = z - 1.0, z
    return e


def _jacobian(X8, xh):
    """DF (n,3,3) with DF[:, :, d] = d x / d xhat_d for a trilinear map."""
    x, y, z = xh
    s = [(1 - x, x), (1 - y, y), (1 - z, z)]
    ds = (-1.0, 1.0)
    DF = np.zeros((X8.shape[0], 3, 3))
    for c in (0, 1):
        for b in (0, 1):
            for a in (0, 1):
                X = X8[:, a + 2 * b + 4 * c, :]
                DF[:, :, 0] += ds[a] * s[1][b] * s[2][c] * X
                DF[:, :, 1] += s[0][a] * ds[b] * s[2][c] * X
                DF[:, :, 2] += s[0][a] * s[1][b] * ds[c] * X
    return DF


def sym_from6(K6):
    K = np.empty((K6.shape[0], 3, 3))
    K[:, 0, 0], K[:, 1, 1], K[:, 2, 2] = K6[:, 0], K6[:, 1], K6[:, 2]
    K[:, 0, 1] = K[:, 1, 0] = K6[:, 3]
    K[:, 0, 2] = K[:, 2, 0] = K6[:, 4]
    K[:, 1, 2] = K[:, 2, 1] = K6[:, 5]
    return K


def element_matrices(X8, K6, gamma):
    """Return B (n,6,6) and cell volume (n,) by 3x3x3 Gauss quadrature."""
    Kinv = np.linalg.inv(sym_from6(K6))
    n = X8.shape[0]
    B = np.zeros((n, 6, 6))
    vol = np.zeros(n)
    for qz, wz in zip(GAUSS_X, GAUSS_W):
        for qy, wy in zip(GAUSS_X, GAUSS_W):
            for qx, wx in zip(GAUSS_X, GAUSS_W):
                xh = (qx, qy, qz)
                w = wx * wy * wz
                DF = _jacobian(X8, xh)
                J = np.linalg.det(DF)
                if np.any(J <= 0):
                    raise ValueError("non-positive Jacobian in a cell")
                V = np.einsum("nij,aj->nai", DF, _ref_basis(xh))   # DF eta_hat_a
                B += w * np.einsum("nai,nij,nbj->nab", V, Kinv, V) / J[:, None, None]
                vol += w * J
    return gamma * B, vol


def is_axis_structure(X8, K6) -> bool:
    """True when every cell is an axis-aligned brick and K is diagonal.

    Then W is block-diagonal with one 2x2 block per direction and the blocks
    are assembled with that (smaller) structural pattern.
    """
    if np.any(K6[:, 3:] != 0.0):
        return False
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                v = X8[:, a + 2 * b + 4 * c, :]
                if (np.any(v[:, 0] != X8[:, a, 0]) or np.any(v[:, 1] != X8[:, 2 * b, 1])
                        or np.any(v[:, 2] != X8[:, 4 * c, 2])):
                    return False
    return True


def struct_mask(axis: bool) -> np.ndarray:
    """S[a, b]: whether W_ab is a structural non-zero."""
    if axis:
        return np.array([[a // 2 == b // 2 for b in range(6)] for a in range(6)])
    return np.ones((6, 6), dtype=bool)


# ----------------------------------------------------------------------------
# Assembly (Appendix A)
# ----------------------------------------------------------------------------
@dataclass
class System:
    topo: Topology
    kind: np.ndarray        # (Nf,) INTERIOR / NEUMANN / DIRICHLET
    uidx: np.ndarray        # (Nf,) unknown index of each face, -1 for Dirichlet
    ufaces: np.ndarray      # (Nfu,) global face of each face unknown
    W: np.ndarray           # (Ne,6,6)
    vol: np.ndarray         # (Ne,)
    axis: bool
    App: sp.csr_matrix      # A_pipi (Nfu x Nfu)
    Apc: sp.csr_matrix      # A_pip  (Nfu x Ne)
    Acp: sp.csr_matrix      # A_ppi  (Ne x Nfu)
    Acc: sp.csr_matrix      # A_pp   (Ne x Ne)
    b: np.ndarray           # (Nfu + Ne,)
    Dcoef: np.ndarray       # (Ne,6) D_a = W_aa/(W_aa+W'_aa) (interior), 1 Neumann, 0 Dirichlet

    @property
    def nfu(self):
        return self.App.shape[0]

    @property
    def ne(self):
        return self.Acc.shape[0]

    @property
    def n(self):
        return self.nfu + self.ne

    def matrix(self) -> sp.csr_matrix:
        return sp.bmat([[self.App, self.Apc], [self.Acp, self.Acc]], format="csr")


def cell_geometry(prob, topo):
    X8 = prob.nodes[topo.cell_nodes]
    return X8


def _assemble_on_pattern(prow, pcol, rows, cols, vals, shape):
    """Sum COO contributions onto a structural pattern (explicit zeros kept).

    Raises if a contribution falls outside the pattern.
    """
    P = sp.csr_matrix((np.zeros(len(prow)), (prow, pcol)), shape=shape)
    P.sum_duplicates()
    M = sp.csr_matrix((np.concatenate([np.zeros(len(prow)), vals]),
                       (np.concatenate([prow, rows]), np.concatenate([pcol, cols]))),
                      shape=shape)
    M.sum_duplicates()
    M.sort_indices()
    if M.nnz != P.nnz:
        raise AssertionError("contribution outside the structural pattern")
    return M


def assemble(prob) -> System:
    """Assemble the 2x2 block system (eq. system) by the Appendix A formulas."""
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    topo = topology(nx, ny, nz)
    ne, nf = topo.ne, topo.nf
    X8 = prob.nodes[topo.cell_nodes]
    K6 = np.asarray(prob.K, dtype=np.float64)
    B, vol = element_matrices(X8, K6, prob.gamma)
    W = np.linalg.inv(B)
    W = 0.5 * (W + W.transpose(0, 2, 1))
    axis = is_axis_structure(X8, K6)
    S = struct_mask(axis)
    if axis:
        W = W * S[None]                      # structural zeros exact
    kind = face_kinds(topo, prob.bc_type)
    bcv = np.asarray(prob.bc_value, dtype=np.float64)
    L = W.sum(axis=2)                        # L_a = sum_b W_ab

    cf = topo.cell_faces
    fc = topo.face_cells
    cells = np.arange(ne)
    # neighbour across local face a and the local index of the shared face there
    nbr = np.where(np.arange(6)[None, :] % 2 == 1, fc[cf, 1], fc[cf, 0])   # (Ne,6)
    loc_in_nbr = np.arange(6) ^ 1
    kE = kind[cf]                                                         # (Ne,6)
    Wd = W[:, np.arange(6), np.arange(6)]                                 # (Ne,6)
    Wn = np.where(nbr >= 0, Wd[np.maximum(nbr, 0), loc_in_nbr[None, :]], 0.0)
    # C_a = W'_aa/(W_aa+W'_aa), D_a = W_aa/(W_aa+W'_aa); Neumann: C=0, D=1; Dirichlet: C=1, D=0
    C = np.where(kE == INTERIOR, Wn / np.where(kE == INTERIOR, Wd + Wn, 1.0), 0.0)
    D = np.where(kE == INTERIOR, Wd / np.where(kE == INTERIOR, Wd + Wn, 1.0), 0.0)
    C = np.where(kE == DIRICHLET, 1.0, C)
    D = np.where(kE == NEUMANN, 1.0, D)

    N = nf + ne
    rows, cols, vals = [], [], []       # full system, faces then cells
    prow, pcol = [], []                 # structural pattern of the full system

    def add(r, c, v):
        rows.append(np.asarray(r).ravel())
        cols.append(np.asarray(c).ravel())
        vals.append(np.broadcast_to(np.asarray(v, dtype=np.float64), np.shape(r)).ravel())

    def pat(r, c):
        prow.append(np.asarray(r).ravel())
        pcol.append(np.asarray(c).ravel())

    # ---- face rows: sum over the cells sharing the face of q_i^E (eq. cont_fluxes)
    for a in range(6):
        fa = cf[:, a]
        for b in range(6):
            if S[a, b]:
                add(fa, cf[:, b], -W[:, a, b])
                pat(fa, cf[:, b])
        add(fa, nf + cells, L[:, a])
        pat(fa, nf + cells)
    # ---- cell rows (eq. discr_bal_FV_2 with eq. fluxes_MHFEM_STRONG)
    diag = (C * L).sum(axis=1) + vol * prob.c / prob.dt
    add(nf + cells, nf + cells, diag)
    pat(nf + cells, nf + cells)
    for b in range(6):
        pat(nf + cells, cf[:, b])                       # own faces always structural
    for a in range(6):
        for b in range(6):
            if b != a and S[a, b]:
                add(nf + cells, cf[:, b], -C[:, a] * W[:, a, b])
        inter = kE[:, a] == INTERIOR
        e_in, nb = cells[inter], nbr[inter, a]
        ap = loc_in_nbr[a]
        add(nf + e_in, nf + nb, -D[inter, a] * L[nb, ap])
        pat(nf + e_in, nf + nb)
        for bp in range(6):
            if bp != ap and S[ap, bp]:
                add(nf + e_in, cf[nb, bp], D[inter, a] * W[nb, ap, bp])
                pat(nf + e_in, cf[nb, bp])
        dir_ = kE[:, a] == DIRICHLET
        add(nf + cells[dir_], cf[dir_, a], -W[dir_, a, a])

    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    Afull = _assemble_on_pattern(np.concatenate(prow), np.concatenate(pcol), r, c, v, (N, N))

    # right-hand side before elimination
    bfull = np.zeros(N)
    neu = kind == NEUMANN
    bfull[:nf][neu] = bcv[neu]                                   # q_i^E = qbar
    src = vol * prob.source + vol * prob.c * prob.p_prev / prob.dt
    neu_flux = np.where(kE == NEUMANN, bcv[cf], 0.0).sum(axis=1)
    bfull[nf:] = src - neu_flux

    # eliminate Dirichlet faces
    dmask = kind == DIRICHLET
    uf = np.nonzero(~dmask)[0]
    uidx = -np.ones(nf, dtype=np.int64)
    uidx[uf] = np.arange(uf.size)
    keep = np.concatenate([uf, nf + cells])
    xd = np.zeros(N)
    xd[:nf][dmask] = bcv[dmask]
    b = (bfull - Afull @ xd)[keep]
    A = Afull[keep][:, keep].tocsr()
    A.sort_indices()
    nfu = uf.size
    App, Apc = A[:nfu, :nfu].tocsr(), A[:nfu, nfu:].tocsr()
    Acp, Acc = A[nfu:, :nfu].tocsr(), A[nfu:, nfu:].tocsr()
    for m in (App, Apc, Acp, Acc):
        m.sort_indices()
    Dcoef = np.where(kE == DIRICHLET, 0.0, D)
    return System(topo, kind, uidx, uf, W, vol, axis, App, Apc, Acp, Acc, b, Dcoef)


def direct_solve(sysm: System, rhs=None) -> np.ndarray:
    A = sysm.matrix().tocsc()
    return spla.splu(A).solve(sysm.b if rhs is None else rhs)


def split(sysm: System, u):
    return u[:sysm.nfu], u[sysm.nfu:]
