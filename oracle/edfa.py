"""Oracle: EDFA preconditioner (test infrastructure only).

Section 3 of the paper.  Stage 1 (Algorithm 1) and stage 2 (Algorithm 2),
restated in the paper's order and notation:

* For every cell m the restricted SPD systems (eq. syst_MRHS_res and
  eq. syst_MRHS_res-F)
      -A_pipi^(m) g~^(m) = R a_ppi^(m),   -A_pipi^(m) f~^(m) = R a_pip^(m),
  with A_pipi^(m) = R A_pipi R^T on the index set Q^(m) (eq. r_r^m), one set
  for both factors.  Q^(m)_0 is the pattern of row m of A_ppi (the structural
  pattern, which always contains the cell's own unknown faces).
* Static technique: Q^(m) = Q_0 (level 0) or Q_0 plus all unknown faces of
  the cells within face-graph distance k of m (level k).
* Dynamic technique: prolonged residual (eq. prol_res)
      r = a_ppi^(m) + A_pipi R^T g~,
  grow Q by at most n = min(n_add, n_ent - n_prog) indices outside Q with
  the largest |r|, re-solve, until n_prog = n_ent or it_max sweeps.
* Pre-filtration of g~ and f~, assembly of G~ (eq. syls_syst_RED) and F~
  (eq. syls_syst_BLACK), H~ = G~ A_pipi F~ (eq. sparse_S), post-filtration.
* Inner preconditioner of A_pipi: factorised sparse approximate inverse of
  -A_pipi on the lower pattern of A_pipi.
* Stage 2: S~ = A_pp - H~, post-filtration, inner preconditioner of S~:
  ILU(0) in a multicolour order; its triangular solves are applied either
  exactly or through incomplete sparse approximate inverses (ISAI) of the
  two factors with optional refinement steps (a fully parallel substitute,
  as the paper allows for the inner solvers).
* Application (eq. EDFA_prec): t = A~^-1 r_pi; y = r_p - A_ppi t;
  z_p = S~^-1 y; z_pi = t - A~^-1 A_pip z_p.

Readings where the paper is silent (stated again in the design notes):
* selection key: |r_j| rounded to 40 significant bits, ties to the smaller
  index; candidates are indices outside Q whose key is non-zero; a sweep that adds
  nothing ends the loop; it_max defaults to n_ent;
* filtration drops |x_i| < tau * ||x||_2 with the vector's own norm (row of
  G~, column of F~, row of H~ or S~ before dropping); diagonals of H~ and S~
  are always kept;
* H~ keeps its structural pattern (entries that cancel to 0 stay stored);
* FSAI: row i on P_i = {j <= i in the pattern of A_pipi}, solve
  (-A_pipi)[P_i,P_i] y = e_i, G_F[i,P_i] = y / sqrt(y_i);  A~^-1 = -G_F^T G_F;
* colouring: greedy first fit, vertices visited by decreasing priority
  fmix32(index) (MurmurHash3 finaliser), on the graph of S~ + S~^T; rows
  reordered colour by colour, ascending index inside a colour.

Pins (tests/test_oracle_edfa.py): Proposition 1 energy minimality; the
identity g~ = c_Q - f~; r = 0 on Q; Remark 3 support; full patterns give the
exact G, F, S and a one-step solve; exact factor identities G = C - F^T and S
symmetric SPD; ILU(0) defining property; FSAI defining property; colouring
validity and agreement with a brute-force greedy; homogeneous media give
translation-invariant dynamic patterns (Test 1 discussion).
tests/test_oracle_pins.py: dynamic selection against a dense brute-force
prolonged residual per sweep, selection tie and rounding rules, pre-filtration
thresholds, Patch(k) face counts by hand and by a face-graph search, density
mu counted by hand on a one-cell grid.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .mhfe import System, NEUMANN, DIRICHLET, INTERIOR


@dataclass
class Params:
    variant: str = "dynamic"      # "static" | "dynamic"
    static_level: int = 0         # static: 0 = base pattern, k = k-ring of cells
    n_add: int = 1
    n_ent: int = 4
    it_max: int | None = None     # default n_ent
    tau: float = 0.0
    filt: str = "none"            # "none" | "pre" | "post_S" | "post_H"
    schur: str = "isai"           # S~^-1 triangular solves: "isai" | "exact"
    isai_steps: int = 1           # ISAI applications per triangular factor (1 = plain ISAI)
    static_axis: int = 0          # static level k: 0 all directions; 1/2/3 only along x/y/z;
                                  # 4 along each cell's axis of largest transmissibility


class NotSPD(RuntimeError):
    def __init__(self, cell):
        super().__init__(f"restricted matrix of cell {cell} is not SPD")
        self.cell = cell


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------
def key40(v):
    """|v| rounded to 40 significant bits, as a monotone uint64 key."""
    b = np.abs(np.asarray(v, dtype=np.float64)).view(np.uint64)
    return (b + np.uint64(1 << 12)) & ~np.uint64((1 << 13) - 1)


def fmix32(x):
    """MurmurHash3 32-bit finaliser (a bijection on uint32)."""
    h = np.asarray(x, dtype=np.uint64) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    h = (h * np.uint64(0x85EBCA6B)) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(13)
    h = (h * np.uint64(0xC2B2AE35)) & np.uint64(0xFFFFFFFF)
    h ^= h >> np.uint64(16)
    return h


def _row(M: sp.csr_matrix, i):
    a, b = M.indptr[i], M.indptr[i + 1]
    return M.indices[a:b], M.data[a:b]


def filter_keep(x, tau):
    """Mask of entries kept by filtration: |x_i| >= tau * ||x||_2."""
    return np.abs(x) >= tau * np.linalg.norm(x)


def base_pattern(s: System, m, base_rows=None):
    """Q_0^(m): structural pattern of row m of A_ppi (or of `base_rows`)."""
    M = s.Acp if base_rows is None else base_rows
    return np.array(_row(M, m)[0], dtype=np.int64)


def cell_neighbours(s: System, m):
    topo = s.topo
    out = []
    for f in topo.cell_faces[m]:
        for e in topo.face_cells[f]:
            if e >= 0 and e != m:
                out.append(int(e))
    return out


def flow_axis(s: System, m):
    """Axis d of cell m with the largest transmissibility W_(d-,d-) + W_(d+,d+): the
    direction in which the element conducts most.  Values within 1e-12 of the largest count
    as ties, which go to the smaller d (so the rounding of W^E does not decide)."""
    t = [s.W[m, 2 * d, 2 * d] + s.W[m, 2 * d + 1, 2 * d + 1] for d in range(3)]
    top = max(t)
    return next(d for d in range(3) if t[d] >= top * (1.0 - 1e-12))


def axis_neighbours(s: System, m, d):
    """Face neighbours of cell m across its two faces normal to axis d."""
    out = []
    for a in (2 * d, 2 * d + 1):
        for e in s.topo.face_cells[s.topo.cell_faces[m, a]]:
            if e >= 0 and e != m:
                out.append(int(e))
    return out


def patch_pattern(s: System, m, level, base_rows=None, axis=0):
    """Q_0 plus the unknown faces of all cells within face-graph distance `level` (axis 0),
    or within `level` steps along one axis only: x, y, z (axis 1, 2, 3) or the cell's own
    axis of largest transmissibility (axis 4), a strip in the spirit of the paper's
    directional static patterns."""
    cells = {m}
    frontier = {m}
    d = None if axis == 0 else (flow_axis(s, m) if axis == 4 else axis - 1)
    for _ in range(level):
        nxt = set()
        for e in frontier:
            nxt.update(cell_neighbours(s, e) if d is None else axis_neighbours(s, e, d))
        nxt -= cells
        cells |= nxt
        frontier = nxt
    faces = set(base_pattern(s, m, base_rows).tolist())
    for e in cells:
        for f in s.topo.cell_faces[e]:
            if s.uidx[f] >= 0:
                faces.add(int(s.uidx[f]))
    return np.array(sorted(faces), dtype=np.int64)


def restricted_matrix(s: System, Q):
    """-A_pipi^(m) = -R A_pipi R^T as a dense s x s matrix."""
    return -s.App[Q][:, Q].toarray()


def prolonged_residual(s: System, a_row_idx, a_row_val, Q, g):
    """r = a_ppi^(m) + A_pipi R^T g~ on its support (eq. prol_res).

    Returns (indices, values) over the union of the support of a and of the
    columns Q of A_pipi.  A_pipi is symmetric, so column k equals row k.
    """
    sub = s.App[Q]                                  # rows Q == columns Q
    rows_rep = np.repeat(np.arange(len(Q)), np.diff(sub.indptr))
    idx = np.concatenate([sub.indices, a_row_idx])
    val = np.concatenate([sub.data * g[rows_rep], a_row_val])
    uniq, inv = np.unique(idx, return_inverse=True)
    r = np.zeros(len(uniq))
    np.add.at(r, inv, val)
    return uniq, r


def select_new(Q, r_idx, r_val, n):
    """At most n indices outside Q with the largest |r| (40-bit key, ties -> smaller index)."""
    outside = ~np.isin(r_idx, Q) & (key40(r_val) > 0)
    cand, val = r_idx[outside], r_val[outside]
    if cand.size == 0:
        return cand
    order = np.lexsort((cand, ~key40(val)))
    return cand[order[:n]]


def _chol_solve(M, rhs, cell):
    try:
        c = sla.cho_factor(M, lower=True, check_finite=True)
    except np.linalg.LinAlgError:
        raise NotSPD(cell)
    return sla.cho_solve(c, rhs)


# ----------------------------------------------------------------------------
# Stage 1 (Algorithm 1)
# ----------------------------------------------------------------------------
@dataclass
class CellResult:
    Q: np.ndarray
    g: np.ndarray
    f: np.ndarray
    sweeps: int = 0
    added: tuple = ()       # number of indices appended by each dynamic sweep


def local_cell(s: System, m, prm: Params, base_rows=None) -> CellResult:
    """Restricted solves of cell m (static or dynamic branch of Algorithm 1)."""
    a_idx, a_val = _row(s.Acp, m)              # a_ppi^(m) (row m of A_ppi)
    f_idx, f_val = _row(s.ApcT, m)             # a_pip^(m) (column m of A_pip)
    dense_a = dict(zip(a_idx.tolist(), a_val.tolist()))
    dense_f = dict(zip(f_idx.tolist(), f_val.tolist()))
    rhs_g = lambda Q: np.array([dense_a.get(int(q), 0.0) for q in Q])
    rhs_f = lambda Q: np.array([dense_f.get(int(q), 0.0) for q in Q])
    if prm.variant == "static":
        Q = (patch_pattern(s, m, prm.static_level, base_rows, prm.static_axis)
             if prm.static_level > 0 else base_pattern(s, m, base_rows))
        M = restricted_matrix(s, Q)
        g = _chol_solve(M, rhs_g(Q), m)
        f = _chol_solve(M, rhs_f(Q), m)
        return CellResult(Q, g, f, 0)
    # dynamic technique
    Q = base_pattern(s, m, base_rows)
    g = _chol_solve(restricted_matrix(s, Q), rhs_g(Q), m)
    r_idx, r_val = prolonged_residual(s, a_idx, a_val, Q, g)
    it_max = prm.n_ent if prm.it_max is None else prm.it_max
    n_prog, k = 0, 0
    added = []
    while n_prog < prm.n_ent and k < it_max:
        k += 1
        n = min(prm.n_add, prm.n_ent - n_prog)
        new = select_new(Q, r_idx, r_val, n)
        if new.size == 0:
            break
        Q = np.concatenate([Q, new])
        added.append(int(new.size))
        n_prog += new.size
        g = _chol_solve(restricted_matrix(s, Q), rhs_g(Q), m)
        r_idx, r_val = prolonged_residual(s, a_idx, a_val, Q, g)
    f = _chol_solve(restricted_matrix(s, Q), rhs_f(Q), m)
    return CellResult(Q, g, f, k, tuple(added))


@dataclass
class Stage1:
    cells: list
    Gt: sp.csr_matrix       # G~ (Ne x Nfu)
    Ft: sp.csr_matrix       # F~ (Nfu x Ne)
    H: sp.csr_matrix        # H~ (Ne x Ne), after post-filtration on H~ if requested
    H_raw: sp.csr_matrix    # H~ before post-filtration
    GF: sp.csr_matrix       # FSAI factor of -A_pipi (lower triangular)
    GFt: sp.csr_matrix


def _ensure_apct(s: System):
    if not hasattr(s, "ApcT") or s.ApcT is None:
        s.ApcT = s.Apc.T.tocsr()
        s.ApcT.sort_indices()


def _ones(M):
    """The structural pattern of M with every stored entry (zeros included) set to 1."""
    P = sp.csr_matrix(M, copy=True)
    P.data = np.ones_like(P.data, dtype=np.float64)
    return P


def structural_product(*mats):
    """Product of sparse matrices on the structural pattern of the product.

    Values are the ordinary product; the pattern is the product of the
    structural patterns (stored entries counted as ones, explicit zeros
    included), so entries that cancel to zero are kept (as 0).
    """
    val = mats[0]
    pat = _ones(mats[0])
    for m in mats[1:]:
        val = val @ m
        pat = pat @ _ones(m)
    pat = pat.tocsr()
    pat.sort_indices()
    val = val.tocsr()
    val.sort_indices()
    out = pat.copy()
    out.data = np.zeros_like(pat.data)
    # place values of `val` on the pattern
    for r in range(out.shape[0]):
        a, b = out.indptr[r], out.indptr[r + 1]
        va, vb = val.indptr[r], val.indptr[r + 1]
        pos = np.searchsorted(out.indices[a:b], val.indices[va:vb])
        out.data[a + pos] = val.data[va:vb]
    return out


def row_filter(M: sp.csr_matrix, tau, keep_diag=True):
    """Drop |a_ij| < tau * ||a_i||_2 (row norm before dropping), diagonal kept."""
    M = M.tocsr()
    rows = []
    keep = np.zeros(M.nnz, dtype=bool)
    for i in range(M.shape[0]):
        a, b = M.indptr[i], M.indptr[i + 1]
        v = M.data[a:b]
        k = np.abs(v) >= tau * np.linalg.norm(v)
        if keep_diag:
            k |= M.indices[a:b] == i
        keep[a:b] = k
    rows = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))
    out = sp.csr_matrix((M.data[keep], (rows[keep], M.indices[keep])), shape=M.shape)
    out.sort_indices()
    return out


def fsai(s: System):
    """Factorised sparse approximate inverse of -A_pipi on the lower pattern of A_pipi."""
    A = s.App
    n = A.shape[0]
    rows, cols, vals = [], [], []
    for i in range(n):
        idx, _ = _row(A, i)
        P = np.sort(idx[idx <= i])
        M = -A[P][:, P].toarray()
        e = np.zeros(len(P))
        e[-1] = 1.0
        y = _chol_solve(M, e, -1 - i)
        y = y / np.sqrt(y[-1])
        rows.append(np.full(len(P), i)); cols.append(P); vals.append(y)
    GF = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(n, n))
    GF.sort_indices()
    return GF


# ----------------------------------------------------------------------------
# Independent per-cell work over a process pool: the restricted solves of
# Algorithm 1 are independent by construction (Remark 5), as the paper's parfor uses.
# The pool only distributes calls; every call is the serial function unchanged.
# ----------------------------------------------------------------------------
_POOL_CTX = None


def _pool_init(ctx):
    global _POOL_CTX
    _POOL_CTX = ctx


def _pool_cells(rng):
    s, prm, base_rows = _POOL_CTX
    return [local_cell(s, m, prm, base_rows) for m in range(*rng)]


def _pool_map(fn, ctx, n, workers):
    """[fn over ranges of [0, n)] concatenated in order; serial when workers <= 1 or when the
    work is too small to pay for starting the pool."""
    if workers <= 1 or n < 2000:
        _pool_init(ctx)
        return fn((0, n))
    import multiprocessing as mp
    step = -(-n // (4 * workers))
    ranges = [(a, min(a + step, n)) for a in range(0, n, step)]
    with mp.get_context("spawn").Pool(workers, initializer=_pool_init, initargs=(ctx,)) as pool:
        parts = pool.map(fn, ranges)
    return [x for part in parts for x in part]


def stage1(s: System, prm: Params, base_rows=None, workers=1) -> Stage1:
    _ensure_apct(s)
    ne, nfu = s.ne, s.nfu
    res = _pool_map(_pool_cells, (s, prm, base_rows), ne, workers)
    gr, gc, gv, fr, fc, fv = [], [], [], [], [], []
    for m, cr in enumerate(res):
        kg = filter_keep(cr.g, prm.tau) if prm.filt == "pre" else np.ones(len(cr.Q), bool)
        kf = filter_keep(cr.f, prm.tau) if prm.filt == "pre" else np.ones(len(cr.Q), bool)
        gr.append(np.full(kg.sum(), m)); gc.append(cr.Q[kg]); gv.append(cr.g[kg])
        fr.append(cr.Q[kf]); fc.append(np.full(kf.sum(), m)); fv.append(cr.f[kf])
    Gt = sp.csr_matrix((np.concatenate(gv), (np.concatenate(gr), np.concatenate(gc))), shape=(ne, nfu))
    Ft = sp.csr_matrix((np.concatenate(fv), (np.concatenate(fr), np.concatenate(fc))), shape=(nfu, ne))
    Gt.sort_indices()
    Ft.sort_indices()
    H_raw = structural_product(Gt, s.App, Ft)
    H = row_filter(H_raw, prm.tau) if prm.filt == "post_H" else H_raw
    GF = fsai(s)
    GFt = GF.T.tocsr()
    GFt.sort_indices()
    return Stage1(res, Gt, Ft, H, H_raw, GF, GFt)


# ----------------------------------------------------------------------------
# Stage 2 (Algorithm 2)
# ----------------------------------------------------------------------------
def greedy_coloring(P: sp.csr_matrix):
    """Greedy first-fit colouring of the graph of P + P^T, vertices by decreasing fmix32.

    The graph is structural: every stored entry is an edge, explicit zeros included (the
    patterns keep entries that cancel to zero), so the sum is taken on patterns of ones."""
    n = P.shape[0]
    ones = _ones(P)
    G = (ones + ones.T).tocsr()
    order = np.argsort(-fmix32(np.arange(n)).astype(np.int64), kind="stable")
    color = -np.ones(n, dtype=np.int64)
    for v in order:
        nb = G.indices[G.indptr[v]:G.indptr[v + 1]]
        used = set(color[nb[(nb != v)]].tolist())
        c = 0
        while c in used:
            c += 1
        color[v] = c
    return color


def color_permutation(color):
    """perm[new] = old: colour by colour, ascending index inside a colour."""
    return np.lexsort((np.arange(len(color)), color))


def ilu0(B: sp.csr_matrix):
    """ILU(0) (IKJ form) of B on its own pattern: B ~ L U, L unit lower (strict part stored)."""
    B = B.tocsr()
    B.sort_indices()
    n = B.shape[0]
    Lr, Lc, Lv, Ur, Uc, Uv = [], [], [], [], [], []
    urow = [None] * n
    for i in range(n):
        cols, vals = _row(B, i)
        row = dict(zip(cols.tolist(), vals.astype(float).tolist()))
        for k in sorted(c for c in row if c < i):
            ucols, uvals, ukk = urow[k]
            lik = row[k] / ukk
            row[k] = lik
            for j, ukj in zip(ucols, uvals):
                if j > k and j in row:
                    row[j] -= lik * ukj
        if i not in row or row[i] == 0.0:
            raise ZeroDivisionError(f"zero pivot in ILU(0) at row {i}")
        lc = sorted(c for c in row if c < i)
        uc = sorted(c for c in row if c >= i)
        Lr += [i] * len(lc); Lc += lc; Lv += [row[c] for c in lc]
        Ur += [i] * len(uc); Uc += uc; Uv += [row[c] for c in uc]
        urow[i] = (np.array(uc), np.array([row[c] for c in uc]), row[i])
    L = sp.csr_matrix((Lv, (Lr, Lc)), shape=(n, n))
    U = sp.csr_matrix((Uv, (Ur, Uc)), shape=(n, n))
    L.sort_indices(); U.sort_indices()
    return L, U


def unit_lower(L: sp.csr_matrix):
    """I + L keeping every stored entry of L (explicit zeros included) in the pattern."""
    L = L.tocoo()
    n = L.shape[0]
    M = sp.csr_matrix((np.concatenate([L.data, np.ones(n)]),
                       (np.concatenate([L.row, np.arange(n)]), np.concatenate([L.col, np.arange(n)]))),
                      shape=L.shape)
    M.sort_indices()
    return M


def _isai_row(T: sp.csr_matrix, i):
    P = T.indices[T.indptr[i]:T.indptr[i + 1]]
    sub = T[P][:, P].toarray()
    e = np.zeros(len(P))
    e[np.searchsorted(P, i)] = 1.0
    return P, np.linalg.solve(sub.T, e)


def isai(T: sp.csr_matrix):
    """Incomplete sparse approximate inverse of a triangular factor on its own pattern.

    Row i of M solves (T[P_i, P_i])^T m = e_i with P_i the pattern of row i of T
    (diagonal included), so that (M T)_ij = delta_ij for j in P_i.
    """
    T = T.tocsr()
    T.sort_indices()
    rows, cols, vals = [], [], []
    for i in range(T.shape[0]):
        P, m = _isai_row(T, i)
        rows.append(np.full(len(P), i)); cols.append(P); vals.append(m)
    M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=T.shape)
    M.sort_indices()
    return M


@dataclass
class Stage2:
    S: sp.csr_matrix         # S~ (after post-filtration on S~ if requested)
    color: np.ndarray
    perm: np.ndarray         # perm[new] = old
    L: sp.csr_matrix         # in the permuted order, strict lower part of the unit factor
    U: sp.csr_matrix         # in the permuted order, upper part with diagonal
    ML: sp.csr_matrix = None  # ISAI of the unit lower factor (I + L)
    MU: sp.csr_matrix = None  # ISAI of U


def structural_sub(A: sp.csr_matrix, H: sp.csr_matrix):
    """A - H on the union of the two structural patterns (zeros kept)."""
    pa, ph = _ones(A), _ones(H)
    pat = (pa + ph).tocsr()
    pat.sort_indices()
    out = pat.copy()
    out.data = np.zeros_like(pat.data)
    for M, sgn in ((A.tocsr(), 1.0), (H.tocsr(), -1.0)):
        M.sort_indices()
        for r in range(out.shape[0]):
            a, b = out.indptr[r], out.indptr[r + 1]
            ma, mb = M.indptr[r], M.indptr[r + 1]
            pos = np.searchsorted(out.indices[a:b], M.indices[ma:mb])
            out.data[a + pos] += sgn * M.data[ma:mb]
    return out


def stage2(s: System, st1: Stage1, prm: Params) -> Stage2:
    S = structural_sub(s.Acc, st1.H)
    if prm.filt == "post_S":
        S = row_filter(S, prm.tau)
    color = greedy_coloring(S)
    perm = color_permutation(color)
    B = S[perm][:, perm].tocsr()
    L, U = ilu0(B)
    ML = MU = None
    if prm.schur == "isai":
        Lf = unit_lower(L)
        ML, MU = isai(Lf), isai(U)
    return Stage2(S, color, perm, L, U, ML, MU)


# ----------------------------------------------------------------------------
# Application (eq. EDFA_prec)
# ----------------------------------------------------------------------------
@dataclass
class Edfa:
    sys: System
    prm: Params
    st1: Stage1
    st2: Stage2
    inv_perm: np.ndarray = field(default=None)

    def __post_init__(self):
        self.inv_perm = np.empty_like(self.st2.perm)
        self.inv_perm[self.st2.perm] = np.arange(len(self.st2.perm))

    def apply_App_inv(self, v):
        """A~_pipi^-1 v = -G_F^T G_F v."""
        return -(self.st1.GFt @ (self.st1.GF @ v))

    def apply_S_inv(self, y):
        """S~^-1 y with the multicolour ILU(0) factors.

        "exact": forward (unit L) and backward (U) substitution.
        "isai":  w = M_L b, then (steps-1) times w += M_L (b - (I+L) w); the same
                 with M_U and U.
        """
        if self.prm.schur == "isai":
            return self._apply_isai(y, transpose=False)
        L, U = self.st2.L, self.st2.U
        b = y[self.st2.perm]
        n = len(b)
        w = np.zeros(n)
        for i in range(n):
            c, v = _row(L, i)
            w[i] = b[i] - v @ w[c]
        z = np.zeros(n)
        for i in range(n - 1, -1, -1):
            c, v = _row(U, i)
            d = v[c == i][0]
            m = c > i
            z[i] = (w[i] - v[m] @ z[c[m]]) / d
        return z[self.inv_perm]

    def _apply_isai(self, y, transpose):
        st = self.st2
        n = len(y)
        Lf = unit_lower(st.L)
        b = y[st.perm]
        k = self.prm.isai_steps
        if not transpose:
            w = st.ML @ b
            for _ in range(k - 1):
                w = w + st.ML @ (b - Lf @ w)
            z = st.MU @ w
            for _ in range(k - 1):
                z = z + st.MU @ (w - st.U @ z)
        else:
            # (M_U M_L)^T = M_L^T M_U^T with the refinement steps transposed
            w = st.MU.T @ b
            for _ in range(k - 1):
                w = w + st.MU.T @ (b - st.U.T @ w)
            z = st.ML.T @ w
            for _ in range(k - 1):
                z = z + st.ML.T @ (w - Lf.T @ z)
        return z[self.inv_perm]

    def apply_S_inv_T(self, y):
        """S~^-T y: solve U^T w = b (forward), then L^T z = w (backward)."""
        if self.prm.schur == "isai":
            return self._apply_isai(y, transpose=True)
        L, U = self.st2.L, self.st2.U
        b = y[self.st2.perm]
        UT, LT = U.T.tocsr(), L.T.tocsr()
        UT.sort_indices(); LT.sort_indices()
        n = len(b)
        w = np.zeros(n)
        for i in range(n):
            c, v = _row(UT, i)
            d = v[c == i][0]
            m = c < i
            w[i] = (b[i] - v[m] @ w[c[m]]) / d
        z = np.zeros(n)
        for i in range(n - 1, -1, -1):
            c, v = _row(LT, i)
            z[i] = w[i] - v @ z[c]
        return z[self.inv_perm]

    def apply(self, r):
        s = self.sys
        r_pi, r_p = r[:s.nfu], r[s.nfu:]
        t = self.apply_App_inv(r_pi)
        y = r_p - s.Acp @ t
        z_p = self.apply_S_inv(y)
        z_pi = t - self.apply_App_inv(s.Apc @ z_p)
        return np.concatenate([z_pi, z_p])

    def apply_T(self, r):
        """P^-T r (transpose of eq. EDFA_prec)."""
        s = self.sys
        r_pi, r_p = r[:s.nfu], r[s.nfu:]
        t = self.apply_App_inv(r_pi)
        y = r_p - s.Apc.T @ t
        z_p = self.apply_S_inv_T(y)
        z_pi = t - self.apply_App_inv(s.Acp.T @ z_p)
        return np.concatenate([z_pi, z_p])

    def density(self):
        """Preconditioner density mu (Section 4).

        nnz() counts the entries stored for the application: the FSAI factor and its
        transpose for A~_pipi^-1, the two coupling blocks, and for S~^-1 the matrices the
        triangular solves read: M_L and M_U (ISAI, one step), plus the factors L and U when
        refinement steps use them, or L and U alone (exact substitution).
        """
        s = self.sys
        st2 = self.st2
        if self.prm.schur == "isai":
            ns = st2.ML.nnz + st2.MU.nnz
            if self.prm.isai_steps > 1:
                ns += st2.L.nnz + st2.U.nnz
        else:
            ns = st2.L.nnz + st2.U.nnz
        num = 2 * self.st1.GF.nnz + s.Apc.nnz + s.Acp.nnz + ns
        den = s.App.nnz + s.Apc.nnz + s.Acp.nnz + s.Acc.nnz
        return num / den


def build(s: System, prm: Params, workers=1) -> Edfa:
    """Stage 1 and stage 2; workers > 1 spreads the per-cell solves of stage 1 over a
    process pool (same results)."""
    st1 = stage1(s, prm, workers=workers)
    st2 = stage2(s, st1, prm)
    return Edfa(s, prm, st1, st2)
