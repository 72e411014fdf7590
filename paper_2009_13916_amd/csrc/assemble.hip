// Assembly of the MHFE-FV block system on the device.
//
// Element matrices follow the paper's eq. B_ij with the Piola map of Section 2.2;
// the rows follow eq. cont_fluxes (faces) and eq. discr_bal_FV_2 with the strong flux of
// eq. fluxes_MHFEM_STRONG (cells), i.e. the entry lists of Appendix A.  Every row is
// built by one thread from the cell matrices it touches (gather, no atomics), so the
// result is deterministic.
#include <algorithm>
#include <cmath>

#include "system.hpp"

namespace edfa {

// 3-point Gauss-Legendre rule on [0, 1].
__constant__ double c_gx[3] = {0.11270166537925831148, 0.5, 0.88729833462074168852};
__constant__ double c_gw[3] = {0.27777777777777777778, 0.44444444444444444444,
                               0.27777777777777777778};

// In-place Cholesky of an SPD n x n row-major matrix (lower part), returns false on a
// non-positive pivot.
template <int N>
__device__ inline bool chol_inplace(double (&M)[N][N]) {
  for (int j = 0; j < N; ++j) {
    double d = M[j][j];
    for (int k = 0; k < j; ++k) d -= M[j][k] * M[j][k];
    if (!(d > 0.0)) return false;
    d = sqrt(d);
    M[j][j] = d;
    for (int i = j + 1; i < N; ++i) {
      double s = M[i][j];
      for (int k = 0; k < j; ++k) s -= M[i][k] * M[j][k];
      M[i][j] = s / d;
    }
  }
  return true;
}

// Inverse of an SPD matrix given its Cholesky factor (lower part of L): out = L^-T L^-1.
template <int N>
__device__ inline void chol_inverse(const double (&L)[N][N], double (&out)[N][N]) {
  double Li[N][N];
  for (int j = 0; j < N; ++j) {
    for (int i = 0; i < N; ++i) Li[i][j] = 0.0;
    Li[j][j] = 1.0 / L[j][j];
    for (int i = j + 1; i < N; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s -= L[i][k] * Li[k][j];
      Li[i][j] = s / L[i][i];
    }
  }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
      for (int k = i; k < N; ++k) s += Li[k][i] * Li[k][j];
      out[i][j] = s;
      out[j][i] = s;
    }
}

// Per cell: B^E by quadrature, volume, W^E = (B^E)^-1, the storage coefficient and the
// previous pressure; clears axis[g] when the cell is not an axis-aligned brick with
// diagonal K (g its grid: the structural pattern is chosen per grid); records the first
// bad cell.
// Smallest tag + index of a non-finite entry of a[0, n) (tag in the bits above 40).
__global__ void k_first_nonfinite(const double *__restrict__ a, long long n, long long tag,
                                  long long *first) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    if (!isfinite(a[i])) atomicMin((unsigned long long *)first, (unsigned long long)(tag | i));
}

__global__ void k_element(const GridDesc *__restrict__ grids, int ngrid, int ne, double *W,
                          double *vol, double *cstore, double *p_prev, int *axis, int *bad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int gi = grid_of(grids, ngrid, e, true);
  const GridDesc G = grids[gi];
  int i, j, k;
  cell_ijk(G, e, i, j, k);
  double X[8][3];
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        const int nid = (i + a) + (G.nx + 1) * ((j + b) + (G.ny + 1) * (k + c));
        for (int d = 0; d < 3; ++d) X[a + 2 * b + 4 * c][d] = G.nodes[3 * (size_t)nid + d];
      }
  const int le = e - G.cell0;
  const double *Kp = G.K + 6 * (size_t)le;
  double Km[3][3] = {{Kp[0], Kp[3], Kp[4]}, {Kp[3], Kp[1], Kp[5]}, {Kp[4], Kp[5], Kp[2]}};
  bool ok = chol_inplace<3>(Km);
  double Ki[3][3];
  if (ok) chol_inverse<3>(Km, Ki);
  bool cell_axis = (Kp[3] == 0.0 && Kp[4] == 0.0 && Kp[5] == 0.0);
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        const int q = a + 2 * b + 4 * c;
        cell_axis = cell_axis && X[q][0] == X[a][0] && X[q][1] == X[2 * b][1] &&
                    X[q][2] == X[4 * c][2];
      }
  double B[6][6];
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) B[a][b] = 0.0;
  double V = 0.0;
  for (int qz = 0; qz < 3 && ok; ++qz)
    for (int qy = 0; qy < 3; ++qy)
      for (int qx = 0; qx < 3; ++qx) {
        const double xh[3] = {c_gx[qx], c_gx[qy], c_gx[qz]};
        const double w = c_gw[qx] * c_gw[qy] * c_gw[qz];
        const double s[3][2] = {{1 - xh[0], xh[0]}, {1 - xh[1], xh[1]}, {1 - xh[2], xh[2]}};
        double DF[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};   // DF[row][col d]
        for (int c = 0; c < 2; ++c)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
              const int q = a + 2 * b + 4 * c;
              const double dx = (a ? 1.0 : -1.0) * s[1][b] * s[2][c];
              const double dy = s[0][a] * (b ? 1.0 : -1.0) * s[2][c];
              const double dz = s[0][a] * s[1][b] * (c ? 1.0 : -1.0);
              for (int r = 0; r < 3; ++r) {
                DF[r][0] += dx * X[q][r];
                DF[r][1] += dy * X[q][r];
                DF[r][2] += dz * X[q][r];
              }
            }
        const double J = DF[0][0] * (DF[1][1] * DF[2][2] - DF[1][2] * DF[2][1]) -
                         DF[0][1] * (DF[1][0] * DF[2][2] - DF[1][2] * DF[2][0]) +
                         DF[0][2] * (DF[1][0] * DF[2][1] - DF[1][1] * DF[2][0]);
        if (!(J > 0.0)) {
          ok = false;
          break;
        }
        V += w * J;
        // Piola image (times J) of the reference fields: column d of DF times phi_a
        double Vf[6][3], KV[6][3];
        for (int a = 0; a < 6; ++a) {
          const int d = a >> 1;
          const double phi = (a & 1) ? xh[d] : xh[d] - 1.0;
          for (int r = 0; r < 3; ++r) Vf[a][r] = DF[r][d] * phi;
          for (int r = 0; r < 3; ++r)
            KV[a][r] = Ki[r][0] * Vf[a][0] + Ki[r][1] * Vf[a][1] + Ki[r][2] * Vf[a][2];
        }
        const double wj = w / J;
        for (int a = 0; a < 6; ++a)
          for (int b = a; b < 6; ++b)
            B[a][b] += wj * (Vf[a][0] * KV[b][0] + Vf[a][1] * KV[b][1] + Vf[a][2] * KV[b][2]);
      }
  if (ok) {
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < a; ++b) B[a][b] = B[b][a];
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b) B[a][b] *= G.gamma;
    ok = chol_inplace<6>(B);
  }
  if (!ok) {
    atomicMin(bad, e);
    return;
  }
  double Wm[6][6];
  chol_inverse<6>(B, Wm);
  if (!cell_axis) atomicAnd(axis + gi, 0);
  double *We = W + 36 * (size_t)e;
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) {
      double v = Wm[a][b];
      if (cell_axis && (a >> 1) != (b >> 1)) v = 0.0;
      We[6 * a + b] = v;
    }
  vol[e] = V;
  cstore[e] = G.c ? G.c[le] : G.c_scalar;
  p_prev[e] = G.p_prev ? G.p_prev[le] : 0.0;
}

// Face classification and unknown flag.
__global__ void k_face_kind(const GridDesc *__restrict__ grids, int ngrid, int nf, int8_t *kind,
                            int *flag) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const GridDesc &G = grids[grid_of(grids, ngrid, f, false)];
  int cm, cp, dir;
  face_cells(G, f, cm, cp, dir);
  int8_t kd = FACE_INTERIOR;
  if (cm < 0 || cp < 0) kd = (G.bc_type[f - G.face0] == EDFA_BC_DIRICHLET) ? FACE_DIRICHLET : FACE_NEUMANN;
  kind[f] = kd;
  flag[f] = kd != FACE_DIRICHLET;
}

__global__ void k_face_unknowns(int nf, const int8_t *__restrict__ kind, int *uidx, int *ufaces) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  if (kind[f] == FACE_DIRICHLET) {
    uidx[f] = -1;
  } else {
    ufaces[uidx[f]] = f;
  }
}

struct RowCtx {
  const GridDesc *grids;
  int ngrid;
  int nfu;
  const double *W;
  const double *vol;
  const double *cstore;
  const double *p_prev;
  double dt;
  const int8_t *kind;
  const int *uidx;
  const int *ufaces;
};

__device__ inline bool structural(int axis, int a, int b) { return !axis || (a >> 1) == (b >> 1); }

__device__ inline double face_bc_value(const GridDesc &G, int f) { return G.bc_value[f - G.face0]; }

constexpr int ROW_MAX = 48;

// Build one row of [A | b].  Entries are appended in a fixed order, then sorted by column
// and duplicates merged in that order.  Returns the entry count.
template <bool FILL>
__device__ int build_row(const RowCtx &X, int r, int *cols, double *vals, double &rhs,
                         double &diag0, double &rhs0) {
  int cnt = 0;
  rhs = 0.0;
  auto add = [&](int c, double v) {
    cols[cnt] = c;
    vals[cnt] = v;
    ++cnt;
  };
  if (r < X.nfu) {
    // ---- face row: sum of the local fluxes q_i^E of the cells sharing the face
    const int f = X.ufaces[r];
    const GridDesc &G = X.grids[grid_of(X.grids, X.ngrid, f, false)];
    int cm, cp, dir;
    face_cells(G, f, cm, cp, dir);
    for (int side = 0; side < 2; ++side) {
      const int E = side == 0 ? cm : cp;
      if (E < 0) continue;
      const int a = 2 * dir + (side == 0 ? 1 : 0);
      int i, j, k;
      cell_ijk(G, E, i, j, k);
      const double *We = X.W + 36 * (size_t)E;
      double L = 0.0;
      for (int b = 0; b < 6; ++b) L += We[6 * a + b];
      for (int b = 0; b < 6; ++b) {
        if (!structural(G.axis, a, b)) continue;
        const int g = cell_face(G, i, j, k, b);
        const double v = -We[6 * a + b];
        const int u = X.uidx[g];
        if (u >= 0)
          add(u, v);
        else
          rhs -= v * face_bc_value(G, g);
      }
      add(X.nfu + E, L);
    }
    if (X.kind[f] == FACE_NEUMANN) rhs += face_bc_value(G, f);
  } else {
    // ---- cell row: FV balance with the strong inter-element fluxes
    const int E = r - X.nfu;
    const GridDesc &G = X.grids[grid_of(X.grids, X.ngrid, E, true)];
    int i, j, k;
    cell_ijk(G, E, i, j, k);
    const double *We = X.W + 36 * (size_t)E;
    int fc[6], nb[6];
    int8_t kd[6];
    double L[6], Cc[6], Dc[6];
    for (int a = 0; a < 6; ++a) {
      fc[a] = cell_face(G, i, j, k, a);
      nb[a] = cell_nbr(G, i, j, k, a);
      kd[a] = X.kind[fc[a]];
      L[a] = 0.0;
      for (int b = 0; b < 6; ++b) L[a] += We[6 * a + b];
      if (kd[a] == FACE_INTERIOR) {
        const double wd = We[7 * a];
        const double wn = X.W[36 * (size_t)nb[a] + 7 * (a ^ 1)];
        Cc[a] = wn / (wd + wn);
        Dc[a] = wd / (wd + wn);
      } else if (kd[a] == FACE_NEUMANN) {
        Cc[a] = 0.0;
        Dc[a] = 1.0;
      } else {
        Cc[a] = 1.0;
        Dc[a] = 0.0;
      }
    }
    double own[6] = {0, 0, 0, 0, 0, 0};
    double dg = 0.0;
    for (int a = 0; a < 6; ++a) dg += Cc[a] * L[a];
    for (int a = 0; a < 6; ++a) {
      for (int b = 0; b < 6; ++b)
        if (b != a && structural(G.axis, a, b)) own[b] -= Cc[a] * We[6 * a + b];
      if (kd[a] == FACE_DIRICHLET) own[a] -= We[7 * a];
    }
    double r0 = 0.0;
    for (int a = 0; a < 6; ++a) {
      if (kd[a] == FACE_INTERIOR) {
        const int En = nb[a];
        const int ap = a ^ 1;
        const double *Wn = X.W + 36 * (size_t)En;
        double Ln = 0.0;
        for (int b = 0; b < 6; ++b) Ln += Wn[6 * ap + b];
        add(X.nfu + En, -Dc[a] * Ln);
        int ni, nj, nk;
        cell_ijk(G, En, ni, nj, nk);
        for (int bp = 0; bp < 6; ++bp) {
          if (bp == ap || !structural(G.axis, ap, bp)) continue;
          const int g = cell_face(G, ni, nj, nk, bp);
          const double v = Dc[a] * Wn[6 * ap + bp];
          const int u = X.uidx[g];
          if (u >= 0)
            add(u, v);
          else
            r0 -= v * face_bc_value(G, g);
        }
      } else if (kd[a] == FACE_NEUMANN) {
        r0 -= face_bc_value(G, fc[a]);
      }
    }
    for (int b = 0; b < 6; ++b) {
      const int u = X.uidx[fc[b]];
      if (u >= 0)
        add(u, own[b]);
      else
        r0 -= own[b] * face_bc_value(G, fc[b]);
    }
    const double V = X.vol[E];
    const int le = E - G.cell0;
    const double src = G.source ? G.source[le] : 0.0;
    r0 += V * src;
    const double stor = V * X.cstore[E] / X.dt;
    add(X.nfu + E, dg + stor);
    diag0 = dg;
    rhs0 = r0;
    rhs = r0 + stor * X.p_prev[E];
  }
  // sort by column (insertion sort) and merge duplicates in insertion order
  for (int p = 1; p < cnt; ++p) {
    const int c = cols[p];
    const double v = vals[p];
    int q = p - 1;
    while (q >= 0 && cols[q] > c) {
      cols[q + 1] = cols[q];
      vals[q + 1] = vals[q];
      --q;
    }
    cols[q + 1] = c;
    vals[q + 1] = v;
  }
  int m = 0;
  for (int p = 0; p < cnt; ++p) {
    if (m > 0 && cols[m - 1] == cols[p])
      vals[m - 1] += vals[p];
    else {
      cols[m] = cols[p];
      vals[m] = vals[p];
      ++m;
    }
  }
  return m;
}

__global__ void k_row_count(RowCtx X, int n, int *len) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int cols[ROW_MAX];
  double vals[ROW_MAX];
  double rhs, d0, r0;
  len[r] = build_row<false>(X, r, cols, vals, rhs, d0, r0);
}

__global__ void k_row_fill(RowCtx X, int n, const int *__restrict__ rowptr, int *col, double *val,
                           double *b, int *split, double *diag0, double *rhs0, int *diag_pos) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int cols[ROW_MAX];
  double vals[ROW_MAX];
  double rhs, d0 = 0.0, r0 = 0.0;
  const int m = build_row<true>(X, r, cols, vals, rhs, d0, r0);
  const int base = rowptr[r];
  int sp = m;
  for (int p = 0; p < m; ++p) {
    col[base + p] = cols[p];
    val[base + p] = vals[p];
    if (sp == m && cols[p] >= X.nfu) sp = p;
    if (r >= X.nfu && cols[p] == r) diag_pos[r - X.nfu] = base + p;
  }
  split[r] = base + sp;
  b[r] = rhs;
  if (r >= X.nfu) {
    diag0[r - X.nfu] = d0;
    rhs0[r - X.nfu] = r0;
  }
}

// Lengths of one block of each row: left (columns < nfu) or right part.
__global__ void k_block_len(const int *__restrict__ rowptr, const int *__restrict__ split, int row0,
                            int rows, int left, int *len) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int R = row0 + r;
  len[r] = left ? split[R] - rowptr[R] : rowptr[R + 1] - split[R];
}

__global__ void k_block_copy(const int *__restrict__ rowptr, const int *__restrict__ split,
                             const int *__restrict__ col, const double *__restrict__ val, int row0,
                             int rows, int left, int shift, const int *__restrict__ orow,
                             int *ocol, double *oval) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int R = row0 + r;
  const int a = left ? rowptr[R] : split[R];
  const int b = left ? split[R] : rowptr[R + 1];
  int o = orow[r];
  for (int p = a; p < b; ++p, ++o) {
    ocol[o] = col[p] - shift;
    oval[o] = val[p];
  }
}

__global__ void k_find_pos(const int *__restrict__ rowptr, const int *__restrict__ col, int rows,
                           int *pos) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  for (int p = rowptr[r]; p < rowptr[r + 1]; ++p)
    if (col[p] == r) pos[r] = p;
}

static void extract_block(edfa_system_s &S, const int *split, int row0, int rows, int left,
                          int shift, int ncols, Csr<double> &out, hipStream_t s) {
  out.rowptr.ensure((size_t)rows + 1);
  if (rows > 0) {
    hipLaunchKernelGGL(k_block_len, dim3(ceil_div(rows, 256)), dim3(256), 0, s, S.A.rowptr.p,
                       split, row0, rows, left, out.rowptr.p);
    EDFA_CHECK_LAUNCH();
  }
  const int64_t nnz = exclusive_scan(out.rowptr.p, out.rowptr.p, rows, S.tmp, s);
  out.rows = rows;
  out.cols = ncols;
  out.nnz = nnz;
  out.col.ensure((size_t)nnz);
  out.val.ensure((size_t)nnz);
  if (rows > 0) {
    hipLaunchKernelGGL(k_block_copy, dim3(ceil_div(rows, 256)), dim3(256), 0, s, S.A.rowptr.p,
                       split, S.A.col.p, S.A.val.p, row0, rows, left, shift, out.rowptr.p,
                       out.col.p, out.val.p);
    EDFA_CHECK_LAUNCH();
  }
}

void compute_ranges(edfa_system_s &S, hipStream_t s);

RowCtx row_ctx(const edfa_system_s &S) {
  RowCtx X;
  X.grids = S.grids.p;
  X.ngrid = S.ngrid;
  X.nfu = S.nfu;
  X.W = S.W.p;
  X.vol = S.vol.p;
  X.cstore = S.cstore.p;
  X.p_prev = S.p_prev.p;
  X.dt = S.dt;
  X.kind = S.kind.p;
  X.uidx = S.uidx.p;
  X.ufaces = S.ufaces.p;
  return X;
}

void assemble_system(edfa_system_s &S, const edfa_problem *probs, int count, hipStream_t s) {
  if (count < 1 || !probs) fail(EDFA_ERR_ARG, "edfa_assemble: need at least one grid");
  long long ne = 0, nf = 0;
  S.grids_h.clear();
  double dt = probs[0].dt;
  for (int g = 0; g < count; ++g) {
    const edfa_problem &P = probs[g];
    if (P.nx < 1 || P.ny < 1 || P.nz < 1)
      fail(EDFA_ERR_ARG, "grid %d: cells per direction must be >= 1", g);
    if (!P.nodes || !P.K || !P.bc_type || !P.bc_value)
      fail(EDFA_ERR_ARG, "grid %d: nodes, K, bc_type and bc_value are required", g);
    if (!(P.gamma > 0.0) || !(P.dt > 0.0)) fail(EDFA_ERR_ARG, "grid %d: gamma and dt must be > 0", g);
    if (P.dt != dt) fail(EDFA_ERR_ARG, "grid %d: all grids of a batch share one dt", g);
    GridDesc G{};
    G.nx = P.nx;
    G.ny = P.ny;
    G.nz = P.nz;
    G.cell0 = (int)ne;
    G.face0 = (int)nf;
    G.nfx = (P.nx + 1) * P.ny * P.nz;
    G.nfy = P.nx * (P.ny + 1) * P.nz;
    G.ncell = P.nx * P.ny * P.nz;
    G.nface = G.nfx + G.nfy + P.nx * P.ny * (P.nz + 1);
    G.nodes = P.nodes;
    G.K = P.K;
    G.c = P.c;
    G.c_scalar = P.c_scalar;
    G.gamma = P.gamma;
    G.bc_type = P.bc_type;
    G.bc_value = P.bc_value;
    G.source = P.source;
    G.p_prev = P.p_prev;
    ne += G.ncell;
    nf += G.nface;
    S.grids_h.push_back(G);
  }
  if (ne + nf > 0x7fffffffLL / 4) fail(EDFA_ERR_ARG, "system too large for 32-bit indices");
  S.ngrid = count;
  S.ne = (int)ne;
  S.nf = (int)nf;
  S.dt = dt;
  S.grids.ensure(count);
  EDFA_HIP(hipMemcpyAsync(S.grids.p, S.grids_h.data(), sizeof(GridDesc) * count,
                          hipMemcpyHostToDevice, s));

  // non-finite inputs: the first offending entry of each array (per grid) is reported
  {
    DBuf<long long> bad;
    bad.ensure(1);
    const long long none = 0x7fffffffffffffffLL;
    EDFA_HIP(hipMemcpyAsync(bad.p, &none, sizeof(none), hipMemcpyHostToDevice, s));
    struct Arr {
      const double *p;
      long long n;
    };
    const char *names[6] = {"nodes", "K", "c", "bc_value", "p_prev", "source"};
    for (int g = 0; g < count; ++g) {
      const GridDesc &G = S.grids_h[g];
      const long long nn = (long long)(G.nx + 1) * (G.ny + 1) * (G.nz + 1);
      const Arr arrs[6] = {{G.nodes, 3 * nn}, {G.K, 6ll * G.ncell}, {G.c, G.c ? G.ncell : 0},
                           {G.bc_value, G.nface}, {G.p_prev, G.p_prev ? G.ncell : 0},
                           {G.source, G.source ? G.ncell : 0}};
      for (int a = 0; a < 6; ++a)
        if (arrs[a].n > 0) {
          hipLaunchKernelGGL(k_first_nonfinite, dim3(std::min<long long>(ceil_div(arrs[a].n, 256), 4096)),
                             dim3(256), 0, s, arrs[a].p, arrs[a].n, (long long)(g * 6 + a) << 40,
                             bad.p);
          EDFA_CHECK_LAUNCH();
        }
    }
    const long long fb = read_scalar(bad.p, s);
    if (fb != none) {
      const int ga = (int)(fb >> 40);
      fail(EDFA_ERR_NAN, "grid %d: %s[%lld] is not finite", ga / 6, names[ga % 6],
           fb & ((1ll << 40) - 1));
    }
    for (int g = 0; g < count; ++g)
      if (!probs[g].c && !std::isfinite(probs[g].c_scalar))
        fail(EDFA_ERR_NAN, "grid %d: c_scalar is not finite", g);
  }

  // element matrices
  S.W.ensure(36 * (size_t)ne);
  S.vol.ensure(ne);
  S.cstore.ensure(ne);
  S.p_prev.ensure(ne);
  // flags: [0, count) the per-grid axis structure, [count] the first bad cell
  DBuf<int> flags;
  flags.ensure((size_t)count + 1);
  std::vector<int> fl((size_t)count + 1, 1);
  fl[count] = 0x7fffffff;
  EDFA_HIP(hipMemcpyAsync(flags.p, fl.data(), sizeof(int) * fl.size(), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_element, dim3(ceil_div(ne, 128)), dim3(128), 0, s, S.grids.p, count,
                     (int)ne, S.W.p, S.vol.p, S.cstore.p, S.p_prev.p, flags.p, flags.p + count);
  EDFA_CHECK_LAUNCH();
  EDFA_HIP(hipMemcpyAsync(fl.data(), flags.p, sizeof(int) * fl.size(), hipMemcpyDeviceToHost, s));
  EDFA_HIP(hipStreamSynchronize(s));
  if (fl[count] != 0x7fffffff)
    fail(EDFA_ERR_NOT_SPD, "cell %d: conductivity tensor not SPD or non-positive Jacobian",
         fl[count]);
  // each grid of a batch keeps its own structural pattern
  S.axis = 1;
  for (int g = 0; g < count; ++g) {
    S.grids_h[g].axis = fl[g];
    S.axis = S.axis && fl[g];
  }
  EDFA_HIP(hipMemcpyAsync(S.grids.p, S.grids_h.data(), sizeof(GridDesc) * count,
                          hipMemcpyHostToDevice, s));

  // faces and unknown numbering
  // the boundary values outlive the call (the adjoint gradient reads them)
  S.bcv.ensure(nf);
  for (int g = 0; g < count; ++g)
    EDFA_HIP(hipMemcpyAsync(S.bcv.p + S.grids_h[g].face0, probs[g].bc_value,
                            sizeof(double) * S.grids_h[g].nface, hipMemcpyDeviceToDevice, s));
  S.kind.ensure(nf);
  S.uidx.ensure((size_t)nf + 1);
  hipLaunchKernelGGL(k_face_kind, dim3(ceil_div(nf, 256)), dim3(256), 0, s, S.grids.p, count,
                     (int)nf, S.kind.p, S.uidx.p);
  EDFA_CHECK_LAUNCH();
  S.nfu = (int)exclusive_scan(S.uidx.p, S.uidx.p, (int)nf, S.tmp, s);
  S.n = S.nfu + S.ne;
  S.ufaces.ensure(S.nfu);
  hipLaunchKernelGGL(k_face_unknowns, dim3(ceil_div(nf, 256)), dim3(256), 0, s, (int)nf, S.kind.p,
                     S.uidx.p, S.ufaces.p);
  EDFA_CHECK_LAUNCH();

  // rows
  RowCtx X = row_ctx(S);
  const int n = S.n;
  S.A.rowptr.ensure((size_t)n + 1);
  hipLaunchKernelGGL(k_row_count, dim3(ceil_div(n, 128)), dim3(128), 0, s, X, n, S.A.rowptr.p);
  EDFA_CHECK_LAUNCH();
  const int64_t nnz = exclusive_scan(S.A.rowptr.p, S.A.rowptr.p, n, S.tmp, s);
  S.A.rows = S.A.cols = n;
  S.A.nnz = nnz;
  S.A.col.ensure(nnz);
  S.A.val.ensure(nnz);
  S.b.ensure(n);
  S.diag0.ensure(ne);
  S.rhs0.ensure(ne);
  S.diag_pos_A.ensure(ne);
  DBuf<int> split;
  split.ensure(n);
  hipLaunchKernelGGL(k_row_fill, dim3(ceil_div(n, 128)), dim3(128), 0, s, X, n, S.A.rowptr.p,
                     S.A.col.p, S.A.val.p, S.b.p, split.p, S.diag0.p, S.rhs0.p, S.diag_pos_A.p);
  EDFA_CHECK_LAUNCH();

  // blocks
  extract_block(S, split.p, 0, S.nfu, 1, 0, S.nfu, S.Afp, s);
  S.afp_max = -1;
  extract_block(S, split.p, 0, S.nfu, 0, S.nfu, S.ne, S.Afc, s);
  extract_block(S, split.p, S.nfu, S.ne, 1, 0, S.nfu, S.Acf, s);
  extract_block(S, split.p, S.nfu, S.ne, 0, S.nfu, S.ne, S.Acc, s);
  S.diag_pos_pp.ensure(ne);
  hipLaunchKernelGGL(k_find_pos, dim3(ceil_div(ne, 256)), dim3(256), 0, s, S.Acc.rowptr.p,
                     S.Acc.col.p, S.ne, S.diag_pos_pp.p);
  EDFA_CHECK_LAUNCH();
  csr_transpose(S.Afc, S.AfcT, S.tmp, S.tmp2, s);
  build_sell(S.A, S.A_s, S.tmp, s);
  build_sell(S.Acf, S.Acf_s, S.tmp, s);
  build_sell(S.Afc, S.Afc_s, S.tmp, s);
  build_sell(S.AfcT, S.AfcT_s, S.tmp, s);
  EDFA_HIP(hipStreamSynchronize(s));

  S.avg_A = S.n ? (float)S.A.nnz / S.n : 0.f;
  S.avg_fp = S.nfu ? (float)S.Afp.nnz / S.nfu : 0.f;
  S.avg_fc = S.nfu ? (float)S.Afc.nnz / S.nfu : 0.f;
  S.avg_cf = S.ne ? (float)S.Acf.nnz / S.ne : 0.f;
  S.avg_cc = S.ne ? (float)S.Acc.nnz / S.ne : 0.f;
  compute_ranges(S, s);
}

// Per-grid unknown ranges from the face-unknown map (host, after assembly).
void compute_ranges(edfa_system_s &S, hipStream_t s) {
  std::vector<int> ufaces(S.nfu);
  if (S.nfu)
    EDFA_HIP(hipMemcpyAsync(ufaces.data(), S.ufaces.p, sizeof(int) * S.nfu, hipMemcpyDeviceToHost, s));
  EDFA_HIP(hipStreamSynchronize(s));
  S.ranges_h.assign(S.ngrid, GridRange{0, 0, 0, 0});
  int u = 0;
  for (int g = 0; g < S.ngrid; ++g) {
    const GridDesc &G = S.grids_h[g];
    GridRange R;
    R.uf0 = u;
    while (u < S.nfu && ufaces[u] < G.face0 + G.nface) ++u;
    R.uf1 = u;
    R.c0 = G.cell0;
    R.c1 = G.cell0 + G.ncell;
    S.ranges_h[g] = R;
  }
  S.ranges.ensure(S.ngrid);
  EDFA_HIP(hipMemcpyAsync(S.ranges.p, S.ranges_h.data(), sizeof(GridRange) * S.ngrid,
                          hipMemcpyHostToDevice, s));
  if (S.ngrid > 1) {
    // grid of every unknown: face unknowns first, then cells
    std::vector<int> seg((size_t)S.nfu + S.ne);
    for (int g = 0; g < S.ngrid; ++g) {
      const GridRange &R = S.ranges_h[g];
      std::fill(seg.begin() + R.uf0, seg.begin() + R.uf1, g);
      std::fill(seg.begin() + S.nfu + R.c0, seg.begin() + S.nfu + R.c1, g);
    }
    S.rowseg.ensure(seg.size());
    EDFA_HIP(hipMemcpyAsync(S.rowseg.p, seg.data(), sizeof(int) * seg.size(), hipMemcpyHostToDevice, s));
  }
  EDFA_HIP(hipStreamSynchronize(s));
}

// dt update: A_pp diagonal and f_p change (eq. expr_A_pp).
__global__ void k_update_dt(int ne, int nfu, double dt, const double *__restrict__ vol,
                            const double *__restrict__ cstore, const double *__restrict__ p_prev,
                            const double *__restrict__ diag0, const double *__restrict__ rhs0,
                            const int *__restrict__ pos_A, const int *__restrict__ pos_pp,
                            double *Aval, double *ppval, double *b) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const double stor = vol[e] * cstore[e] / dt;
  const double d = diag0[e] + stor;
  Aval[pos_A[e]] = d;
  ppval[pos_pp[e]] = d;
  b[nfu + e] = rhs0[e] + stor * p_prev[e];
}

void update_dt(edfa_system_s &S, double dt, const double *p_prev, hipStream_t s) {
  if (!(dt > 0.0)) fail(EDFA_ERR_ARG, "dt must be > 0");
  S.dt = dt;
  if (p_prev)
    EDFA_HIP(hipMemcpyAsync(S.p_prev.p, p_prev, sizeof(double) * S.ne, hipMemcpyDeviceToDevice, s));
  if (S.ne)
    hipLaunchKernelGGL(k_update_dt, dim3(ceil_div(S.ne, 256)), dim3(256), 0, s, S.ne, S.nfu, dt,
                       S.vol.p, S.cstore.p, S.p_prev.p, S.diag0.p, S.rhs0.p, S.diag_pos_A.p,
                       S.diag_pos_pp.p, S.A.val.p, S.Acc.val.p, S.b.p);
  EDFA_CHECK_LAUNCH();
  // copies of A follow its new diagonal: SELL now, the transpose on its next use
  build_sell(S.A, S.A_s, S.tmp, s);
  S.AT.rows = 0;
  S.AT_s.rows = 0;
}

}  // namespace edfa
