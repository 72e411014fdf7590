// Assembled MHFE-FV block system (internal layout of an edfa_system handle).
#pragma once

#include "common.hpp"

namespace edfa {

enum FaceKind : int8_t { FACE_INTERIOR = 0, FACE_NEUMANN = 1, FACE_DIRICHLET = 2 };

// One grid of a (possibly batched) system, as seen by device kernels.
struct GridDesc {
  int nx, ny, nz;
  int cell0;        // first global cell
  int face0;        // first global face
  int nfx, nfy;     // x- and y-face counts of this grid
  int ncell, nface;
  int axis;         // every cell an axis-aligned brick with diagonal K (smaller pattern)
  const double *nodes;
  const double *K;
  const double *c;
  double c_scalar;
  double gamma;
  const int8_t *bc_type;
  const double *bc_value;
  const double *source;
  const double *p_prev;
};

// Per-grid ranges of the unknown vector, used by segmented (per-grid) reductions.
struct GridRange {
  int uf0, uf1;     // face unknowns [uf0, uf1)
  int c0, c1;       // cell unknowns, as rows nfu + [c0, c1)
};

__host__ __device__ inline int grid_of(const GridDesc *g, int ng, int idx, bool by_cell) {
  int lo = 0, hi = ng - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    int start = by_cell ? g[mid].cell0 : g[mid].face0;
    if (start <= idx)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Global face of local face a (0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+) of cell (i,j,k).
__host__ __device__ inline int cell_face(const GridDesc &G, int i, int j, int k, int a) {
  switch (a >> 1) {
    case 0: return G.face0 + i + (a & 1) + (G.nx + 1) * (j + G.ny * k);
    case 1: return G.face0 + G.nfx + i + G.nx * (j + (a & 1) + (G.ny + 1) * k);
    default: return G.face0 + G.nfx + G.nfy + i + G.nx * (j + G.ny * (k + (a & 1)));
  }
}

// Face neighbour of cell (i,j,k) across local face a, or -1.
__host__ __device__ inline int cell_nbr(const GridDesc &G, int i, int j, int k, int a) {
  const int e = G.cell0 + i + G.nx * (j + G.ny * k);
  switch (a) {
    case 0: return i > 0 ? e - 1 : -1;
    case 1: return i + 1 < G.nx ? e + 1 : -1;
    case 2: return j > 0 ? e - G.nx : -1;
    case 3: return j + 1 < G.ny ? e + G.nx : -1;
    case 4: return k > 0 ? e - G.nx * G.ny : -1;
    default: return k + 1 < G.nz ? e + G.nx * G.ny : -1;
  }
}

__host__ __device__ inline void cell_ijk(const GridDesc &G, int e, int &i, int &j, int &k) {
  int l = e - G.cell0;
  i = l % G.nx;
  l /= G.nx;
  j = l % G.ny;
  k = l / G.ny;
}

// The two cells of a global face f of grid G: cm on the minus side (f is its plus face),
// cp on the plus side; -1 when absent.  dir = 0/1/2.
__host__ __device__ inline void face_cells(const GridDesc &G, int f, int &cm, int &cp, int &dir) {
  int l = f - G.face0;
  int i, j, k;
  if (l < G.nfx) {
    dir = 0;
    i = l % (G.nx + 1);
    l /= (G.nx + 1);
    j = l % G.ny;
    k = l / G.ny;
    cm = i > 0 ? G.cell0 + (i - 1) + G.nx * (j + G.ny * k) : -1;
    cp = i < G.nx ? G.cell0 + i + G.nx * (j + G.ny * k) : -1;
  } else if (l < G.nfx + G.nfy) {
    l -= G.nfx;
    dir = 1;
    i = l % G.nx;
    l /= G.nx;
    j = l % (G.ny + 1);
    k = l / (G.ny + 1);
    cm = j > 0 ? G.cell0 + i + G.nx * ((j - 1) + G.ny * k) : -1;
    cp = j < G.ny ? G.cell0 + i + G.nx * (j + G.ny * k) : -1;
  } else {
    l -= G.nfx + G.nfy;
    dir = 2;
    i = l % G.nx;
    l /= G.nx;
    j = l % G.ny;
    k = l / G.ny;
    cm = k > 0 ? G.cell0 + i + G.nx * (j + G.ny * (k - 1)) : -1;
    cp = k < G.nz ? G.cell0 + i + G.nx * (j + G.ny * k) : -1;
  }
}

}  // namespace edfa

struct edfa_system_s {
  int ngrid = 0;
  int ne = 0, nf = 0, nfu = 0, n = 0;
  int axis = 0;
  double dt = 1.0;
  std::vector<edfa::GridDesc> grids_h;
  std::vector<edfa::GridRange> ranges_h;
  edfa::DBuf<edfa::GridDesc> grids;
  edfa::DBuf<edfa::GridRange> ranges;
  edfa::DBuf<int> rowseg;        // batches only: grid of every unknown (faces, then cells)
  // per cell
  edfa::DBuf<double> W;          // Ne x 36
  edfa::DBuf<double> vol;        // Ne
  edfa::DBuf<double> cstore;     // Ne storage coefficient
  edfa::DBuf<double> p_prev;     // Ne
  edfa::DBuf<double> bcv;        // Nf boundary values, copied from the inputs at assembly
  edfa::DBuf<double> diag0;      // Ne: A_pp diagonal without the storage term
  edfa::DBuf<double> rhs0;       // Ne: f_p without the storage term
  edfa::DBuf<int> diag_pos_A;    // Ne: position of (cell, cell) in A.val
  edfa::DBuf<int> diag_pos_pp;   // Ne: position of (cell, cell) in App-block val
  // per face
  edfa::DBuf<int8_t> kind;       // Nf
  edfa::DBuf<int> uidx;          // Nf -> unknown or -1
  edfa::DBuf<int> ufaces;        // Nfu -> global face
  // matrices (FP64)
  edfa::Csr<double> A;           // N x N
  edfa::Csr<double> Afp, Afc, Acf, Acc;   // A_pipi, A_pip, A_ppi, A_pp
  int afp_max = -1;   // longest row of A_pipi (found by the first setup; -1: not yet)
  edfa::Csr<double> AfcT;        // A_pip^T (N_e x Nfu): row m = column m of A_pip
  edfa::Csr<double> AT;          // A^T (built on first use)
  edfa::Csr<double> AcfT;        // A_ppi^T (Nfu x N_e, built on first use)
  // SELL-64 copies used by the iteration (transposes built on first use)
  edfa::Sell<double> A_s, AT_s, Acf_s, Afc_s, AfcT_s, AcfT_s;
  edfa::DBuf<double> b;          // N
  edfa::DBuf<int> tmp, tmp2;     // scratch for scans and transposes
  float avg_A = 0, avg_fp = 0, avg_fc = 0, avg_cf = 0, avg_cc = 0;
};
