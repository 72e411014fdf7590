// EDFA stage 1 (the paper's Algorithm 1) on the device.
//
//  * k_base / k_patch   initial pattern Q_0 of every cell (row of A_ppi, or a k-ring patch)
//  * k_local_reg        one wavefront per cell: restricted SPD matrix -A_pipi^(m) gathered
//                       into LDS, Cholesky factor held one row per lane in registers,
//                       solves for g~ and f~ (eqs. syst_MRHS_res, syst_MRHS_res-F); the
//                       dynamic variant grows Q from the prolonged residual (eq. prol_res)
//                       and extends the factor by bordering instead of refactoring
//  * k_local            the same with the factor in LDS, for patterns longer than 48
//  * G~, F~^T           compacted (pre-filtration) into CSR
//  * k_htilde           row m of H~ = (A_pipi R^T g~)^T F~ (eq. sparse_S), one wavefront per
//                       cell, LDS hash maps, deterministic sums
//  * k_fsai             factorised sparse approximate inverse of -A_pipi on lower(A_pipi)
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "precond.hpp"

namespace edfa {

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

template <int SIZE>
__device__ inline unsigned hslot(int key) {
  return ((unsigned)key * 2654435761u) >> (32 - ilog2c(SIZE));
}

// Find key in an LDS open-addressing table; returns the slot or -1.
template <int SIZE>
__device__ inline int h_find(const int *keys, int key) {
  unsigned h = hslot<SIZE>(key);
  for (int p = 0; p < SIZE; ++p) {
    const int k = keys[h];
    if (k == key) return (int)h;
    if (k == -1) return -1;
    h = (h + 1) & (SIZE - 1);
  }
  return -1;
}

// h_find given the key k0 read at the key's first slot h: the first probe can be issued
// early, beside other reads.
template <int SIZE>
__device__ inline int h_resolve(const int *keys, int key, unsigned h, int k0) {
  for (int p = 0; p < SIZE; ++p) {
    if (k0 == key) return (int)h;
    if (k0 == -1) return -1;
    h = (h + 1) & (SIZE - 1);
    k0 = keys[h];
  }
  return -1;
}

// Insert key (idempotent); returns the slot, or -1 when the table is full.  fresh tells
// whether this call inserted it.
template <int SIZE>
__device__ inline int h_insert(int *keys, int key, bool &fresh) {
  unsigned h = hslot<SIZE>(key);
  for (int p = 0; p < SIZE; ++p) {
    const int old = atomicCAS(&keys[h], -1, key);
    if (old == -1) {
      fresh = true;
      return (int)h;
    }
    if (old == key) {
      fresh = false;
      return (int)h;
    }
    h = (h + 1) & (SIZE - 1);
  }
  fresh = false;
  return -1;
}

template <class T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ inline int pidx(int i, int j) { return i * (i + 1) / 2 + j; }   // packed lower
__device__ inline int sidx(int i, int j) { return i * (i - 1) / 2 + j; }   // strictly lower, j < i

#define EDFA_INLINE __attribute__((always_inline))

// Visit the column indices of CSR row r in blocks of RB: every index of a block is
// requested before f runs on any of them, so a row's loads are in flight together instead
// of one behind each hash lookup.  Positions past the row's end re-read its last entry
// (always in bounds) and are not passed to f.
template <int RB, class F>
__device__ __forceinline__ void row_cols(const int *__restrict__ rp, const int *__restrict__ col,
                                         int r, F &&f) {
  const int p0 = rp[r], p1 = rp[r + 1];
  for (int b = p0; b < p1; b += RB) {
    int c[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) c[k] = col[min(b + k, p1 - 1)];
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (b + k < p1) f(c[k]);
  }
}

// |r| rounded to 40 significant bits, as a monotone unsigned key.
__device__ inline unsigned long long key40(double r) {
  unsigned long long b = (unsigned long long)__double_as_longlong(fabs(r));
  return (b + (1ull << 12)) & ~((1ull << 13) - 1ull);
}

// ------------------------------------------------------------------------------------
// Initial patterns
// ------------------------------------------------------------------------------------
__global__ void k_base(const int *__restrict__ rp, const int *__restrict__ col, int ne, int smax,
                       int *Q, int *qlen) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= ne) return;
  const int a = rp[m], n = rp[m + 1] - a;
  for (int t = 0; t < n && t < smax; ++t) Q[(size_t)m * smax + t] = col[a + t];
  qlen[m] = n;
}

// Base pattern plus the unknown faces of every cell within `level` face-neighbour steps
// (Manhattan distance on the structured grid; axis = 0), or within `level` steps along one
// axis only (axis 1/2/3: x/y/z; axis 4: the cell's axis of largest transmissibility
// W_(d-,d-) + W_(d+,d+), values within 1e-12 of the largest counting as ties that go to the
// smaller axis), sorted.
__global__ void k_patch(const GridDesc *__restrict__ grids, int ngrid, const int *__restrict__ uidx,
                        const int *__restrict__ rp, const int *__restrict__ col, int ne, int level,
                        int axis, const double *__restrict__ W, int smax, int *Q, int *qlen,
                        int *err_cap) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= ne) return;
  const GridDesc &G = grids[grid_of(grids, ngrid, m, true)];
  int i0, j0, k0;
  cell_ijk(G, m, i0, j0, k0);
  int dsel = axis - 1;   // -1: every direction
  if (axis == 4) {
    const double *We = W + 36 * (size_t)m;
    double t[3], top = 0.0;
    for (int d = 0; d < 3; ++d) {
      t[d] = We[7 * (2 * d)] + We[7 * (2 * d + 1)];
      top = fmax(top, t[d]);
    }
    dsel = t[0] >= top * (1.0 - 1e-12) ? 0 : t[1] >= top * (1.0 - 1e-12) ? 1 : 2;
  }
  int buf[PATCH_MAX];
  int n = 0;
  bool over = false;
  auto add = [&](int u) {
    for (int t = 0; t < n; ++t)
      if (buf[t] == u) return;
    if (n < PATCH_MAX)
      buf[n++] = u;
    else
      over = true;
  };
  for (int p = rp[m]; p < rp[m + 1]; ++p) add(col[p]);
  for (int dk = -level; dk <= level; ++dk)
    for (int dj = -level; dj <= level; ++dj)
      for (int di = -level; di <= level; ++di) {
        if (abs(di) + abs(dj) + abs(dk) > level) continue;
        if (dsel >= 0 && ((dsel != 0 && di) || (dsel != 1 && dj) || (dsel != 2 && dk))) continue;
        const int i = i0 + di, j = j0 + dj, k = k0 + dk;
        if (i < 0 || j < 0 || k < 0 || i >= G.nx || j >= G.ny || k >= G.nz) continue;
        for (int a = 0; a < 6; ++a) {
          const int u = uidx[cell_face(G, i, j, k, a)];
          if (u >= 0) add(u);
        }
      }
  for (int p = 1; p < n; ++p) {
    const int v = buf[p];
    int q = p - 1;
    while (q >= 0 && buf[q] > v) {
      buf[q + 1] = buf[q];
      --q;
    }
    buf[q + 1] = v;
  }
  if (over || n > smax) {
    atomicMin(err_cap, m);
    n = min(n, smax);
  }
  for (int t = 0; t < n; ++t) Q[(size_t)m * smax + t] = buf[t];
  qlen[m] = n;
}

// total of n int32 lengths (64-bit accumulator)
__global__ void k_len_sum(const int *__restrict__ len, int n, unsigned long long *out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long v = r < n ? (unsigned long long)len[r] : 0ull;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(out, v);
}

__global__ void k_repack(const int *__restrict__ src, const int *__restrict__ len, int n, int s0,
                         int s1, int *dst) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int t = 0; t < len[r]; ++t) dst[(size_t)r * s1 + t] = src[(size_t)r * s0 + t];
}

// *out = max(*out, longest row): rows given by a row pointer (len null) or by lengths; one
// atomic per wavefront after a shuffle reduction
__global__ __launch_bounds__(256) void k_row_max(const int *__restrict__ rp,
                                                 const int *__restrict__ len, int rows,
                                                 int *out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  int v = 0;
  if (r < rows) v = len ? len[r] : rp[r + 1] - rp[r];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0 && v > 0) atomicMax(out, v);
}

// A_pipi rows padded to ELL_W entries, for the candidate residuals of k_local_reg: a row's
// entries then load from its index alone, in a few wide loads.  A face couples to the
// faces of its one or two hexahedra, at most 11 entries.
constexpr int ELL_W = 12;
__global__ void k_ell_fill(const int *__restrict__ rp, const int *__restrict__ col,
                           const double *__restrict__ val, int rows, int *ecol, double *eval) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)rows * ELL_W) return;
  const int r = (int)(t / ELL_W), k = (int)(t % ELL_W);
  const int p = rp[r] + k;
  const bool in = p < rp[r + 1];
  ecol[t] = in ? col[p] : -1;
  eval[t] = in ? val[p] : 0.0;
}

// Rows of a CSR matrix padded to w entries (w a multiple of 16, rows of at most w entries).
template <class T>
__global__ void k_pad_rows(const int *__restrict__ rp, const int *__restrict__ col,
                           const T *__restrict__ val, int rows, int w, int *ecol, T *eval) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)rows * w) return;
  const int r = (int)(t / w), k = (int)(t % w);
  const int p = rp[r] + k;
  const bool in = p < rp[r + 1];
  ecol[t] = in ? col[p] : -1;
  eval[t] = in ? val[p] : T(0);
}

// ------------------------------------------------------------------------------------
// Restricted local solves, one 64-lane wavefront per cell
// ------------------------------------------------------------------------------------
template <class T>
struct LocalArgs {
  int ne;
  const int *app_rp, *app_col;
  const double *app_val;
  const int *ell_col;   // A_pipi as ELL_W-entry rows (k_local_reg)
  const double *ell_val;
  const int *acf_rp, *acf_col;
  const double *acf_val;
  const int *afcT_rp, *afcT_col;
  const double *afcT_val;
  int dynamic, n_add, n_ent, it_max;
  int *Q, *qlen;
  T *gout, *fout;
  int *err_spd, *err_cap;
  int qstride;          // entries per cell in Q, gout, fout (>= the kernel's capacity)
  const int *cells;     // cells of this launch (NULL: cell = block index)
};

template <class T, int SMAX>
__global__ __launch_bounds__(64) void k_local(LocalArgs<T> A) {
  constexpr int QH = (2 * SMAX < 64) ? 64 : 2 * SMAX;
  constexpr int CH = 8 * SMAX;
  constexpr int LP = SMAX * (SMAX + 1) / 2;
  __shared__ T Lp[LP];
  __shared__ int q[SMAX];
  __shared__ int qk[QH], qv[QH];
  __shared__ T bg[SMAX], bf[SMAX], yg[SMAX], yf[SMAX], xg[SMAX], xf[SMAX], rowt[SMAX];
  __shared__ int ck[CH], clist[CH];
  __shared__ T cr[CH];
  __shared__ int ccount, sflag;

  const int m = A.cells ? A.cells[blockIdx.x] : blockIdx.x;
  const int lane = threadIdx.x;
  if (m >= A.ne) return;
  int s = A.qlen[m];
  if (s > SMAX) {
    if (lane == 0) atomicMin(A.err_cap, m);
    return;
  }
  for (int t = lane; t < SMAX; t += 64) {
    q[t] = t < s ? A.Q[(size_t)m * A.qstride + t] : -1;
    bg[t] = 0;
    bf[t] = 0;
  }
  for (int h = lane; h < QH; h += 64) qk[h] = -1;
  if (lane == 0) sflag = 0;
  __syncthreads();
  for (int t = lane; t < s; t += 64) {
    bool fr;
    const int h = h_insert<QH>(qk, q[t], fr);
    qv[h] = t;
  }
  __syncthreads();
  // right-hand sides: a_ppi^(m) (row m of A_ppi) and a_pip^(m) (column m of A_pip)
  for (int p = A.acf_rp[m] + lane; p < A.acf_rp[m + 1]; p += 64) {
    const int h = h_find<QH>(qk, A.acf_col[p]);
    if (h >= 0) bg[qv[h]] = (T)A.acf_val[p];
  }
  for (int p = A.afcT_rp[m] + lane; p < A.afcT_rp[m + 1]; p += 64) {
    const int h = h_find<QH>(qk, A.afcT_col[p]);
    if (h >= 0) bf[qv[h]] = (T)A.afcT_val[p];
  }
  // restricted matrix -R A_pipi R^T, lower part in Q order
  for (int t = lane; t < LP; t += 64) Lp[t] = 0;
  __syncthreads();
  for (int t = lane; t < s; t += 64) {
    const int r = q[t];
    for (int p = A.app_rp[r]; p < A.app_rp[r + 1]; ++p) {
      const int h = h_find<QH>(qk, A.app_col[p]);
      if (h >= 0) {
        const int k = qv[h];
        if (k <= t) Lp[pidx(t, k)] = -(T)A.app_val[p];
      }
    }
  }
  __syncthreads();

  // right-looking Cholesky
  for (int j = 0; j < s; ++j) {
    const T d = Lp[pidx(j, j)];
    if (!(d > T(0))) {
      if (lane == 0) atomicMin(A.err_spd, m);
      return;
    }
    const T ljj = sqrt(d);
    __syncthreads();
    if (lane == 0) Lp[pidx(j, j)] = ljj;
    for (int i = j + 1 + lane; i < s; i += 64) Lp[pidx(i, j)] /= ljj;
    __syncthreads();
    for (int i = j + 1 + lane; i < s; i += 64) {
      const T lij = Lp[pidx(i, j)];
      for (int k = j + 1; k <= i; ++k) Lp[pidx(i, k)] -= lij * Lp[pidx(k, j)];
    }
    __syncthreads();
  }

  // solves with the current factor: two right-hand sides (g and f) or g only
  auto solve = [&](bool with_f) {
    for (int t = lane; t < s; t += 64) {
      rowt[t] = bg[t];
      if (with_f) xf[t] = bf[t];
    }
    __syncthreads();
    for (int k = 0; k < s; ++k) {   // forward: L y = b (rowt, xf as work vectors)
      const T dk = Lp[pidx(k, k)];
      const T y1 = rowt[k] / dk;
      const T y2 = with_f ? xf[k] / dk : T(0);
      for (int i = k + 1 + lane; i < s; i += 64) {
        const T l = Lp[pidx(i, k)];
        rowt[i] -= l * y1;
        if (with_f) xf[i] -= l * y2;
      }
      if (lane == 0) {
        yg[k] = y1;
        if (with_f) yf[k] = y2;
      }
      __syncthreads();
    }
    for (int k = s - 1; k >= 0; --k) {   // backward: L^T x = y (in place on yg, yf)
      const T dk = Lp[pidx(k, k)];
      const T x1 = yg[k] / dk;
      const T x2 = with_f ? yf[k] / dk : T(0);
      for (int i = lane; i < k; i += 64) {
        const T l = Lp[pidx(k, i)];
        yg[i] -= l * x1;
        if (with_f) yf[i] -= l * x2;
      }
      __syncthreads();
      if (lane == 0) {
        xg[k] = x1;
        if (with_f) xf[k] = x2;
      }
    }
    __syncthreads();
  };

  if (!A.dynamic) {
    solve(true);
  } else {
    solve(false);
    const int it_max = A.it_max > 0 ? A.it_max : A.n_ent;
    int n_prog = 0, sweep = 0;
    while (n_prog < A.n_ent && sweep < it_max) {
      ++sweep;
      const int n = min(A.n_add, A.n_ent - n_prog);
      // candidate set: A_pipi neighbours of Q outside Q (support of the prolonged residual)
      for (int h = lane; h < CH; h += 64) ck[h] = -1;
      if (lane == 0) ccount = 0;
      __syncthreads();
      for (int t = lane; t < s; t += 64) {
        const int r = q[t];
        for (int p = A.app_rp[r]; p < A.app_rp[r + 1]; ++p) {
          const int c = A.app_col[p];
          if (h_find<QH>(qk, c) < 0) {
            bool fr;
            if (h_insert<CH>(ck, c, fr) < 0) sflag = 1;
          }
        }
      }
      __syncthreads();
      if (sflag) {
        if (lane == 0) atomicMin(A.err_cap, m);
        return;
      }
      for (int h = lane; h < CH; h += 64)
        if (ck[h] >= 0) clist[atomicAdd(&ccount, 1)] = ck[h];
      __syncthreads();
      const int nc = ccount;
      // r_j = (A_pipi R^T g~)_j for j outside Q (a_ppi^(m) vanishes there)
      for (int c = lane; c < nc; c += 64) {
        const int j = clist[c];
        T acc = 0;
        for (int p = A.app_rp[j]; p < A.app_rp[j + 1]; ++p) {
          const int h = h_find<QH>(qk, A.app_col[p]);
          if (h >= 0) acc += (T)A.app_val[p] * xg[qv[h]];
        }
        cr[c] = acc;
      }
      __syncthreads();
      int added = 0;
      for (int rnd = 0; rnd < n; ++rnd) {
        unsigned long long bk = 0;
        int bj = 0x7fffffff, bc = -1;
        for (int c = lane; c < nc; c += 64) {
          const unsigned long long k = key40((double)cr[c]);
          const int j = clist[c];
          if (k > bk || (k == bk && k != 0 && j < bj)) {
            bk = k;
            bj = j;
            bc = c;
          }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const unsigned lo = __shfl_xor((unsigned)(bk & 0xffffffffull), o);
          const unsigned hi = __shfl_xor((unsigned)(bk >> 32), o);
          const unsigned long long ok = ((unsigned long long)hi << 32) | lo;
          const int oj = __shfl_xor(bj, o);
          const int oc = __shfl_xor(bc, o);
          if (ok > bk || (ok == bk && oj < bj)) {
            bk = ok;
            bj = oj;
            bc = oc;
          }
        }
        if (bk == 0) break;   // uniform: every lane holds the reduced value
        if (s >= SMAX) {
          if (lane == 0) atomicMin(A.err_cap, m);
          return;
        }
        const int t = s;
        if (lane == 0) {
          cr[bc] = 0;
          q[t] = bj;
          bool fr;
          const int h = h_insert<QH>(qk, bj, fr);
          qv[h] = t;
          bg[t] = 0;
          bf[t] = 0;
        }
        __syncthreads();
        // bordered Cholesky: gather row t of -A_pipi[Q,Q], solve L l = m, new diagonal
        for (int k = lane; k <= t; k += 64) rowt[k] = 0;
        __syncthreads();
        for (int p = A.app_rp[bj] + lane; p < A.app_rp[bj + 1]; p += 64) {
          const int h = h_find<QH>(qk, A.app_col[p]);
          if (h >= 0) rowt[qv[h]] = -(T)A.app_val[p];
        }
        __syncthreads();
        for (int k = 0; k < t; ++k) {
          const T lk = rowt[k] / Lp[pidx(k, k)];
          for (int i = k + 1 + lane; i < t; i += 64) rowt[i] -= Lp[pidx(i, k)] * lk;
          if (lane == 0) Lp[pidx(t, k)] = lk;
          __syncthreads();
        }
        T part = 0;
        for (int k = lane; k < t; k += 64) {
          const T l = Lp[pidx(t, k)];
          part += l * l;
        }
        const T d = rowt[t] - wave_sum(part);
        if (!(d > T(0))) {
          if (lane == 0) atomicMin(A.err_spd, m);
          return;
        }
        if (lane == 0) Lp[pidx(t, t)] = sqrt(d);
        __syncthreads();
        ++s;
        ++added;
      }
      if (added == 0) break;
      n_prog += added;
      solve(false);
    }
    // f~ on the final pattern: its right-hand side was placed when the base was loaded
    solve(true);
  }
  for (int t = lane; t < s; t += 64) {
    A.Q[(size_t)m * A.qstride + t] = q[t];
    A.gout[(size_t)m * A.qstride + t] = xg[t];
    A.fout[(size_t)m * A.qstride + t] = xf[t];
  }
  if (lane == 0) A.qlen[m] = s;
}

// Pattern table of the register kernel: a slot holds a column in its low and its index in
// Q in its high 32 bits, so a lookup is one LDS read per probe.  Columns are inserted once.
constexpr unsigned long long Q_EMPTY = ~0ull;
template <int SIZE>
__device__ inline int q_resolve(const unsigned long long *tab, int key, unsigned h,
                                unsigned long long e) {   // e = tab[h], h = hslot(key)
  for (int p = 0; p < SIZE; ++p) {
    const int k = (int)(unsigned)e;
    if (k == key) return (int)(e >> 32);
    if (k == -1) return -1;
    h = (h + 1) & (SIZE - 1);
    e = tab[h];
  }
  return -1;
}
template <int SIZE>
__device__ inline int q_find(const unsigned long long *tab, int key) {
  const unsigned h = hslot<SIZE>(key);
  return q_resolve<SIZE>(tab, key, h, tab[h]);
}
template <int SIZE>
__device__ inline void q_insert(unsigned long long *tab, int key, int pos) {
  const unsigned long long e = ((unsigned long long)(unsigned)pos << 32) | (unsigned)key;
  unsigned h = hslot<SIZE>(key);
  for (int p = 0; p < SIZE; ++p) {
    if (atomicCAS(&tab[h], Q_EMPTY, e) == Q_EMPTY) return;
    h = (h + 1) & (SIZE - 1);
  }
}

// Visit the entries of row r of an ELL_W-entry copy in order (column -1 ends a row): the
// row is requested in a few wide loads before f runs on any entry.  val may be null.
template <class F>
__device__ __forceinline__ void ell_row(const int *__restrict__ ecol,
                                        const double *__restrict__ eval, int r, F &&f) {
  const int4 *pc = reinterpret_cast<const int4 *>(ecol + (size_t)r * ELL_W);
  int c[ELL_W];
  double v[ELL_W];
#pragma unroll
  for (int u = 0; u < ELL_W / 4; ++u) {
    const int4 w = pc[u];
    c[4 * u] = w.x;
    c[4 * u + 1] = w.y;
    c[4 * u + 2] = w.z;
    c[4 * u + 3] = w.w;
  }
  if (eval) {
    const double2 *pv = reinterpret_cast<const double2 *>(eval + (size_t)r * ELL_W);
#pragma unroll
    for (int u = 0; u < ELL_W / 2; ++u) {
      const double2 w = pv[u];
      v[2 * u] = w.x;
      v[2 * u + 1] = w.y;
    }
  } else {
#pragma unroll
    for (int u = 0; u < ELL_W; ++u) v[u] = 0;
  }
#pragma unroll
  for (int u = 0; u < ELL_W; ++u)
    if (c[u] >= 0) f(c[u], v[u]);
}

// ------------------------------------------------------------------------------------
// Restricted local solves with the factor held in registers (patterns of at most 48).
//
// Lane t owns row t of the Cholesky factor L of -A_pipi^(m) in registers (compile-time
// indexed), plus its diagonal.  The right-looking factorisation, the forward
// substitutions and the bordering of appended rows broadcast the pivot row's entry with
// a lane read, so they run without barriers; the backward substitution reads L from a
// packed copy in LDS.  Pattern bookkeeping (hash of Q, candidates, residual, selection)
// is the same as in k_local.
// ------------------------------------------------------------------------------------
constexpr int pow2ceil(int x) { return x <= 1 ? 1 : 2 * pow2ceil((x + 1) / 2); }

// f(std::integral_constant<int, i>) for i = B .. E-1: register arrays indexed by i stay in
// registers (the bodies must be inlined: lambdas passed here are marked EDFA_INLINE).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Value of v held by lane `src` (uniform index), for every lane.
template <class T>
__device__ inline T lane_value(T v, int src) {
  if constexpr (sizeof(T) == 8) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  } else {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
  }
}

template <class T, int SMAX>
__global__ __launch_bounds__(64) void k_local_reg(LocalArgs<T> A) {
  static_assert(SMAX <= 64, "one lane per pattern entry");
  constexpr int QH = pow2ceil(2 * SMAX < 64 ? 64 : 2 * SMAX);
  // candidate table: 256 slots at capacities 40..48 (the largest candidate set measured on
  // hexahedral grids is about 100; a full table is a capacity error), which keeps the
  // wavefront's LDS small enough for three per SIMD
  constexpr int CH = (SMAX >= 40 && SMAX <= 48) ? 256 : pow2ceil(8 * SMAX);
  constexpr int LP = SMAX * (SMAX - 1) / 2;   // strictly lower triangle (diagonal apart)
  __shared__ T Lp[LP];
  __shared__ int q[SMAX];
  __shared__ unsigned long long qt[QH];   // column -> index in Q (q_find)
  // xs holds the solution for the candidate residuals and, after them, the bordering column
  // (rowt); the right-hand sides live in registers (one entry per lane)
  __shared__ T xs[SMAX];
  T *const rowt = xs;
  __shared__ int ck[CH], clist[CH];
  __shared__ T cr[CH];
  __shared__ int ccount, sflag;

  const int m = A.cells ? A.cells[blockIdx.x] : blockIdx.x;
  const int lane = threadIdx.x;
  if (m >= A.ne) return;
  int s = A.qlen[m];
  if (s > SMAX) {
    if (lane == 0) atomicMin(A.err_cap, m);
    return;
  }
  for (int t = lane; t < SMAX; t += 64) {
    q[t] = t < s ? A.Q[(size_t)m * A.qstride + t] : -1;
    cr[t] = 0;          // the right-hand sides are gathered in cr, then read into registers
    cr[SMAX + t] = 0;
  }
  for (int h = lane; h < QH; h += 64) qt[h] = Q_EMPTY;
  if (lane == 0) sflag = 0;
  __syncthreads();
  for (int t = lane; t < s; t += 64) q_insert<QH>(qt, q[t], t);
  __syncthreads();
  // right-hand sides: a_ppi^(m) (row m of A_ppi) and a_pip^(m) (column m of A_pip)
  for (int p = A.acf_rp[m] + lane; p < A.acf_rp[m + 1]; p += 64) {
    const int k = q_find<QH>(qt, A.acf_col[p]);
    if (k >= 0) cr[k] = (T)A.acf_val[p];
  }
  for (int p = A.afcT_rp[m] + lane; p < A.afcT_rp[m + 1]; p += 64) {
    const int k = q_find<QH>(qt, A.afcT_col[p]);
    if (k >= 0) cr[SMAX + k] = (T)A.afcT_val[p];
  }
  // restricted matrix -R A_pipi R^T, lower part in Q order
  for (int t = lane; t < LP; t += 64) Lp[t] = 0;
  __syncthreads();
  // lane t's entries of the two right-hand sides (zero past the pattern and for every entry
  // appended later: a_ppi^(m) and a_pip^(m) vanish outside the base pattern)
  const T bgl = lane < SMAX ? cr[lane] : T(0);
  const T bfl = lane < SMAX ? cr[SMAX + lane] : T(0);
  T d0 = 0;   // lane's diagonal entry (the packed copy holds the strictly lower part)
  if (lane < s) {
    ell_row(A.ell_col, A.ell_val, q[lane], [&](int c, double v) EDFA_INLINE {
      const int k = q_find<QH>(qt, c);
      if (k >= 0 && k < lane) Lp[sidx(lane, k)] = -(T)v;
      if (k == lane) d0 = -(T)v;
    });
  }
  __syncthreads();

  // row `lane` into registers and right-looking Cholesky.  Lane i keeps row i of L strictly
  // below the diagonal, and L_ii and 1/L_ii apart; the updates of a step also touch the
  // slots at and past the diagonal, which no later step reads, so they are cleared at the
  // end.  The triangular solves below then need no per-step selects.
  T Lr[SMAX];
  static_for<0, SMAX>([&](auto K) EDFA_INLINE {
    constexpr int k = K;
    Lr[k] = (lane < s && k < lane) ? Lp[sidx(lane, k)] : (lane < s && k == lane ? d0 : T(0));
  });
  T dg = 1;
  bool spd = true;
  static_for<0, SMAX>([&](auto J) EDFA_INLINE {
    constexpr int j = J;
    if (!spd || j >= s) return;
    const T d = lane_value(Lr[j], j);
    if (!(d > T(0))) {
      spd = false;
      return;
    }
    const T ljj = sqrt(d);
    const T inv = T(1) / ljj;
    Lr[j] = lane == j ? ljj : Lr[j] * inv;
    if (lane == j) dg = ljj;
    static_for<j + 1, SMAX>([&](auto K) EDFA_INLINE {
      constexpr int k = K;
      if (k < s) Lr[k] -= Lr[j] * lane_value(Lr[j], k);
    });
  });
  if (!spd) {
    if (lane == 0) atomicMin(A.err_spd, m);
    return;
  }
  T invd = T(1) / dg;
  static_for<0, SMAX>([&](auto K) EDFA_INLINE {
    constexpr int k = K;
    Lr[k] = k < lane ? Lr[k] : T(0);
  });
  __syncthreads();
  static_for<0, SMAX>([&](auto K) EDFA_INLINE {
    constexpr int k = K;
    if (lane < s && k < lane) Lp[sidx(lane, k)] = Lr[k];
  });
  __syncthreads();

  const int it_max = A.it_max > 0 ? A.it_max : A.n_ent;
  int n_prog = 0, sweep = 0;
  int scanned = 0;   // pattern entries whose A_pipi rows are in the candidate set
  bool fin = !A.dynamic;
  T xg = 0, xf = 0;
  for (;;) {
    const bool last = fin || !(n_prog < A.n_ent && sweep < it_max);
    // forward L y = b, then backward L^T x = y (g~, and f~ on the last pass).  Lane k's
    // entry is final when step k reads it (its row has no entry at or past k), so each lane
    // ends holding its own entry and divides it by L_kk there: the same operations, on the
    // same operands, as dividing at step k.
    {
      T b1 = lane < s ? bgl : T(0);
      if (!last) {
        // both substitutions run all SMAX steps without branches, so the reads of later
        // steps issue early: the entries past s are zero and so are their updates
        static_for<0, SMAX>([&](auto K) EDFA_INLINE {
          constexpr int k = K;
          b1 -= Lr[k] * (lane_value(b1, k) * lane_value(invd, k));
        });
        b1 *= invd;
        static_for<0, SMAX>([&](auto K) EDFA_INLINE {
          constexpr int k = SMAX - 1 - K;
          const T l = lane < k ? Lp[sidx(k, lane)] : T(0);
          b1 -= l * (lane_value(b1, k) * lane_value(invd, k));
        });
        b1 *= invd;
      } else {
        T b2 = lane < s ? bfl : T(0);
        static_for<0, SMAX>([&](auto K) EDFA_INLINE {
          constexpr int k = K;
          const T ik = lane_value(invd, k);
          b1 -= Lr[k] * (lane_value(b1, k) * ik);
          b2 -= Lr[k] * (lane_value(b2, k) * ik);
        });
        b1 *= invd;
        b2 *= invd;
        static_for<0, SMAX>([&](auto K) EDFA_INLINE {
          constexpr int k = SMAX - 1 - K;
          const T ik = lane_value(invd, k);
          const T l = lane < k ? Lp[sidx(k, lane)] : T(0);
          b1 -= l * (lane_value(b1, k) * ik);
          b2 -= l * (lane_value(b2, k) * ik);
        });
        b1 *= invd;
        b2 *= invd;
        xf = b2;
      }
      xg = b1;
    }
    if (last) break;
    ++sweep;
    const int n = min(A.n_add, A.n_ent - n_prog);
    if (lane < s) xs[lane] = xg;
    // candidate set: A_pipi neighbours of Q outside Q (support of the prolonged residual),
    // kept across sweeps: only the rows of the entries appended since the last sweep are
    // scanned, fresh candidates are appended to clist, and candidates that have joined Q
    // get a zero residual below
    if (sweep == 1) {
      for (int h = lane; h < CH; h += 64) ck[h] = -1;
      if (lane == 0) ccount = 0;
    }
    __syncthreads();
    for (int t = scanned + lane; t < s; t += 64) {
      ell_row(A.ell_col, nullptr, q[t], [&](int c, double) EDFA_INLINE {
        if (q_find<QH>(qt, c) < 0) {
          bool fr;
          if (h_insert<CH>(ck, c, fr) < 0)
            sflag = 1;
          else if (fr)
            clist[atomicAdd(&ccount, 1)] = c;
        }
      });
    }
    scanned = s;
    __syncthreads();
    if (sflag) {
      if (lane == 0) atomicMin(A.err_cap, m);
      return;
    }
    const int nc = ccount;
    // r_j = (A_pipi R^T g~)_j for j outside Q (a_ppi^(m) vanishes there).  Lane l takes the
    // candidates l, l + 64, ...; the ELL row of its next candidate is in flight while the
    // current one is looked up (two register slots used in place; the loads are issued
    // without branches, past the list's end re-reading its last candidate).  A row's
    // entries are looked up as one batch of first table probes, then one batch of x~
    // reads at the entries found; the sum runs in the row's order.
    struct EllRow {
      int4 c[ELL_W / 4];
      double2 v[ELL_W / 2];
    };
    auto rfetch = [&](int c, EllRow &r) EDFA_INLINE {
      const int j = clist[min(c, nc - 1)];
      const int4 *pc = reinterpret_cast<const int4 *>(A.ell_col + (size_t)j * ELL_W);
      const double2 *pv = reinterpret_cast<const double2 *>(A.ell_val + (size_t)j * ELL_W);
#pragma unroll
      for (int u = 0; u < ELL_W / 4; ++u) r.c[u] = pc[u];
#pragma unroll
      for (int u = 0; u < ELL_W / 2; ++u) r.v[u] = pv[u];
    };
    auto residual = [&](int c, const EllRow &r) EDFA_INLINE {
      if (c >= nc) return;
      const int j = clist[c];
      T acc = 0;
      if (q_find<QH>(qt, j) < 0) {
        int cc[ELL_W], kq[ELL_W];
        double vv[ELL_W];
        unsigned long long ee[ELL_W];
        T xv[ELL_W];
#pragma unroll
        for (int u = 0; u < ELL_W / 4; ++u) {
          cc[4 * u] = r.c[u].x;
          cc[4 * u + 1] = r.c[u].y;
          cc[4 * u + 2] = r.c[u].z;
          cc[4 * u + 3] = r.c[u].w;
        }
#pragma unroll
        for (int u = 0; u < ELL_W / 2; ++u) {
          vv[2 * u] = r.v[u].x;
          vv[2 * u + 1] = r.v[u].y;
        }
#pragma unroll
        for (int u = 0; u < ELL_W; ++u) ee[u] = qt[hslot<QH>(cc[u])];
#pragma unroll
        for (int u = 0; u < ELL_W; ++u)
          kq[u] = cc[u] >= 0 ? q_resolve<QH>(qt, cc[u], hslot<QH>(cc[u]), ee[u]) : -1;
#pragma unroll
        for (int u = 0; u < ELL_W; ++u) xv[u] = xs[kq[u] >= 0 ? kq[u] : 0];
#pragma unroll
        for (int u = 0; u < ELL_W; ++u)
          if (kq[u] >= 0) acc += (T)vv[u] * xv[u];
      }
      cr[c] = acc;
    };
    if (nc > 0) {
      if constexpr (sizeof(T) == 4) {
        // one row in flight (fewer registers: the FP32 kernel then fits four wavefronts per
        // SIMD)
        EllRow ra;
        rfetch(lane, ra);
        for (int base = 0; base < nc; base += 64) {
          residual(base + lane, ra);
          rfetch(base + lane + 64, ra);
        }
      } else {
        EllRow ra, rb;
        rfetch(lane, ra);
        rfetch(lane + 64, rb);
        for (int base = 0; base < nc; base += 128) {
          residual(base + lane, ra);
          rfetch(base + lane + 128, ra);
          residual(base + lane + 64, rb);
          rfetch(base + lane + 192, rb);
        }
      }
    }
    __syncthreads();
    // the factor rows back into registers from the packed copy (the same values): the
    // register copy is dead during the candidate residuals, which then have its registers
    static_for<0, SMAX>([&](auto K) EDFA_INLINE {
      constexpr int k = K;
      Lr[k] = (k < lane && lane < s) ? Lp[sidx(lane, k)] : T(0);
    });
    int added = 0;
    for (int rnd = 0; rnd < n; ++rnd) {
      unsigned long long bk = 0;
      int bj = 0x7fffffff, bc = -1;
      for (int c = lane; c < nc; c += 64) {
        const unsigned long long k = key40((double)cr[c]);
        const int j = clist[c];
        if (k > bk || (k == bk && k != 0 && j < bj)) {
          bk = k;
          bj = j;
          bc = c;
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned lo = __shfl_xor((unsigned)(bk & 0xffffffffull), o);
        const unsigned hi = __shfl_xor((unsigned)(bk >> 32), o);
        const unsigned long long ok = ((unsigned long long)hi << 32) | lo;
        const int oj = __shfl_xor(bj, o);
        const int oc = __shfl_xor(bc, o);
        if (ok > bk || (ok == bk && oj < bj)) {
          bk = ok;
          bj = oj;
          bc = oc;
        }
      }
      if (bk == 0) break;   // uniform: every lane holds the reduced value
      if (s >= SMAX) {
        if (lane == 0) atomicMin(A.err_cap, m);
        return;
      }
      const int t = s;
      if (lane == 0) {
        cr[bc] = 0;
        q[t] = bj;
        q_insert<QH>(qt, bj, t);
      }
      if (lane <= t) rowt[lane] = 0;
      __syncthreads();
      // bordering: column of -A_pipi[Q, j] and its diagonal, L l = a, l_tt^2 = a_tt - l.l
      if (lane < ELL_W) {
        const int c = A.ell_col[(size_t)bj * ELL_W + lane];
        const int k = c >= 0 ? q_find<QH>(qt, c) : -1;
        if (k >= 0) rowt[k] = -(T)A.ell_val[(size_t)bj * ELL_W + lane];
      }
      __syncthreads();
      T a = lane <= t ? rowt[lane] : T(0);
      const T att = lane_value(a, t);
      T dsum = 0;
      static_for<0, SMAX>([&](auto K) EDFA_INLINE {
        constexpr int k = K;
        if (k >= t) return;
        const T lk = lane_value(a, k) * lane_value(invd, k);
        a -= Lr[k] * lk;
        Lr[k] = lane == t ? lk : Lr[k];   // a select, not a store to Lr[t]
        if (lane == 0) Lp[sidx(t, k)] = lk;
        dsum += lk * lk;
      });
      const T d = att - dsum;
      if (!(d > T(0))) {
        if (lane == 0) atomicMin(A.err_spd, m);
        return;
      }
      const T ltt = sqrt(d);
      if (lane == t) {
        dg = ltt;
        invd = T(1) / ltt;
      }
      __syncthreads();
      ++s;
      ++added;
    }
    if (added == 0)
      fin = true;
    else
      n_prog += added;
  }
  if (lane < s) {
    A.Q[(size_t)m * A.qstride + lane] = q[lane];
    A.gout[(size_t)m * A.qstride + lane] = xg;
    A.fout[(size_t)m * A.qstride + lane] = xf;
  }
  if (lane == 0) A.qlen[m] = s;
}

// ------------------------------------------------------------------------------------
// G~ and F~^T as CSR (sorted columns), with optional pre-filtration
// ------------------------------------------------------------------------------------
template <class T>
__global__ void k_vec_count(const int *__restrict__ qlen, const T *__restrict__ v, int ne, int smax,
                            int pre, double tau, int *len) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= ne) return;
  const int s = qlen[m];
  if (!pre) {
    len[m] = s;
    return;
  }
  const T *x = v + (size_t)m * smax;
  double nrm = 0;
  for (int t = 0; t < s; ++t) nrm += (double)x[t] * (double)x[t];
  const double thr = tau * sqrt(nrm);
  int c = 0;
  for (int t = 0; t < s; ++t) c += fabs((double)x[t]) >= thr;
  len[m] = c;
}

template <class T, int CAP>
__global__ void k_vec_write(const int *__restrict__ Q, const int *__restrict__ qlen,
                            const T *__restrict__ v, int ne, int smax, int pre, double tau,
                            const int *__restrict__ rp, int *col, T *val) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= ne) return;
  const int s = qlen[m];
  const T *x = v + (size_t)m * smax;
  const int *qq = Q + (size_t)m * smax;
  double thr = -1.0;
  if (pre) {
    double nrm = 0;
    for (int t = 0; t < s; ++t) nrm += (double)x[t] * (double)x[t];
    thr = tau * sqrt(nrm);
  }
  int base = rp[m];
  int n = 0;
  int c[CAP];
  T w[CAP];
  for (int t = 0; t < s; ++t) {
    if (pre && !(fabs((double)x[t]) >= thr)) continue;
    const int cc = qq[t];
    const T vv = x[t];
    int p = n - 1;
    while (p >= 0 && c[p] > cc) {
      c[p + 1] = c[p];
      w[p + 1] = w[p];
      --p;
    }
    c[p + 1] = cc;
    w[p + 1] = vv;
    ++n;
  }
  for (int t = 0; t < n; ++t) {
    col[base + t] = c[t];
    val[base + t] = w[t];
  }
}

// Patterns of at most 64 entries: one wavefront per cell (four per block), lane t holding
// entry t; the pre-filtration norm is a fixed butterfly sum (the count and the write pass
// compute it the same way), and each kept entry's slot is its rank by column.
template <class T>
__device__ inline bool vec_keep(T xv, bool in, int pre, double tau) {
  if (!pre) return in;
  const double thr = tau * sqrt(wave_sum((double)xv * (double)xv));
  return in && fabs((double)xv) >= thr;
}

template <class T>
__global__ __launch_bounds__(256) void k_vec_count_w(const int *__restrict__ qlen,
                                                     const T *__restrict__ v, int ne, int smax,
                                                     int pre, double tau, int *len) {
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (m >= ne) return;
  const int s = qlen[m];
  const bool in = lane < s;
  const T xv = in ? v[(size_t)m * smax + lane] : T(0);
  const bool keep = vec_keep(xv, in, pre, tau);
  const int k = __popcll(__ballot(keep));
  if (lane == 0) len[m] = k;
}

template <class T>
__global__ __launch_bounds__(256) void k_vec_write_w(const int *__restrict__ Q,
                                                     const int *__restrict__ qlen,
                                                     const T *__restrict__ v, int ne, int smax,
                                                     int pre, double tau,
                                                     const int *__restrict__ rp, int *col, T *val) {
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (m >= ne) return;
  const int s = qlen[m];
  const bool in = lane < s;
  const T xv = in ? v[(size_t)m * smax + lane] : T(0);
  const int c = in ? Q[(size_t)m * smax + lane] : 0x7fffffff;
  const bool keep = vec_keep(xv, in, pre, tau);
  int rank = 0;
  for (int j = 0; j < s; ++j) {
    const int cj = __shfl(c, j);
    const int kj = __shfl((int)keep, j);
    rank += kj && cj < c;
  }
  if (keep) {
    col[rp[m] + rank] = c;
    val[rp[m] + rank] = xv;
  }
}

// ------------------------------------------------------------------------------------
// H~ rows: h_m = (A_pipi R^T g~_m)^T F~, one wavefront per cell
// ------------------------------------------------------------------------------------
template <class T>
struct HArgs {
  int ne;
  const int *g_rp, *g_col;
  const T *g_val;
  const int *ell_col;   // A_pipi as ELL_W-entry rows
  const double *ell_val;
  const int *ff_rp, *ff_col;   // F~ by face rows (cells)
  const int *ft_rp;            // F~^T by cell rows (faces): row pointer, and the rows padded
  const int *ft_ecol;          //   to ft_w entries
  const T *ft_eval;
  int ft_w;
  int *Hcol, *Hlen;
  T *Hval;
  int *err_cap;
  const int *cells;      // rows to compute (NULL: row = block index)
  int *retry_count;      // non-NULL: a row whose tables pass half full is listed here
  int *retry_list;       //   instead of computed (first pass with small tables)
  int t_retry;           // first pass: a support of t over this many faces retries
};

// Tables: g~ (GH slots), the support of t (TH slots, listed in tlist: TH/2 entries for the
// small tables, a first-pass row that fills them past half retries; TH for the large ones)
// and the candidate cells (LH slots; at most LH/2 candidates are kept, listed in llist).
template <class T, int GH, int TH, int LH>
__global__ __launch_bounds__(64) void k_htilde(HArgs<T> A) {
  constexpr int CL = LH / 2;
  constexpr int TL = TH <= 512 ? TH / 2 : TH;
  __shared__ int gk[GH];
  __shared__ T gv[GH];
  __shared__ int tk[TH], tlist[TL];
  __shared__ T tv[TH];
  __shared__ int lk[LH], llist[CL];
  __shared__ int tcount, lcount, sflag;
  const int m = A.cells ? A.cells[blockIdx.x] : blockIdx.x;
  const int lane = threadIdx.x;
  if (m >= A.ne) return;
  // retry: row m goes to the large-table pass (first pass only; all lanes agree)
  auto retry = [&]() {
    if (lane == 0) A.retry_list[atomicAdd(A.retry_count, 1)] = m;
  };
  for (int h = lane; h < GH; h += 64) gk[h] = -1;
  for (int h = lane; h < TH; h += 64) tk[h] = -1;
  for (int h = lane; h < LH; h += 64) lk[h] = -1;
  if (lane == 0) {
    tcount = 0;
    lcount = 0;
    sflag = 0;
  }
  __syncthreads();
  const int g0 = A.g_rp[m], g1 = A.g_rp[m + 1];
  for (int p = g0 + lane; p < g1; p += 64) {
    bool fr;
    const int h = h_insert<GH>(gk, A.g_col[p], fr);
    if (h < 0)
      sflag = 1;
    else
      gv[h] = A.g_val[p];
  }
  // support of t = A_pipi R^T g~: A_pipi neighbours of the pattern of g~
  auto add_t = [&](int c, double) EDFA_INLINE {
    bool fr;
    const int h = h_insert<TH>(tk, c, fr);
    if (h < 0) {
      sflag = 1;
    } else if (fr) {
      const int i = atomicAdd(&tcount, 1);
      if (i < TL) tlist[i] = h;
    }
  };
  for (int p = g0 + lane; p < g1; p += 64) ell_row(A.ell_col, nullptr, A.g_col[p], add_t);
  __syncthreads();
  if (A.retry_count && (sflag || tcount > A.t_retry)) {
    retry();
    return;
  }
  if (sflag || tcount > TL) {
    if (lane == 0) atomicMin(A.err_cap, m);
    return;
  }
  const int nt = tcount;
  for (int c = lane; c < nt; c += 64) {
    const int h = tlist[c];
    T acc = 0;
    {
      // the row's first table probes as one batch of LDS reads, then the reads of g~ at
      // the entries found; the sum runs in the row's order
      const int r = tk[h];
      const int4 *pc = reinterpret_cast<const int4 *>(A.ell_col + (size_t)r * ELL_W);
      const double2 *pv = reinterpret_cast<const double2 *>(A.ell_val + (size_t)r * ELL_W);
      int cc[ELL_W], kk[ELL_W], sl[ELL_W];
      double vv[ELL_W];
      T xv[ELL_W];
#pragma unroll
      for (int u = 0; u < ELL_W / 4; ++u) {
        const int4 w = pc[u];
        cc[4 * u] = w.x;
        cc[4 * u + 1] = w.y;
        cc[4 * u + 2] = w.z;
        cc[4 * u + 3] = w.w;
      }
#pragma unroll
      for (int u = 0; u < ELL_W / 2; ++u) {
        const double2 w = pv[u];
        vv[2 * u] = w.x;
        vv[2 * u + 1] = w.y;
      }
#pragma unroll
      for (int u = 0; u < ELL_W; ++u) kk[u] = gk[hslot<GH>(cc[u])];
#pragma unroll
      for (int u = 0; u < ELL_W; ++u)
        sl[u] = cc[u] >= 0 ? h_resolve<GH>(gk, cc[u], hslot<GH>(cc[u]), kk[u]) : -1;
#pragma unroll
      for (int u = 0; u < ELL_W; ++u) xv[u] = gv[sl[u] >= 0 ? sl[u] : 0];
#pragma unroll
      for (int u = 0; u < ELL_W; ++u)
        if (sl[u] >= 0) acc += (T)vv[u] * xv[u];
    }
    tv[h] = acc;
  }
  // candidate cells: all l with F~[j, l] != 0 for j in the support of t
  for (int c = lane; c < nt; c += 64) {
    row_cols<16>(A.ff_rp, A.ff_col, tk[tlist[c]], [&](int l) EDFA_INLINE {
      bool fr;
      const int q = h_insert<LH>(lk, l, fr);
      if (q < 0) {
        sflag = 1;
      } else if (fr) {
        const int i = atomicAdd(&lcount, 1);
        if (i < CL) llist[i] = l;
      }
    });
  }
  __syncthreads();
  const int nl = lcount;
  if (A.retry_count && (sflag || nl > CL)) {
    retry();
    return;
  }
  if (sflag || nl > CL || nl > HMAX) {
    if (lane == 0) atomicMin(A.err_cap, m);
    return;
  }
  // h_ml = sum over the pattern of f~_l of t_j f~_l[j] (F~^T row l, ascending j), written
  // sorted by column: slot = number of smaller candidate cells
  for (int c = lane; c < nl; c += 64) {
    const int l = llist[c];
    T acc = 0;
    // a block of the row is looked up at once: the first table probes of all its entries,
    // then the reads of t at the entries found, each one batch of LDS reads; the sum runs
    // in the row's order
    // (the row is read from its padded copy: 16 entries as four int4 and eight 16-byte
    // value loads, instead of one load per entry)
    const int len = A.ft_rp[l + 1] - A.ft_rp[l];
    const int *ec = A.ft_ecol + (size_t)l * A.ft_w;
    const T *ev = A.ft_eval + (size_t)l * A.ft_w;
    for (int b = 0; b < len; b += 16) {
      int cc[16], kk[16], sl[16];
      T vv[16], xv[16];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int4 w4 = reinterpret_cast<const int4 *>(ec + b)[u];
        cc[4 * u] = w4.x;
        cc[4 * u + 1] = w4.y;
        cc[4 * u + 2] = w4.z;
        cc[4 * u + 3] = w4.w;
      }
      if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const double2 w2 = reinterpret_cast<const double2 *>(ev + b)[u];
          vv[2 * u] = w2.x;
          vv[2 * u + 1] = w2.y;
        }
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float4 w4 = reinterpret_cast<const float4 *>(ev + b)[u];
          vv[4 * u] = w4.x;
          vv[4 * u + 1] = w4.y;
          vv[4 * u + 2] = w4.z;
          vv[4 * u + 3] = w4.w;
        }
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) kk[u] = tk[hslot<TH>(cc[u])];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        sl[u] = b + u < len ? h_resolve<TH>(tk, cc[u], hslot<TH>(cc[u]), kk[u]) : -1;
#pragma unroll
      for (int u = 0; u < 16; ++u) xv[u] = tv[sl[u] >= 0 ? sl[u] : 0];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (sl[u] >= 0) acc += xv[u] * vv[u];
    }
    int rank = 0;
    for (int c2 = 0; c2 < nl; ++c2) rank += llist[c2] < l;
    A.Hcol[(size_t)m * HMAX + rank] = l;
    A.Hval[(size_t)m * HMAX + rank] = acc;
  }
  if (lane == 0) A.Hlen[m] = nl;
}

// Post-filtration on H~ (row norm before dropping, diagonal kept) and compaction: one
// wavefront per row (four rows per block of 256), lanes across the row's entries; the
// norm is a fixed butterfly sum, and the kept entries keep their order (ballot prefix).
template <class T>
__device__ inline double hrow_threshold(const T *v, int n, int lane, int filt, double tau) {
  if (!filt) return -1.0;
  double nrm = 0;
  for (int t = lane; t < n; t += 64) nrm += (double)v[t] * (double)v[t];
  return tau * sqrt(wave_sum(nrm));
}

template <class T>
__global__ __launch_bounds__(256) void k_hcount(const int *__restrict__ Hcol,
                                                const T *__restrict__ Hval,
                                                const int *__restrict__ Hlen, int ne, int filt,
                                                double tau, int *len) {
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (m >= ne) return;
  const int n = Hlen[m];
  const T *v = Hval + (size_t)m * HMAX;
  const int *c = Hcol + (size_t)m * HMAX;
  const double thr = hrow_threshold(v, n, lane, filt, tau);
  int k = 0;
  for (int t0 = 0; t0 < n; t0 += 64) {
    const int t = t0 + lane;
    const bool keep = t < n && (!filt || fabs((double)v[t]) >= thr || c[t] == m);
    k += __popcll(__ballot(keep));
  }
  if (lane == 0) len[m] = k;
}

template <class T>
__global__ __launch_bounds__(256) void k_hwrite(const int *__restrict__ Hcol,
                                                const T *__restrict__ Hval,
                                                const int *__restrict__ Hlen, int ne, int filt,
                                                double tau, const int *__restrict__ rp, int *col,
                                                T *val) {
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (m >= ne) return;
  const int n = Hlen[m];
  const T *v = Hval + (size_t)m * HMAX;
  const int *c = Hcol + (size_t)m * HMAX;
  const double thr = hrow_threshold(v, n, lane, filt, tau);
  const unsigned long long below = (1ull << lane) - 1;
  int o = rp[m];
  for (int t0 = 0; t0 < n; t0 += 64) {
    const int t = t0 + lane;
    const bool keep = t < n && (!filt || fabs((double)v[t]) >= thr || c[t] == m);
    const unsigned long long mask = __ballot(keep);
    if (keep) {
      const int q = o + __popcll(mask & below);
      col[q] = c[t];
      val[q] = v[t];
    }
    o += __popcll(mask);
  }
}

// ------------------------------------------------------------------------------------
// FSAI of -A_pipi: row i on P_i = {j <= i in the pattern of A_pipi}; with M = -A[P,P] =
// L L^T, the solution of M y = e_last has y_last = 1/L_ll^2, so G_F[i, P_i] = y L_ll.
// ------------------------------------------------------------------------------------
__global__ void k_fsai_count(const int *__restrict__ rp, const int *__restrict__ col, int n,
                             int *len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = 0;
  for (int p = rp[i]; p < rp[i + 1]; ++p) c += col[p] <= i;
  len[i] = c;
}

template <class T>
__global__ void k_fsai(const int *__restrict__ rp, const int *__restrict__ col,
                       const double *__restrict__ val, int n, const int *__restrict__ grp,
                       int *gcol, T *gval, int *err_spd, int *err_cap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int P[FSAI_MAX];
  int np = 0;
  for (int p = rp[i]; p < rp[i + 1]; ++p)
    if (col[p] <= i) {
      if (np == FSAI_MAX) {
        atomicMin(err_cap, i);
        return;
      }
      P[np++] = col[p];
    }
  T M[FSAI_MAX * (FSAI_MAX + 1) / 2];
  for (int t = 0; t < np * (np + 1) / 2; ++t) M[t] = 0;
  for (int a = 0; a < np; ++a) {
    const int r = P[a];
    for (int p = rp[r]; p < rp[r + 1]; ++p) {
      const int c = col[p];
      for (int b = 0; b <= a; ++b)
        if (P[b] == c) M[pidx(a, b)] = -(T)val[p];
    }
  }
  for (int j = 0; j < np; ++j) {
    T d = M[pidx(j, j)];
    for (int k = 0; k < j; ++k) d -= M[pidx(j, k)] * M[pidx(j, k)];
    if (!(d > T(0))) {
      atomicMin(err_spd, i);
      return;
    }
    d = sqrt(d);
    M[pidx(j, j)] = d;
    for (int r = j + 1; r < np; ++r) {
      T s = M[pidx(r, j)];
      for (int k = 0; k < j; ++k) s -= M[pidx(r, k)] * M[pidx(j, k)];
      M[pidx(r, j)] = s / d;
    }
  }
  T y[FSAI_MAX];
  const int l = np - 1;
  const T Ll = M[pidx(l, l)];
  y[l] = T(1) / (Ll * Ll);
  for (int k = l - 1; k >= 0; --k) {
    T s = 0;
    for (int r = k + 1; r <= l; ++r) s -= M[pidx(r, k)] * y[r];
    y[k] = s / M[pidx(k, k)];
  }
  const int o = grp[i];
  for (int t = 0; t < np; ++t) {
    gcol[o + t] = P[t];
    gval[o + t] = y[t] * Ll;
  }
}

// ------------------------------------------------------------------------------------
// Host driver of stage 1
// ------------------------------------------------------------------------------------
template <class T>
static void build_vec_csr(edfa_system_s &S, PrecData<T> &D, const DBuf<T> &v, int smax, int pre,
                          double tau, Csr<T> &out, hipStream_t s) {
  const int ne = S.ne;
  out.rowptr.ensure((size_t)ne + 1);
  // patterns of up to 64 entries: wavefront kernels (the count and the write pass must
  // share the way the filtration norm is summed)
  const bool wave = smax <= 64;
  if (wave)
    hipLaunchKernelGGL(k_vec_count_w<T>, dim3(ceil_div(ne, 4)), dim3(256), 0, s, D.qlen.p, v.p,
                       ne, smax, pre, tau, out.rowptr.p);
  else
    hipLaunchKernelGGL(k_vec_count<T>, dim3(ceil_div(ne, 256)), dim3(256), 0, s, D.qlen.p, v.p,
                       ne, smax, pre, tau, out.rowptr.p);
  EDFA_CHECK_LAUNCH();
  const int64_t nnz = exclusive_scan(out.rowptr.p, out.rowptr.p, ne, S.tmp, s);
  out.rows = ne;
  out.cols = S.nfu;
  out.nnz = nnz;
  out.col.ensure(nnz);
  out.val.ensure(nnz);
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(ceil_div(ne, 64)), dim3(64), 0, s, D.Q.p, D.qlen.p, v.p, ne, smax,
                       pre, tau, out.rowptr.p, out.col.p, out.val.p);
    EDFA_CHECK_LAUNCH();
  };
  if (wave) {
    hipLaunchKernelGGL(k_vec_write_w<T>, dim3(ceil_div(ne, 4)), dim3(256), 0, s, D.Q.p, D.qlen.p,
                       v.p, ne, smax, pre, tau, out.rowptr.p, out.col.p, out.val.p);
    EDFA_CHECK_LAUNCH();
  } else if (smax <= 128)
    launch(k_vec_write<T, 128>);
  else
    launch(k_vec_write<T, PATCH_MAX>);
}

// Reads the error flags at `at` (and returns flags[at + 2], the scratch value of the last
// step).
static int check_flags(edfa_precond_s &P, hipStream_t s, const char *where, int at = 0) {
  int fl[3];
  read_small(fl, P.flags.p + at, 3, s);
  if (fl[0] != 0x7fffffff)
    fail(EDFA_ERR_NOT_SPD, "%s: restricted system of row/cell %d is not SPD", where, fl[0]);
  if (fl[1] != 0x7fffffff)
    fail(EDFA_ERR_CAPACITY, "%s: pattern capacity exceeded at row/cell %d", where, fl[1]);
  return fl[2];
}

static void reset_flags(edfa_precond_s &P, hipStream_t s) {
  P.flags.ensure(8);
  const int init[8] = {0x7fffffff, 0x7fffffff, 0, 0, 0x7fffffff, 0x7fffffff, 0, 0};
  EDFA_HIP(hipMemcpyAsync(P.flags.p, init, sizeof(init), hipMemcpyHostToDevice, s));
}

// Buckets of pattern capacity: a cell goes to the smallest compiled capacity that holds its
// pattern (its base or static pattern plus n_ent for the dynamic technique), and each bucket
// runs the restricted-solve kernel of its own capacity (or a larger one the setup tuner
// found faster).  40 and 44 keep the register kernel (its code grows with the square of
// the capacity) close to the patterns of the usual hexahedral grids (a base pattern of 36
// faces plus a few dynamic entries).
struct Capacities {
  int c[NCAP];
};
__global__ void k_need_bucket(const int *__restrict__ rp, const int *__restrict__ qlen, int ne,
                              int extra, Capacities caps, int *bucket) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= ne) return;
  const int need = (rp ? rp[m + 1] - rp[m] : qlen[m]) + extra;
  int b = NCAP;
  for (int i = NCAP - 1; i >= 0; --i)
    if (need <= caps.c[i]) b = i;
  bucket[m] = b;
}

template <class T>
static void launch_local(int cap, int cells, const LocalArgs<T> &la, hipStream_t s) {
  if (cells <= 0) return;
  switch (cap) {
    case 16: hipLaunchKernelGGL((k_local_reg<T, 16>), dim3(cells), dim3(64), 0, s, la); break;
    case 32: hipLaunchKernelGGL((k_local_reg<T, 32>), dim3(cells), dim3(64), 0, s, la); break;
    case 40: hipLaunchKernelGGL((k_local_reg<T, 40>), dim3(cells), dim3(64), 0, s, la); break;
    case 44: hipLaunchKernelGGL((k_local_reg<T, 44>), dim3(cells), dim3(64), 0, s, la); break;
    case 48: hipLaunchKernelGGL((k_local_reg<T, 48>), dim3(cells), dim3(64), 0, s, la); break;
    case 64: hipLaunchKernelGGL((k_local<T, 64>), dim3(cells), dim3(64), 0, s, la); break;
    case 128: hipLaunchKernelGGL((k_local<T, 128>), dim3(cells), dim3(64), 0, s, la); break;
    default: fail(EDFA_ERR_CAPACITY, "no restricted-solve kernel of capacity %d", cap);
  }
  EDFA_CHECK_LAUNCH();
}

// Kernel capacity of bucket b: the tuned one when set (never below the bucket's own).
static int bucket_capacity(const edfa_precond_s &P, int b) {
  const int own = kCapacities[b];
  return P.cap_map[b] > own ? P.cap_map[b] : own;
}

// FSAI of -A_pipi, its transpose and their SELL copies, on stream `ss` with the branch's own
// scratch and error flags (flags[4], [5]): nothing here depends on the restricted solves,
// so it runs beside them.  Records P.side.done at its end.
template <class T>
static void fsai_branch(edfa_precond_s &P, PrecData<T> &D, hipStream_t ss) {
  edfa_system_s &S = *P.sys;
  const int nfu = S.nfu;
  D.GF.rowptr.ensure((size_t)nfu + 1);
  hipLaunchKernelGGL(k_fsai_count, dim3(ceil_div(nfu, 256)), dim3(256), 0, ss, S.Afp.rowptr.p,
                     S.Afp.col.p, nfu, D.GF.rowptr.p);
  EDFA_CHECK_LAUNCH();
  const int64_t gnnz = exclusive_scan(D.GF.rowptr.p, D.GF.rowptr.p, nfu, P.side_tmp, ss);
  D.GF.rows = D.GF.cols = nfu;
  D.GF.nnz = gnnz;
  D.GF.col.ensure(gnnz);
  D.GF.val.ensure(gnnz);
  if (nfu > 0) {
    hipLaunchKernelGGL(k_fsai<T>, dim3(ceil_div(nfu, 64)), dim3(64), 0, ss, S.Afp.rowptr.p,
                       S.Afp.col.p, S.Afp.val.p, nfu, D.GF.rowptr.p, D.GF.col.p, D.GF.val.p,
                       P.flags.p + 4, P.flags.p + 5);
    EDFA_CHECK_LAUNCH();
  }
  check_flags(P, ss, "FSAI", 4);
  csr_transpose(D.GF, D.GFT, P.side_tmp, P.side_tmp2, ss);
  build_sell(D.GF, D.GF_s, P.side_tmp, ss);
  build_sell(D.GFT, D.GFT_s, P.side_tmp, ss);
  EDFA_HIP(hipEventRecord(P.side.done, ss));
}

template <class T>
static void stage1_impl(edfa_precond_s &P, PrecData<T> &D, hipStream_t s) {
  edfa_system_s &S = *P.sys;
  const edfa_params &prm = P.prm;
  const int ne = S.ne, nfu = S.nfu;
  reset_flags(P, s);
  int *err_spd = P.flags.p, *err_cap = P.flags.p + 1;

  // the register kernel and the rows of H~ read A_pipi as ELL_W-entry rows (its pattern is
  // fixed by the assembly: its longest row is found once)
  if (S.afp_max < 0) {
    EDFA_HIP(hipMemsetAsync(P.flags.p + 2, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_row_max, dim3(ceil_div(nfu, 256)), dim3(256), 0, s, S.Afp.rowptr.p,
                       nullptr, nfu, P.flags.p + 2);
    EDFA_CHECK_LAUNCH();
    S.afp_max = read_scalar(P.flags.p + 2, s);
  }
  const int afp_max = S.afp_max;
  if (afp_max > ELL_W)
    fail(EDFA_ERR_CAPACITY, "a row of A_pipi has %d > %d entries (hexahedra give at most 11)",
         afp_max, ELL_W);
  const bool dynamic = prm.variant == EDFA_DYNAMIC;
  const bool patches = !dynamic && prm.static_level > 0;
  D.qlen.ensure(ne);
  if (patches) {
    if (prm.static_level > 3) fail(EDFA_ERR_ARG, "static_level must be 0..3");
    // patches are built with the widest stride, then repacked to the storage stride
    D.wide.ensure((size_t)ne * PATCH_MAX);
    hipLaunchKernelGGL(k_patch, dim3(ceil_div(ne, 64)), dim3(64), 0, s, S.grids.p, S.ngrid,
                       S.uidx.p, S.Acf.rowptr.p, S.Acf.col.p, ne, prm.static_level,
                       prm.static_axis, S.W.p, PATCH_MAX, D.wide.p, D.qlen.p, err_cap);
    EDFA_CHECK_LAUNCH();
    check_flags(P, s, "static patch");
  }
  // cells by capacity bucket (from their base or static pattern length)
  D.bucket.ensure(std::max(ne, 1));
  D.bcells.ensure(std::max(ne, 1));
  std::vector<int> counts(NCAP + 1, 0);
  if (ne > 0) {
    Capacities caps;
    for (int i = 0; i < NCAP; ++i) caps.c[i] = kCapacities[i];
    hipLaunchKernelGGL(k_need_bucket, dim3(ceil_div(ne, 256)), dim3(256), 0, s,
                       patches ? nullptr : S.Acf.rowptr.p, D.qlen.p, ne,
                       dynamic ? std::max(0, prm.n_ent) : 0, caps, D.bucket.p);
    EDFA_CHECK_LAUNCH();
    stable_partition(D.bucket.p, ne, NCAP + 1, D.bcells.p, D.bhist, S.tmp, s, counts);
  }
  if (counts[NCAP] > 0)
    fail(EDFA_ERR_CAPACITY, "%d cells have patterns of more than %d entries", counts[NCAP],
         kCapacities[NCAP - 1]);
  int smax = kCapacities[0];
  for (int b = 0; b < NCAP; ++b) {
    P.bucket_cells[b] = counts[b];
    if (counts[b]) smax = std::max(smax, bucket_capacity(P, b));
  }
  D.Q.ensure((size_t)ne * smax);
  if (patches && ne > 0) {
    hipLaunchKernelGGL(k_repack, dim3(ceil_div(ne, 256)), dim3(256), 0, s, D.wide.p, D.qlen.p, ne,
                       PATCH_MAX, smax, D.Q.p);
    EDFA_CHECK_LAUNCH();
  }
  D.gbuf.ensure((size_t)ne * smax);
  D.fbuf.ensure((size_t)ne * smax);
  P.smax = smax;

  LocalArgs<T> la;
  la.ne = ne;
  la.app_rp = S.Afp.rowptr.p;
  la.app_col = S.Afp.col.p;
  la.app_val = S.Afp.val.p;
  la.ell_col = nullptr;
  la.ell_val = nullptr;
  if (nfu > 0) {
    D.ell_col.ensure((size_t)nfu * ELL_W);
    D.ell_val.ensure((size_t)nfu * ELL_W);
    hipLaunchKernelGGL(k_ell_fill, dim3(ceil_div((long long)nfu * ELL_W, 256)), dim3(256), 0, s,
                       S.Afp.rowptr.p, S.Afp.col.p, S.Afp.val.p, nfu, D.ell_col.p, D.ell_val.p);
    EDFA_CHECK_LAUNCH();
    la.ell_col = D.ell_col.p;
    la.ell_val = D.ell_val.p;
  }
  la.acf_rp = S.Acf.rowptr.p;
  la.acf_col = S.Acf.col.p;
  la.acf_val = S.Acf.val.p;
  la.afcT_rp = S.AfcT.rowptr.p;
  la.afcT_col = S.AfcT.col.p;
  la.afcT_val = S.AfcT.val.p;
  la.dynamic = dynamic;
  la.n_add = std::max(1, prm.n_add);
  la.n_ent = std::max(0, prm.n_ent);
  la.it_max = prm.it_max;
  la.Q = D.Q.p;
  la.qlen = D.qlen.p;
  la.gout = D.gbuf.p;
  la.fout = D.fbuf.p;
  la.err_spd = err_spd;
  la.err_cap = err_cap;
  la.qstride = smax;
  if (!patches && ne > 0) {
    hipLaunchKernelGGL(k_base, dim3(ceil_div(ne, 256)), dim3(256), 0, s, S.Acf.rowptr.p,
                       S.Acf.col.p, ne, smax, D.Q.p, D.qlen.p);
    EDFA_CHECK_LAUNCH();
  }
  // the FSAI branch runs on the side stream beside the restricted solves: ordered after what
  // s held before them (the flags' reset, any earlier use of G_F), and its host part, which
  // waits on the side stream only, is issued once the solves are queued
  hipStream_t ss = P.side.get();
  EDFA_HIP(hipEventRecord(P.side.start, s));
  // one launch per capacity bucket, over the bucket's cells
  for (int b = 0, off = 0; b < NCAP; off += counts[b], ++b) {
    la.cells = D.bcells.p + off;
    launch_local<T>(bucket_capacity(P, b), counts[b], la, s);
  }
  EDFA_HIP(hipStreamWaitEvent(ss, P.side.start, 0));
  fsai_branch<T>(P, D, ss);
  // longest final pattern (sizes the H~ tables), read with the error flags
  EDFA_HIP(hipMemsetAsync(P.flags.p + 2, 0, sizeof(int), s));
  if (ne > 0) {
    hipLaunchKernelGGL(k_row_max, dim3(ceil_div(ne, 256)), dim3(256), 0, s, nullptr, D.qlen.p,
                       ne, P.flags.p + 2);
    EDFA_CHECK_LAUNCH();
  }
  P.max_pattern = check_flags(P, s, "restricted solves");

  // G~ and F~^T (pre-filtration), F~ by faces
  const int pre = prm.filt_mode == EDFA_FILT_PRE;
  build_vec_csr(S, D, D.gbuf, smax, pre, prm.tau_filt, D.G, s);
  build_vec_csr(S, D, D.fbuf, smax, pre, prm.tau_filt, D.FT, s);
  csr_transpose(D.FT, D.Fface, S.tmp, S.tmp2, s, false);   // only its pattern is used

  // H~ = G~ A_pipi F~
  D.Hcol.ensure((size_t)ne * HMAX);
  D.Hval.ensure((size_t)ne * HMAX);
  D.Hlen.ensure(ne);
  HArgs<T> ha;
  ha.ne = ne;
  ha.g_rp = D.G.rowptr.p;
  ha.g_col = D.G.col.p;
  ha.g_val = D.G.val.p;
  ha.ell_col = la.ell_col;
  ha.ell_val = la.ell_val;
  ha.ff_rp = D.Fface.rowptr.p;
  ha.ff_col = D.Fface.col.p;
  // F~^T with its rows padded to a multiple of 16 entries (a row holds at most smax)
  D.ft_w = (smax + 15) / 16 * 16;
  D.ft_ecol.ensure((size_t)std::max(ne, 1) * D.ft_w);
  D.ft_eval.ensure((size_t)std::max(ne, 1) * D.ft_w);
  if (ne > 0) {
    hipLaunchKernelGGL(k_pad_rows<T>, dim3(ceil_div((long long)ne * D.ft_w, 256)), dim3(256), 0,
                       s, D.FT.rowptr.p, D.FT.col.p, D.FT.val.p, ne, D.ft_w, D.ft_ecol.p,
                       D.ft_eval.p);
    EDFA_CHECK_LAUNCH();
  }
  ha.ft_rp = D.FT.rowptr.p;
  ha.ft_ecol = D.ft_ecol.p;
  ha.ft_eval = D.ft_eval.p;
  ha.ft_w = D.ft_w;
  ha.Hcol = D.Hcol.p;
  ha.Hlen = D.Hlen.p;
  ha.Hval = D.Hval.p;
  ha.err_cap = err_cap;
  const int support = P.max_pattern * (S.axis ? 3 : 11);
  ha.cells = nullptr;
  ha.retry_count = nullptr;
  ha.retry_list = nullptr;
  // half of the small table of t (its hash probes stay short) unless the caller asks for less
  ha.t_retry = prm.htilde_retry > 0 ? std::min(prm.htilde_retry, 256) : 256;
  // large-table pass over `rows` rows (all cells, or the listed ones)
  auto large_pass = [&](int rows) {
    if (rows <= 0) return;
    if (P.max_pattern <= 32 && support <= 128)
      hipLaunchKernelGGL((k_htilde<T, 64, 256, 1024>), dim3(rows), dim3(64), 0, s, ha);
    else if (P.max_pattern <= 64 && support <= 512)
      hipLaunchKernelGGL((k_htilde<T, 128, 1024, 1024>), dim3(rows), dim3(64), 0, s, ha);
    else
      hipLaunchKernelGGL((k_htilde<T, 256, 2048, 1024>), dim3(rows), dim3(64), 0, s, ha);
    EDFA_CHECK_LAUNCH();
  };
  if (ne > 0 && P.max_pattern <= 64) {
    // first pass with small tables (about twice the occupancy); rows that fill them past
    // their limits are listed and recomputed with the large tables
    D.hretry.ensure(ne);
    EDFA_HIP(hipMemsetAsync(P.flags.p + 3, 0, sizeof(int), s));
    ha.retry_count = P.flags.p + 3;
    ha.retry_list = D.hretry.p;
    if (P.max_pattern <= 32)
      hipLaunchKernelGGL((k_htilde<T, 64, 512, 512>), dim3(ne), dim3(64), 0, s, ha);
    else
      hipLaunchKernelGGL((k_htilde<T, 128, 512, 512>), dim3(ne), dim3(64), 0, s, ha);
    EDFA_CHECK_LAUNCH();
    const int nretry = read_scalar(P.flags.p + 3, s);
    P.htilde_retry_rows = nretry;
    ha.retry_count = nullptr;
    ha.retry_list = nullptr;
    ha.cells = D.hretry.p;
    large_pass(nretry);
    ha.cells = nullptr;
  } else {
    P.htilde_retry_rows = 0;
    large_pass(ne);
  }
  check_flags(P, s, "H~ rows");
  {
    // entries of H~ before the post-filtration (diagnostic of what the filter drops)
    DBuf<unsigned long long> &acc = P.counter;
    acc.ensure(1);
    EDFA_HIP(hipMemsetAsync(acc.p, 0, sizeof(unsigned long long), s));
    if (ne > 0) {
      hipLaunchKernelGGL(k_len_sum, dim3(ceil_div(ne, 256)), dim3(256), 0, s, D.Hlen.p, ne, acc.p);
      EDFA_CHECK_LAUNCH();
    }
    EDFA_HIP(hipMemcpyAsync(P.nnz_h_raw.ensure(1), acc.p, sizeof(unsigned long long),
                            hipMemcpyDeviceToHost, s));
  }
  const int postH = prm.filt_mode == EDFA_FILT_POST_H;
  D.H.rowptr.ensure((size_t)ne + 1);
  hipLaunchKernelGGL(k_hcount<T>, dim3(ceil_div(ne, 4)), dim3(256), 0, s, D.Hcol.p, D.Hval.p,
                     D.Hlen.p, ne, postH, prm.tau_filt, D.H.rowptr.p);
  EDFA_CHECK_LAUNCH();
  const int64_t hnnz = exclusive_scan(D.H.rowptr.p, D.H.rowptr.p, ne, S.tmp, s);
  D.H.rows = D.H.cols = ne;
  D.H.nnz = hnnz;
  D.H.col.ensure(hnnz);
  D.H.val.ensure(hnnz);
  hipLaunchKernelGGL(k_hwrite<T>, dim3(ceil_div(ne, 4)), dim3(256), 0, s, D.Hcol.p, D.Hval.p,
                     D.Hlen.p, ne, postH, prm.tau_filt, D.H.rowptr.p, D.H.col.p, D.H.val.p);
  EDFA_CHECK_LAUNCH();

  // the FSAI branch joins here
  EDFA_HIP(hipStreamWaitEvent(s, P.side.done, 0));
}

// Setup tuner: each non-empty capacity bucket of the last stage 1 is timed (best of three
// launches over its cells, from the base or static patterns in scratch copies) with its own
// kernel capacity and the next two larger ones; the fastest, unless the default is within
// 3%, is kept for later setups.  The handle's preconditioner is left as it was built.
template <class T>
static void tune_setup_impl(edfa_precond_s &P, PrecData<T> &D, hipStream_t s,
                            edfa_setup_tune *rep) {
  edfa_system_s &S = *P.sys;
  const edfa_params &prm = P.prm;
  const int ne = S.ne;
  const bool dynamic = prm.variant == EDFA_DYNAMIC;
  const bool patches = !dynamic && prm.static_level > 0;
  if (rep) *rep = edfa_setup_tune{};
  if (rep) rep->buckets = NCAP;
  if (ne <= 0 || D.bcells.n < (size_t)ne) return;
  DBuf<int> Qt, qt;
  DBuf<T> gt, ft;
  qt.ensure(ne);
  hipEvent_t e0, e1;
  EDFA_HIP(hipEventCreate(&e0));
  EDFA_HIP(hipEventCreate(&e1));
  LocalArgs<T> la;
  la.ne = ne;
  la.app_rp = S.Afp.rowptr.p;
  la.app_col = S.Afp.col.p;
  la.app_val = S.Afp.val.p;
  la.ell_col = D.ell_col.p;
  la.ell_val = D.ell_val.p;
  la.acf_rp = S.Acf.rowptr.p;
  la.acf_col = S.Acf.col.p;
  la.acf_val = S.Acf.val.p;
  la.afcT_rp = S.AfcT.rowptr.p;
  la.afcT_col = S.AfcT.col.p;
  la.afcT_val = S.AfcT.val.p;
  la.dynamic = dynamic;
  la.n_add = std::max(1, prm.n_add);
  la.n_ent = std::max(0, prm.n_ent);
  la.it_max = prm.it_max;
  la.err_spd = P.flags.p;
  la.err_cap = P.flags.p + 1;
  try {
    for (int b = 0, off = 0; b < NCAP; off += P.bucket_cells[b], ++b) {
      const int nb = P.bucket_cells[b];
      if (rep) {
        rep->capacity[b] = kCapacities[b];
        rep->cells[b] = nb;
        rep->chosen[b] = bucket_capacity(P, b);
      }
      if (nb <= 0) continue;
      float best_us = INFINITY, own_us = INFINITY;
      int best = b;
      for (int c = b; c < std::min(NCAP, b + 3); ++c) {
        const int cap = kCapacities[c];
        Qt.ensure((size_t)ne * cap);
        gt.ensure((size_t)ne * cap);
        ft.ensure((size_t)ne * cap);
        la.Q = Qt.p;
        la.qlen = qt.p;
        la.gout = gt.p;
        la.fout = ft.p;
        la.qstride = cap;
        la.cells = D.bcells.p + off;
        float t = INFINITY;
        for (int r = 0; r < 3; ++r) {
          if (patches) {
            EDFA_HIP(hipMemcpyAsync(qt.p, D.qlen.p, sizeof(int) * ne, hipMemcpyDeviceToDevice, s));
            hipLaunchKernelGGL(k_repack, dim3(ceil_div(ne, 256)), dim3(256), 0, s, D.wide.p,
                               qt.p, ne, PATCH_MAX, cap, Qt.p);
          } else {
            hipLaunchKernelGGL(k_base, dim3(ceil_div(ne, 256)), dim3(256), 0, s, S.Acf.rowptr.p,
                               S.Acf.col.p, ne, cap, Qt.p, qt.p);
          }
          EDFA_CHECK_LAUNCH();
          EDFA_HIP(hipEventRecord(e0, s));
          launch_local<T>(cap, nb, la, s);
          EDFA_HIP(hipEventRecord(e1, s));
          EDFA_HIP(hipEventSynchronize(e1));
          float ms = 0;
          EDFA_HIP(hipEventElapsedTime(&ms, e0, e1));
          t = std::min(t, 1e3f * ms);
        }
        check_flags(P, s, "setup tuner");
        if (rep) rep->us[b][c] = t;
        if (c == b) own_us = t;
        if (t < best_us) {
          best_us = t;
          best = c;
        }
      }
      if (best != b && best_us > own_us * 0.97f) best = b;
      P.cap_map[b] = kCapacities[best];
      if (rep) rep->chosen[b] = kCapacities[best];
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

void tune_setup(edfa_precond_s &P, hipStream_t s, edfa_setup_tune *report) {
  if (P.prm.precision == 1)
    tune_setup_impl<float>(P, P.f, s, report);
  else
    tune_setup_impl<double>(P, P.d, s, report);
}

// Raw (unfiltered) H~ as CSR, for export.
template <class T>
void build_hraw(edfa_precond_s &P, PrecData<T> &D, hipStream_t s) {
  edfa_system_s &S = *P.sys;
  const int ne = S.ne;
  D.Hraw.rowptr.ensure((size_t)ne + 1);
  hipLaunchKernelGGL(k_hcount<T>, dim3(ceil_div(ne, 4)), dim3(256), 0, s, D.Hcol.p, D.Hval.p,
                     D.Hlen.p, ne, 0, 0.0, D.Hraw.rowptr.p);
  const int64_t nnz = exclusive_scan(D.Hraw.rowptr.p, D.Hraw.rowptr.p, ne, S.tmp, s);
  D.Hraw.rows = D.Hraw.cols = ne;
  D.Hraw.nnz = nnz;
  D.Hraw.col.ensure(nnz);
  D.Hraw.val.ensure(nnz);
  hipLaunchKernelGGL(k_hwrite<T>, dim3(ceil_div(ne, 4)), dim3(256), 0, s, D.Hcol.p, D.Hval.p,
                     D.Hlen.p, ne, 0, 0.0, D.Hraw.rowptr.p, D.Hraw.col.p, D.Hraw.val.p);
  EDFA_CHECK_LAUNCH();
}
template void build_hraw<double>(edfa_precond_s &, PrecData<double> &, hipStream_t);
template void build_hraw<float>(edfa_precond_s &, PrecData<float> &, hipStream_t);

void precond_stage1(edfa_precond_s &P, hipStream_t s) {
  if (P.prm.precision == 1)
    stage1_impl<float>(P, P.f, s);
  else
    stage1_impl<double>(P, P.d, s);
}

}  // namespace edfa
