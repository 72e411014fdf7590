// EDFA stage 2 (the paper's Algorithm 2) on the device, plus the inner preconditioner of S~.
//
//  * S~ = A_pp - H~ on the union pattern; optional post-filtration on S~ (diagonal kept)
//  * colouring of the graph of S~ + S~^T: Jones-Plassmann rounds whose result equals greedy
//    first fit over vertices by decreasing fmix32 priority (a vertex is coloured only after
//    all its higher-priority neighbours), so the colouring is deterministic
//  * stable permutation colour by colour, permuted matrix B = P S~ P^T
//  * ILU(0) of B, one launch per colour (rows of one colour are independent)
//  * sparse approximate inverses of the two triangular factors (row i of M solves
//    T[P_i,P_i]^T m = e_i on the pattern P_i of row i), used to apply the triangular solves
#include <algorithm>

#include "precond.hpp"

namespace edfa {

__device__ inline unsigned fmix32(unsigned h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// ---------------------------------------------------------------------------------------
// S~ = A_pp - H~
// ---------------------------------------------------------------------------------------
template <class T, bool WRITE>
__device__ int merge_row(const int *arp, const int *acol, const double *aval, const int *hrp,
                         const int *hcol, const T *hval, int i, int filt, double tau,
                         int *ocol, T *oval) {
  const int a0 = arp[i], a1 = arp[i + 1], h0 = hrp[i], h1 = hrp[i + 1];
  double thr = -1.0;
  if (filt) {
    double nrm = 0;
    int p = a0, q = h0;
    while (p < a1 || q < h1) {
      double v;
      if (q >= h1 || (p < a1 && acol[p] < hcol[q])) {
        v = aval[p++];
      } else if (p >= a1 || hcol[q] < acol[p]) {
        v = -(double)hval[q++];
      } else {
        v = (double)((T)aval[p] - hval[q]);
        ++p;
        ++q;
      }
      nrm += v * v;
    }
    thr = tau * sqrt(nrm);
  }
  int n = 0;
  int p = a0, q = h0;
  while (p < a1 || q < h1) {
    int c;
    T v;
    if (q >= h1 || (p < a1 && acol[p] < hcol[q])) {
      c = acol[p];
      v = (T)aval[p++];
    } else if (p >= a1 || hcol[q] < acol[p]) {
      c = hcol[q];
      v = -hval[q++];
    } else {
      c = acol[p];
      v = (T)aval[p++] - hval[q++];
    }
    if (filt && !(fabs((double)v) >= thr || c == i)) continue;
    if (WRITE) {
      ocol[n] = c;
      oval[n] = v;
    }
    ++n;
  }
  return n;
}

template <class T>
__global__ void k_merge_count(const int *arp, const int *acol, const double *aval, const int *hrp,
                              const int *hcol, const T *hval, int ne, int filt, double tau, int *len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  len[i] = merge_row<T, false>(arp, acol, aval, hrp, hcol, hval, i, filt, tau, nullptr, nullptr);
}

template <class T>
__global__ void k_merge_write(const int *arp, const int *acol, const double *aval, const int *hrp,
                              const int *hcol, const T *hval, int ne, int filt, double tau,
                              const int *orp, int *ocol, T *oval) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  merge_row<T, true>(arp, acol, aval, hrp, hcol, hval, i, filt, tau, ocol + orp[i], oval + orp[i]);
}

// Without post-filtration on S~: one wavefront per row (four per block of 256).  Lane j holds
// entry j of the A_pp row (rows of up to 64 entries; a longer row is merged by lane 0 with
// merge_row); the H~ row streams through in chunks of 64.  Pass 1 finds, for each A_pp
// entry, whether H~ holds its column and how many H~ columns are smaller; pass 2 places
// each H~ entry at its index plus the number of smaller A_pp-only columns, and each
// A_pp-only entry after the smaller H~ columns and the A_pp-only entries before it: the
// union sorted by column, with the same values as merge_row.
template <class T, bool WRITE>
__device__ int merge_row_wave(const int *arp, const int *acol, const double *aval, const int *hrp,
                              const int *hcol, const T *hval, int i, int lane, int *ocol,
                              T *oval) {
  const int a0 = arp[i], na = arp[i + 1] - a0, h0 = hrp[i], nh = hrp[i + 1] - h0;
  if (na > 64) {   // uniform
    int n = 0;
    if (lane == 0) n = merge_row<T, WRITE>(arp, acol, aval, hrp, hcol, hval, i, 0, 0.0, ocol, oval);
    return __shfl(n, 0);
  }
  const bool ina = lane < na;
  const int ac = ina ? acol[a0 + lane] : 0x7fffffff;
  const T av = ina ? (T)aval[a0 + lane] : T(0);
  int lessH = 0;      // for this lane's A_pp entry: H~ entries with smaller columns
  bool inH = false;   // ... and whether H~ holds its column
  for (int q0 = 0; q0 < nh; q0 += 64) {
    const int q = q0 + lane;
    const bool inh = q < nh;
    const int hc = inh ? hcol[h0 + q] : 0x7fffffff;
    for (int j = 0; j < na; ++j) {
      const int cj = __shfl(ac, j);
      const unsigned long long lt = __ballot(inh && hc < cj), eq = __ballot(inh && hc == cj);
      if (lane == j) {
        lessH += __popcll(lt);
        inH = inH || eq != 0;
      }
    }
  }
  const bool aonly = ina && !inH;
  const unsigned long long amask = __ballot(aonly);
  if (!WRITE) return nh + __popcll(amask);
  if (aonly) {
    const int o = lessH + __popcll(amask & ((1ull << lane) - 1));
    ocol[o] = ac;
    oval[o] = av;
  }
  for (int q0 = 0; q0 < nh; q0 += 64) {
    const int q = q0 + lane;
    const bool inh = q < nh;
    const int hc = inh ? hcol[h0 + q] : 0x7fffffff;
    const T hv = inh ? hval[h0 + q] : T(0);
    int less = 0, match = -1;
    for (int j = 0; j < na; ++j) {
      const int cj = __shfl(ac, j);
      less += ((amask >> j) & 1) && cj < hc;
      if (cj == hc) match = j;
    }
    const T am = __shfl(av, match < 0 ? 0 : match);
    if (inh) {
      ocol[q + less] = hc;
      oval[q + less] = match >= 0 ? am - hv : -hv;
    }
  }
  return nh + __popcll(amask);
}

template <class T>
__global__ __launch_bounds__(256) void k_merge_count_w(const int *arp, const int *acol,
                                                       const double *aval, const int *hrp,
                                                       const int *hcol, const T *hval, int ne,
                                                       int *len) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= ne) return;
  const int n = merge_row_wave<T, false>(arp, acol, aval, hrp, hcol, hval, i, lane, nullptr, nullptr);
  if (lane == 0) len[i] = n;
}

template <class T>
__global__ __launch_bounds__(256) void k_merge_write_w(const int *arp, const int *acol,
                                                       const double *aval, const int *hrp,
                                                       const int *hcol, const T *hval, int ne,
                                                       const int *orp, int *ocol, T *oval) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= ne) return;
  merge_row_wave<T, true>(arp, acol, aval, hrp, hcol, hval, i, lane, ocol + orp[i], oval + orp[i]);
}

// ---------------------------------------------------------------------------------------
// Colouring
// ---------------------------------------------------------------------------------------
// Priorities use the cell index local to its grid, so a batch of grids is coloured exactly
// as each grid alone (neighbours never cross grids).  One lane per vertex checks the common
// case: a vertex whose recorded blocker is still uncoloured stays blocked (two loads).  The
// wavefront then takes its other uncoloured vertices four at a time (16 lanes each), reading
// all neighbour entries (S~ row, then S~^T row) and their colours at once; the first uncoloured
// higher-priority neighbour blocks the vertex for this round and is recorded.  A vertex
// with no blocker takes the smallest colour unused by its neighbours (all coloured ones have
// higher priority), so the colouring does not depend on the order in which a round visits
// the vertices.
constexpr int JP_BATCH = 14;
__global__ __launch_bounds__(256) void k_jp_round(const int *__restrict__ srp,
                                                  const int *__restrict__ scol,
                                                  const int *__restrict__ trp,
                                                  const int *__restrict__ tcol, int ne,
                                                  const GridDesc *__restrict__ grids, int ngrid,
                                                  const int *__restrict__ list, int nlist,
                                                  int *color, int *blocker,
                                                  int *ncolored, int *err) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int v = -1, vs0 = 0, vls = 0, vt0 = 0, vlt = 0;
  bool need = false;
  if (slot < (list ? nlist : ne)) {
    v = list ? list[slot] : slot;
    // the vertex's colour and its recorded blocker are loaded together (one latency, not
    // two), and beside them the extents of its S~ and S~^T rows, which the full check below
    // takes from this lane
    const int bv = blocker[v];
    const int cv = __atomic_load_n(&color[v], __ATOMIC_RELAXED);
    vs0 = srp[v];
    vls = srp[v + 1] - vs0;
    vt0 = trp[v];
    vlt = trp[v + 1] - vt0;
    if (cv < 0) need = !(bv >= 0 && __atomic_load_n(&color[bv], __ATOMIC_RELAXED) < 0);
  }
  unsigned long long work = __ballot(need);
  const int g = lane >> 4, l = lane & 15;   // four groups of 16 lanes
  while (work) {   // uniform: the same mask in every lane
    // the next four vertices of the wavefront's list, one per group
    int mine = -1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (work) {
        if (q == g) mine = __ffsll((long long)work) - 1;
        work &= work - 1;
      }
    }
    const int src = mine >= 0 ? mine : 0;
    const int w = __shfl(v, src);
    const int s0 = __shfl(vs0, src), ls = __shfl(vls, src);
    const int t0 = __shfl(vt0, src), lt = __shfl(vlt, src);
    if (mine < 0) continue;
    const int c0 = grids[grid_of(grids, ngrid, w, true)].cell0;
    const unsigned pw = fmix32((unsigned)(w - c0));
    const int tot = ls + lt;
    // JP_BATCH entries per lane: the neighbour indices, then their colours, are each one
    // batch of independent loads; the same colours serve the blocking test and the choice
    // of colour (a coloured neighbour always has the higher priority)
    unsigned used[MAX_COLORS / 32];
#pragma unroll
    for (int q = 0; q < MAX_COLORS / 32; ++q) used[q] = 0;
    int first = -1;   // position of the first blocking entry (the same in the group)
    for (int base = 0; base < tot && first < 0; base += 16 * JP_BATCH) {
      int u[JP_BATCH], cu[JP_BATCH];
#pragma unroll
      for (int k = 0; k < JP_BATCH; ++k) {
        const int p = base + 16 * k + l;
        u[k] = p < tot ? (p < ls ? scol[s0 + p] : tcol[t0 + p - ls]) : w;
      }
#pragma unroll
      for (int k = 0; k < JP_BATCH; ++k) cu[k] = __atomic_load_n(&color[u[k]], __ATOMIC_RELAXED);
#pragma unroll
      for (int k = 0; k < JP_BATCH; ++k) {
        const bool blk = u[k] != w && cu[k] < 0 && fmix32((unsigned)(u[k] - c0)) > pw;
        const unsigned gm = (unsigned)(__ballot(blk) >> (16 * g)) & 0xffffu;
        if (first < 0 && gm) first = base + 16 * k + __ffs(gm) - 1;
        if (u[k] != w && cu[k] >= 0) used[cu[k] >> 5] |= 1u << (cu[k] & 31);
      }
    }
    if (first >= 0) {   // blocked for this round
      if (l == (first & 15)) blocker[w] = first < ls ? scol[s0 + first] : tcol[t0 + first - ls];
      continue;
    }
#pragma unroll
    for (int q = 0; q < MAX_COLORS / 32; ++q)
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) used[q] |= __shfl_xor(used[q], o, 16);
    if (l == 0) {
      int c = -1;
      for (int q = 0; q < MAX_COLORS / 32 && c < 0; ++q)
        if (~used[q]) c = q * 32 + __ffs(~used[q]) - 1;
      if (c < 0) {
        atomicMin(err, w);
        c = MAX_COLORS - 1;
      }
      __atomic_store_n(&color[w], c, __ATOMIC_RELAXED);
      atomicAdd(ncolored, 1);
    }
  }
}

// Worklist of the vertices still uncoloured (any order: a vertex's colour depends only on
// its coloured higher-priority neighbours, not on when it is visited).
__global__ __launch_bounds__(256) void k_uncolored(const int *__restrict__ color, int n, int *list,
                                                   int *count) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const bool keep = v < n && color[v] < 0;
  // one atomic per wavefront: lanes take consecutive slots after the wavefront's base
  const unsigned long long mask = __ballot(keep);
  if (!mask) return;
  const int lane = threadIdx.x & 63, leader = __ffsll((long long)mask) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, __popcll(mask));
  base = __shfl(base, leader);
  if (keep) list[base + __popcll(mask & ((1ull << lane) - 1))] = v;
}

// *out = max(*out, largest colour), one atomic per wavefront (colours are >= 0)
__global__ __launch_bounds__(256) void k_color_max(const int *__restrict__ color, int n,
                                                   int *out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  int c = -1;
  if (v < n) c = color[v];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c = max(c, __shfl_xor(c, o));
  if ((threadIdx.x & 63) == 0 && c >= 0) atomicMax(out, c);
}

// starts[c] = hist[c * nb] (the scanned histogram's first entry of each colour)
__global__ void k_color_starts(const int *__restrict__ hist, int nb, int ncol, int *starts) {
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) starts[c] = hist[(size_t)c * nb];
}

// per-block colour histograms, laid out colour-major: hist[c * nb + b]
__global__ __launch_bounds__(256) void k_color_hist(const int *__restrict__ color, int n, int ncol,
                                                    int nb, int *hist) {
  __shared__ int h[MAX_COLORS];
  for (int c = threadIdx.x; c < ncol; c += 256) h[c] = 0;
  __syncthreads();
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v < n) atomicAdd(&h[color[v]], 1);
  __syncthreads();
  for (int c = threadIdx.x; c < ncol; c += 256) hist[(size_t)c * nb + blockIdx.x] = h[c];
}

__global__ __launch_bounds__(256) void k_color_scatter(const int *__restrict__ color, int n, int nb,
                                                       const int *__restrict__ offs, int *perm,
                                                       int *iperm) {
  __shared__ int cl[256];
  const int v = blockIdx.x * 256 + threadIdx.x;
  cl[threadIdx.x] = v < n ? color[v] : -1;
  __syncthreads();
  if (v >= n) return;
  const int c = cl[threadIdx.x];
  int rank = 0;
  for (int t = 0; t < (int)threadIdx.x; ++t) rank += cl[t] == c;
  const int pos = offs[(size_t)c * nb + blockIdx.x] + rank;
  perm[pos] = v;
  iperm[v] = pos;
}

__global__ void k_gather_len(const int *__restrict__ rp, const int *__restrict__ perm, int n, int *len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) len[i] = rp[perm[i] + 1] - rp[perm[i]];
}

// B row i = S~ row perm[i] with columns mapped by iperm, sorted; one wavefront per row
template <class T>
__global__ __launch_bounds__(64) void k_permute_rows(const int *__restrict__ srp,
                                                     const int *__restrict__ scol,
                                                     const T *__restrict__ sval,
                                                     const int *__restrict__ perm,
                                                     const int *__restrict__ iperm, int n,
                                                     const int *__restrict__ brp, int *bcol,
                                                     T *bval, int *diag) {
  __shared__ int c[HMAX + 64];
  const int i = blockIdx.x;
  if (i >= n) return;
  const int r = perm[i];
  const int a = srp[r], len = srp[r + 1] - a;
  for (int t = threadIdx.x; t < len; t += 64) c[t] = iperm[scol[a + t]];
  __syncthreads();
  const int o = brp[i];
  for (int t = threadIdx.x; t < len; t += 64) {
    const int ct = c[t];
    int rank = 0;
    for (int u = 0; u < len; ++u) rank += c[u] < ct;
    bcol[o + rank] = ct;
    bval[o + rank] = sval[a + t];
    if (ct == i) diag[i] = o + rank;
  }
}

// Column -> position table of one row in LDS (open addressing, `bits` = log2 of its size,
// at least twice the row length).  A slot holds the key in its low and the position in its
// high 32 bits, so a probe is one LDS read; most lookups end at the first probe.  It sits at
// the start of the dynamic LDS (8-byte slots).
using RowSlot = unsigned long long;
constexpr RowSlot ROW_EMPTY = ~0ull;
__device__ inline unsigned row_slot(int key, int bits) {
  return ((unsigned)key * 2654435761u) >> (32 - bits);
}
__device__ inline void row_clear(RowSlot *tab, int bits) {
  for (int t = threadIdx.x; t < (1 << bits); t += blockDim.x) tab[t] = ROW_EMPTY;
}
__device__ inline void row_insert(RowSlot *tab, int bits, int key, int pos) {   // distinct keys
  const unsigned mask = (1u << bits) - 1;
  const RowSlot e = ((RowSlot)(unsigned)pos << 32) | (unsigned)key;
  unsigned h = row_slot(key, bits);
  while (atomicCAS(&tab[h], ROW_EMPTY, e) != ROW_EMPTY) h = (h + 1) & mask;
}
// Position of key (-1 when absent), given the content e of its first slot h: the first
// probe can then be issued early, beside other reads.
__device__ inline int row_resolve(const RowSlot *tab, int bits, int key, unsigned h, RowSlot e) {
  const unsigned mask = (1u << bits) - 1;
  for (;;) {
    const int k = (int)(unsigned)e;
    if (k == key) return (int)(e >> 32);
    if (k == -1) return -1;
    h = (h + 1) & mask;
    e = tab[h];
  }
}
__device__ inline int row_find(const RowSlot *tab, int bits, int key) {
  const unsigned h = row_slot(key, bits);
  return row_resolve(tab, bits, key, h, tab[h]);
}

// ILU(0), IKJ form, rows [r0, r1) of one colour; one wavefront per row.  The row lives in
// LDS; for each pivot column k (ascending) the lanes stream the U part of row k and update
// the matching entries of the row (found by binary search), so row i's updates keep the
// IKJ order exactly.
// Dynamic LDS of the per-row kernels below, `cap` entries per array (cap = the longest row
// of S~): the T arrays first, then the int arrays.
extern __shared__ __align__(16) unsigned char row_lds[];

template <class T>
__global__ __launch_bounds__(64) void k_ilu_color(const int *__restrict__ rp,
                                                  const int *__restrict__ col, T *val,
                                                  const int *__restrict__ diag, int r0, int r1,
                                                  int cap, int hbits, int *err) {
  RowSlot *tab = (RowSlot *)row_lds;   // column -> position of row i
  T *vi = (T *)(tab + (1 << hbits));
  int *ci = (int *)(vi + cap), *sdk = ci + cap, *sek = sdk + cap;
  const int i = r0 + blockIdx.x;
  if (i >= r1) return;
  const int a = rp[i], n = rp[i + 1] - a, d = diag[i] - a;
  row_clear(tab, hbits);
  for (int t = threadIdx.x; t < n; t += 64) {
    ci[t] = col[a + t];
    vi[t] = val[a + t];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n; t += 64) row_insert(tab, hbits, ci[t], t);
  // diagonal position and end of every pivot row, all at once
  for (int t = threadIdx.x; t < d; t += 64) {
    const int k = ci[t];
    sdk[t] = diag[k];
    sek[t] = rp[k + 1];
  }
  __syncthreads();
  // Software pipeline over the pivots: u_kk and the first 128 upper entries of pivot rows
  // (two entries per lane, in registers) are loaded three steps ahead.  The loop is
  // unrolled over three register slots used in place: moving a register whose load is in
  // flight would wait for that load.
  // Every step issues the same loads without a branch (entries past the row's end read
  // its diagonal; a clamped step index re-reads the last pivot), so the compiler can wait
  // for exactly the oldest slot's loads.
  struct Piv {
    T uk, v0, v1;
    int c0, c1;
    bool ok0, ok1;
  };
  auto fetch = [&](int p, Piv &g) {
    const int dk = sdk[p], ek = sek[p];
    const int q = dk + 1 + threadIdx.x;
    g.ok0 = q < ek;
    g.ok1 = q + 64 < ek;
    const int q0 = g.ok0 ? q : dk, q1 = g.ok1 ? q + 64 : dk;
    g.uk = val[dk];
    g.c0 = col[q0];
    g.v0 = val[q0];
    g.c1 = col[q1];
    g.v1 = val[q1];
  };
  auto step = [&](int p, Piv &f) {
    const int cdk = sdk[p], cek = sek[p];
    // the first probes of both entries issue with the read of the row's entry p, so the
    // chain of a step is one LDS read, the division and one read-modify-write
    const unsigned h0 = row_slot(f.c0, hbits), h1 = row_slot(f.c1, hbits);
    const RowSlot e0 = tab[h0], e1 = tab[h1];
    const T lik = vi[p] / f.uk;
    // a pivot row's columns exceed k = ci[p], so the positions found lie past p; its
    // columns are distinct, so are the two positions, and both reads may go first
    const int pos0 = f.ok0 ? row_resolve(tab, hbits, f.c0, h0, e0) : -1;
    const int pos1 = f.ok1 ? row_resolve(tab, hbits, f.c1, h1, e1) : -1;
    const T a0 = vi[pos0 >= 0 ? pos0 : p], a1 = vi[pos1 >= 0 ? pos1 : p];
    if (pos0 >= 0) vi[pos0] = a0 - lik * f.v0;
    if (pos1 >= 0) vi[pos1] = a1 - lik * f.v1;
    for (int q = cdk + 129 + threadIdx.x; q < cek; q += 64) {   // pivot rows past 128 entries
      const int pos = row_find(tab, hbits, col[q]);
      if (pos >= 0) vi[pos] -= lik * val[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) vi[p] = lik;
    fetch(min(p + 3, d - 1), f);   // this slot serves step p + 3
  };
  Piv fa, fb, fc;
  if (d > 0) {
    fetch(0, fa);
    fetch(min(1, d - 1), fb);
    fetch(min(2, d - 1), fc);
  }
  // whole groups of three steps, then the tail: every path around the loop issues the
  // same loads, so the wait before a step covers only its own slot
  int p = 0;
  for (; p + 3 <= d; p += 3) {
    step(p, fa);
    step(p + 1, fb);
    step(p + 2, fc);
  }
  if (p < d) step(p, fa);
  if (p + 1 < d) step(p + 1, fb);
  __syncthreads();
  for (int t = threadIdx.x; t < n; t += 64) val[a + t] = vi[t];
  if (threadIdx.x == 0) {
    const T piv = vi[d];
    if (!(piv != T(0)) || !isfinite((double)piv)) atomicMin(err, i);
  }
}

__global__ void k_check_diag(const int *__restrict__ diag, int n, int *err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && diag[i] < 0) atomicMin(err, i);
}

__global__ void k_split_len(const int *__restrict__ rp, const int *__restrict__ diag, int n,
                            int *llen, int *ulen) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  llen[i] = diag[i] - rp[i];
  ulen[i] = rp[i + 1] - diag[i];
}

// L and U parts of each row (one wavefront per row, four rows per block of 256)
template <class T>
__global__ __launch_bounds__(256) void k_split(const int *__restrict__ rp,
                                               const int *__restrict__ col,
                                               const T *__restrict__ val,
                                               const int *__restrict__ diag, int n,
                                               const int *__restrict__ lrp, int *lcol, T *lval,
                                               const int *__restrict__ urp, int *ucol, T *uval) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= n) return;
  const int a = rp[i], e = rp[i + 1], d = diag[i];
  const int lo = lrp[i] - a, uo = urp[i] - d;
  for (int p = a + lane; p < e; p += 64) {
    if (p < d) {
      lcol[lo + p] = col[p];
      lval[lo + p] = val[p];
    } else {
      ucol[uo + p] = col[p];
      uval[uo + p] = val[p];
    }
  }
}

// ISAI of the unit lower factor (I + L): row i on P = cols(L row i) + {i}.
// (T[P,P])^T m = e_i, solved from the last index down: m_k = delta_ik - sum_{j>k} T[j,k] m_j.
// The extents of all rows k in P are read at once; the first 64 entries of the rows of the
// next two steps are in flight (one per lane, in registers) while a step runs, and rows
// past 64 entries read their remainder in the step.  The order of the updates of each
// acc entry is the order of the steps, as without the prefetch.
template <class T>
__global__ __launch_bounds__(64) void k_isai_lower(const int *__restrict__ lrp,
                                                   const int *__restrict__ lcol,
                                                   const T *__restrict__ lval, int n, int cap,
                                                   int hbits, const int *__restrict__ mrp,
                                                   int *mcol, T *mval) {
  RowSlot *tab = (RowSlot *)row_lds;   // column -> index in P
  T *acc = (T *)(tab + (1 << hbits));
  int *P = (int *)(acc + cap), *rb = P + cap, *re = rb + cap;
  const int i = blockIdx.x;
  if (i >= n) return;
  const int a = lrp[i], nl = lrp[i + 1] - a, np = nl + 1;
  row_clear(tab, hbits);
  __syncthreads();
  for (int t = threadIdx.x; t < np; t += 64) {
    const int k = t < nl ? lcol[a + t] : i;
    P[t] = k;
    rb[t] = lrp[k];
    re[t] = lrp[k + 1];
    acc[t] = 0;
    row_insert(tab, hbits, k, t);
  }
  __syncthreads();
  const int o = mrp[i];
  // branch-free loads (an entry past the row's end reads entry 0, unused), so every step
  // issues the same loads and the compiler waits for exactly the oldest slot's
  auto fetch = [&](int idx, int &c, T &v) {
    const int q = rb[idx] + threadIdx.x;
    const int qc = q < re[idx] ? q : 0;
    c = lcol[qc];
    v = lval[qc];
  };
  // three register slots used in place (see k_ilu_color), loaded three steps ahead
  auto step = [&](int idx, int &c0, T &v0) {
    const unsigned h0 = row_slot(c0, hbits);
    const RowSlot e0 = tab[h0];   // first probe, beside the reads below
    const int k = P[idx];
    const T mk = (k == i ? T(1) : T(0)) - acc[idx];
    // acc[idx] is final once read: it keeps m_k until the row is written out at the end
    // (no global store inside the loop, so the barrier waits for no memory operation)
    if (threadIdx.x == 0) acc[idx] = mk;
    // row k's columns are below k = P[idx], so the indices found lie before idx
    if (rb[idx] + (int)threadIdx.x < re[idx]) {
      const int pos = row_resolve(tab, hbits, c0, h0, e0);
      if (pos >= 0) acc[pos] += v0 * mk;
    }
    for (int p = rb[idx] + 64 + threadIdx.x; p < re[idx]; p += 64) {
      const int pos = row_find(tab, hbits, lcol[p]);
      if (pos >= 0) acc[pos] += lval[p] * mk;
    }
    __syncthreads();
    fetch(max(idx - 3, 0), c0, v0);
  };
  int ca, cb, cc;
  T va, vb, vc;
  fetch(np - 1, ca, va);
  fetch(max(np - 2, 0), cb, vb);
  fetch(max(np - 3, 0), cc, vc);
  int idx = np - 1;   // whole groups of three, then the tail (see k_ilu_color)
  for (; idx >= 2; idx -= 3) {
    step(idx, ca, va);
    step(idx - 1, cb, vb);
    step(idx - 2, cc, vc);
  }
  if (idx >= 0) step(idx, ca, va);
  if (idx >= 1) step(idx - 1, cb, vb);
  for (int t = threadIdx.x; t < np; t += 64) {
    mcol[o + t] = P[t];
    mval[o + t] = acc[t];
  }
}

// ISAI of U (diagonal first in each row): row i on P = cols(U row i).
// (U[P,P])^T m = e_i, solved upward: m_k = (delta_ik - sum_{j<k} U[j,k] m_j) / U[k,k].
// Same prefetch scheme as the lower factor (rows k start with their diagonal, read with the
// extents).
template <class T>
__global__ __launch_bounds__(64) void k_isai_upper(const int *__restrict__ urp,
                                                   const int *__restrict__ ucol,
                                                   const T *__restrict__ uval, int n, int cap,
                                                   int hbits, int *mcol, T *mval) {
  RowSlot *tab = (RowSlot *)row_lds;   // column -> index in P
  T *acc = (T *)(tab + (1 << hbits)), *ud = acc + cap;
  int *P = (int *)(ud + cap), *rb = P + cap, *re = rb + cap;
  const int i = blockIdx.x;
  if (i >= n) return;
  const int a = urp[i], np = urp[i + 1] - a;
  row_clear(tab, hbits);
  __syncthreads();
  for (int t = threadIdx.x; t < np; t += 64) {
    const int k = ucol[a + t];
    P[t] = k;
    const int kb = urp[k];
    rb[t] = kb + 1;
    re[t] = urp[k + 1];
    ud[t] = uval[kb];
    acc[t] = 0;
    row_insert(tab, hbits, k, t);
  }
  __syncthreads();
  auto fetch = [&](int idx, int &c, T &v) {   // as in k_isai_lower
    const int q = rb[idx] + threadIdx.x;
    const int qc = q < re[idx] ? q : 0;
    c = ucol[qc];
    v = uval[qc];
  };
  // three register slots used in place (see k_ilu_color), loaded three steps ahead
  auto step = [&](int idx, int &c0, T &v0) {
    const unsigned h0 = row_slot(c0, hbits);
    const RowSlot e0 = tab[h0];   // first probe, beside the reads below
    const int k = P[idx];
    const T mk = ((k == i ? T(1) : T(0)) - acc[idx]) / ud[idx];
    if (threadIdx.x == 0) acc[idx] = mk;   // kept until the row is written out
    // row k's columns past its diagonal exceed k = P[idx]: the indices found lie past idx
    if (rb[idx] + (int)threadIdx.x < re[idx]) {
      const int pos = row_resolve(tab, hbits, c0, h0, e0);
      if (pos >= 0) acc[pos] += v0 * mk;
    }
    for (int p = rb[idx] + 64 + threadIdx.x; p < re[idx]; p += 64) {
      const int pos = row_find(tab, hbits, ucol[p]);
      if (pos >= 0) acc[pos] += uval[p] * mk;
    }
    __syncthreads();
    fetch(min(idx + 3, np - 1), c0, v0);
  };
  if (np <= 0) return;
  int ca, cb, cc;
  T va, vb, vc;
  fetch(0, ca, va);
  fetch(min(1, np - 1), cb, vb);
  fetch(min(2, np - 1), cc, vc);
  int idx = 0;   // whole groups of three, then the tail (see k_ilu_color)
  for (; idx + 3 <= np; idx += 3) {
    step(idx, ca, va);
    step(idx + 1, cb, vb);
    step(idx + 2, cc, vc);
  }
  if (idx < np) step(idx, ca, va);
  if (idx + 1 < np) step(idx + 1, cb, vb);
  for (int t = threadIdx.x; t < np; t += 64) {
    mcol[a + t] = P[t];
    mval[a + t] = acc[t];
  }
}

__global__ void k_ml_rowptr(const int *__restrict__ lrp, int n, int *mrp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n) mrp[i] = lrp[i] + i;
}

// *out = max(*out, longest row), one atomic per wavefront after a shuffle reduction
__global__ __launch_bounds__(256) void k_row_len_max(const int *__restrict__ rp, int rows,
                                                     int *out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  int v = 0;
  if (r < rows) v = rp[r + 1] - rp[r];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0 && v > 0) atomicMax(out, v);
}

// ---------------------------------------------------------------------------------------
// N = P^T M P: row o of N is row iperm[o] of M (colour order) with columns mapped back by
// perm, sorted.
template <class T>
static void to_natural_order(const Csr<T> &M, Csr<T> &N, PrecData<T> &D, edfa_system_s &S,
                             hipStream_t s) {
  const int n = M.rows;
  N.alloc(n, n, M.nnz);
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather_len, dim3(ceil_div(n, 256)), dim3(256), 0, s, M.rowptr.p, D.iperm.p,
                     n, N.rowptr.p);
  EDFA_CHECK_LAUNCH();
  exclusive_scan(N.rowptr.p, N.rowptr.p, n, S.tmp, s);
  D.scratch_diag.ensure(n);
  hipLaunchKernelGGL(k_permute_rows<T>, dim3(n), dim3(64), 0, s, M.rowptr.p, M.col.p, M.val.p,
                     D.iperm.p, D.perm.p, n, N.rowptr.p, N.col.p, N.val.p, D.scratch_diag.p);
  EDFA_CHECK_LAUNCH();
}

template <class T>
static void stage2_impl(edfa_precond_s &P, PrecData<T> &D, hipStream_t s) {
  edfa_system_s &S = *P.sys;
  const edfa_params &prm = P.prm;
  const int ne = S.ne;
  P.flags.ensure(4);
  const int init[4] = {0x7fffffff, 0x7fffffff, 0, 0};
  EDFA_HIP(hipMemcpyAsync(P.flags.p, init, sizeof(init), hipMemcpyHostToDevice, s));

  // S~ = A_pp - H~, post-filtration on S~
  const int postS = prm.filt_mode == EDFA_FILT_POST_S;
  D.S.rowptr.ensure((size_t)ne + 1);
  if (postS)
    hipLaunchKernelGGL(k_merge_count<T>, dim3(ceil_div(ne, 256)), dim3(256), 0, s,
                       S.Acc.rowptr.p, S.Acc.col.p, S.Acc.val.p, D.H.rowptr.p, D.H.col.p,
                       D.H.val.p, ne, postS, prm.tau_filt, D.S.rowptr.p);
  else
    hipLaunchKernelGGL(k_merge_count_w<T>, dim3(ceil_div(ne, 4)), dim3(256), 0, s,
                       S.Acc.rowptr.p, S.Acc.col.p, S.Acc.val.p, D.H.rowptr.p, D.H.col.p,
                       D.H.val.p, ne, D.S.rowptr.p);
  EDFA_CHECK_LAUNCH();
  const int64_t snnz = exclusive_scan(D.S.rowptr.p, D.S.rowptr.p, ne, S.tmp, s);
  D.S.rows = D.S.cols = ne;
  D.S.nnz = snnz;
  D.S.col.ensure(snnz);
  D.S.val.ensure(snnz);
  if (postS)
    hipLaunchKernelGGL(k_merge_write<T>, dim3(ceil_div(ne, 256)), dim3(256), 0, s,
                       S.Acc.rowptr.p, S.Acc.col.p, S.Acc.val.p, D.H.rowptr.p, D.H.col.p,
                       D.H.val.p, ne, postS, prm.tau_filt, D.S.rowptr.p, D.S.col.p, D.S.val.p);
  else
    hipLaunchKernelGGL(k_merge_write_w<T>, dim3(ceil_div(ne, 4)), dim3(256), 0, s,
                       S.Acc.rowptr.p, S.Acc.col.p, S.Acc.val.p, D.H.rowptr.p, D.H.col.p,
                       D.H.val.p, ne, D.S.rowptr.p, D.S.col.p, D.S.val.p);
  EDFA_CHECK_LAUNCH();
  EDFA_HIP(hipMemsetAsync(P.flags.p + 2, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_row_len_max, dim3(ceil_div(ne, 256)), dim3(256), 0, s, D.S.rowptr.p, ne,
                     P.flags.p + 2);
  EDFA_CHECK_LAUNCH();
  const int smaxrow = read_scalar(P.flags.p + 2, s);
  if (smaxrow > HMAX + 64) fail(EDFA_ERR_CAPACITY, "a row of S~ has %d > %d entries", smaxrow, HMAX + 64);
  csr_transpose(D.S, D.ST, S.tmp, S.tmp2, s, false);   // pattern only (colouring)

  // colouring
  D.color.ensure(ne);
  EDFA_HIP(hipMemsetAsync(D.color.p, 0xff, sizeof(int) * ne, s));
  EDFA_HIP(hipMemsetAsync(P.flags.p + 2, 0, sizeof(int), s));
  D.blocker.ensure(ne);
  EDFA_HIP(hipMemsetAsync(D.blocker.p, 0xff, sizeof(int) * (size_t)ne, s));
  int rounds = 0, list_rounds = 0;
  int nlist = ne;                 // vertices each round visits
  const int *list = nullptr;      // nullptr: all of them
  D.jplist.ensure(ne);
  while (true) {
    // a round is cheap (one load per vertex still blocked), so check completion rarely
    const int batch = rounds < 64 ? 16 : 32;
    for (int r = 0; r < batch; ++r)
      hipLaunchKernelGGL(k_jp_round, dim3(ceil_div(nlist, 256)), dim3(256), 0, s,
                         D.S.rowptr.p, D.S.col.p, D.ST.rowptr.p, D.ST.col.p, ne, S.grids.p,
                         S.ngrid, list, nlist, D.color.p, D.blocker.p,
                         P.flags.p + 2, P.flags.p + 1);
    EDFA_CHECK_LAUNCH();
    rounds += batch;
    if (list) list_rounds += batch;
    const int done = read_scalar(P.flags.p + 2, s);
    if (done >= ne) break;
    if (rounds > 2 * ne + 64) fail(EDFA_ERR_BREAKDOWN, "colouring did not finish");
    if (10 * (ne - done) < 7 * nlist) {
      // under 70% of the visited vertices are left: visit only those from now on
      EDFA_HIP(hipMemsetAsync(P.flags.p + 3, 0, sizeof(int), s));
      hipLaunchKernelGGL(k_uncolored, dim3(ceil_div(ne, 256)), dim3(256), 0, s, D.color.p, ne,
                         D.jplist.p, P.flags.p + 3);
      EDFA_CHECK_LAUNCH();
      nlist = read_scalar(P.flags.p + 3, s);
      list = D.jplist.p;
    }
  }
  P.color_rounds = rounds;
  P.color_list_rounds = list_rounds;
  if (read_scalar(P.flags.p + 1, s) != 0x7fffffff)
    fail(EDFA_ERR_CAPACITY, "more than %d colours needed", MAX_COLORS);
  EDFA_HIP(hipMemsetAsync(P.flags.p + 3, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_color_max, dim3(ceil_div(ne, 256)), dim3(256), 0, s, D.color.p, ne,
                     P.flags.p + 3);
  EDFA_CHECK_LAUNCH();
  const int ncol = ne ? read_scalar(P.flags.p + 3, s) + 1 : 0;
  P.n_colors = ncol;

  // stable permutation by colour
  const int nb = ceil_div(ne, 256);

  D.hist.ensure((size_t)ncol * nb + 1 + (size_t)ncol);   // scan, then the colour starts
  D.perm.ensure(ne);
  D.iperm.ensure(ne);
  if (ne) {
    hipLaunchKernelGGL(k_color_hist, dim3(nb), dim3(256), 0, s, D.color.p, ne, ncol, nb, D.hist.p);
    EDFA_CHECK_LAUNCH();
    exclusive_scan_async(D.hist.p, D.hist.p, ncol * nb, S.tmp, s);
    hipLaunchKernelGGL(k_color_scatter, dim3(nb), dim3(256), 0, s, D.color.p, ne, nb, D.hist.p,
                       D.perm.p, D.iperm.p);
    EDFA_CHECK_LAUNCH();
  }
  D.cstart.assign(ncol + 1, ne);
  if (ne) {
    // the first position of colour c is the scanned count of (c, block 0): gathered behind
    // the histogram, then one small read
    int *starts = D.hist.p + (size_t)ncol * nb + 1;
    hipLaunchKernelGGL(k_color_starts, dim3(1), dim3(256), 0, s, D.hist.p, nb, ncol, starts);
    EDFA_CHECK_LAUNCH();
    read_small(D.cstart.data(), starts, (size_t)ncol, s);
  }

  // permuted matrix
  D.B.rowptr.ensure((size_t)ne + 1);
  hipLaunchKernelGGL(k_gather_len, dim3(ceil_div(ne, 256)), dim3(256), 0, s, D.S.rowptr.p,
                     D.perm.p, ne, D.B.rowptr.p);
  EDFA_CHECK_LAUNCH();
  exclusive_scan(D.B.rowptr.p, D.B.rowptr.p, ne, S.tmp, s);
  D.B.rows = D.B.cols = ne;
  D.B.nnz = snnz;
  D.B.col.ensure(snnz);
  D.B.val.ensure(snnz);
  D.diag.ensure(ne);
  EDFA_HIP(hipMemsetAsync(D.diag.p, 0xff, sizeof(int) * (size_t)ne, s));
  if (ne) {
    hipLaunchKernelGGL(k_permute_rows<T>, dim3(ne), dim3(64), 0, s, D.S.rowptr.p, D.S.col.p,
                       D.S.val.p, D.perm.p, D.iperm.p, ne, D.B.rowptr.p, D.B.col.p, D.B.val.p,
                       D.diag.p);
    EDFA_CHECK_LAUNCH();
  }

  hipLaunchKernelGGL(k_check_diag, dim3(ceil_div(ne, 256)), dim3(256), 0, s, D.diag.p, ne,
                     P.flags.p + 1);
  EDFA_CHECK_LAUNCH();
  if (read_scalar(P.flags.p + 1, s) != 0x7fffffff)
    fail(EDFA_ERR_BREAKDOWN, "S~ row %d has no diagonal entry", read_scalar(P.flags.p + 1, s));
  // ILU(0) colour by colour; the per-row kernels size their LDS by the longest row
  const int cap = std::max(smaxrow, 1);
  int hbits = 1;
  while ((1 << hbits) < 2 * cap) ++hbits;
  const size_t lds_ilu = (size_t)cap * (sizeof(T) + 3 * sizeof(int)) + sizeof(int) * (2u << hbits);
  for (int c = 0; c < ncol; ++c) {
    const int r0 = D.cstart[c], r1 = D.cstart[c + 1];
    if (r1 > r0)
      hipLaunchKernelGGL(k_ilu_color<T>, dim3(r1 - r0), dim3(64), lds_ilu, s, D.B.rowptr.p,
                         D.B.col.p, D.B.val.p, D.diag.p, r0, r1, cap, hbits, P.flags.p);
  }
  EDFA_CHECK_LAUNCH();
  if (read_scalar(P.flags.p, s) != 0x7fffffff)
    fail(EDFA_ERR_BREAKDOWN, "ILU(0) of S~: zero or non-finite pivot at row %d", read_scalar(P.flags.p, s));

  // L (strict lower, unit factor) and U (with diagonal)
  D.L.rowptr.ensure((size_t)ne + 1);
  D.U.rowptr.ensure((size_t)ne + 1);
  hipLaunchKernelGGL(k_split_len, dim3(ceil_div(ne, 256)), dim3(256), 0, s, D.B.rowptr.p, D.diag.p,
                     ne, D.L.rowptr.p, D.U.rowptr.p);
  EDFA_CHECK_LAUNCH();
  const int64_t lnnz = exclusive_scan(D.L.rowptr.p, D.L.rowptr.p, ne, S.tmp, s);
  const int64_t unnz = exclusive_scan(D.U.rowptr.p, D.U.rowptr.p, ne, S.tmp, s);
  D.L.rows = D.L.cols = D.U.rows = D.U.cols = ne;
  D.L.nnz = lnnz;
  D.U.nnz = unnz;
  D.L.col.ensure(lnnz);
  D.L.val.ensure(lnnz);
  D.U.col.ensure(unnz);
  D.U.val.ensure(unnz);
  hipLaunchKernelGGL(k_split<T>, dim3(ceil_div(ne, 4)), dim3(256), 0, s, D.B.rowptr.p, D.B.col.p,
                     D.B.val.p, D.diag.p, ne, D.L.rowptr.p, D.L.col.p, D.L.val.p, D.U.rowptr.p,
                     D.U.col.p, D.U.val.p);
  EDFA_CHECK_LAUNCH();

  if (prm.schur_solver == EDFA_SCHUR_ISAI) {
    D.ML.alloc(ne, ne, lnnz + ne);
    D.MU.alloc(ne, ne, unnz);
    hipLaunchKernelGGL(k_ml_rowptr, dim3(ceil_div(ne + 1, 256)), dim3(256), 0, s, D.L.rowptr.p, ne,
                       D.ML.rowptr.p);
    EDFA_CHECK_LAUNCH();
    EDFA_HIP(hipMemcpyAsync(D.MU.rowptr.p, D.U.rowptr.p, sizeof(int) * ((size_t)ne + 1),
                            hipMemcpyDeviceToDevice, s));
    if (ne) {
      const size_t lds_tab = sizeof(int) * (2u << hbits);
      hipLaunchKernelGGL(k_isai_lower<T>, dim3(ne), dim3(64),
                         (size_t)cap * (sizeof(T) + 3 * sizeof(int)) + lds_tab, s, D.L.rowptr.p,
                         D.L.col.p, D.L.val.p, ne, cap, hbits, D.ML.rowptr.p, D.ML.col.p,
                         D.ML.val.p);
      EDFA_CHECK_LAUNCH();
      hipLaunchKernelGGL(k_isai_upper<T>, dim3(ne), dim3(64),
                         (size_t)cap * (2 * sizeof(T) + 3 * sizeof(int)) + lds_tab, s,
                         D.U.rowptr.p, D.U.col.p, D.U.val.p, ne, cap, hbits, D.MU.col.p,
                         D.MU.val.p);
      EDFA_CHECK_LAUNCH();
    }
  }
  if (prm.schur_solver == EDFA_SCHUR_ISAI) {
    // the application works in the natural cell order: P^T M P for every factor it uses
    // (the factors themselves only in the refinement steps)
    if (prm.isai_steps > 1) {
      to_natural_order(D.L, D.Ln, D, S, s);
      to_natural_order(D.U, D.Un, D, S, s);
      build_sell(D.Ln, D.L_s, S.tmp, s);
      build_sell(D.Un, D.U_s, S.tmp, s);
    } else {
      D.L_s.rows = D.U_s.rows = 0;
    }
    to_natural_order(D.ML, D.MLn, D, S, s);
    to_natural_order(D.MU, D.MUn, D, S, s);
    build_sell(D.MLn, D.ML_s, S.tmp, s);
    build_sell(D.MUn, D.MU_s, S.tmp, s);
  } else {
    build_sell(D.L, D.L_s, S.tmp, s);
    build_sell(D.U, D.U_s, S.tmp, s);
  }
  // transposes are rebuilt lazily for the transposed application
  D.LT.rows = D.UT.rows = D.MLT.rows = D.MUT.rows = 0;
  EDFA_HIP(hipStreamSynchronize(s));
}

void precond_stage2(edfa_precond_s &P, hipStream_t s) {
  if (P.prm.precision == 1)
    stage2_impl<float>(P, P.f, s);
  else
    stage2_impl<double>(P, P.d, s);
}

}  // namespace edfa
