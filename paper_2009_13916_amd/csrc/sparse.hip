// Primitive device algorithms: prefix sums, CSR transpose, CSR SpMV.
#include <hip/hip_ext.h>

#include <vector>

#include "common.hpp"

namespace edfa {

// ----------------------------------------------------------------------------------
// Exclusive scan.  Tiles of 2048 int32 per 256-thread block, tile totals scanned
// recursively.  The output has n_out = n_in + 1 slots so that out[n_in] is the total.
// ----------------------------------------------------------------------------------
constexpr int SCAN_T = 256;
constexpr int SCAN_I = 8;
constexpr int SCAN_TILE = SCAN_T * SCAN_I;

__global__ __launch_bounds__(SCAN_T) void k_scan_tile(const int *__restrict__ in, int *out,
                                                      int n_in, int n_out, int *totals) {
  __shared__ int sh[SCAN_T];
  const int tid = threadIdx.x;
  const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)tid * SCAN_I;
  int v[SCAN_I];
  int sum = 0;
#pragma unroll
  for (int i = 0; i < SCAN_I; ++i) {
    long long idx = base + i;
    int x = (idx < n_in) ? in[idx] : 0;
    v[i] = sum;
    sum += x;
  }
  sh[tid] = sum;
  __syncthreads();
  for (int off = 1; off < SCAN_T; off <<= 1) {
    int t = (tid >= off) ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += t;
    __syncthreads();
  }
  const int excl = sh[tid] - sum;
#pragma unroll
  for (int i = 0; i < SCAN_I; ++i) {
    long long idx = base + i;
    if (idx < n_out) out[idx] = v[i] + excl;
  }
  if (tid == SCAN_T - 1) totals[blockIdx.x] = sh[SCAN_T - 1];
}

__global__ __launch_bounds__(SCAN_T) void k_scan_add(int *out, int n, const int *__restrict__ offs) {
  const int add = offs[blockIdx.x];
  const long long base = (long long)blockIdx.x * SCAN_TILE;
  for (int i = threadIdx.x; i < SCAN_TILE; i += SCAN_T) {
    long long idx = base + i;
    if (idx < n) out[idx] += add;
  }
}

static size_t scan_tmp_size(long long n) {
  size_t s = 0;
  long long m = n;
  do {
    m = (m + SCAN_TILE - 1) / SCAN_TILE;
    s += (size_t)m + 1;
  } while (m > 1);
  return s + 16;
}

static void scan_rec(const int *in, int *out, int n_in, int n_out, int *tmp, hipStream_t s) {
  const int nb = ceil_div(n_out, SCAN_TILE);
  int *totals = tmp;
  hipLaunchKernelGGL(k_scan_tile, dim3(nb), dim3(SCAN_T), 0, s, in, out, n_in, n_out, totals);
  EDFA_CHECK_LAUNCH();
  if (nb > 1) {
    scan_rec(totals, totals, nb, nb, tmp + nb + 1, s);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(SCAN_T), 0, s, out, n_out, totals);
    EDFA_CHECK_LAUNCH();
  }
}

void exclusive_scan_async(const int *in, int *out, int n, DBuf<int> &tmp, hipStream_t s) {
  if (n < 0) fail(EDFA_ERR_ARG, "scan of negative length");
  tmp.ensure(scan_tmp_size((long long)n + 1));
  scan_rec(in, out, n, n + 1, tmp.p, s);
}

int64_t exclusive_scan(const int *in, int *out, int n, DBuf<int> &tmp, hipStream_t s) {
  exclusive_scan_async(in, out, n, tmp, s);
  return read_scalar(out + n, s);
}

// ----------------------------------------------------------------------------------
// Stable partition by a small key: per-block key histograms (key-major), one scan, and a
// scatter that keeps the index order inside a key.
// ----------------------------------------------------------------------------------
constexpr int PART_MAX_KEYS = 64;
__global__ __launch_bounds__(256) void k_part_hist(const int *__restrict__ key, int n, int nkey,
                                                   int nb, int *hist) {
  __shared__ int h[PART_MAX_KEYS];
  for (int c = threadIdx.x; c < nkey; c += 256) h[c] = 0;
  __syncthreads();
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v < n) atomicAdd(&h[key[v]], 1);
  __syncthreads();
  for (int c = threadIdx.x; c < nkey; c += 256) hist[(size_t)c * nb + blockIdx.x] = h[c];
}

__global__ __launch_bounds__(256) void k_part_scatter(const int *__restrict__ key, int n, int nb,
                                                      const int *__restrict__ offs, int *out) {
  __shared__ int kl[256];
  const int v = blockIdx.x * 256 + threadIdx.x;
  kl[threadIdx.x] = v < n ? key[v] : -1;
  __syncthreads();
  if (v >= n) return;
  const int c = kl[threadIdx.x];
  int rank = 0;
  for (int t = 0; t < (int)threadIdx.x; ++t) rank += kl[t] == c;
  out[offs[(size_t)c * nb + blockIdx.x] + rank] = v;
}

__global__ void k_part_starts(const int *__restrict__ hist, int nb, int count, int *starts) {
  for (int c = threadIdx.x; c < count; c += blockDim.x) starts[c] = hist[(size_t)c * nb];
}

void stable_partition(const int *key, int n, int nkey, int *out, DBuf<int> &hist, DBuf<int> &tmp,
                      hipStream_t s, std::vector<int> &counts) {
  if (nkey < 1 || nkey > PART_MAX_KEYS) fail(EDFA_ERR_ARG, "partition into %d keys", nkey);
  counts.assign(nkey, 0);
  if (n <= 0) return;
  const int nb = ceil_div(n, 256);
  hist.ensure((size_t)nkey * nb + 1 + (size_t)(nkey + 1));   // scan, then the gathered starts
  hipLaunchKernelGGL(k_part_hist, dim3(nb), dim3(256), 0, s, key, n, nkey, nb, hist.p);
  EDFA_CHECK_LAUNCH();
  exclusive_scan_async(hist.p, hist.p, nkey * nb, tmp, s);
  hipLaunchKernelGGL(k_part_scatter, dim3(nb), dim3(256), 0, s, key, n, nb, hist.p, out);
  EDFA_CHECK_LAUNCH();
  std::vector<int> start(nkey + 1);
  // the start of key c sits at hist[c * nb]: gathered on the device behind the histogram,
  // then one contiguous copy
  int *starts = hist.p + (size_t)nkey * nb + 1;
  hipLaunchKernelGGL(k_part_starts, dim3(1), dim3(64), 0, s, hist.p, nb, nkey + 1, starts);
  EDFA_CHECK_LAUNCH();
  read_small(start.data(), starts, (size_t)(nkey + 1), s);   // nkey <= PART_MAX_KEYS
  for (int c = 0; c < nkey; ++c) counts[c] = start[c + 1] - start[c];
}

// ----------------------------------------------------------------------------------
// CSR transpose: count per column, scan, scatter with atomic cursors, sort each row.
// ----------------------------------------------------------------------------------
__global__ void k_count_cols(const int *__restrict__ col, int64_t nnz, int *cnt) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nnz) atomicAdd(&cnt[col[k]], 1);
}

// L lanes per source row, across its entries (the order inside a target row is fixed by the
// sort that follows)
template <class V, int L>
__global__ __launch_bounds__(256) void k_transpose_fill(const int *__restrict__ rowptr,
                                                        const int *__restrict__ col,
                                                        const V *__restrict__ val, int rows,
                                                        int *cursor, int *colT, V *valT) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  const int r = t / L;
  if (r >= rows) return;
  const int e = rowptr[r + 1];
  for (int k = rowptr[r] + t % L; k < e; k += L) {
    const int pos = atomicAdd(&cursor[col[k]], 1);
    colT[pos] = r;
    valT[pos] = val[k];
  }
}

constexpr int SORT_WAVE_CAP = 1024;

// Sort the entries of each row by column: rows longer than SORT_WAVE_CAP here (insertion
// sort, one thread per row); shorter rows are sorted by k_sort_rows_wave.
template <class V>
__global__ void k_sort_rows(const int *__restrict__ rowptr, int rows, int *col, V *val,
                            int min_len) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  const int a = rowptr[r], b = rowptr[r + 1];
  if (b - a < min_len) return;
  for (int i = a + 1; i < b; ++i) {
    int c = col[i];
    V v = val[i];
    int j = i - 1;
    while (j >= a && col[j] > c) {
      col[j + 1] = col[j];
      val[j + 1] = val[j];
      --j;
    }
    col[j + 1] = c;
    val[j + 1] = v;
  }
}

// One wavefront per row (rows up to SORT_WAVE_CAP entries): rank of each entry = number of
// smaller columns in the row (columns are unique within a row).
template <class V>
__global__ __launch_bounds__(64) void k_sort_rows_wave(const int *__restrict__ rowptr, int rows,
                                                       int *col, V *val) {
  __shared__ int c[SORT_WAVE_CAP];
  __shared__ V v[SORT_WAVE_CAP];
  const int r = blockIdx.x;
  if (r >= rows) return;
  const int a = rowptr[r], n = rowptr[r + 1] - a;
  if (n < 2 || n > SORT_WAVE_CAP) return;
  for (int t = threadIdx.x; t < n; t += 64) {
    c[t] = col[a + t];
    v[t] = val[a + t];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n; t += 64) {
    const int ct = c[t];
    int rank = 0;
    for (int u = 0; u < n; ++u) rank += c[u] < ct;
    col[a + rank] = ct;
    val[a + rank] = v[t];
  }
}

template <class V>
void csr_transpose(const Csr<V> &src, Csr<V> &dst, DBuf<int> &tmp, DBuf<int> &cursor,
                   hipStream_t s, bool sort) {
  dst.alloc(src.cols, src.rows, src.nnz);
  EDFA_HIP(hipMemsetAsync(dst.rowptr.p, 0, sizeof(int) * ((size_t)src.cols + 1), s));
  if (src.nnz > 0) {
    hipLaunchKernelGGL(k_count_cols, dim3(ceil_div(src.nnz, 256)), dim3(256), 0, s, src.col.p,
                       src.nnz, dst.rowptr.p);
    EDFA_CHECK_LAUNCH();
  }
  exclusive_scan_async(dst.rowptr.p, dst.rowptr.p, src.cols, tmp, s);

  cursor.ensure((size_t)src.cols + 1);
  EDFA_HIP(hipMemcpyAsync(cursor.p, dst.rowptr.p, sizeof(int) * ((size_t)src.cols + 1),
                          hipMemcpyDeviceToDevice, s));
  if (src.rows > 0) {
    if ((double)src.nnz > 16.0 * src.rows)
      hipLaunchKernelGGL((k_transpose_fill<V, 16>), dim3(ceil_div((long long)src.rows * 16, 256)),
                         dim3(256), 0, s, src.rowptr.p, src.col.p, src.val.p, src.rows, cursor.p,
                         dst.col.p, dst.val.p);
    else
      hipLaunchKernelGGL((k_transpose_fill<V, 4>), dim3(ceil_div((long long)src.rows * 4, 256)),
                         dim3(256), 0, s, src.rowptr.p, src.col.p, src.val.p, src.rows, cursor.p,
                         dst.col.p, dst.val.p);
    EDFA_CHECK_LAUNCH();
  }
  if (src.cols > 0 && sort) {
    const double avg = src.cols ? (double)src.nnz / src.cols : 0.0;
    if (avg > 8.0) {
      hipLaunchKernelGGL(k_sort_rows_wave<V>, dim3(src.cols), dim3(64), 0, s, dst.rowptr.p,
                         src.cols, dst.col.p, dst.val.p);
      hipLaunchKernelGGL(k_sort_rows<V>, dim3(ceil_div(src.cols, 256)), dim3(256), 0, s,
                         dst.rowptr.p, src.cols, dst.col.p, dst.val.p, SORT_WAVE_CAP + 1);
    } else {
      hipLaunchKernelGGL(k_sort_rows<V>, dim3(ceil_div(src.cols, 256)), dim3(256), 0, s,
                         dst.rowptr.p, src.cols, dst.col.p, dst.val.p, 0);
    }
    EDFA_CHECK_LAUNCH();
  }

}

template void csr_transpose<double>(const Csr<double> &, Csr<double> &, DBuf<int> &, DBuf<int> &,
                                    hipStream_t, bool);
template void csr_transpose<float>(const Csr<float> &, Csr<float> &, DBuf<int> &, DBuf<int> &,
                                   hipStream_t, bool);

// ----------------------------------------------------------------------------------
// SpMV: a group of LANES lanes per row, shuffle reduction inside the group.
// ----------------------------------------------------------------------------------
template <class V, class X> struct AccT { using type = double; };
template <> struct AccT<float, float> { using type = float; };

template <class V, class X, int LANES>
__global__ __launch_bounds__(256) void k_spmv(const int *__restrict__ rowptr,
                                              const int *__restrict__ col,
                                              const V *__restrict__ val, int rows,
                                              const X *__restrict__ x, X *__restrict__ y,
                                              double alpha, const X *__restrict__ b,
                                              double beta, double gamma) {
  using A = typename AccT<V, X>::type;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int row = (int)(gid / LANES);
  const int lane = (int)(gid % LANES);
  if (row >= rows) return;
  A sum = 0;
  const int end = rowptr[row + 1];
  for (int k = rowptr[row] + lane; k < end; k += LANES) sum += (A)val[k] * (A)x[col[k]];
#pragma unroll
  for (int off = LANES / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, LANES);
  if (lane == 0) {
    A r = (A)alpha * sum;
    if (b) r += (A)beta * (A)b[row];
    if (gamma != 0.0) r += (A)gamma * (A)x[row];
    y[row] = (X)r;
  }
}

template <class V, class X>
void spmv(const int *rowptr, const int *col, const V *val, int rows, const X *x, X *y,
          double alpha, const X *b, double beta, float avg_nnz, hipStream_t s, double gamma) {
  if (rows <= 0) return;
  auto launch = [&](auto kern, int lanes) {
    long long threads = (long long)rows * lanes;
    hipLaunchKernelGGL(kern, dim3(ceil_div(threads, 256)), dim3(256), 0, s, rowptr, col, val,
                       rows, x, y, alpha, b, beta, gamma);
    EDFA_CHECK_LAUNCH();
  };
  if (avg_nnz <= 3.f)
    launch(k_spmv<V, X, 2>, 2);
  else if (avg_nnz <= 6.f)
    launch(k_spmv<V, X, 4>, 4);
  else if (avg_nnz <= 14.f)
    launch(k_spmv<V, X, 8>, 8);
  else if (avg_nnz <= 40.f)
    launch(k_spmv<V, X, 16>, 16);
  else
    launch(k_spmv<V, X, 32>, 32);
}

template void spmv<double, double>(const int *, const int *, const double *, int, const double *,
                                   double *, double, const double *, double, float, hipStream_t,
                                   double);
template void spmv<float, float>(const int *, const int *, const float *, int, const float *,
                                 float *, double, const float *, double, float, hipStream_t, double);

}  // namespace edfa

namespace edfa {

// ----------------------------------------------------------------------------------
// SELL-64
// ----------------------------------------------------------------------------------
__global__ void k_sell_width(const int *__restrict__ rowptr, int rows, int nslice, int *w64) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= nslice) return;
  int w = 0;
  for (int r = sl * 64; r < min(rows, sl * 64 + 64); ++r) w = max(w, rowptr[r + 1] - rowptr[r]);
  w64[sl] = w * 64;
}

// Sorted layout (SELL-C-sigma with C = 64, sigma = SELL_SIGMA): inside each window of
// SELL_SIGMA rows, positions hold the rows by descending length (ties by row index), so a
// slice of 64 positions holds rows of similar length.  One block of 256 threads per window:
// bitonic sort of (length, row) keys in LDS.  perm[position] = row.
constexpr int SELL_SIGMA = 1024;
__global__ __launch_bounds__(256) void k_sell_sort(const int *__restrict__ rowptr, int rows,
                                                   int *perm) {
  __shared__ unsigned long long key[SELL_SIGMA];
  const int w0 = blockIdx.x * SELL_SIGMA;
  for (int t = threadIdx.x; t < SELL_SIGMA; t += 256) {
    const int r = w0 + t;
    // ascending keys = descending lengths; rows past the end sort last
    key[t] = r < rows ? ((unsigned long long)(0x7fffffff - (rowptr[r + 1] - rowptr[r])) << 32) |
                            (unsigned)r
                      : ~0ull;
  }
  __syncthreads();
  for (int k = 2; k <= SELL_SIGMA; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < SELL_SIGMA; t += 256) {
        const int o = t ^ j;
        if (o > t) {
          const unsigned long long a = key[t], b = key[o];
          if (((t & k) == 0) == (a > b)) {
            key[t] = b;
            key[o] = a;
          }
        }
      }
      __syncthreads();
    }
  for (int t = threadIdx.x; t < SELL_SIGMA; t += 256)
    if (w0 + t < rows) perm[w0 + t] = (int)(key[t] & 0xffffffffu);
}

// slice widths of the sorted layout: the longest row of each slice of 64 positions
__global__ void k_sell_width_perm(const int *__restrict__ rowptr, const int *__restrict__ perm,
                                  int rows, int nslice, int *w64) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= nslice) return;
  int w = 0;
  for (int p = sl * 64; p < min(rows, sl * 64 + 64); ++p) {
    const int r = perm[p];
    w = max(w, rowptr[r + 1] - rowptr[r]);
  }
  w64[sl] = w * 64;
}

// position p holds row perm[p] (perm NULL: row p)
template <class V>
__global__ void k_sell_fill(const int *__restrict__ rowptr, const int *__restrict__ col,
                            const V *__restrict__ val, int rows, const int *__restrict__ perm,
                            const int *__restrict__ sptr, int *rlen, int *scol, V *sval) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= rows) return;
  const int r = perm ? perm[p] : p;
  const int a = rowptr[r], n = rowptr[r + 1] - a;
  const int base = sptr[p >> 6] + (p & 63);
  rlen[p] = n;
  // eight entries of the row in flight at once (clamped reads, guarded stores)
  for (int k0 = 0; k0 < n; k0 += 8) {
    int c[8];
    V v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = min(k0 + u, n - 1);
      c[u] = col[a + k];
      v[u] = val[a + k];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u < n) {
        scol[base + 64 * (k0 + u)] = c[u];
        sval[base + 64 * (k0 + u)] = v[u];
      }
  }
}

// Lanes per row for a matrix with the given mean row length: one lane per row (SELL) for
// short rows, a CSR group of lanes for long ones.
constexpr double SPMV_VEC_MIN_ROW = 24.0;
// SELL-64 padding (stored / true entries) above which the rows are sorted by length
constexpr double SELL_SORT_PAD = 1.2;
int default_spmv_lanes(double mean_row) {
  return mean_row < SPMV_VEC_MIN_ROW ? 0 : SPMV_CHUNKED;
}

// The SELL layout of S from its CSR arrays (rows sorted by length inside windows when plain
// slices would pad by more than SELL_SORT_PAD).  Synchronises to size the storage.
template <class V>
static void sell_layout(const Sell<V> &S, DBuf<int> &tmp, hipStream_t s) {
  S.nslice = ceil_div(S.rows, 64);
  S.sptr.ensure((size_t)S.nslice + 1);
  S.rlen.ensure((size_t)std::max(S.rows, 1));
  S.sorted = false;
  S.padded = 0;
  S.sell_ready = true;
  if (S.nslice == 0) return;
  hipLaunchKernelGGL(k_sell_width, dim3(ceil_div(S.nslice, 256)), dim3(256), 0, s, S.csr_rp,
                     S.rows, S.nslice, S.sptr.p);
  EDFA_CHECK_LAUNCH();
  S.padded = exclusive_scan(S.sptr.p, S.sptr.p, S.nslice, tmp, s);
  if (S.padded > SELL_SORT_PAD * (double)S.nnz) {
    // rows of very different lengths side by side: sort them inside windows
    S.perm.ensure((size_t)S.rows);
    hipLaunchKernelGGL(k_sell_sort, dim3(ceil_div(S.rows, SELL_SIGMA)), dim3(256), 0, s,
                       S.csr_rp, S.rows, S.perm.p);
    hipLaunchKernelGGL(k_sell_width_perm, dim3(ceil_div(S.nslice, 256)), dim3(256), 0, s,
                       S.csr_rp, S.perm.p, S.rows, S.nslice, S.sptr.p);
    EDFA_CHECK_LAUNCH();
    S.padded = exclusive_scan(S.sptr.p, S.sptr.p, S.nslice, tmp, s);
    S.sorted = true;
  }
  S.col.ensure((size_t)std::max<int64_t>(S.padded, 1));
  S.val.ensure((size_t)std::max<int64_t>(S.padded, 1));
  hipLaunchKernelGGL(k_sell_fill<V>, dim3(ceil_div(S.rows, 256)), dim3(256), 0, s, S.csr_rp,
                     S.csr_col, S.csr_val, S.rows, S.sorted ? S.perm.p : nullptr, S.sptr.p,
                     S.rlen.p, S.col.p, S.val.p);
  EDFA_CHECK_LAUNCH();
}

template <class V>
void ensure_sell(const Sell<V> &S, hipStream_t s) {
  if (!S.sell_ready) sell_layout(S, S.scan_tmp, s);
}
template void ensure_sell<double>(const Sell<double> &, hipStream_t);
template void ensure_sell<float>(const Sell<float> &, hipStream_t);

template <class V>
void build_sell(const Csr<V> &M, Sell<V> &S, DBuf<int> &tmp, hipStream_t s) {
  S.rows = M.rows;
  S.cols = M.cols;
  S.nnz = M.nnz;
  S.csr_rp = M.rowptr.p;
  S.csr_col = M.col.p;
  S.csr_val = M.val.p;
  S.lanes = M.rows > 0 ? default_spmv_lanes((double)M.nnz / M.rows) : 0;
  S.depth = 0;
  S.chunk_k = 0;   // the CSR arrays may have changed: descriptors are rebuilt on demand
  S.sell_ready = false;
  if (S.lanes == SPMV_CHUNKED)
    build_row_chunks(S, CHUNK_K, s);   // the SELL layout waits for a SELL variant
  else
    sell_layout(S, tmp, s);
}

template void build_sell<double>(const Csr<double> &, Sell<double> &, DBuf<int> &, hipStream_t);
template void build_sell<float>(const Csr<float> &, Sell<float> &, DBuf<int> &, hipStream_t);

// One lane per row.  Each round issues the loads of the next U entries of the row at once
// (predicated past the row's end), so a row of up to U entries costs one dependent chain
// (column index -> x) instead of one per entry.  ROLE only separates the system-operator
// launches (0) from the preconditioner's (1) in kernel traces.
constexpr int SPMV_T = 256;

// y[row] = alpha sum + beta b[row] + gamma x[row]; y and b are FP64 or FP32 each, whatever
// x is (io bit 0: y is FP64, bit 1: b is FP64), so the FP32 application reads and writes
// the FP64 vectors of the iteration directly.
template <class A, class X>
__device__ __forceinline__ void store_row(void *y, const void *b, int io, int row, A sum,
                                          double alpha, double beta, double gamma,
                                          const X *__restrict__ x) {
  A out = (A)alpha * sum;
  if (b) out += (A)beta * (io & 2 ? (A)((const double *)b)[row] : (A)((const float *)b)[row]);
  if (gamma != 0.0) out += (A)gamma * (A)x[row];
  if (io & 1)
    ((double *)y)[row] = (double)out;
  else
    ((float *)y)[row] = (float)out;
}

template <class V, class X, int ROLE, int U>
__global__ __launch_bounds__(SPMV_T) void k_spmv_sell(const int *__restrict__ sptr,
                                                      const int *__restrict__ rlen,
                                                      const int *__restrict__ col,
                                                      const V *__restrict__ val,
                                                      const int *__restrict__ perm, int rows,
                                                      const X *__restrict__ x, void *y,
                                                      double alpha, const void *b, double beta,
                                                      double gamma, int io, RowMask mk) {
  using A = typename AccT<V, X>::type;
  // Prologue without a branch before its loads: positions past the end are clamped to the
  // last row (they load it and store nothing); the stop flag of a single system, the slice
  // offset, the row length and the terms of the addend are all in flight before the first
  // wait, and a row that stores nothing runs no entry round.
  const int r0 = blockIdx.x * SPMV_T + threadIdx.x;   // position in the layout
  const int r = min(r0, rows - 1);
  const int flag = *(mk.act ? mk.act : sptr);           // any valid address without a mask
  // a wavefront holds exactly one slice of 64 rows: its offset is a scalar load
  const int sb = sptr[__builtin_amdgcn_readfirstlane(r >> 6)];
  const int n0 = rlen[r];
  const int row = perm ? perm[r] : r;
  double bd = 0;   // the addend as stored (converted where it is used)
  float bf = 0;
  X xr = 0;
  if (b) {
    if (io & 2)
      bd = ((const double *)b)[row];
    else
      bf = ((const float *)b)[row];
  }
  if (gamma != 0.0) xr = x[row];
  const bool live = r0 < rows && !(mk.act && !mk.seg && flag == 0) && !row_off(mk, row);
  const int n = live ? n0 : 0;
  const int base = sb + (r & 63);
  A s[U];
#pragma unroll
  for (int u = 0; u < U; ++u) s[u] = 0;
  for (int k = 0; k < n; k += U) {
    // entries past the row's end re-read its last entry (always valid, no branch) and
    // contribute zero, so every load of the round is issued before the first wait
    int c[U];
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = base + 64 * min(k + u, n - 1);
      c[u] = col[p];
      v[u] = val[p];
    }
    X xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] += (k + u < n ? (A)v[u] : A(0)) * (A)xv[u];
  }
#pragma unroll
  for (int h = U / 2; h > 0; h >>= 1)
#pragma unroll
    for (int u = 0; u < h; ++u) s[u] += s[u + h];
  if (!live) return;
  // store_row's arithmetic with the addend terms loaded above
  A out = (A)alpha * s[0];
  if (b) out += (A)beta * (io & 2 ? (A)bd : (A)bf);
  if (gamma != 0.0) out += (A)gamma * (A)xr;
  if (io & 1)
    ((double *)y)[row] = (double)out;
  else
    ((float *)y)[row] = (float)out;
}

// L lanes per row on the CSR arrays, for matrices with long rows: the lanes of a row read
// consecutive entries (coalesced), each round issuing U entries per lane at once
// (predicated past the row's end), and a shuffle tree sums the lanes' partials.
template <class V, class X, int L, int U>
__global__ __launch_bounds__(SPMV_T) void k_spmv_csr_vec(const int *__restrict__ rp,
                                                         const int *__restrict__ col,
                                                         const V *__restrict__ val, int rows,
                                                         const X *__restrict__ x, void *y,
                                                         double alpha, const void *b, double beta,
                                                         double gamma, int io, RowMask mk) {
  using A = typename AccT<V, X>::type;
  if (all_off(mk)) return;
  const int t = blockIdx.x * SPMV_T + threadIdx.x;
  const int r = t / L, l = t % L;
  if (r >= rows) return;   // all L lanes of a row leave together
  if (row_off(mk, r)) return;
  const int a = rp[r], e = rp[r + 1];
  A s[U];
#pragma unroll
  for (int u = 0; u < U; ++u) s[u] = 0;
  for (int p0 = a + l; p0 < e; p0 += L * U) {
    // entries past the row's end re-read entry p0 (valid, no branch) and contribute zero
    int c[U];
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u * L < e ? p0 + u * L : p0;
      c[u] = col[p];
      v[u] = val[p];
    }
    X xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] += (p0 + u * L < e ? (A)v[u] : A(0)) * (A)xv[u];
  }
#pragma unroll
  for (int h = U / 2; h > 0; h >>= 1)
#pragma unroll
    for (int u = 0; u < h; ++u) s[u] += s[u + h];
  A sum = s[0];
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
  if (l == 0) store_row<A, X>(y, b, io, r, sum, alpha, beta, gamma, x);
}

// ----------------------------------------------------------------------------------
// Chunk kernel for matrices whose rows are long and of uneven length (the approximate
// inverses of the ILU(0) factors: 1 to ~160 entries, in the natural order).  The CSR arrays
// are cut into chunks of whole consecutive rows holding at most 64 K entries.
// One wavefront per chunk: its lanes load the chunk's entries with unit stride, K loads of
// column index and value in flight per lane, gather x, and leave the products in LDS;
// then G lanes per row sum each row's products (strided, then a shuffle tree).  Every load
// is useful (no lane idles on a short row) and the x gathers keep the natural order's
// locality.  A row longer than 64 K entries forms a chunk of its own, summed by the whole
// wavefront.
// ----------------------------------------------------------------------------------
// Greedy row-aligned chunks of at most `cap` entries (a longer row is a chunk of its own),
// built on the device.  The greedy pass closes the chunk that starts at row r0 before the
// first row r > r0 with rp[r + 1] - rp[r0] > cap, so its successor is
// nxt(r0) = min(max(ub - 1, r0 + 1), rows), ub the first index with rp[ub] > rp[r0] + cap
// (a binary search on the sorted row pointer); the chunk starts are the orbit of row 0 under
// nxt, marked by pointer doubling (after k rounds every nxt^i(0) with i < 2^k is marked),
// then compacted in row order.  Same chunks as the sequential pass.
__global__ void k_chunk_next(const int *__restrict__ rp, int rows, int cap, int *nxt,
                             int *mark) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r > rows) return;
  mark[r] = r == 0 ? 1 : 0;
  if (r == rows) {
    nxt[r] = rows;
    return;
  }
  const long long thr = (long long)rp[r] + cap;
  int lo = r + 1, hi = rows + 1;   // rp[r] <= thr: the first index past thr is above r
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((long long)rp[mid] > thr)
      hi = mid;
    else
      lo = mid + 1;
  }
  nxt[r] = min(max(lo - 1, r + 1), rows);
}

// One doubling round: every marked row marks its jump target (marks only grow, and every
// mark lies on the orbit), and jump_out = jump_in o jump_in.  The end row `rows`, where
// every orbit ends, is never marked (only rows below it start chunks): in the late rounds
// most jumps land there, and their stores would all queue on one address.
__global__ void k_chunk_double(const int *__restrict__ jin, int *jout, int *mark, int rows) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r > rows) return;
  const int j = jin[r];
  if (j < rows && __hip_atomic_load(mark + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &&
      !__hip_atomic_load(mark + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    __hip_atomic_store(mark + j, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  jout[r] = jin[j];
}

__global__ void k_chunk_write(const int *__restrict__ rp, const int *__restrict__ mark,
                              const int *__restrict__ pos, int rows, int nchunk, int2 *d) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < rows && mark[r]) d[pos[r]] = make_int2(r, rp[r]);
  if (r == rows) d[nchunk] = make_int2(rows, rp[rows]);
}

static void device_chunks(const int *rp_dev, int rows, int cap, DBuf<int2> &out, int &count,
                          DBuf<int> &work, DBuf<int> &scan_tmp, hipStream_t s) {
  // work: nxt and a second jump array (rows + 1 each), the marks (rows + 1), positions (rows)
  const size_t n1 = (size_t)rows + 1;
  work.ensure(4 * n1);
  int *ja = work.p, *jb = work.p + n1, *mark = work.p + 2 * n1, *pos = work.p + 3 * n1;
  const int gb = ceil_div((long long)n1, 256);
  hipLaunchKernelGGL(k_chunk_next, dim3(gb), dim3(256), 0, s, rp_dev, rows, cap, ja, mark);
  EDFA_CHECK_LAUNCH();
  int rounds = 1;
  while ((1ll << rounds) < (long long)n1) ++rounds;
  for (int k = 0; k < rounds; ++k) {
    hipLaunchKernelGGL(k_chunk_double, dim3(gb), dim3(256), 0, s, ja, jb, mark, rows);
    std::swap(ja, jb);
  }
  EDFA_CHECK_LAUNCH();
  count = (int)exclusive_scan(mark, pos, rows, scan_tmp, s);
  out.ensure((size_t)count + 1);
  hipLaunchKernelGGL(k_chunk_write, dim3(gb), dim3(256), 0, s, rp_dev, mark, pos, rows, count,
                     out.p);
  EDFA_CHECK_LAUNCH();
}

template <class V>
void build_row_chunks(Sell<V> &S, int k, hipStream_t s) {
  if (S.chunk_k == k || S.rows <= 0) return;
  device_chunks(S.csr_rp, S.rows, 64 * k, S.chunk, S.nchunk, S.chunk_work, S.scan_tmp, s);
  S.nchunk_alt = -1;
  S.chunk_k = k;
}
template void build_row_chunks<double>(Sell<double> &, int, hipStream_t);
template void build_row_chunks<float>(Sell<float> &, int, hipStream_t);

constexpr int CHUNK_G = 8;   // lanes per row in the sums

template <class V, class X, int K>
__global__ __launch_bounds__(SPMV_T) void k_spmv_chunk(const int *__restrict__ rp,
                                                       const int *__restrict__ col,
                                                       const V *__restrict__ val,
                                                       const int2 *__restrict__ desc,
                                                       int nchunk, const X *__restrict__ x,
                                                       void *y, double alpha, const void *b,
                                                       double beta, double gamma, int io,
                                                       RowMask mk) {
  using A = typename AccT<V, X>::type;
  constexpr int CAP = 64 * K;
  __shared__ A buf[SPMV_T / 64][CAP];
  if (all_off(mk)) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int c = blockIdx.x * (SPMV_T / 64) + wv;
  if (c >= nchunk) return;
  const int2 d0 = desc[c], d1 = desc[c + 1];
  const int r0 = d0.x, r1 = d1.x, e0 = d0.y, e1 = d1.y;
  if (mk.seg) {
    // the whole chunk in one stopped grid
    const int s0 = mk.seg[r0], s1 = mk.seg[r1 - 1];
    if (s0 == s1 && !mk.act[s0 * mk.stride]) return;
  }
  auto finish = [&](int row, A sum) {
    if (row_off(mk, row)) return;
    store_row<A, X>(y, b, io, row, sum, alpha, beta, gamma, x);
  };
  if (e1 - e0 > CAP) {
    // one long row: the wavefront strides over it, K entries in flight per lane
    A s = 0;
    for (int p0 = e0 + lane; p0 < e1; p0 += 64 * K) {
      int cc[K];
      V v[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int p = min(p0 + 64 * k, e1 - 1);
        cc[k] = col[p];
        v[k] = val[p];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) s += (p0 + 64 * k < e1 ? (A)v[k] : A(0)) * (A)x[cc[k]];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) finish(r0, s);
    return;
  }
  // row starts of the chunk's first 64 rows (one load per lane, beside the entry loads)
  const int rpl = rp[min(r0 + lane, r1)];
  int cc[K];
  V v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    // past the chunk's end: re-read its last entry (valid, weight zero)
    const int p = max(min(e0 + 64 * k + lane, e1 - 1), 0);
    cc[k] = col[p];
    v[k] = val[p];
  }
  A *mine = buf[wv];
#pragma unroll
  for (int k = 0; k < K; ++k)
    mine[64 * k + lane] = (e0 + 64 * k + lane < e1 ? (A)v[k] : A(0)) * (A)x[cc[k]];
  // the products of other lanes of this wavefront are read below
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const int nr = r1 - r0;
  const int g = lane / CHUNK_G, gl = lane % CHUNK_G;
  for (int q = 0; q < nr; q += 64 / CHUNK_G) {   // uniform trip count
    const int ri = q + g;
    int a = __shfl(rpl, min(ri, 63)), e = __shfl(rpl, min(ri + 1, 63));
    if (ri >= 64) a = rp[min(r0 + ri, r1)];
    if (ri + 1 >= 64) e = rp[min(r0 + ri + 1, r1)];
    A s = 0;
    if (ri < nr)
      for (int p = a - e0 + gl; p < e - e0; p += CHUNK_G) s += mine[p];
#pragma unroll
    for (int o = CHUNK_G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, CHUNK_G);
    if (gl == 0 && ri < nr) finish(r0 + ri, s);
  }
}

// Launch helper: the extended launch records e0/e1 around the kernel when given; plain
// launches otherwise (the form stream capture records).
template <class K, class... Args>
static void launch_timed(K kern, int blocks, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                         Args... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kern, dim3(blocks), dim3(SPMV_T), 0, s, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(SPMV_T), 0, s, args...);
}

template <class V, class X>
void spmv_sell_io(const Sell<V> &M, const X *x, void *y, bool y64, double alpha, const void *b,
                  bool b64, double beta, hipStream_t s, double gamma, int role, hipEvent_t e0,
                  hipEvent_t e1, RowMask mk) {
  if (M.rows <= 0) return;
  const int io = (y64 ? 1 : 0) | (b64 ? 2 : 0);
  if (M.lanes == SPMV_CHUNKED) {
    if (M.chunk_k != CHUNK_K)
      fail(EDFA_ERR_ARG, "the chunk kernel needs the chunk descriptors of its matrix");
    if (M.depth == CHUNK_K_ALT) {
      if (M.nchunk_alt < 0)
        device_chunks(M.csr_rp, M.rows, 64 * CHUNK_K_ALT, M.chunk_alt, M.nchunk_alt,
                      M.chunk_work, M.scan_tmp, s);
      const int nb = ceil_div(M.nchunk_alt, SPMV_T / 64);
      launch_timed(k_spmv_chunk<V, X, CHUNK_K_ALT>, nb, s, e0, e1, M.csr_rp, M.csr_col,
                   M.csr_val, (const int2 *)M.chunk_alt.p, M.nchunk_alt, x, y, alpha, b, beta,
                   gamma, io, mk);
    } else {
      const int nb = ceil_div(M.nchunk, SPMV_T / 64);
      launch_timed(k_spmv_chunk<V, X, CHUNK_K>, nb, s, e0, e1, M.csr_rp, M.csr_col, M.csr_val,
                   (const int2 *)M.chunk.p, M.nchunk, x, y, alpha, b, beta, gamma, io, mk);
    }
  } else if (M.lanes > 1) {
    const int nb = ceil_div((long long)M.rows * M.lanes, SPMV_T);
    const bool deep = M.depth == 4;
#define EDFA_VEC(LN, UU)                                                                      \
  launch_timed(k_spmv_csr_vec<V, X, LN, UU>, nb, s, e0, e1, M.csr_rp, M.csr_col, M.csr_val,    \
               M.rows, x, y, alpha, b, beta, gamma, io, mk)
#define EDFA_VEC2(LN) \
  if (deep) EDFA_VEC(LN, 4); else EDFA_VEC(LN, 2)
    switch (M.lanes) {
      case 2: EDFA_VEC2(2); break;
      case 4: EDFA_VEC2(4); break;
      case 8: EDFA_VEC2(8); break;
      case 16: EDFA_VEC2(16); break;
      default: EDFA_VEC2(32); break;
    }
#undef EDFA_VEC2
#undef EDFA_VEC
  } else {
    ensure_sell(M, s);
    const int nb = ceil_div(M.rows, SPMV_T);
    const bool deep = M.depth == 8;
#define EDFA_SELL(RL, UU)                                                                     \
  launch_timed(k_spmv_sell<V, X, RL, UU>, nb, s, e0, e1, M.sptr.p, M.rlen.p, M.col.p, M.val.p, \
               M.sorted ? M.perm.p : nullptr, M.rows, x, y, alpha, b, beta, gamma, io, mk)
    if (role == SPMV_OPERATOR) {
      if (deep) EDFA_SELL(SPMV_OPERATOR, 8); else EDFA_SELL(SPMV_OPERATOR, 4);
    } else {
      if (deep) EDFA_SELL(SPMV_PRECOND, 8); else EDFA_SELL(SPMV_PRECOND, 4);
    }
#undef EDFA_SELL
  }
  EDFA_CHECK_LAUNCH();
}

template <class V, class X>
void spmv_sell(const Sell<V> &M, const X *x, X *y, double alpha, const X *b, double beta,
               hipStream_t s, double gamma, int role, hipEvent_t e0, hipEvent_t e1,
               RowMask mk) {
  constexpr bool w = sizeof(X) == 8;
  spmv_sell_io<V, X>(M, x, y, w, alpha, b, w, beta, s, gamma, role, e0, e1, mk);
}

template void spmv_sell<double, double>(const Sell<double> &, const double *, double *, double,
                                        const double *, double, hipStream_t, double, int,
                                        hipEvent_t, hipEvent_t, RowMask);
template void spmv_sell<float, float>(const Sell<float> &, const float *, float *, double,
                                      const float *, double, hipStream_t, double, int, hipEvent_t,
                                      hipEvent_t, RowMask);
template void spmv_sell_io<float, float>(const Sell<float> &, const float *, void *, bool, double,
                                         const void *, bool, double, hipStream_t, double, int,
                                         hipEvent_t, hipEvent_t, RowMask);
template void spmv_sell_io<float, double>(const Sell<float> &, const double *, void *, bool,
                                          double, const void *, bool, double, hipStream_t, double,
                                          int, hipEvent_t, hipEvent_t, RowMask);

}  // namespace edfa
