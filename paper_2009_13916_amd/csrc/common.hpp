// Internal helpers of the EDFA library: errors, device buffers, launch shapes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "edfa.h"

namespace edfa {

struct Error {
  edfa_status status;
  std::string msg;
};

[[noreturn]] void fail(edfa_status st, const char *fmt, ...);
void set_last_error(const std::string &msg);

#define EDFA_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      ::edfa::fail(e_ == hipErrorOutOfMemory ? EDFA_ERR_NOMEM : EDFA_ERR_HIP, "%s: %s (%s:%d)", \
                   #call, hipGetErrorString(e_), __FILE__, __LINE__);                    \
  } while (0)

#define EDFA_CHECK_LAUNCH() EDFA_HIP(hipGetLastError())

// Growable device buffer owned by a handle.  ensure() keeps the allocation when it is
// already large enough, so repeated setups reuse memory.
template <class T>
struct DBuf {
  T *p = nullptr;
  size_t cap = 0;
  size_t n = 0;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  DBuf(DBuf &&o) noexcept : p(o.p), cap(o.cap), n(o.n) { o.p = nullptr; o.cap = o.n = 0; }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = n = 0;
  }
  T *ensure(size_t count) {
    n = count;
    if (count <= cap && p) return p;
    release();
    size_t bytes = (count ? count : 1) * sizeof(T);
    EDFA_HIP(hipMalloc(&p, bytes));
    cap = count ? count : 1;
    n = count;
    return p;
  }
  T *get() const { return p; }
  operator T *() const { return p; }
};

// Pinned host buffer: device-to-host copies into it run asynchronously.
template <class T>
struct HBuf {
  T *p = nullptr;
  size_t cap = 0;
  HBuf() = default;
  HBuf(const HBuf &) = delete;
  HBuf &operator=(const HBuf &) = delete;
  ~HBuf() {
    if (p) (void)hipHostFree(p);
  }
  T *ensure(size_t count) {
    if (count <= cap && p) return p;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    const size_t c = count ? count : 1;
    EDFA_HIP(hipHostMalloc((void **)&p, c * sizeof(T), hipHostMallocDefault));
    cap = c;
    return p;
  }
};

// CSR matrix in device memory (int32 indices).
template <class V>
struct Csr {
  int rows = 0, cols = 0;
  int64_t nnz = 0;
  DBuf<int> rowptr;
  DBuf<int> col;
  DBuf<V> val;
  void alloc(int r, int c, int64_t z) {
    rows = r;
    cols = c;
    nnz = z;
    rowptr.ensure((size_t)r + 1);
    col.ensure((size_t)z);
    val.ensure((size_t)z);
  }
};

// Sliced ELLPACK with slices of 64 rows (one wavefront): the k-th entries of the 64 rows of
// a slice are contiguous, so a lane per row reads coalesced without cross-lane reductions.
// Each row stops at its own length (padding is stored but never read).
template <class V>
struct Sell {
  int rows = 0, cols = 0;
  int64_t nnz = 0;
  // The SELL layout.  Matrices whose default kernel is the chunk kernel (long rows) get it
  // only when a SELL variant first multiplies them (sell_ready false until then), so the
  // fields below are filled on demand from the CSR arrays.
  mutable bool sell_ready = false;
  mutable int nslice = 0;
  mutable int64_t padded = 0;
  mutable DBuf<int> sptr;   // nslice + 1 element offsets
  mutable DBuf<int> rlen;   // rows
  mutable DBuf<int> col;
  mutable DBuf<V> val;
  // sorted layout: position p of the slices holds row perm[p] (rows sorted by length
  // inside windows); otherwise position p holds row p
  mutable bool sorted = false;
  mutable DBuf<int> perm;
  mutable DBuf<int> scan_tmp;     // scratch of the on-demand builds
  mutable DBuf<int> chunk_work;   // scratch of the chunk descriptor build
  // Kernel choice: lanes = 0 or 1 runs the SELL kernel; lanes = 2..32 runs the CSR kernel
  // with that many lanes per row on the source CSR arrays (which must outlive this copy);
  // lanes = SPMV_CHUNKED runs the chunk kernel on the CSR arrays (below).
  // depth: entries in flight per lane and round (SELL 4 or 8, CSR 2 or 4; other values
  // take 4 and 2; the chunk kernel CHUNK_K, or CHUNK_K_ALT on its own descriptors).
  int lanes = 0;
  int depth = 0;
  const int *csr_rp = nullptr, *csr_col = nullptr;
  const V *csr_val = nullptr;
  // Row-aligned chunks of the CSR arrays for the chunk kernel: chunk c holds rows
  // [chunk[c].x, chunk[c+1].x) and entries [chunk[c].y, chunk[c+1].y), at most 64 * chunk_k
  // entries unless it is a single longer row (chunk_k = 0: not built).  Built with the
  // copy for matrices whose rows are long (the kernel's default there).
  DBuf<int2> chunk;
  int nchunk = 0;
  int chunk_k = 0;
  // The same for the chunk kernel with CHUNK_K_ALT (chunks of at most 64 * CHUNK_K_ALT
  // entries), built on the first product that uses them (nchunk_alt < 0: not built).
  mutable DBuf<int2> chunk_alt;
  mutable int nchunk_alt = -1;
};
constexpr int SPMV_CHUNKED = -1;
constexpr int CHUNK_K = 12;       // chunk kernel: 12 entries in flight per lane, 768 per chunk
constexpr int CHUNK_K_ALT = 8;    // narrower chunks: 8 per lane, 512 per chunk

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }


// Pinned host staging for small device reads, one block per host thread (allocated on
// first use and kept for the life of the process): a copy into pinned memory returns about
// a third sooner than one into pageable memory.
constexpr size_t PINNED_SLOT = 4096;
inline void *pinned_slot(size_t bytes) {
  constexpr size_t SLOT = PINNED_SLOT;
  static thread_local void *slot = nullptr;
  if (bytes > SLOT) fail(EDFA_ERR_ARG, "pinned read of %zu bytes", bytes);
  if (!slot) EDFA_HIP(hipHostMalloc(&slot, SLOT, hipHostMallocDefault));
  return slot;
}

// Host read of `count` device values (synchronises the stream; count * sizeof(T) <=
// PINNED_SLOT).
template <class T>
void read_small(T *out, const T *dptr, size_t count, hipStream_t s) {
  T *pin = static_cast<T *>(pinned_slot(sizeof(T) * count));
  EDFA_HIP(hipMemcpyAsync(pin, dptr, sizeof(T) * count, hipMemcpyDeviceToHost, s));
  EDFA_HIP(hipStreamSynchronize(s));
  for (size_t i = 0; i < count; ++i) out[i] = pin[i];
}

// Host read of one device scalar (synchronises the stream).
template <class T>
T read_scalar(const T *dptr, hipStream_t s) {
  T v{};
  read_small(&v, dptr, 1, s);
  return v;
}

// Events for device-side timing on a stream.
struct EventTimer {
  hipEvent_t a{}, b{};
  EventTimer() {
    EDFA_HIP(hipEventCreate(&a));
    EDFA_HIP(hipEventCreate(&b));
  }
  ~EventTimer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
  void start(hipStream_t s) { EDFA_HIP(hipEventRecord(a, s)); }
  void stop(hipStream_t s) { EDFA_HIP(hipEventRecord(b, s)); }
  float ms() {
    EDFA_HIP(hipEventSynchronize(b));
    float t = 0;
    EDFA_HIP(hipEventElapsedTime(&t, a, b));
    return t;
  }
};

// ---------------------------------------------------------------------------------
// Primitive device algorithms (sparse.hip)
// ---------------------------------------------------------------------------------
// Exclusive prefix sum of n int32 values into out (out may alias in); returns the total
// (synchronises the stream).  tmp is scratch owned by the caller.
int64_t exclusive_scan(const int *in, int *out, int n, DBuf<int> &tmp, hipStream_t s);
// Same, without reading the total back (asynchronous).
void exclusive_scan_async(const int *in, int *out, int n, DBuf<int> &tmp, hipStream_t s);
// Stable partition of [0, n) by key[i] in [0, nkey): out lists the indices key by key,
// ascending inside a key; counts (host) receives each key's size.  Synchronises.
void stable_partition(const int *key, int n, int nkey, int *out, DBuf<int> &hist, DBuf<int> &tmp,
                      hipStream_t s, std::vector<int> &counts);

// Transpose of a CSR matrix (rows x cols) into dst (cols x rows).  With sort, columns are
// sorted within rows (deterministic layout, needed where values are summed); without,
// the order inside a row is arbitrary (pattern-only uses).
template <class V>
void csr_transpose(const Csr<V> &src, Csr<V> &dst, DBuf<int> &tmp, DBuf<int> &cursor,
                   hipStream_t s, bool sort = true);

// y[i] = alpha * (A x)[i] + beta * b[i] + gamma * x[i]   (b may be null; gamma needs a
// square A).  A in CSR with values V, vectors of type X; accumulation in the wider type.
// y may alias b (each row reads only its own b entry), never x.
template <class V, class X>
void spmv(const int *rowptr, const int *col, const V *val, int rows, const X *x, X *y,
          double alpha, const X *b, double beta, float avg_nnz, hipStream_t s,
          double gamma = 0.0);

// SELL-64 copy of a CSR matrix (device-side conversion; synchronises to size the storage).
// Matrices with long rows get the chunk descriptors of their default chunk kernel instead;
// their SELL layout is built by ensure_sell when a SELL variant first multiplies them.
template <class V>
void build_sell(const Csr<V> &M, Sell<V> &S, DBuf<int> &tmp, hipStream_t s);
template <class V>
void ensure_sell(const Sell<V> &S, hipStream_t s);
// Chunk descriptors of S's CSR arrays for chunks of at most 64 * k entries (the greedy
// row-aligned cut, computed on the device; synchronises once for the chunk count).  No-op
// when they exist for this k.
template <class V>
void build_row_chunks(Sell<V> &S, int k, hipStream_t s);
// Default lanes per row for a mean row length (0: the SELL kernel).
int default_spmv_lanes(double mean_row);

// Rows to skip in a product: row r is computed only if act[seg[r] * stride] != 0 (the
// activity flag of its grid).  seg == NULL computes every row.
// Rows to skip in a product: row r belongs to grid seg[r], whose flag act[g * stride] is
// zero once it stops iterating.  seg = null with act set: every row belongs to grid 0 (a
// single system, masked after convergence); act = null: no mask.
struct RowMask {
  const int *seg = nullptr;
  const int *act = nullptr;
  int stride = 0;
  RowMask offset(int rows) const { return RowMask{seg ? seg + rows : nullptr, act, stride}; }
};
// A stopped single system: one uniform check at a kernel's start, before any divergence.
__device__ __forceinline__ bool all_off(const RowMask &mk) {
  return mk.act && !mk.seg && !mk.act[0];
}
// A row of a stopped grid of a batch.
__device__ __forceinline__ bool row_off(const RowMask &mk, int row) {
  return mk.seg && !mk.act[mk.seg[row] * mk.stride];
}

// Same contract as spmv() for a SELL-64 matrix.  `role` picks the kernel symbol:
// SPMV_OPERATOR for products with the system matrix, SPMV_PRECOND for everything else.
// Non-null events e0/e1 are recorded by the launch itself around the kernel.
enum { SPMV_OPERATOR = 0, SPMV_PRECOND = 1 };
template <class V, class X>
void spmv_sell(const Sell<V> &M, const X *x, X *y, double alpha, const X *b, double beta,
               hipStream_t s, double gamma = 0.0, int role = SPMV_PRECOND,
               hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, RowMask mask = {});
// The same with y and b in FP64 (y64, b64) or FP32 each, whatever the type of x.
template <class V, class X>
void spmv_sell_io(const Sell<V> &M, const X *x, void *y, bool y64, double alpha, const void *b,
                  bool b64, double beta, hipStream_t s, double gamma, int role, hipEvent_t e0,
                  hipEvent_t e1, RowMask mask);

}  // namespace edfa
