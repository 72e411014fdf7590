// Launch-shape autotuner for the sparse products of the iteration.
//
// Every matrix the solve multiplies (the system matrix, the FSAI factor and its transpose,
// the coupling blocks, the ILU(0) factors and their approximate inverses, and their
// transposes once built) is timed with the SELL kernel (one lane per row, 4 or 8 entries
// in flight per lane), with the CSR kernel at 2, 4, 8, 16 and 32 lanes per row (2 or 4
// entries in flight per lane) and, for matrices with long rows, with the chunk kernel; the
// fastest choice is kept in the preconditioner handle and re-applied whenever the copies
// are rebuilt (the next setup rebuilds them with the default choice).
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>

#include "precond.hpp"

namespace edfa {

namespace {

struct Variant {
  int lanes, depth;
};
constexpr Variant kVariants[EDFA_TUNE_VARIANTS] = {
    {0, 4},  {0, 8},  {2, 2},  {2, 4},  {4, 2},  {4, 4},           {8, 2},
    {8, 4},  {16, 2}, {16, 4}, {32, 2}, {32, 4}, {SPMV_CHUNKED, CHUNK_K},
    {SPMV_CHUNKED, CHUNK_K_ALT}};
constexpr int CHUNK_VARIANT = 12;

// The chunk kernel runs only on matrices that carry chunk descriptors (long rows); others
// keep their kernel.
template <class M_>
bool can_run(const M_ &M, const Variant &v) {
  return v.lanes != SPMV_CHUNKED || M.chunk_k == CHUNK_K;
}

template <class M_>
void set_kernel(M_ &M, const Variant &v) {
  if (!can_run(M, v)) return;
  M.lanes = v.lanes;
  M.depth = v.depth;
}

// Visit every tunable matrix of the active precision path: fn(slot, Sell<V>&, role).
template <class F>
void for_each_slot(edfa_precond_s &P, F &&fn) {
  edfa_system_s &S = *P.sys;
  fn(0, S.A_s, SPMV_OPERATOR);
  fn(1, S.AT_s, SPMV_OPERATOR);
  auto prec = [&](auto &D) {
    fn(2, D.GF_s, SPMV_PRECOND);
    fn(3, D.GFT_s, SPMV_PRECOND);
    fn(4, D.L_s, SPMV_PRECOND);
    fn(5, D.U_s, SPMV_PRECOND);
    fn(6, D.ML_s, SPMV_PRECOND);
    fn(7, D.MU_s, SPMV_PRECOND);
    fn(8, D.LT_s, SPMV_PRECOND);
    fn(9, D.UT_s, SPMV_PRECOND);
    fn(10, D.MLT_s, SPMV_PRECOND);
    fn(11, D.MUT_s, SPMV_PRECOND);
  };
  if (P.prm.precision == 1) {
    prec(P.f);
    for (int q = 0; q < 4; ++q) fn(12 + q, P.coupling_fs[q], SPMV_PRECOND);
  } else {
    prec(P.d);
    fn(12, S.Acf_s, SPMV_PRECOND);
    fn(13, S.Afc_s, SPMV_PRECOND);
    fn(14, S.AfcT_s, SPMV_PRECOND);
    fn(15, S.AcfT_s, SPMV_PRECOND);
  }
}

// Reads a buffer larger than the last-level cache, so the next launch finds the matrix in
// HBM as it does inside the solve (where a full iteration streams between two products
// with the same matrix); the conditional store keeps the loads.
constexpr long long FLUSH_DOUBLES = 64ll << 20;   // 512 MiB
__global__ void k_flush(const double *__restrict__ buf, long long n, double *sink) {
  double acc = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    acc += buf[i];
  if (acc == 1.0) sink[0] = acc;
}

template <class V>
float time_variant(Sell<V> &M, Variant v, int role, DBuf<V> &x, DBuf<V> &y, DBuf<double> &fl,
                   hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const int saved = M.lanes, saved_depth = M.depth;
  set_kernel(M, v);
  spmv_sell<V, V>(M, x.p, y.p, 1.0, nullptr, 0.0, s, 0.0, role);   // warm-up
  float best = 1e30f;
  for (int r = 0; r < 5; ++r) {
    if (fl.p) {
      hipLaunchKernelGGL(k_flush, dim3(4096), dim3(256), 0, s, fl.p, FLUSH_DOUBLES, fl.p);
      EDFA_CHECK_LAUNCH();
    }
    spmv_sell<V, V>(M, x.p, y.p, 1.0, nullptr, 0.0, s, 0.0, role, e0, e1);
    EDFA_HIP(hipEventSynchronize(e1));
    float ms = 0;
    EDFA_HIP(hipEventElapsedTime(&ms, e0, e1));
    best = std::min(best, ms);
  }
  M.lanes = saved;
  M.depth = saved_depth;
  return best;
}

template <class V>
__global__ void k_fill_ones(V *x, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = V(1);
}

}  // namespace

void apply_tuned(edfa_precond_s &P) {
  for_each_slot(P, [&](int slot, auto &M, int) {
    if (P.tuned[slot] >= 0 && M.rows > 0) set_kernel(M, kVariants[P.tuned[slot]]);
  });
}

bool layouts_pending(edfa_precond_s &P) {
  bool pending = false;
  for_each_slot(P, [&](int, auto &M, int) {
    if (M.rows > 0 && M.lanes == SPMV_CHUNKED && M.depth == CHUNK_K_ALT && M.nchunk_alt < 0)
      pending = true;
    if (M.rows > 0 && (M.lanes == 0 || M.lanes == 1) && !M.sell_ready) pending = true;
  });
  return pending;
}

void set_variant(edfa_precond_s &P, int slot, int variant) {
  for (int q = 0; q < EDFA_TUNE_SLOTS; ++q)
    if (slot < 0 || q == slot) P.tuned[q] = variant;
  apply_tuned(P);
}

namespace {
struct TuneBufs {
  DBuf<double> flush;   // cache eviction between timed launches (empty: none)
  DBuf<double> xd, yd;
  DBuf<float> xf, yf;
  DBuf<double> &x(double *) { return xd; }
  DBuf<double> &y(double *) { return yd; }
  DBuf<float> &x(float *) { return xf; }
  DBuf<float> &y(float *) { return yf; }
};

constexpr float TUNE_MARGIN = 0.03f;

template <class V>
int tune_one(Sell<V> &M, int role, TuneBufs &B, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
             float *us) {
  DBuf<V> &x = B.x((V *)nullptr);
  DBuf<V> &y = B.y((V *)nullptr);
  const int nx = std::max(M.cols, 1);
  x.ensure(nx);
  y.ensure(std::max(M.rows, 1));
  hipLaunchKernelGGL(k_fill_ones<V>, dim3(ceil_div(nx, 256)), dim3(256), 0, s, x.p, (long long)nx);
  EDFA_CHECK_LAUNCH();
  // the default kernel (SELL, 4 in flight, for short rows; the chunk kernel for long ones)
  // is kept unless another variant is at least TUNE_MARGIN faster; otherwise the first
  // variant (in table order) within TUNE_MARGIN of the fastest is taken, so timing noise
  // does not flip the choice between equivalent kernels from one run to the next
  const int dflt =
      M.rows > 0 && default_spmv_lanes((double)M.nnz / M.rows) == SPMV_CHUNKED ? CHUNK_VARIANT : 0;
  float fastest = INFINITY;
  for (int v = 0; v < EDFA_TUNE_VARIANTS; ++v) {
    us[v] = can_run(M, kVariants[v])
                ? 1e3f * time_variant(M, kVariants[v], role, x, y, B.flush, s, e0, e1)
                : INFINITY;
    fastest = std::min(fastest, us[v]);
  }
  if (!(us[dflt] * (1.0f - TUNE_MARGIN) > fastest)) return dflt;
  for (int v = 0; v < EDFA_TUNE_VARIANTS; ++v)
    if (us[v] * (1.0f - TUNE_MARGIN) <= fastest) return v;
  return dflt;
}
}  // namespace

// EDFA parameter choice: every candidate is set up and solved on the system, timed with
// events on the stream (setup + solve), and the fastest converged candidate wins.
int tune_params(edfa_system_s &S, const edfa_params *cand, int ncand,
                const edfa_solve_params &sp, hipStream_t s, double *times_ms, int *iterations,
                int *status) {
  DBuf<double> x;
  x.ensure(std::max(S.n, 1));
  int best = -1;
  double best_t = INFINITY;
  for (int c = 0; c < ncand; ++c) {
    double t = INFINITY;
    int its = -1, st = EDFA_OK;
    try {
      edfa_precond_s P;
      P.sys = &S;
      P.prm = cand[c];
      EventTimer tm;
      tm.start(s);
      precond_stage1(P, s);
      precond_stage2(P, s);
      edfa_solve_info info{};
      st = sp.method == EDFA_BICGSTAB ? bicgstab(S, P, S.b.p, x.p, sp, s, &info)
                                      : gmres(S, P, S.b.p, x.p, sp, s, &info);
      tm.stop(s);
      its = info.iterations;
      if (st == EDFA_OK) t = tm.ms();
    } catch (const Error &e) {
      // a candidate the system cannot take (capacity, breakdown) is skipped
      st = e.status;
      (void)hipStreamSynchronize(s);
    }
    if (times_ms) times_ms[c] = t;
    if (iterations) iterations[c] = its;
    if (status) status[c] = st;
    if (t < best_t) {
      best_t = t;
      best = c;
    }
  }
  return best;
}

int autotune(edfa_precond_s &P, hipStream_t s, edfa_tune_slot *slots) {
  hipEvent_t e0, e1;
  EDFA_HIP(hipEventCreate(&e0));
  EDFA_HIP(hipEventCreate(&e1));
  TuneBufs B;
  // matrices larger than an XCD's L2 are timed cold: a zeroed 512 MiB buffer is read
  // before every timed launch
  int64_t biggest = 0;
  for_each_slot(P, [&](int, auto &M, int) { biggest = std::max<int64_t>(biggest, M.nnz); });
  if (biggest * 12 > (8ll << 20)) {
    B.flush.ensure((size_t)FLUSH_DOUBLES);
    EDFA_HIP(hipMemsetAsync(B.flush.p, 0, sizeof(double) * FLUSH_DOUBLES, s));
  }
  // CGS2 block width: one dot pass over 24 basis vectors of the system's size
  {
    edfa_system_s &S = *P.sys;
    if (!P.ws) P.ws.reset(new SolveWork());
    SolveWork &W = *P.ws;
    build_chunks(S, W, s);
    const int n = S.n, nv = 24, ld = 2 * nv + 4;
    DBuf<double> Vt, pt;
    DBuf<SegState> st;
    Vt.ensure((size_t)(nv + 2) * std::max(n, 1));
    pt.ensure((size_t)W.nchunk * ld);
    st.ensure(S.ngrid);
    std::vector<SegState> hs(S.ngrid);
    for (auto &q : hs) {
      q = SegState{};
      q.active = 1;
    }
    EDFA_HIP(hipMemcpyAsync(st.p, hs.data(), sizeof(SegState) * hs.size(), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_fill_ones<double>, dim3(ceil_div((long long)(nv + 2) * n, 256)), dim3(256),
                       0, s, Vt.p, (long long)(nv + 2) * n);
    EDFA_CHECK_LAUNCH();
    float best = INFINITY, dflt = INFINITY;
    int width = 4;
    for (int wd : {4, 2, 8}) {
      float t = INFINITY;
      for (int r = 0; r < 5; ++r) {
        if (B.flush.p) {
          hipLaunchKernelGGL(k_flush, dim3(4096), dim3(256), 0, s, B.flush.p, FLUSH_DOUBLES, B.flush.p);
          EDFA_CHECK_LAUNCH();
        }
        EDFA_HIP(hipEventRecord(e0, s));
        launch_dots2(wd, nv, W.nchunk, s, Vt.p, (long long)n, Vt.p + (size_t)nv * n,
                     Vt.p + (size_t)(nv + 1) * n, W.chunks.p, st.p, pt.p, ld);
        EDFA_HIP(hipEventRecord(e1, s));
        EDFA_HIP(hipEventSynchronize(e1));
        float ms = 0;
        EDFA_HIP(hipEventElapsedTime(&ms, e0, e1));
        t = std::min(t, ms);
      }
      if (wd == 4) dflt = t;
      if (t < best) {
        best = t;
        width = wd;
      }
    }
    P.cgs2_width = best < dflt * (1.0f - TUNE_MARGIN) ? width : 4;
  }
  int tuned = 0;
  if (slots)
    for (int q = 0; q < EDFA_TUNE_SLOTS; ++q) slots[q] = edfa_tune_slot{};
  for_each_slot(P, [&](int slot, auto &M, int role) {
    if (M.rows <= 0) return;
    edfa_tune_slot rec{};
    const int best = tune_one(M, role, B, s, e0, e1, rec.us);
    P.tuned[slot] = best;
    set_kernel(M, kVariants[best]);
    ++tuned;
    if (slots) {
      rec.rows = M.rows;
      rec.cols = M.cols;
      rec.nnz = M.nnz;
      rec.variant = best;
      rec.value_bytes = (int32_t)sizeof(*M.val.p);
      rec.sell_sorted = M.sorted ? 1 : 0;
      rec.sell_padding = M.nnz > 0 ? (float)((double)M.padded / (double)M.nnz) : 1.0f;
      slots[slot] = rec;
    }
  });
  EDFA_HIP(hipStreamSynchronize(s));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return tuned;
}

}  // namespace edfa
