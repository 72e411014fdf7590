// Launch-shape autotuner for the sparse products of the iteration.
//
// Every matrix the solve multiplies (the system matrix, the FSAI factor and its transpose,
// the coupling blocks, the ILU(0) factors and their approximate inverses, and their
// transposes once built) is timed with the SELL kernel (one lane per row) and with the
// CSR kernel at 2, 4, 8, 16 and 32 lanes per row; the fastest choice is kept in the
// preconditioner handle and re-applied whenever the copies are rebuilt (the next setup
// rebuilds them with the default choice).
#include <hip/hip_ext.h>

#include <algorithm>

#include "precond.hpp"

namespace edfa {

namespace {

constexpr int kVariants[] = {0, 2, 4, 8, 16, 32};

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

template <class V>
float time_lanes(Sell<V> &M, int lanes, int role, DBuf<V> &x, DBuf<V> &y, hipStream_t s,
                 hipEvent_t e0, hipEvent_t e1) {
  const int saved = M.lanes;
  M.lanes = lanes;
  spmv_sell<V, V>(M, x.p, y.p, 1.0, nullptr, 0.0, s, 0.0, role);   // warm-up
  float best = 1e30f;
  for (int r = 0; r < 5; ++r) {
    spmv_sell<V, V>(M, x.p, y.p, 1.0, nullptr, 0.0, s, 0.0, role, e0, e1);
    EDFA_HIP(hipEventSynchronize(e1));
    float ms = 0;
    EDFA_HIP(hipEventElapsedTime(&ms, e0, e1));
    best = std::min(best, ms);
  }
  M.lanes = saved;
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
    if (P.tuned[slot] >= 0 && M.rows > 0) M.lanes = P.tuned[slot];
  });
}

namespace {
struct TuneBufs {
  DBuf<double> xd, yd;
  DBuf<float> xf, yf;
  DBuf<double> &x(double *) { return xd; }
  DBuf<double> &y(double *) { return yd; }
  DBuf<float> &x(float *) { return xf; }
  DBuf<float> &y(float *) { return yf; }
};

template <class V>
int tune_one(Sell<V> &M, int role, TuneBufs &B, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  DBuf<V> &x = B.x((V *)nullptr);
  DBuf<V> &y = B.y((V *)nullptr);
  const int nx = std::max(M.cols, 1);
  x.ensure(nx);
  y.ensure(std::max(M.rows, 1));
  hipLaunchKernelGGL(k_fill_ones<V>, dim3(ceil_div(nx, 256)), dim3(256), 0, s, x.p, (long long)nx);
  EDFA_CHECK_LAUNCH();
  int best = 0;
  float tbest = 1e30f;
  for (int lanes : kVariants) {
    const float t = time_lanes(M, lanes, role, x, y, s, e0, e1);
    if (t < tbest) {
      tbest = t;
      best = lanes;
    }
  }
  return best;
}
}  // namespace

int autotune(edfa_precond_s &P, hipStream_t s) {
  hipEvent_t e0, e1;
  EDFA_HIP(hipEventCreate(&e0));
  EDFA_HIP(hipEventCreate(&e1));
  TuneBufs B;
  int tuned = 0;
  for_each_slot(P, [&](int slot, auto &M, int role) {
    if (M.rows <= 0) return;
    const int best = tune_one(M, role, B, s, e0, e1);
    P.tuned[slot] = best;
    M.lanes = best;
    ++tuned;
  });
  EDFA_HIP(hipStreamSynchronize(s));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return tuned;
}

}  // namespace edfa
