// Application of the EDFA preconditioner (eq. EDFA_prec) and of its transpose.
//
//   t   = A~^-1 r_pi            A~^-1 = -G_F^T G_F   (two SpMVs)
//   y   = r_p - A_ppi t
//   z_p = S~^-1 y               multicolour ILU(0): ISAI of the factors (+ refinement) in
//                               the natural cell order, or colour-by-colour substitution
//   z_pi = A~^-1 (r_pi - A_pip z_p)
// The transpose swaps A_ppi <-> A_pip^T and uses (LU)^-T.
#include <mutex>

#include "precond.hpp"

namespace edfa {

template <class T>
__global__ void k_gather(const T *__restrict__ x, const int *__restrict__ idx, int n, T *y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[idx[i]];
}

template <class T>
__global__ void k_scatter(const T *__restrict__ x, const int *__restrict__ idx, int n, T *y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[idx[i]] = x[i];
}

template <class A, class B>
__global__ void k_convert(const A *__restrict__ x, long long n, B *y, RowMask mk) {
  if (all_off(mk)) return;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (row_off(mk, (int)i)) return;
  y[i] = (B)x[i];
}

// Colour-by-colour substitution on rows [r0, r1): y_i = (b_i - sum_{j != diag} a_ij y_j) / d
// where d = a_ii when the row stores its diagonal (first or last entry), else 1.
template <class T>
__global__ void k_sweep(const int *__restrict__ rp, const int *__restrict__ col,
                        const T *__restrict__ val, int r0, int r1, int diag_where,
                        const T *__restrict__ b, T *y) {
  const int i = r0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= r1) return;
  int a = rp[i], e = rp[i + 1];
  T d = T(1);
  if (diag_where == 1) d = val[a++];        // diagonal first (U)
  else if (diag_where == 2) d = val[--e];   // diagonal last (U^T)
  T s = b[i];
  for (int p = a; p < e; ++p) s -= val[p] * y[col[p]];
  y[i] = s / d;
}

// FP32 copy of an FP64 CSR matrix (pattern copied, values rounded); kept across calls.
static void to_fp32(const Csr<double> &M, Csr<float> &F, hipStream_t s) {
  F.alloc(M.rows, M.cols, M.nnz);
  EDFA_HIP(hipMemcpyAsync(F.rowptr.p, M.rowptr.p, sizeof(int) * ((size_t)M.rows + 1),
                          hipMemcpyDeviceToDevice, s));
  if (M.nnz) {
    EDFA_HIP(hipMemcpyAsync(F.col.p, M.col.p, sizeof(int) * M.nnz, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL((k_convert<double, float>), dim3(ceil_div(M.nnz, 256)), dim3(256), 0, s,
                       M.val.p, (long long)M.nnz, F.val.p, RowMask{});
    EDFA_CHECK_LAUNCH();
  }
}

// Events of one product of a profiled solve (none otherwise).
struct Ev {
  hipEvent_t a = nullptr, b = nullptr;
};
static Ev prod_events(edfa_precond_s &P, int slot) {
  if (!P.prof) return {};
  Ev e{P.prof->get(), P.prof->get()};
  P.prof->rec.emplace_back(slot, e.a, e.b);
  return e;
}

// Workspace vectors of one application: t1, t2 (N_f^u), r, w, res, y, zq (N_e).
template <class T>
struct ApplyWork {
  T *t1, *t2, *r, *w, *res, *y, *zq;
};
template <class T>
static ApplyWork<T> handle_work(PrecData<T> &D, int nfu, int ne) {
  return {D.t1.ensure(nfu), D.t2.ensure(nfu), D.r.ensure(ne), D.w.ensure(ne),
          D.res.ensure(ne),  D.y.ensure(ne),   D.zq.ensure(ne)};
}

// z_p = S~^-1 y.  ISAI: products with the approximate inverses of (I + L) and U (and
// Richardson steps with the factors), all stored in the natural cell order, so y and z_p
// are used as they are.  Exact: colour-by-colour substitution in the colour order, between
// a gather and a scatter of the vector.
template <class T>
static void sinv(edfa_precond_s &P, PrecData<T> &D, const ApplyWork<T> &W, int transpose,
                 const T *y, T *zp, hipStream_t s, RowMask cm) {
  const int ne = P.sys->ne;
  const int gb = ceil_div(ne, 256);
  const int steps = std::max(1, P.prm.isai_steps);
  if (P.prm.schur_solver == EDFA_SCHUR_ISAI) {
    // first factor (L, or U^T for the transpose), then the second
    const Sell<T> &M1 = transpose ? D.MUT_s : D.ML_s;
    const Sell<T> &T1 = transpose ? D.UT_s : D.L_s;
    const Sell<T> &M2 = transpose ? D.MLT_s : D.MU_s;
    const Sell<T> &T2 = transpose ? D.LT_s : D.U_s;
    const double g1 = transpose ? 0.0 : -1.0;   // (I + L) w = L w + w
    const double g2 = transpose ? -1.0 : 0.0;
    // tuner slots of M1, T1, M2, T2
    const int sM1 = transpose ? 11 : 6, sT1 = transpose ? 9 : 4;
    const int sM2 = transpose ? 10 : 7, sT2 = transpose ? 8 : 5;
    const int R = SPMV_PRECOND;
    auto prod = [&](const Sell<T> &M, int slot, const T *in, T *out, double alpha, const T *bb,
                    double beta, double gamma) {
      const Ev e = prod_events(P, slot);
      spmv_sell<T, T>(M, in, out, alpha, bb, beta, s, gamma, R, e.a, e.b, cm);
    };
    prod(M1, sM1, y, W.w, 1.0, nullptr, 0.0, 0.0);
    for (int k = 1; k < steps; ++k) {
      prod(T1, sT1, W.w, W.res, -1.0, y, 1.0, g1);
      prod(M1, sM1, W.res, W.w, 1.0, W.w, 1.0, 0.0);
    }
    prod(M2, sM2, W.w, zp, 1.0, nullptr, 0.0, 0.0);
    for (int k = 1; k < steps; ++k) {
      prod(T2, sT2, zp, W.res, -1.0, W.w, 1.0, g2);
      prod(M2, sM2, W.res, zp, 1.0, zp, 1.0, 0.0);
    }
    return;
  }
  hipLaunchKernelGGL(k_gather<T>, dim3(gb), dim3(256), 0, s, y, D.perm.p, ne, W.y);
  EDFA_CHECK_LAUNCH();
  const int nc = P.n_colors;
  if (!transpose) {
    for (int c = 0; c < nc; ++c) {
      const int r0 = D.cstart[c], r1 = D.cstart[c + 1];
      if (r1 > r0)
        hipLaunchKernelGGL(k_sweep<T>, dim3(ceil_div(r1 - r0, 64)), dim3(64), 0, s, D.L.rowptr.p,
                           D.L.col.p, D.L.val.p, r0, r1, 0, W.y, W.w);
    }
    for (int c = nc - 1; c >= 0; --c) {
      const int r0 = D.cstart[c], r1 = D.cstart[c + 1];
      if (r1 > r0)
        hipLaunchKernelGGL(k_sweep<T>, dim3(ceil_div(r1 - r0, 64)), dim3(64), 0, s, D.U.rowptr.p,
                           D.U.col.p, D.U.val.p, r0, r1, 1, W.w, W.zq);
    }
  } else {
    for (int c = 0; c < nc; ++c) {
      const int r0 = D.cstart[c], r1 = D.cstart[c + 1];
      if (r1 > r0)
        hipLaunchKernelGGL(k_sweep<T>, dim3(ceil_div(r1 - r0, 64)), dim3(64), 0, s, D.UT.rowptr.p,
                           D.UT.col.p, D.UT.val.p, r0, r1, 2, W.y, W.w);
    }
    for (int c = nc - 1; c >= 0; --c) {
      const int r0 = D.cstart[c], r1 = D.cstart[c + 1];
      if (r1 > r0)
        hipLaunchKernelGGL(k_sweep<T>, dim3(ceil_div(r1 - r0, 64)), dim3(64), 0, s, D.LT.rowptr.p,
                           D.LT.col.p, D.LT.val.p, r0, r1, 0, W.w, W.zq);
    }
  }
  EDFA_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_scatter<T>, dim3(gb), dim3(256), 0, s, W.zq, D.perm.p, ne, zp);
  EDFA_CHECK_LAUNCH();
}

template <class T>
static void ensure_transposed_factors(edfa_precond_s &P, PrecData<T> &D, hipStream_t s) {
  edfa_system_s &S = *P.sys;
  if (D.MUT.rows == 0 && D.UT.rows == 0 && S.ne) {
    // ISAI: transposes of the natural-order copies (of the factors only for refinement
    // steps); exact substitution: colour order
    const bool isai = P.prm.schur_solver == EDFA_SCHUR_ISAI;
    if (!isai || P.prm.isai_steps > 1) {
      csr_transpose(isai ? D.Un : D.U, D.UT, S.tmp, S.tmp2, s);
      csr_transpose(isai ? D.Ln : D.L, D.LT, S.tmp, S.tmp2, s);
      build_sell(D.UT, D.UT_s, S.tmp, s);
      build_sell(D.LT, D.LT_s, S.tmp, s);
    } else {
      D.UT_s.rows = D.LT_s.rows = 0;
    }
    if (isai) {
      csr_transpose(D.MLn, D.MLT, S.tmp, S.tmp2, s);
      csr_transpose(D.MUn, D.MUT, S.tmp, S.tmp2, s);
      build_sell(D.MLT, D.MLT_s, S.tmp, s);
      build_sell(D.MUT, D.MUT_s, S.tmp, s);
    }
  }
  if (S.AcfT.rows == 0 && S.nfu) csr_transpose(S.Acf, S.AcfT, S.tmp, S.tmp2, s);
  if (S.AcfT_s.rows == 0 && S.nfu) build_sell(S.AcfT, S.AcfT_s, S.tmp, s);
}

// z = P^-1 r (or P^-T r) in precision T; c1 = A_ppi (A_pip^T), c2 = A_pip (A_ppi^T).
// fm / cm: rows of face / cell unknowns to skip (grids of a batch that have converged).
template <class T>
static void apply_typed(edfa_precond_s &P, PrecData<T> &D, const ApplyWork<T> &W, const T *r,
                        T *z, const Sell<T> &c1, const Sell<T> &c2, int transpose,
                        hipStream_t s, RowMask fm, RowMask cm) {
  edfa_system_s &S = *P.sys;
  const int nfu = S.nfu;
  const int R = SPMV_PRECOND;
  const T *rpi = r, *rp = r + nfu;
  T *zpi = z, *zp = z + nfu;
  // tuner slots of the coupling products
  const int s1 = transpose ? 14 : 12, s2 = transpose ? 15 : 13;
  auto prod = [&](const Sell<T> &M, int slot, const T *in, T *out, double alpha, const T *bb,
                  double beta, RowMask mk) {
    const Ev e = prod_events(P, slot);
    spmv_sell<T, T>(M, in, out, alpha, bb, beta, s, 0.0, R, e.a, e.b, mk);
  };
  // t = A~^-1 r_pi = -G_F^T G_F r_pi
  prod(D.GF_s, 2, rpi, W.t1, 1.0, nullptr, 0.0, fm);
  prod(D.GFT_s, 3, W.t1, W.t2, -1.0, nullptr, 0.0, fm);
  // y = r_p - A_ppi t
  prod(c1, s1, W.t2, W.r, -1.0, rp, 1.0, cm);
  // z_p = S~^-1 y
  sinv<T>(P, D, W, transpose, W.r, zp, s, cm);
  // z_pi = A~^-1 (r_pi - A_pip z_p)
  prod(c2, s2, zp, W.t1, -1.0, rpi, 1.0, fm);
  prod(D.GF_s, 2, W.t1, W.t2, 1.0, nullptr, 0.0, fm);
  prod(D.GFT_s, 3, W.t2, zpi, -1.0, nullptr, 0.0, fm);
}

// FP32 application reading r and writing z in FP64 directly (no conversion passes of the
// whole vector): the first products read r_pi and r_p, the last ones write z_p and z_pi,
// in FP64; everything between stays FP32.  Used for the approximate inverses of the ILU(0)
// factors without refinement steps (the default), forward application.
static void apply_fp32_direct(edfa_precond_s &P, PrecData<float> &D, const ApplyWork<float> &W,
                              const double *r, double *z, const Sell<float> &c1,
                              const Sell<float> &c2, hipStream_t s, RowMask fm, RowMask cm) {
  const int nfu = P.sys->nfu;
  const int R = SPMV_PRECOND;
  const double *rpi = r, *rp = r + nfu;
  double *zpi = z, *zp = z + nfu;
  // out (FP64 when o64), x of type X, addend bb FP64 when given
  auto prod = [&](const Sell<float> &M, int slot, const auto *in, void *out, bool o64,
                  double alpha, const double *bb, RowMask mk) {
    const Ev e = prod_events(P, slot);
    spmv_sell_io(M, in, out, o64, alpha, bb, true, bb ? 1.0 : 0.0, s, 0.0, R, e.a, e.b, mk);
  };
  // t = A~^-1 r_pi = -G_F^T G_F r_pi
  prod(D.GF_s, 2, rpi, W.t1, false, 1.0, nullptr, fm);
  prod(D.GFT_s, 3, W.t1, W.t2, false, -1.0, nullptr, fm);
  // y = r_p - A_ppi t
  prod(c1, 12, W.t2, W.r, false, -1.0, rp, cm);
  // z_p = M_U (M_L y)
  prod(D.ML_s, 6, W.r, W.w, false, 1.0, nullptr, cm);
  prod(D.MU_s, 7, W.w, zp, true, 1.0, nullptr, cm);
  // z_pi = A~^-1 (r_pi - A_pip z_p)
  prod(c2, 13, zp, W.t1, false, -1.0, rpi, fm);
  prod(D.GF_s, 2, W.t1, W.t2, false, 1.0, nullptr, fm);
  prod(D.GFT_s, 3, W.t2, zpi, true, -1.0, nullptr, fm);
}

// Device memory for the allocation-free application: a static array per GPU, its
// address looked up once per device.  Every call on a device uses the same bytes, so calls
// that overlap on one GPU race.
constexpr size_t SCRATCH_BYTES = EDFA_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[MAX_DEVICES];

static void *scratch_ptr() {
  int dev = 0;
  EDFA_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) fail(EDFA_ERR_ARG, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    EDFA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

// Carves aligned vectors out of a fixed region.
struct Carver {
  unsigned char *base;
  size_t cap, used = 0;
  template <class T>
  T *take(size_t n) {
    const size_t bytes = ((n * sizeof(T) + 255) / 256) * 256;
    T *p = reinterpret_cast<T *>(base + used);
    used += bytes;
    return p;
  }
};

template <class T>
static ApplyWork<T> carve_work(Carver &C, int nfu, int ne) {
  ApplyWork<T> W;
  W.t1 = C.take<T>(nfu);
  W.t2 = C.take<T>(nfu);
  W.r = C.take<T>(ne);
  W.w = C.take<T>(ne);
  W.res = C.take<T>(ne);
  W.y = C.take<T>(ne);
  W.zq = C.take<T>(ne);
  return W;
}

// Bytes of scratch an application needs (the layout of carve_work, plus the FP32 copies
// of the vector in and out).
static size_t scratch_need(const edfa_precond_s &P) {
  const edfa_system_s &S = *P.sys;
  auto al = [](size_t b) { return ((b + 255) / 256) * 256; };
  const size_t vb = P.prm.precision == 1 ? sizeof(float) : sizeof(double);
  size_t need = 2 * al(vb * S.nfu) + 5 * al(vb * S.ne);
  if (P.prm.precision == 1) need += 2 * al(sizeof(float) * (size_t)S.n);
  return need;
}

static bool transposed_ready(const edfa_precond_s &P) {
  const edfa_system_s &S = *P.sys;
  auto ready = [&](const auto &D) {
    const bool isai = P.prm.schur_solver == EDFA_SCHUR_ISAI;
    if (isai && (D.MUT_s.rows != S.ne || D.MLT_s.rows != S.ne)) return false;
    if ((!isai || P.prm.isai_steps > 1) && (D.UT_s.rows != S.ne || D.LT_s.rows != S.ne))
      return false;
    return true;
  };
  if (S.nfu && S.AcfT_s.rows != S.nfu) return false;
  return S.ne == 0 || (P.prm.precision == 1 ? ready(P.f) : ready(P.d));
}

static void apply_impl(edfa_precond_s &P, int transpose, const double *r, double *z,
                       hipStream_t s, RowMask mask, void *scr) {
  edfa_system_s &S = *P.sys;
  const RowMask fm = mask, cm = mask.offset(S.nfu);
  Carver C{static_cast<unsigned char *>(scr), SCRATCH_BYTES};
  if (transpose) {
    if (!scr) {
      if (P.prm.precision == 1)
        ensure_transposed_factors(P, P.f, s);
      else
        ensure_transposed_factors(P, P.d, s);
    } else if (!transposed_ready(P)) {
      fail(EDFA_ERR_ARG, "the transposed factors do not exist yet: build them with one "
                         "edfa_apply(transpose = 1) or transposed solve first");
    }
    apply_tuned(P);
  }
  if (P.prm.precision != 1) {
    const ApplyWork<double> W = scr ? carve_work<double>(C, S.nfu, S.ne)
                                    : handle_work(P.d, S.nfu, S.ne);
    apply_typed<double>(P, P.d, W, r, z, transpose ? S.AfcT_s : S.Acf_s,
                        transpose ? S.AcfT_s : S.Afc_s, transpose, s, fm, cm);
    return;
  }
  // FP32 application: convert in, apply, convert out
  PrecData<float> &D = P.f;
  auto &cf = P.coupling_f;
  auto &cs = P.coupling_fs;
  const Csr<double> *src[4] = {&S.Acf, &S.Afc, &S.AfcT, &S.AcfT};
  bool rebuilt = false;
  for (int q = 0; q < (transpose ? 4 : 2); ++q) {
    if (cf[q].rows != src[q]->rows || cf[q].nnz != src[q]->nnz) {
      if (scr)
        fail(EDFA_ERR_ARG, "the FP32 coupling blocks do not exist yet: build them with one "
                           "edfa_apply (of the same transpose) first");
      to_fp32(*src[q], cf[q], s);
      build_sell(cf[q], cs[q], S.tmp, s);
      rebuilt = true;
    }
  }
  if (rebuilt) apply_tuned(P);
  const int n = S.n;
  float *rin, *zf;
  ApplyWork<float> W;
  if (scr) {
    W = carve_work<float>(C, S.nfu, S.ne);
    rin = C.take<float>(n);
    zf = C.take<float>(n);
  } else {
    W = handle_work(D, S.nfu, S.ne);
    rin = P.rin_f.ensure(n);
    zf = D.z.ensure(n);
  }
  if (!transpose && P.prm.schur_solver == EDFA_SCHUR_ISAI && P.prm.isai_steps <= 1) {
    apply_fp32_direct(P, D, W, r, z, cs[0], cs[1], s, fm, cm);
    return;
  }
  hipLaunchKernelGGL((k_convert<double, float>), dim3(ceil_div(n, 256)), dim3(256), 0, s, r,
                     (long long)n, rin, mask);
  EDFA_CHECK_LAUNCH();
  apply_typed<float>(P, D, W, rin, zf, transpose ? cs[2] : cs[0], transpose ? cs[3] : cs[1],
                     transpose, s, fm, cm);
  hipLaunchKernelGGL((k_convert<float, double>), dim3(ceil_div(n, 256)), dim3(256), 0, s, zf,
                     (long long)n, z, mask);
  EDFA_CHECK_LAUNCH();
}

void precond_apply(edfa_precond_s &P, int transpose, const double *r, double *z, hipStream_t s,
                   RowMask mask) {
  apply_impl(P, transpose, r, z, s, mask, nullptr);
}

void precond_apply_noalloc(edfa_precond_s &P, int transpose, const double *r, double *z,
                           hipStream_t s) {
  const size_t need = scratch_need(P);
  if (need > SCRATCH_BYTES)
    fail(EDFA_ERR_ARG,
         "the allocation-free application needs %zu bytes of workspace for this system "
         "(2 N_f^u + 5 N_e preconditioner values, plus 2 N floats in FP32); its static "
         "array holds %zu",
         need, SCRATCH_BYTES);
  if (layouts_pending(P))
    fail(EDFA_ERR_ARG, "a product kernel chosen by the tuner needs its chunk descriptors or SELL "
                       "layout: build them with one edfa_apply (or solve) first");
  apply_impl(P, transpose, r, z, s, RowMask{}, scratch_ptr());
}

}  // namespace edfa
