// extern "C" entry points of libedfa: argument checks, error translation, dispatch.
#include <cstdarg>

#include "precond.hpp"
#include "system.hpp"

namespace edfa {

static thread_local std::string g_last_error;

void set_last_error(const std::string &msg) { g_last_error = msg; }

void fail(edfa_status st, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Error{st, std::string(buf)};
}

void assemble_system(edfa_system_s &S, const edfa_problem *probs, int count, hipStream_t s);
void update_dt(edfa_system_s &S, double dt, const double *p_prev, hipStream_t s);

template <class F>
static edfa_status guard(F &&f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const Error &e) {
    g_last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return EDFA_ERR_NOMEM;
  } catch (const std::exception &e) {
    g_last_error = e.what();
    return EDFA_ERR_ARG;
  }
}

static void ensure_transposes(edfa_system_s &S, hipStream_t s) {
  if (S.AT.rows == 0 && S.n > 0) csr_transpose(S.A, S.AT, S.tmp, S.tmp2, s);
  if (S.AcfT.rows == 0 && S.nfu > 0) csr_transpose(S.Acf, S.AcfT, S.tmp, S.tmp2, s);
}

}  // namespace edfa

using namespace edfa;

extern "C" {

const char *edfa_last_error(void) { return g_last_error.c_str(); }

edfa_status edfa_assemble(const edfa_problem *grids, int32_t count, hipStream_t stream,
                          edfa_system *out) {
  return guard([&] {
    if (!out) fail(EDFA_ERR_ARG, "out is NULL");
    *out = nullptr;
    auto *S = new edfa_system_s();
    try {
      assemble_system(*S, grids, count, stream);
    } catch (...) {
      delete S;
      throw;
    }
    *out = S;
    return EDFA_OK;
  });
}

void edfa_system_destroy(edfa_system sys) { delete sys; }

edfa_status edfa_system_get_info(edfa_system sys, edfa_system_info *info) {
  return guard([&] {
    if (!sys || !info) fail(EDFA_ERR_ARG, "NULL argument");
    info->n_grids = sys->ngrid;
    info->n_cells = sys->ne;
    info->n_faces = sys->nf;
    info->n_face_unknowns = sys->nfu;
    info->n = sys->n;
    info->axis_structure = sys->axis;
    info->nnz = sys->A.nnz;
    info->nnz_block[0] = sys->Afp.nnz;
    info->nnz_block[1] = sys->Afc.nnz;
    info->nnz_block[2] = sys->Acf.nnz;
    info->nnz_block[3] = sys->Acc.nnz;
    return EDFA_OK;
  });
}

edfa_status edfa_update_dt(edfa_system sys, double dt, const double *p_prev, hipStream_t stream) {
  return guard([&] {
    if (!sys) fail(EDFA_ERR_ARG, "NULL system");
    update_dt(*sys, dt, p_prev, stream);
    return EDFA_OK;
  });
}

edfa_status edfa_export_block(edfa_system sys, int32_t block, int32_t *rowptr, int32_t *col,
                              double *val, hipStream_t stream) {
  return guard([&] {
    if (!sys) fail(EDFA_ERR_ARG, "NULL system");
    const Csr<double> *M = nullptr;
    switch (block) {
      case 0: M = &sys->Afp; break;
      case 1: M = &sys->Afc; break;
      case 2: M = &sys->Acf; break;
      case 3: M = &sys->Acc; break;
      case 4: M = &sys->A; break;
      default: fail(EDFA_ERR_ARG, "block must be 0..4");
    }
    if (rowptr)
      EDFA_HIP(hipMemcpyAsync(rowptr, M->rowptr.p, sizeof(int) * ((size_t)M->rows + 1),
                              hipMemcpyDeviceToDevice, stream));
    if (col && M->nnz)
      EDFA_HIP(hipMemcpyAsync(col, M->col.p, sizeof(int) * M->nnz, hipMemcpyDeviceToDevice, stream));
    if (val && M->nnz)
      EDFA_HIP(hipMemcpyAsync(val, M->val.p, sizeof(double) * M->nnz, hipMemcpyDeviceToDevice, stream));
    return EDFA_OK;
  });
}

edfa_status edfa_export_rhs(edfa_system sys, double *b, double *W, double *vol, hipStream_t stream) {
  return guard([&] {
    if (!sys) fail(EDFA_ERR_ARG, "NULL system");
    if (b) EDFA_HIP(hipMemcpyAsync(b, sys->b.p, sizeof(double) * sys->n, hipMemcpyDeviceToDevice, stream));
    if (W)
      EDFA_HIP(hipMemcpyAsync(W, sys->W.p, sizeof(double) * 36 * (size_t)sys->ne,
                              hipMemcpyDeviceToDevice, stream));
    if (vol)
      EDFA_HIP(hipMemcpyAsync(vol, sys->vol.p, sizeof(double) * sys->ne, hipMemcpyDeviceToDevice, stream));
    return EDFA_OK;
  });
}

edfa_status edfa_spmv(edfa_system sys, int32_t transpose, const double *x, double *y,
                      hipStream_t stream) {
  return guard([&] {
    if (!sys || !x || !y) fail(EDFA_ERR_ARG, "NULL argument");
    if (transpose) {
      ensure_transposes(*sys, stream);
      if (sys->AT_s.rows == 0) build_sell(sys->AT, sys->AT_s, sys->tmp, stream);
    }
    spmv_sell<double, double>(transpose ? sys->AT_s : sys->A_s, x, y, 1.0, nullptr, 0.0, stream,
                              0.0, SPMV_OPERATOR);
    return EDFA_OK;
  });
}

}  // extern "C"

namespace edfa {
template <class T>
static const Csr<T> *precond_art(edfa_precond_s &P, PrecData<T> &D, int what, hipStream_t s) {
  switch (what) {
    case 0: return &D.G;
    case 1: return &D.FT;
    case 2:
      build_hraw(P, D, s);
      return &D.Hraw;
    case 3: return &D.H;
    case 4: return &D.S;
    case 5: return &D.GF;
    case 6: return &D.L;
    case 7: return &D.U;
    case 8: return &D.ML;
    case 9: return &D.MU;
    default: fail(EDFA_ERR_ARG, "unknown artefact %d", what);
  }
}

__global__ void k_f2d(const float *__restrict__ x, long long n, double *y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}

template <class T>
static void export_art(edfa_precond_s &P, PrecData<T> &D, int what, int32_t *rowptr, int32_t *col,
                       double *val, int32_t *perm, int64_t *nnz, int32_t *rows, hipStream_t s) {
  const Csr<T> *M = precond_art(P, D, what, s);
  if ((what == 8 || what == 9) && P.prm.schur_solver != EDFA_SCHUR_ISAI)
    fail(EDFA_ERR_ARG, "no sparse approximate inverses with the exact substitution solver");
  if (nnz) *nnz = M->nnz;
  if (rows) *rows = M->rows;
  if (!rowptr) return;
  EDFA_HIP(hipMemcpyAsync(rowptr, M->rowptr.p, sizeof(int) * ((size_t)M->rows + 1),
                          hipMemcpyDeviceToDevice, s));
  if (M->nnz) {
    if (col) EDFA_HIP(hipMemcpyAsync(col, M->col.p, sizeof(int) * M->nnz, hipMemcpyDeviceToDevice, s));
    if (val) {
      if (sizeof(T) == sizeof(double))
        EDFA_HIP(hipMemcpyAsync(val, M->val.p, sizeof(double) * M->nnz, hipMemcpyDeviceToDevice, s));
      else
        hipLaunchKernelGGL(k_f2d, dim3(ceil_div(M->nnz, 256)), dim3(256), 0, s,
                           (const float *)M->val.p, (long long)M->nnz, val);
    }
  }
  if (perm && what >= 6)
    EDFA_HIP(hipMemcpyAsync(perm, D.perm.p, sizeof(int) * P.sys->ne, hipMemcpyDeviceToDevice, s));
  EDFA_HIP(hipStreamSynchronize(s));
}

template <class T>
static void fill_info(edfa_precond_s &P, PrecData<T> &D, edfa_precond_info *info) {
  edfa_system_s &S = *P.sys;
  info->nnz_G = D.G.nnz;
  info->nnz_F = D.FT.nnz;
  info->nnz_H = D.H.nnz;
  info->nnz_S = D.S.nnz;
  info->nnz_GF = D.GF.nnz;
  info->nnz_L = D.L.nnz;
  info->nnz_U = D.U.nnz;
  const bool isai = P.prm.schur_solver == EDFA_SCHUR_ISAI;
  info->nnz_ML = isai ? D.ML.nnz : 0;
  info->nnz_MU = isai ? D.MU.nnz : 0;
  info->n_colors = P.n_colors;
  info->max_pattern = P.max_pattern;
  // mu of Section 4 with nnz() counting what the application stores and reads: G_F and
  // G_F^T for A~_pipi^-1, the coupling blocks, and for S~^-1 the approximate inverses M_L,
  // M_U (plus L and U when refinement steps multiply by them) or L and U (substitution)
  const double den = (double)(S.Afp.nnz + S.Afc.nnz + S.Acf.nnz + S.Acc.nnz);
  double ns = (double)(D.L.nnz + D.U.nnz);
  if (isai) ns = (double)(D.ML.nnz + D.MU.nnz) + (P.prm.isai_steps > 1 ? ns : 0.0);
  const double num = 2.0 * D.GF.nnz + S.Afc.nnz + S.Acf.nnz + ns;
  info->mu = den > 0 ? num / den : 0.0;
  info->t_stage1_ms = P.t_stage1_ms;
  info->t_stage2_ms = P.t_stage2_ms;
  info->nnz_H_raw = P.nnz_h_raw.p ? (int64_t)*P.nnz_h_raw.p : 0;
  info->htilde_retry_rows = P.htilde_retry_rows;
  info->color_rounds = P.color_rounds;
  info->color_list_rounds = P.color_list_rounds;
  info->cgs2_width = P.cgs2_width;
  info->chunks_ML = D.ML_s.chunk_k == CHUNK_K ? D.ML_s.nchunk : 0;
  info->chunks_MU = D.MU_s.chunk_k == CHUNK_K ? D.MU_s.nchunk : 0;
}

void check_params(const edfa_params &p) {
  const edfa_params *prm = &p;
  if (prm->variant != EDFA_STATIC && prm->variant != EDFA_DYNAMIC)
    fail(EDFA_ERR_ARG, "variant must be EDFA_STATIC or EDFA_DYNAMIC");
  if (prm->variant == EDFA_DYNAMIC && (prm->n_add < 1 || prm->n_ent < 0))
    fail(EDFA_ERR_ARG, "dynamic variant needs n_add >= 1 and n_ent >= 0");
  if (prm->filt_mode < EDFA_FILT_NONE || prm->filt_mode > EDFA_FILT_POST_H)
    fail(EDFA_ERR_ARG, "filt_mode out of range");
  if (prm->filt_mode != EDFA_FILT_NONE && !(prm->tau_filt >= 0.0))
    fail(EDFA_ERR_ARG, "tau_filt must be >= 0");
  if (prm->precision != 0 && prm->precision != 1) fail(EDFA_ERR_ARG, "precision must be 0 or 1");
  if (prm->schur_solver != EDFA_SCHUR_ISAI && prm->schur_solver != EDFA_SCHUR_EXACT)
    fail(EDFA_ERR_ARG, "schur_solver out of range");
  if (prm->isai_steps < 1) fail(EDFA_ERR_ARG, "isai_steps must be >= 1");
  if (prm->static_axis < 0 || prm->static_axis > 4) fail(EDFA_ERR_ARG, "static_axis must be 0..4");
  if (prm->htilde_retry < 0 || prm->htilde_retry > 256)
    fail(EDFA_ERR_ARG, "htilde_retry must be in 0..256");
}
}  // namespace edfa

extern "C" {

edfa_status edfa_setup(edfa_system sys, const edfa_params *prm, hipStream_t stream,
                       edfa_precond *out) {
  return guard([&] {
    if (!sys || !prm || !out) fail(EDFA_ERR_ARG, "NULL argument");
    *out = nullptr;
    check_params(*prm);
    auto *P = new edfa_precond_s();
    P->sys = sys;
    P->prm = *prm;
    try {
      EventTimer t1, t2;
      t1.start(stream);
      precond_stage1(*P, stream);
      t1.stop(stream);
      P->t_stage1_ms = t1.ms();
      t2.start(stream);
      precond_stage2(*P, stream);
      t2.stop(stream);
      P->t_stage2_ms = t2.ms();
    } catch (...) {
      delete P;
      throw;
    }
    *out = P;
    return EDFA_OK;
  });
}

edfa_status edfa_setup_stage2(edfa_precond pre, hipStream_t stream) {
  return guard([&] {
    if (!pre) fail(EDFA_ERR_ARG, "NULL preconditioner");
    EventTimer t2;
    t2.start(stream);
    precond_stage2(*pre, stream);
    t2.stop(stream);
    pre->t_stage2_ms = t2.ms();
    return EDFA_OK;
  });
}

edfa_status edfa_resetup(edfa_precond pre, hipStream_t stream) {
  return guard([&] {
    if (!pre) fail(EDFA_ERR_ARG, "NULL preconditioner");
    EventTimer t1, t2;
    t1.start(stream);
    precond_stage1(*pre, stream);
    t1.stop(stream);
    pre->t_stage1_ms = t1.ms();
    t2.start(stream);
    precond_stage2(*pre, stream);
    t2.stop(stream);
    pre->t_stage2_ms = t2.ms();
    return EDFA_OK;
  });
}

void edfa_precond_destroy(edfa_precond pre) { delete pre; }

edfa_status edfa_precond_get_info(edfa_precond pre, edfa_precond_info *info) {
  return guard([&] {
    if (!pre || !info) fail(EDFA_ERR_ARG, "NULL argument");
    if (pre->prm.precision == 1)
      fill_info(*pre, pre->f, info);
    else
      fill_info(*pre, pre->d, info);
    return EDFA_OK;
  });
}

edfa_status edfa_export_precond(edfa_precond pre, int32_t what, int32_t *rowptr, int32_t *col,
                                double *val, int32_t *perm, int64_t *nnz, int32_t *rows,
                                hipStream_t stream) {
  return guard([&] {
    if (!pre) fail(EDFA_ERR_ARG, "NULL preconditioner");
    if (pre->prm.precision == 1)
      export_art(*pre, pre->f, what, rowptr, col, val, perm, nnz, rows, stream);
    else
      export_art(*pre, pre->d, what, rowptr, col, val, perm, nnz, rows, stream);
    return EDFA_OK;
  });
}

edfa_status edfa_apply(edfa_precond pre, int32_t transpose, const double *r, double *z,
                       hipStream_t stream) {
  return guard([&] {
    if (!pre || !r || !z) fail(EDFA_ERR_ARG, "NULL argument");
    if (r == z) fail(EDFA_ERR_ARG, "r and z must not alias");
    precond_apply(*pre, transpose ? 1 : 0, r, z, stream);
    return EDFA_OK;
  });
}

edfa_status edfa_apply_noalloc(edfa_precond pre, int32_t transpose, const double *r, double *z,
                               hipStream_t stream) {
  return guard([&] {
    if (!pre || !r || !z) fail(EDFA_ERR_ARG, "NULL argument");
    if (r == z) fail(EDFA_ERR_ARG, "r and z must not alias");
    precond_apply_noalloc(*pre, transpose ? 1 : 0, r, z, stream);
    return EDFA_OK;
  });
}

edfa_status edfa_solve(edfa_system sys, edfa_precond pre, const double *b, double *x,
                       const edfa_solve_params *prm, hipStream_t stream, edfa_solve_info *info) {
  return guard([&] {
    if (!sys || !pre || !b || !x || !prm) fail(EDFA_ERR_ARG, "NULL argument");
    if (pre->sys != sys) fail(EDFA_ERR_ARG, "preconditioner built for another system");
    if (b == x) fail(EDFA_ERR_ARG, "b and x must not alias");
    if (prm->max_iter < 1) fail(EDFA_ERR_ARG, "max_iter must be >= 1");
    if (prm->method == EDFA_BICGSTAB) return bicgstab(*sys, *pre, b, x, *prm, stream, info);
    if (prm->method != EDFA_GMRES) fail(EDFA_ERR_ARG, "method must be EDFA_GMRES or EDFA_BICGSTAB");
    return gmres(*sys, *pre, b, x, *prm, stream, info);
  });
}

edfa_status edfa_transient(edfa_system sys, edfa_precond pre, const edfa_transient_params *prm,
                           double *u, hipStream_t stream, edfa_step_info *steps, int32_t *taken) {
  return guard([&] {
    if (!sys || !pre || !prm || !u) fail(EDFA_ERR_ARG, "NULL argument");
    int k = 0;
    const edfa_status st = transient(*sys, *pre, *prm, u, stream, steps, &k);
    if (taken) *taken = k;
    return st;
  });
}

edfa_status edfa_tune_params(edfa_system sys, const edfa_params *cand, int32_t ncand,
                             const edfa_solve_params *solve, hipStream_t stream, int32_t *best,
                             double *times_ms, int32_t *iterations, int32_t *status) {
  return guard([&] {
    if (!sys || !cand || !solve || !best) fail(EDFA_ERR_ARG, "NULL argument");
    if (ncand < 1) fail(EDFA_ERR_ARG, "need at least one candidate");
    if (solve->max_iter < 1 || !(solve->rtol > 0.0)) fail(EDFA_ERR_ARG, "bad solve parameters");
    for (int c = 0; c < ncand; ++c) check_params(cand[c]);
    *best = tune_params(*sys, cand, ncand, *solve, stream, times_ms, iterations, status);
    if (*best < 0) fail(EDFA_ERR_BREAKDOWN, "no candidate converged");
    return EDFA_OK;
  });
}

edfa_status edfa_autotune(edfa_precond pre, hipStream_t stream, int32_t *tuned,
                          edfa_tune_slot *slots) {
  return guard([&] {
    if (!pre) fail(EDFA_ERR_ARG, "NULL preconditioner");
    const int n = autotune(*pre, stream, slots);
    if (tuned) *tuned = n;
    return EDFA_OK;
  });
}

edfa_status edfa_autotune_setup(edfa_precond pre, hipStream_t stream, edfa_setup_tune *report) {
  return guard([&] {
    if (!pre) fail(EDFA_ERR_ARG, "NULL preconditioner");
    tune_setup(*pre, stream, report);
    return EDFA_OK;
  });
}

edfa_status edfa_set_variant(edfa_precond pre, int32_t slot, int32_t variant) {
  return guard([&] {
    if (!pre) fail(EDFA_ERR_ARG, "NULL preconditioner");
    if (slot < -1 || slot >= EDFA_TUNE_SLOTS) fail(EDFA_ERR_ARG, "slot %d out of range", slot);
    if (variant < -1 || variant >= EDFA_TUNE_VARIANTS)
      fail(EDFA_ERR_ARG, "variant %d out of range", variant);
    set_variant(*pre, slot, variant);
    return EDFA_OK;
  });
}

edfa_status edfa_grad_logk(edfa_system sys, const double *u, const double *lambda, double *g,
                           hipStream_t stream) {
  return guard([&] {
    if (!sys || !u || !lambda || !g) fail(EDFA_ERR_ARG, "NULL argument");
    grad_logk(*sys, u, lambda, g, stream);
    return EDFA_OK;
  });
}

}  // extern "C"
