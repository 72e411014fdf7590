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
  if (S.AT.rows == 0 && S.n > 0) csr_transpose(S.A, S.AT, S.tmp, s);
  if (S.AcfT.rows == 0 && S.nfu > 0) csr_transpose(S.Acf, S.AcfT, S.tmp, s);
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
      spmv<double, double>(sys->AT.rowptr.p, sys->AT.col.p, sys->AT.val.p, sys->n, x, y, 1.0,
                           nullptr, 0.0, sys->avg_A, stream);
    } else {
      spmv<double, double>(sys->A.rowptr.p, sys->A.col.p, sys->A.val.p, sys->n, x, y, 1.0,
                           nullptr, 0.0, sys->avg_A, stream);
    }
    return EDFA_OK;
  });
}

}  // extern "C"
