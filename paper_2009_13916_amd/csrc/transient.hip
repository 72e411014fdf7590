// Transient sequence with adaptive time steps (Section 4): per step, A_pp and f_p follow
// (dt, p_prev), stage 2 of the preconditioner is rebuilt on the recycled stage 1 (stage 1
// depends only on A_pipi, A_pip and A_ppi; Section 3, implementation details), the system
// is solved from x0 = 0, and the step size follows eq. delta_t_dyn,
//   dt_{n+1} = min(dt_n min(dt_mult, dp_T / dp_max), dt_max),
// with dp_max the largest absolute pressure change of the step.  Each step also reports the
// largest Courant number of eq. CFL_number, chi^E = Q^E dt / (Omega^E phi), where Q^E is
// half the absolute sum of the element's outward face fluxes q^E = W^E (p^E 1 - pi^E).
#include <cmath>
#include <cstring>

#include "precond.hpp"

namespace edfa {

void update_dt(edfa_system_s &S, double dt, const double *p_prev, hipStream_t s);

namespace {

// Non-negative doubles order as their bit patterns: the maximum by an integer atomic.
__device__ inline void atomic_max_nonneg(unsigned long long *dst, double v) {
  atomicMax(dst, (unsigned long long)__double_as_longlong(v));
}

// out[0] = max_E |p^E - p_prev^E|, out[1] = max_E chi^E (both >= 0)
__global__ __launch_bounds__(256) void k_step_measures(
    const GridDesc *__restrict__ grids, int ngrid, int ne, int nfu, const double *__restrict__ u,
    const double *__restrict__ p_prev, const double *__restrict__ W,
    const double *__restrict__ vol, const int *__restrict__ uidx, const double *__restrict__ bcv,
    double dt, double porosity, unsigned long long *out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double dp = 0.0, chi = 0.0;
  if (e < ne) {
    const GridDesc &G = grids[grid_of(grids, ngrid, e, true)];
    int i, j, k;
    cell_ijk(G, e, i, j, k);
    const double p = u[nfu + e];
    dp = fabs(p - p_prev[e]);
    double d[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const int f = cell_face(G, i, j, k, a);
      const int q = uidx[f];
      d[a] = p - (q >= 0 ? u[q] : bcv[f]);
    }
    const double *We = W + 36 * (size_t)e;
    double Q = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      double qa = 0.0;
#pragma unroll
      for (int b = 0; b < 6; ++b) qa += We[6 * a + b] * d[b];
      Q += fabs(qa);
    }
    chi = 0.5 * Q * dt / (vol[e] * porosity);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    dp = fmax(dp, __shfl_xor(dp, o));
    chi = fmax(chi, __shfl_xor(chi, o));
  }
  if ((threadIdx.x & 63) == 0) {
    atomic_max_nonneg(out, dp);
    atomic_max_nonneg(out + 1, chi);
  }
}

}  // namespace

edfa_status transient(edfa_system_s &S, edfa_precond_s &P, const edfa_transient_params &prm,
                      double *u, hipStream_t s, edfa_step_info *steps, int *taken) {
  if (prm.n_steps < 1) fail(EDFA_ERR_ARG, "n_steps must be >= 1");
  if (!(prm.dt0 > 0.0) || !(prm.dt_max > 0.0)) fail(EDFA_ERR_ARG, "dt0 and dt_max must be > 0");
  if (!(prm.dt_mult >= 1.0)) fail(EDFA_ERR_ARG, "dt_mult must be >= 1");
  if (!(prm.dp_target > 0.0)) fail(EDFA_ERR_ARG, "dp_target must be > 0 (infinity: no goal)");
  if (!(prm.porosity > 0.0)) fail(EDFA_ERR_ARG, "porosity must be > 0");
  if (prm.stage1_every < 0) fail(EDFA_ERR_ARG, "stage1_every must be >= 0");
  if (P.sys != &S) fail(EDFA_ERR_ARG, "preconditioner built for another system");
  DBuf<unsigned long long> meas;
  meas.ensure(2);
  double dt = prm.dt0, t = 0.0;
  edfa_status last = EDFA_OK;
  int k = 0;
  for (; k < prm.n_steps; ++k) {
    update_dt(S, dt, k == 0 ? nullptr : u + S.nfu, s);
    EventTimer ts, tv;
    ts.start(s);
    if (prm.stage1_every > 0 && k % prm.stage1_every == 0)
      precond_stage1(P, s);
    precond_stage2(P, s);
    ts.stop(s);
    tv.start(s);
    edfa_solve_info si{};
    last = prm.solve.method == EDFA_BICGSTAB ? bicgstab(S, P, S.b.p, u, prm.solve, s, &si)
                                             : gmres(S, P, S.b.p, u, prm.solve, s, &si);
    tv.stop(s);
    EDFA_HIP(hipMemsetAsync(meas.p, 0, 2 * sizeof(unsigned long long), s));
    if (S.ne) {
      hipLaunchKernelGGL(k_step_measures, dim3(ceil_div(S.ne, 256)), dim3(256), 0, s, S.grids.p,
                         S.ngrid, S.ne, S.nfu, u, S.p_prev.p, S.W.p, S.vol.p, S.uidx.p, S.bcv.p,
                         dt, prm.porosity, meas.p);
      EDFA_CHECK_LAUNCH();
    }
    unsigned long long mh[2];
    read_small(mh, meas.p, 2, s);
    double dp, chi;
    memcpy(&dp, &mh[0], sizeof(double));
    memcpy(&chi, &mh[1], sizeof(double));
    t += dt;
    if (steps) {
      edfa_step_info &r = steps[k];
      r = edfa_step_info{};
      r.t = t;
      r.dt = dt;
      r.dp_max = dp;
      r.chi_inf = chi;
      r.converged = last == EDFA_OK ? 1 : 0;
      r.t_setup_ms = ts.ms();
      r.t_solve_ms = tv.ms();
      r.iterations = si.iterations;
    }
    if (last != EDFA_OK || (prm.t_end > 0.0 && t >= prm.t_end)) {
      ++k;
      break;
    }
    // eq. delta_t_dyn
    const double grow = dp > 0.0 ? std::min(prm.dt_mult, prm.dp_target / dp) : prm.dt_mult;
    dt = std::min(dt * grow, prm.dt_max);
  }
  if (taken) *taken = k;
  return last;
}

}  // namespace edfa
