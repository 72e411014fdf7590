// Right-preconditioned Bi-CGStab, the paper's outer solver (Section 4, after van der Vorst
// 1992): x0 = 0, exit when ||r_k|| <= tol ||r_0||, an iteration cap ("NC" past it).
//
//   rho = (r^, r); beta = (rho / rho_old)(alpha / omega)
//   p = r + beta (p - omega v);  p^ = P^-1 p;  v = A p^;  alpha = rho / (r^, v)
//   s = r - alpha v                       (converged at the half step: x += alpha p^)
//   s^ = P^-1 s;  t = A s^;  omega = (t, s) / (t, t)
//   x += alpha p^ + omega s^;  r = s - omega t
//
// Every grid of a batch ("segment") keeps its own scalars and convergence state; vector
// kernels run over the chunks of the GMRES solver (never straddling a grid), their dot
// products are summed per chunk and then per segment in a fixed order (deterministic), and
// the products skip the rows of segments that have stopped.  When every segment has
// stopped, the true FP64 residual b - A x confirms convergence; a segment whose recurrence
// drifted past the target or broke down (rho, (r^, v) or omega zero) restarts from its
// current iterate with r^ = r.
#include <cmath>

#include "precond.hpp"

namespace edfa {

namespace {

constexpr int BT = 256;
constexpr int BI_CHECK = 4;   // iterations between host reads of the segment states

// p = r + beta (p - omega v); first iteration after a (re)start: p = r
__global__ __launch_bounds__(BT) void k_bi_p(const double *__restrict__ r, double *p,
                                             const double *__restrict__ v,
                                             const Chunk *__restrict__ ch,
                                             const BiSeg *__restrict__ st) {
  const Chunk c = ch[blockIdx.x];
  const BiSeg S = st[c.seg];
  if (!S.active) return;
#pragma unroll
  for (int k = 0; k < SOLVE_CHUNK / BT; ++k) {
    const int e = c.start + threadIdx.x + k * BT;
    if (e < c.end) p[e] = S.first ? r[e] : r[e] + S.beta * (p[e] - S.omega * v[e]);
  }
}

// Per-chunk partial sums of NC dot products a_i . b_i into part[chunk * ld + i].
template <int NC>
__device__ void chunk_dots(const double (&s)[NC], const Chunk &c, double *part, int ld) {
  __shared__ double red[BT / 64][NC];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    double x = s[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0) red[wv][i] = x;
  }
  __syncthreads();
  if (threadIdx.x < NC)
    part[(long long)blockIdx.x * ld + threadIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

// (r^, v)
__global__ __launch_bounds__(BT) void k_bi_dot_rv(const double *__restrict__ rh,
                                                  const double *__restrict__ v,
                                                  const Chunk *__restrict__ ch,
                                                  const BiSeg *__restrict__ st, double *part,
                                                  int ld) {
  const Chunk c = ch[blockIdx.x];
  if (!st[c.seg].active) return;
  double s[1] = {0.0};
#pragma unroll
  for (int k = 0; k < SOLVE_CHUNK / BT; ++k) {
    const int e = c.start + threadIdx.x + k * BT;
    if (e < c.end) s[0] += rh[e] * v[e];
  }
  chunk_dots<1>(s, c, part, ld);
}

// s = r - alpha v, partial (s, s)
__global__ __launch_bounds__(BT) void k_bi_s(const double *__restrict__ r,
                                             const double *__restrict__ v, double *sv,
                                             const Chunk *__restrict__ ch,
                                             const BiSeg *__restrict__ st, double *part, int ld) {
  const Chunk c = ch[blockIdx.x];
  const BiSeg S = st[c.seg];
  if (!S.active) return;
  double q[1] = {0.0};
#pragma unroll
  for (int k = 0; k < SOLVE_CHUNK / BT; ++k) {
    const int e = c.start + threadIdx.x + k * BT;
    if (e < c.end) {
      const double x = r[e] - S.alpha * v[e];
      sv[e] = x;
      q[0] += x * x;
    }
  }
  chunk_dots<1>(q, c, part, ld);
}

// (t, s), (t, t)
__global__ __launch_bounds__(BT) void k_bi_dot_ts(const double *__restrict__ t,
                                                  const double *__restrict__ sv,
                                                  const Chunk *__restrict__ ch,
                                                  const BiSeg *__restrict__ st, double *part,
                                                  int ld) {
  const Chunk c = ch[blockIdx.x];
  if (!st[c.seg].active) return;
  double q[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < SOLVE_CHUNK / BT; ++k) {
    const int e = c.start + threadIdx.x + k * BT;
    if (e < c.end) {
      q[0] += t[e] * sv[e];
      q[1] += t[e] * t[e];
    }
  }
  chunk_dots<2>(q, c, part, ld);
}

// x += alpha p^ + omega s^, r = s - omega t (half step: x += alpha p^, r = s);
// partial (r^, r), (r, r)
__global__ __launch_bounds__(BT) void k_bi_update(double *x, double *r,
                                                  const double *__restrict__ rh,
                                                  const double *__restrict__ ph,
                                                  const double *__restrict__ sh,
                                                  const double *__restrict__ sv,
                                                  const double *__restrict__ t,
                                                  const Chunk *__restrict__ ch,
                                                  const BiSeg *__restrict__ st, double *part,
                                                  int ld) {
  const Chunk c = ch[blockIdx.x];
  const BiSeg S = st[c.seg];
  if (!S.active) return;
  double q[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < SOLVE_CHUNK / BT; ++k) {
    const int e = c.start + threadIdx.x + k * BT;
    if (e < c.end) {
      double rn;
      if (S.half) {
        x[e] += S.alpha * ph[e];
        rn = sv[e];
      } else {
        x[e] += S.alpha * ph[e] + S.omega * sh[e];
        rn = sv[e] - S.omega * t[e];
      }
      r[e] = rn;
      q[0] += rh[e] * rn;
      q[1] += rn * rn;
    }
  }
  chunk_dots<2>(q, c, part, ld);
}

// r^ = r on the segments that (re)start
__global__ __launch_bounds__(BT) void k_bi_copy_active(const double *__restrict__ r, double *rh,
                                                       const Chunk *__restrict__ ch,
                                                       const BiSeg *__restrict__ st) {
  const Chunk c = ch[blockIdx.x];
  if (!st[c.seg].active) return;
#pragma unroll
  for (int k = 0; k < SOLVE_CHUNK / BT; ++k) {
    const int e = c.start + threadIdx.x + k * BT;
    if (e < c.end) rh[e] = r[e];
  }
}

enum { STEP_START = 0, STEP_RESTART, STEP_ALPHA, STEP_HALF, STEP_OMEGA, STEP_END };

// One block per segment: sum the NC chunk partials of the segment (thread-strided, then a
// fixed tree), then take the scalar step.  STEP_START / STEP_RESTART read ||r||^2.
template <int NC>
__global__ __launch_bounds__(BT) void k_bi_reduce_step(const double *__restrict__ part, int ld,
                                                       const int *__restrict__ segptr,
                                                       BiSeg *st, int step, double rtol,
                                                       int max_iter) {
  __shared__ double red[BT][NC];
  const int g = blockIdx.x;
  BiSeg S = st[g];
  const bool starting = step == STEP_START || step == STEP_RESTART;
  if (!starting && !S.active) return;
  if (step == STEP_RESTART && S.done) return;
  const int c0 = segptr[g], c1 = segptr[g + 1];
  double acc[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) acc[i] = 0.0;
  for (int c = c0 + (int)threadIdx.x; c < c1; c += BT)
#pragma unroll
    for (int i = 0; i < NC; ++i) acc[i] += part[(long long)c * ld + i];
#pragma unroll
  for (int i = 0; i < NC; ++i) red[threadIdx.x][i] = acc[i];
  __syncthreads();
  for (int h = BT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
#pragma unroll
      for (int i = 0; i < NC; ++i) red[threadIdx.x][i] += red[threadIdx.x + h][i];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double d0 = red[0][0], d1 = NC > 1 ? red[0][NC > 1 ? 1 : 0] : 0.0;
  switch (step) {
    case STEP_START:
    case STEP_RESTART: {
      const double rn = sqrt(d0);
      if (step == STEP_START) {
        S = BiSeg{};
        S.bnorm = rn;
        S.tol = rtol * rn;
      }
      S.rnorm = rn;
      S.relres = S.bnorm > 0 ? rn / S.bnorm : 0.0;
      S.active = 0;
      S.half = 0;
      S.breakdown = 0;
      if (!(rn > S.tol)) {
        S.done = 1;
        S.converged = isfinite(rn) ? 1 : 0;
      } else if (S.total >= max_iter || !isfinite(rn)) {
        S.done = 1;
      } else {
        S.active = 1;
        S.first = 1;
        S.rho = d0;   // (r^, r) with r^ = r
        S.alpha = S.omega = 1.0;
        S.beta = 0.0;
      }
      break;
    }
    case STEP_ALPHA:
      if (d0 == 0.0 || !isfinite(d0)) {
        // the iteration counts, so repeated breakdowns end at the cap
        S.active = 0;
        S.breakdown = 1;
        S.total += 1;
      } else {
        S.alpha = S.rho / d0;
      }
      break;
    case STEP_HALF:
      S.half = sqrt(d0) <= S.tol ? 1 : 0;
      break;
    case STEP_OMEGA:
      S.omega = d1 > 0 ? d0 / d1 : 0.0;
      break;
    case STEP_END: {
      S.total += 1;
      S.first = 0;
      S.rnorm = sqrt(d1);
      if (S.half || S.rnorm <= S.tol) {
        S.active = 0;
      } else if (S.omega == 0.0 || d0 == 0.0 || !isfinite(d0) || !isfinite(S.rnorm)) {
        S.active = 0;
        S.breakdown = 1;
      } else if (S.total >= max_iter) {
        S.active = 0;
      } else {
        S.beta = (d0 / S.rho) * (S.alpha / S.omega);
        S.rho = d0;
      }
      S.half = 0;
      break;
    }
    default: break;
  }
  st[g] = S;
}

// partial ||r||^2 (segments not done)
__global__ __launch_bounds__(BT) void k_bi_nrm(const double *__restrict__ r,
                                               const Chunk *__restrict__ ch, double *part,
                                               int ld) {
  const Chunk c = ch[blockIdx.x];
  double q[1] = {0.0};
#pragma unroll
  for (int k = 0; k < SOLVE_CHUNK / BT; ++k) {
    const int e = c.start + threadIdx.x + k * BT;
    if (e < c.end) q[0] += r[e] * r[e];
  }
  chunk_dots<1>(q, c, part, ld);
}

}  // namespace

edfa_status bicgstab(edfa_system_s &S, edfa_precond_s &P, const double *b, double *x,
                     const edfa_solve_params &prm, hipStream_t s, edfa_solve_info *info) {
  if (!(prm.rtol > 0.0)) fail(EDFA_ERR_ARG, "rtol must be > 0");
  if (prm.use_graph) fail(EDFA_ERR_ARG, "graph-captured cycles are a GMRES option");
  if (!P.ws) P.ws.reset(new SolveWork());
  SolveWork &W = *P.ws;
  const int n = S.n, nseg = S.ngrid;
  const int tr = prm.transpose ? 1 : 0;
  build_chunks(S, W, s);
  const int nch = W.nchunk;
  constexpr int LD = 2;
  W.part.ensure((size_t)nch * LD);
  for (DBuf<double> *v : {&W.r, &W.rhat, &W.p, &W.v, &W.ph, &W.sv, &W.sh, &W.t}) v->ensure(n);
  W.bst.ensure(nseg);
  if (tr && S.AT.rows == 0) csr_transpose(S.A, S.AT, S.tmp, S.tmp2, s);
  if (tr && S.AT_s.rows == 0) build_sell(S.AT, S.AT_s, S.tmp, s);
  apply_tuned(P);
  const Sell<double> &A = tr ? S.AT_s : S.A_s;

  std::vector<hipEvent_t> evs;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_spmv, ev_apply;
  auto ev = [&]() {
    hipEvent_t e;
    EDFA_HIP(hipEventCreate(&e));
    evs.push_back(e);
    return e;
  };
  struct EvFree {
    std::vector<hipEvent_t> &v;
    ~EvFree() {
      for (auto e : v) (void)hipEventDestroy(e);
    }
  } evfree{evs};
  RowMask live;
  if (nseg > 1) {
    if (S.rowseg.n < (size_t)n) fail(EDFA_ERR_ARG, "batch without its row-to-grid map");
    live = RowMask{S.rowseg.p, &W.bst.p->active, (int)(sizeof(BiSeg) / sizeof(int))};
  }
  auto spmvA = [&](const double *in, double *out, const double *bb, RowMask mk) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prm.profile) {
      e0 = ev();
      e1 = ev();
      ev_spmv.emplace_back(e0, e1);
    }
    spmv_sell<double, double>(A, in, out, bb ? -1.0 : 1.0, bb, 1.0, s, 0.0, SPMV_OPERATOR, e0, e1,
                              mk);
  };
  ProdProfile pp;
  auto applyP = [&](const double *in, double *out) {
    hipEvent_t e0{}, e1{};
    if (prm.profile) {
      e0 = ev();
      EDFA_HIP(hipEventRecord(e0, s));
      if (prm.profile >= 2) P.prof = &pp;
    }
    precond_apply(P, tr, in, out, s, live);
    P.prof = nullptr;
    if (prm.profile) {
      e1 = ev();
      EDFA_HIP(hipEventRecord(e1, s));
      ev_apply.emplace_back(e0, e1);
    }
  };
  auto reduce = [&](int nc, int step) {
    if (nc == 1)
      hipLaunchKernelGGL(k_bi_reduce_step<1>, dim3(nseg), dim3(BT), 0, s, W.part.p, LD, W.segptr.p,
                         W.bst.p, step, prm.rtol, prm.max_iter);
    else
      hipLaunchKernelGGL(k_bi_reduce_step<2>, dim3(nseg), dim3(BT), 0, s, W.part.p, LD, W.segptr.p,
                         W.bst.p, step, prm.rtol, prm.max_iter);
    EDFA_CHECK_LAUNCH();
  };
  std::vector<BiSeg> hst(nseg);
  auto read_states = [&]() {
    EDFA_HIP(hipMemcpyAsync(hst.data(), W.bst.p, sizeof(BiSeg) * nseg, hipMemcpyDeviceToHost, s));
    EDFA_HIP(hipStreamSynchronize(s));
    int a = 0;
    for (auto &q : hst) a += q.active;
    return a;
  };

  EventTimer total;
  total.start(s);
  // start: x = 0, r = b, r^ = r
  EDFA_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
  EDFA_HIP(hipMemcpyAsync(W.r.p, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_bi_nrm, dim3(nch), dim3(BT), 0, s, W.r.p, W.chunks.p, W.part.p, LD);
  EDFA_CHECK_LAUNCH();
  reduce(1, STEP_START);
  hipLaunchKernelGGL(k_bi_copy_active, dim3(nch), dim3(BT), 0, s, W.r.p, W.rhat.p, W.chunks.p,
                     W.bst.p);
  EDFA_CHECK_LAUNCH();
  int nact = read_states();
  for (int g = 0; g < nseg; ++g)
    if (!std::isfinite(hst[g].bnorm))
      fail(EDFA_ERR_NAN, "grid %d: the right-hand side has a non-finite entry", g);
  int starts = 1;
  while (true) {
    if (!nact) {
      // every segment stopped: confirm on the true residual, restart the others
      spmvA(x, W.r.p, b, RowMask{});
      hipLaunchKernelGGL(k_bi_nrm, dim3(nch), dim3(BT), 0, s, W.r.p, W.chunks.p, W.part.p, LD);
      EDFA_CHECK_LAUNCH();
      reduce(1, STEP_RESTART);
      hipLaunchKernelGGL(k_bi_copy_active, dim3(nch), dim3(BT), 0, s, W.r.p, W.rhat.p,
                         W.chunks.p, W.bst.p);
      EDFA_CHECK_LAUNCH();
      nact = read_states();
      if (!nact) break;
      ++starts;
    }
    for (int it = 0; it < BI_CHECK; ++it) {
      hipLaunchKernelGGL(k_bi_p, dim3(nch), dim3(BT), 0, s, W.r.p, W.p.p, W.v.p, W.chunks.p,
                         W.bst.p);
      EDFA_CHECK_LAUNCH();
      applyP(W.p.p, W.ph.p);
      spmvA(W.ph.p, W.v.p, nullptr, live);
      hipLaunchKernelGGL(k_bi_dot_rv, dim3(nch), dim3(BT), 0, s, W.rhat.p, W.v.p, W.chunks.p,
                         W.bst.p, W.part.p, LD);
      EDFA_CHECK_LAUNCH();
      reduce(1, STEP_ALPHA);
      hipLaunchKernelGGL(k_bi_s, dim3(nch), dim3(BT), 0, s, W.r.p, W.v.p, W.sv.p, W.chunks.p,
                         W.bst.p, W.part.p, LD);
      EDFA_CHECK_LAUNCH();
      reduce(1, STEP_HALF);
      applyP(W.sv.p, W.sh.p);
      spmvA(W.sh.p, W.t.p, nullptr, live);
      hipLaunchKernelGGL(k_bi_dot_ts, dim3(nch), dim3(BT), 0, s, W.t.p, W.sv.p, W.chunks.p,
                         W.bst.p, W.part.p, LD);
      EDFA_CHECK_LAUNCH();
      reduce(2, STEP_OMEGA);
      hipLaunchKernelGGL(k_bi_update, dim3(nch), dim3(BT), 0, s, x, W.r.p, W.rhat.p, W.ph.p,
                         W.sh.p, W.sv.p, W.t.p, W.chunks.p, W.bst.p, W.part.p, LD);
      EDFA_CHECK_LAUNCH();
      reduce(2, STEP_END);
    }
    nact = read_states();
  }
  total.stop(s);
  const float tms = total.ms();
  int conv = 0, iters = 0;
  double rt = 0, est = 0;
  for (auto &q : hst) {
    conv += q.converged;
    iters = std::max(iters, q.total);
    rt = std::max(rt, q.relres);
    est = std::max(est, q.bnorm > 0 ? q.rnorm / q.bnorm : 0.0);
  }
  if (info) {
    info->iterations = iters;
    info->converged = conv;
    info->cycles = starts;
    info->relres_est = est;
    info->relres_true = rt;
    info->t_solve_ms = tms;
    auto avg = [&](auto &v) {
      double t = 0;
      for (auto &pr : v) {
        float ms = 0;
        EDFA_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
        t += ms;
      }
      return v.empty() ? 0.0 : t / v.size();
    };
    info->spmv_avg_ms = prm.profile ? avg(ev_spmv) : 0.0;
    info->spmv_count = (int)ev_spmv.size();
    info->apply_avg_ms = prm.profile ? avg(ev_apply) : 0.0;
    info->apply_count = (int)ev_apply.size();
    pp.summarise(info->slot_ms, info->slot_launches, EDFA_TUNE_SLOTS);
    info->slot_ms[tr] = info->spmv_avg_ms;
    info->slot_launches[tr] = info->spmv_count;
  }
  return conv == nseg ? EDFA_OK : EDFA_NOT_CONVERGED;
}

}  // namespace edfa
