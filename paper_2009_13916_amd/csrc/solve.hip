// Restarted right-preconditioned GMRES / flexible GMRES, x0 = 0, exit on the true FP64
// relative residual (the paper's stopping test, Section 4).
//
// Every grid of a batch ("segment") has its own Krylov basis coefficients, Hessenberg
// matrix, Givens rotations and convergence state; all segments advance together and a
// converged segment is masked out of the vector kernels.  Vectors are processed in
// chunks that never straddle a segment, so every reduction is per segment and fixed in
// order (deterministic).
//
// Orthogonalisation: classical Gram-Schmidt with the second (re-orthogonalisation) pass of
// each basis vector delayed to the next iteration, where it shares the passes over the
// basis with the first pass of the new vector (delayed CGS2, after Swirydowicz, Langou,
// Ananthan, Yang and Thomas, 2020).  Iteration j holds Q = [q_0 .. q_{j-1}] and u_j, the
// vector projected once but not yet re-orthogonalised or normalised; with w = A M^-1 u_j,
//   one pass     a = Q^T u_j,  b = Q^T w,  nu = u_j . u_j,  beta = u_j . w
//   per segment  rho = sqrt(nu - a.a); Hessenberg column j-1 becomes final (+= a, subdiagonal
//                rho) and gets its Givens rotation; c = [b; (beta - a.b)/rho] = [Q q_j]^T w;
//                the provisional column j is (c - Hbar a)/rho
//   one pass     q_j = (u_j - Q a)/rho,  u_{j+1} = (w - Q b - q_j c_j)/rho
// (w = rho A M^-1 q_j + A M^-1 Q a and A M^-1 Q = Q_{j+1} Hbar give these).  FGMRES keeps
// z_j = M^-1 u_j as applied: with u_j = rho_j q_j + Q a_j, the columns M^-1 q_j are
// Z T^-1 for the upper triangular T with columns [a_j; rho_j], so the end of a cycle adds
// Z (T^-1 y) instead of correcting every z_j with a pass over Z.  The last column of a
// cycle is finalised by one more pass of dots.
#include <cmath>

#include "precond.hpp"

namespace edfa {

constexpr int CHUNK = SOLVE_CHUNK;   // elements per chunk: 256 threads x 8
constexpr int RT = 256;

// Partial dots tiled over (chunk, group of DG basis vectors): block (c, q) forms Q_i . u and
// Q_i . w on chunk c for i in [DG q, DG q + DG); blocks with q = 0 also form u . u and u . w.
// Components per chunk row: [Q^T u (nv) | Q^T w (nv) | u.u | u.w].  The group width DG
// (the CGS2 block width: 2, 4 or 8 basis vectors per block) trades re-reads of u and w
// against blocks in flight; the solve tuner picks it (groups of 16 leave too few blocks).
template <int DG>
__global__ __launch_bounds__(RT) void k_dots2(const double *__restrict__ Q, long long ldq, int nv,
                                              const double *__restrict__ u,
                                              const double *__restrict__ w,
                                              const Chunk *__restrict__ ch,
                                              const SegState *__restrict__ st, double *part,
                                              int ldp, int nch, int ng) {
  __shared__ double red[4][2 * DG + 2];
  // XCD-aware order: workgroups are dealt to the 8 XCDs in turn, so block b runs on XCD b % 8
  // as that XCD's (b / 8)-th block; there the groups of one chunk follow each other, and the
  // chunk's u and w come from that XCD's L2 after the first group
  const int xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
  const int chunk = (slot / ng) * 8 + xcd, grp = slot % ng;
  if (chunk >= nch) return;
  const Chunk c = ch[chunk];
  if (!st[c.seg].active) return;
  const int i0 = grp * DG;
  const bool self = grp == 0;
  // Branch-free loads: elements past the chunk end re-read its last element with weight
  // zero, and basis slots past nv re-read slot nv - 1 (their sums are not stored), so every
  // load of the block is issued before the first wait.
  int ek[8];
  bool ok[8];
  double ue[8], we[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int e = c.start + threadIdx.x + k * RT;
    ok[k] = e < c.end;
    ek[k] = ok[k] ? e : c.end - 1;
    ue[k] = u[ek[k]];
    we[k] = w[ek[k]];
  }
  double au[DG], aw[DG], uu = 0.0, uw = 0.0;
#pragma unroll
  for (int g = 0; g < DG; ++g) au[g] = aw[g] = 0.0;
  if (nv > 0) {
#pragma unroll
    for (int g = 0; g < DG; ++g) {
      const double *qg = Q + (long long)min(i0 + g, nv - 1) * ldq;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const double q = ok[k] ? qg[ek[k]] : 0.0;
        au[g] += q * ue[k];
        aw[g] += q * we[k];
      }
    }
  }
  if (self) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double uk = ok[k] ? ue[k] : 0.0;
      uu += uk * uk;
      uw += uk * we[k];
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int g = 0; g < 2 * DG + 2; ++g) {
    double v = g < DG ? au[g] : g < 2 * DG ? aw[g - DG] : g == 2 * DG ? uu : uw;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[wave][g] = v;
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < 2 * DG + 2) {
    const double v = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
    double *row = part + (long long)chunk * ldp;
    if (t < DG) {
      if (i0 + t < nv) row[i0 + t] = v;
    } else if (t < 2 * DG) {
      if (i0 + t - DG < nv) row[nv + i0 + t - DG] = v;
    } else if (self) {
      row[2 * nv + (t - 2 * DG)] = v;
    }
  }
}

void launch_dots2(int width, int j, int nch, hipStream_t s, const double *Q, long long ldq,
                  const double *u, const double *w, const Chunk *ch, const SegState *st,
                  double *part, int ld) {
  // one dimension: 8 x ceil(nch / 8) chunk slots (those past nch return) times the ng groups
  // of basis vectors, in the order the kernel maps to (chunk, group)
  auto go = [&](auto kern, int dg) {
    const int ng = std::max(1, ceil_div(j, dg));
    hipLaunchKernelGGL(kern, dim3(8 * ceil_div(nch, 8) * ng), dim3(RT), 0, s, Q, ldq, j, u, w,
                       ch, st, part, ld, nch, ng);
  };
  if (width == 2)
    go(k_dots2<2>, 2);
  else if (width == 8)
    go(k_dots2<8>, 8);
  else
    go(k_dots2<4>, 4);
  EDFA_CHECK_LAUNCH();
}

// Per-segment sums of chunk partials: one wavefront per (segment, component), lanes strided
// over the segment's chunks, then a fixed shuffle tree (no block barriers).
// which: SEG_ALL or SEG_ACTIVE (only segments still iterating).
enum { SEG_ALL = 0, SEG_ACTIVE = 1 };
__global__ __launch_bounds__(256) void k_seg_reduce_w(const double *__restrict__ part, int ldp,
                                                      int ncomp, const int *__restrict__ segptr,
                                                      const SegState *__restrict__ st,
                                                      int which, double *out, int ldo) {
  const int g = blockIdx.y;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= ncomp) return;
  const int c0 = segptr[g], c1 = segptr[g + 1];   // loaded beside the state, not after it
  if (which != SEG_ALL && !st[g].active) return;
  double s = 0;
  // eight of the lane's chunks per round, their loads issued together (the sum keeps the
  // chunk order)
  int c = c0 + lane;
  for (; c + 7 * 64 < c1; c += 8 * 64) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(long long)(c + u * 64) * ldp + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; c < c1; c += 64) s += part[(long long)c * ldp + i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) out[(long long)g * ldo + i] = s;
}

// partial sum of squares of x over each chunk (all non-done segments)
__global__ __launch_bounds__(RT) void k_nrm2_part(const double *__restrict__ x,
                                                  const Chunk *__restrict__ ch, double *part,
                                                  int ldp) {
  __shared__ double red[4];
  const Chunk c = ch[blockIdx.x];
  double s = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int e = c.start + threadIdx.x + k * RT;
    if (e < c.end) s += x[e] * x[e];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[(long long)blockIdx.x * ldp] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Per segment, one wavefront: finish column j-1 of the Hessenberg matrix with the
// re-orthogonalisation coefficients a and rho, rotate it, update the residual estimate and
// the convergence state; then (unless `final`) form the provisional column j and the
// coefficients of the update pass: coef = [a (j) | c (j + 1)], scale = 1/rho.
// d = reduced dots [a | b | nu | beta] of this iteration.  Hbar: unrotated columns, column k
// at Hb + (g m + k)(m + 1).  j = 0: q_0 is already normalised (rho = 1, no column to finish).
__global__ __launch_bounds__(64) void k_dcgs_step(int nseg, int m, int j, int final_, SegState *st,
                                                  const double *__restrict__ d, int ldd,
                                                  double *Hb, double *R, double *cs, double *sn,
                                                  double *gv, double *coef, double *scale,
                                                  int max_iter, double *Tz) {
  __shared__ double a[MAXV], b[MAXV], col[MAXV], hf[MAXV], cc[MAXV], c_[MAXV], s_[MAXV];
  __shared__ double sh_rho;
  __shared__ int sh_live;
  const int g = blockIdx.x;
  if (g >= nseg) return;
  const int lane = threadIdx.x;
  const double *dd = d + (long long)g * ldd;
  double *H = Hb + (long long)g * m * (m + 1);
  const int jf = j - 1;                          // the column that becomes final (j > 0)
  double *hc = H + (long long)jf * (m + 1);
  // the loads that depend on nothing computed here go out together before the first wait
  // (no branch between them): the segment's state, the reduced sums, column jf, the
  // rotations before it (entry jf, in bounds, is loaded and not used) and g_jf.  Every
  // global store comes after the last barrier, so no barrier waits for one; column jf as
  // finished here (hf) is read from LDS.
  const int active = st[g].active, total = st[g].total;
  const double tol = st[g].tol;
  const double nu = dd[2 * j], beta = dd[2 * j + 1];
  const double gj = gv[(long long)g * (m + 1) + max(jf, 0)];
  for (int i = lane; i < j; i += 64) {
    const double ai = dd[i], bi = dd[j + i], hi = hc[i];
    const double ci = cs[(long long)g * m + i], si = sn[(long long)g * m + i];
    a[i] = ai;
    b[i] = bi;
    hf[i] = hi + ai;   // Hbar[0:j, jf] += a
    c_[i] = ci;
    s_[i] = si;
  }
  if (!active) return;   // the same for the whole wavefront
  __syncthreads();
  double aa = 0, ab = 0;
  for (int i = lane; i < j; i += 64) {
    aa += a[i] * a[i];
    ab += a[i] * b[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    aa += __shfl_xor(aa, o);
    ab += __shfl_xor(ab, o);
  }
  // lane 0's results of the rotation, stored after the barriers
  double cj = 0, sj = 0, gn = 0, est = 0;
  int tot = 0;
  bool live = true;
  if (j > 0) {
    // column jf = j - 1 becomes final: Hbar[0:j, jf] += a, Hbar[j, jf] = rho
    const double r2 = nu - aa;
    const double rho = r2 > 0 ? sqrt(r2) : 0.0;
    for (int i = lane; i < j; i += 64) col[i] = hf[i];
    if (lane == 0) {
      hf[j] = rho;
      col[j] = rho;
    }
    __syncthreads();
    if (lane == 0) {
      for (int i = 0; i < jf; ++i) {
        const double t = c_[i] * col[i] + s_[i] * col[i + 1];
        col[i + 1] = -s_[i] * col[i] + c_[i] * col[i + 1];
        col[i] = t;
      }
      const double den = hypot(col[jf], col[jf + 1]);
      cj = den > 0 ? col[jf] / den : 1.0;
      sj = den > 0 ? col[jf + 1] / den : 0.0;
      col[jf] = den;
      gn = -sj * gj;
      est = fabs(gn);
      tot = total + 1;
      live = !(final_ || !(est > tol) || !(rho > 0) || tot >= max_iter || !isfinite(est));
      sh_live = live;
      sh_rho = rho;
    }
    __syncthreads();
    // the finished column, its rotated form and lane 0's rotation and state
    for (int i = lane; i <= j; i += 64) hc[i] = hf[i];
    for (int i = lane; i <= jf; i += 64) R[((long long)g * m + i) * m + jf] = col[i];
    if (lane == 0) {
      cs[(long long)g * m + jf] = cj;
      sn[(long long)g * m + jf] = sj;
      double *gg = gv + (long long)g * (m + 1);
      gg[jf + 1] = gn;
      gg[jf] = cj * gj;
      st[g].est = est;
      st[g].j = j;
      st[g].total = tot;
      if (!live) st[g].active = 0;
    }
    if (!sh_live) return;
  } else {
    if (lane == 0) {
      sh_rho = 1.0;
      sh_live = 1;
    }
    __syncthreads();
  }
  // provisional column j: (c - Hbar[0:j+1, 0:j] a) / rho, c = [b ; (beta - a.b)/rho]
  const double rho = sh_rho;
  for (int i = lane; i < j; i += 64) cc[i] = b[i];
  if (lane == 0) cc[j] = (beta - ab) / rho;
  __syncthreads();
  double *hn = H + (long long)j * (m + 1);
  for (int i = lane; i <= j; i += 64) {
    // the entries of row i of Hbar are read 32 columns at a time (clamped loads issued
    // together, no branch; column jf from LDS), the sum still runs in ascending column order
    double t = cc[i];
    for (int k = i > 0 ? i - 1 : 0; k < j; k += 32) {
      double h[32];
#pragma unroll
      for (int u = 0; u < 32; ++u) h[u] = H[(long long)min(k + u, j - 1) * (m + 1) + i];
#pragma unroll
      for (int u = 0; u < 32; ++u)
        if (k + u < j) t -= (k + u == jf ? hf[i] : h[u]) * a[k + u];
    }
    hn[i] = t / rho;
  }
  double *cf = coef + (long long)g * (2 * m + 2);
  for (int i = lane; i < j; i += 64) cf[i] = a[i];
  for (int i = lane; i <= j; i += 64) cf[j + i] = cc[i];
  if (lane == 0) scale[g] = 1.0 / rho;
  if (Tz && j < m) {
    // column j of T: u_j = rho q_j + Q a (FGMRES)
    double *T = Tz + (long long)g * m * m;
    for (int i = lane; i < j; i += 64) T[(long long)i * m + j] = a[i];
    if (lane == 0) T[(long long)j * m + j] = rho;
  }
}

// q_j = (u_j - Q a) / rho (in place in slot j) and u_{j+1} = (w - Q b - q_j c_j) / rho
// (into slot j + 1); coef = [a (j) | b (j) | c_j], scale = 1/rho.
__global__ __launch_bounds__(RT) void k_dcgs_update(double *Q, long long ldq, int j,
                                                    const double *__restrict__ w,
                                                    const Chunk *__restrict__ ch,
                                                    const SegState *__restrict__ st,
                                                    const double *__restrict__ coef, int ldc,
                                                    const double *__restrict__ scale) {
  __shared__ double sa[MAXV], sb[MAXV];
  const Chunk c = ch[blockIdx.x];
  if (!st[c.seg].active) return;
  const double *cf = coef + (long long)c.seg * ldc;
  for (int i = threadIdx.x; i < j; i += RT) {
    sa[i] = cf[i];
    sb[i] = cf[j + i];
  }
  __syncthreads();
  const double cj = cf[2 * j], ir = scale[c.seg];
  double *uj = Q + (long long)j * ldq;
  double *un = Q + (long long)(j + 1) * ldq;
  // block (c, h) updates half h of the chunk (twice the blocks of one per chunk keep more
  // loads in flight); basis vectors outermost, each step issuing the UE loads of one vector
  // without a branch (elements past the chunk end re-read its last element, unstored)
  constexpr int UE = CHUNK / RT / 2;
  const int e0 = c.start + blockIdx.y * (UE * RT) + threadIdx.x;
  int ek[UE];
  double u[UE], x[UE];
#pragma unroll
  for (int k = 0; k < UE; ++k) {
    ek[k] = min(e0 + k * RT, c.end - 1);
    u[k] = uj[ek[k]];
    x[k] = w[ek[k]];
  }
  for (int i = 0; i < j; ++i) {
    const double a = sa[i], bb = sb[i];
    const double *qi = Q + (long long)i * ldq;
#pragma unroll
    for (int k = 0; k < UE; ++k) {
      const double q = qi[ek[k]];
      u[k] -= a * q;
      x[k] -= bb * q;
    }
  }
#pragma unroll
  for (int k = 0; k < UE; ++k) {
    const int e = e0 + k * RT;
    if (e < c.end) {
      const double qj = u[k] * ir;
      uj[e] = qj;
      un[e] = (x[k] - cj * qj) * ir;
    }
  }
}

// V_{j+1} = w * scale[seg] (active segments); with j < 0: V_0 = r / beta for starting ones.
__global__ __launch_bounds__(RT) void k_scale(const double *__restrict__ w, double *v,
                                              const Chunk *__restrict__ ch,
                                              const SegState *__restrict__ st,
                                              const double *__restrict__ scale) {
  const Chunk c = ch[blockIdx.x];
  if (!st[c.seg].active) return;
  const double f = scale[c.seg];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int e = c.start + threadIdx.x + k * RT;
    if (e < c.end) v[e] = w[e] * f;
  }
}

// Cycle start: beta = ||r||, decide convergence on the true residual, set g = beta e_1.
__global__ void k_seg_start(int nseg, int m, SegState *st, const double *__restrict__ rn2, int ldh,
                            double *gv, double *scale, int max_iter, int first) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nseg) return;
  SegState S = st[g];
  const double r = sqrt(rn2[(long long)g * ldh]);
  if (first) {
    S.bnorm = r;
    S.tol = S.rtol * r;
    S.total = 0;
    S.done = 0;
    S.converged = 0;
  }
  S.relres = S.bnorm > 0 ? r / S.bnorm : 0.0;
  S.j = 0;
  S.active = 0;
  if (!S.done) {
    if (!(r > S.tol)) {
      S.done = 1;
      S.converged = isfinite(r) ? 1 : 0;
    } else if (S.total >= max_iter || !isfinite(r)) {
      S.done = 1;
    } else {
      S.active = 1;
      S.beta = r;
      double *gg = gv + (long long)g * (m + 1);
      gg[0] = r;
      for (int i = 1; i <= m; ++i) gg[i] = 0.0;
      scale[g] = 1.0 / r;
    }
  }
  st[g] = S;
}

// Least squares of the cycle, one wavefront per segment: R y = g (upper triangular, size
// k = the columns that ran), by columns (y_i = s_i / R_ii, then s_l -= R_li y_i for l < i),
// with the triangle staged in LDS when it fits (`staged`); FGMRES (Tz non-null) then
// replaces y by T^-1 y, the coefficients of the stored z_j, the same way.
extern __shared__ double lsq_lds[];
__global__ __launch_bounds__(64) void k_lsq(int nseg, int m, const SegState *__restrict__ st,
                                            const double *__restrict__ R,
                                            const double *__restrict__ gv, double *y,
                                            const int *__restrict__ ran,
                                            const double *__restrict__ Tz, int staged) {
  const int g = blockIdx.x;
  if (g >= nseg) return;
  const int lane = threadIdx.x;
  const int k = __builtin_amdgcn_readfirstlane(ran[g]);
  double *ys = lsq_lds, *Ms = lsq_lds + m;
  const double *gg = gv + (long long)g * (m + 1);
  for (int i = lane; i < m; i += 64) ys[i] = i < k ? gg[i] : 0.0;
  auto solve = [&](const double *Mg) {   // entry (i, l) at Mg[i m + l]
    const double *M = Mg;
    if (staged) {
      for (int t = lane; t < k * k; t += 64) {
        const int i = t / k, l = t % k;
        Ms[i * m + l] = Mg[(long long)i * m + l];
      }
      M = Ms;
    }
    __syncthreads();
    for (int i = k - 1; i >= 0; --i) {
      const double yi = ys[i] / M[(long long)i * m + i];
      for (int l = lane; l < i; l += 64) ys[l] -= M[(long long)l * m + i] * yi;
      __syncthreads();
      if (lane == 0) ys[i] = yi;
      __syncthreads();
    }
  };
  solve(R + (long long)g * m * m);
  if (Tz) solve(Tz + (long long)g * m * m);
  double *yy = y + (long long)g * m;
  for (int i = lane; i < m; i += 64) yy[i] = ys[i];
}

// out[e] (+)= sum_{i<m} y[seg][i] B_i[e]
__global__ __launch_bounds__(RT) void k_combine(const double *__restrict__ B, long long ldb, int m,
                                                const Chunk *__restrict__ ch,
                                                const double *__restrict__ y, const int *__restrict__ ran,
                                                double *out, int accumulate) {
  const Chunk c = ch[blockIdx.x];
  const int k = ran[c.seg];
  const double *yy = y + (long long)c.seg * m;
  int ek[8];
  double s[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    ek[q] = min(c.start + (int)threadIdx.x + q * RT, c.end - 1);
    s[q] = accumulate ? out[ek[q]] : 0.0;
  }
#pragma unroll 2
  for (int i = 0; i < k; ++i) {
    const double a = yy[i];
    const double *bi = B + (long long)i * ldb;
#pragma unroll
    for (int q = 0; q < 8; ++q) s[q] += a * bi[ek[q]];
  }
#pragma unroll
  for (int q = 0; q < 8; ++q)
    if (c.start + (int)threadIdx.x + q * RT < c.end) out[c.start + threadIdx.x + q * RT] = s[q];
}

__global__ void k_axpy(long long n, const double *__restrict__ x, double *y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

__global__ void k_record_ran(int nseg, const SegState *__restrict__ st, int *ran) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < nseg) ran[g] = st[g].j;
}

// ---------------------------------------------------------------------------------------
void ProdProfile::summarise(double *ms, int32_t *count, int nslot) const {
  std::vector<double> tot(nslot, 0.0);
  std::vector<int> cnt(nslot, 0);
  for (const auto &r : rec) {
    const int q = std::get<0>(r);
    if (q < 0 || q >= nslot) continue;
    float t = 0;
    EDFA_HIP(hipEventElapsedTime(&t, std::get<1>(r), std::get<2>(r)));
    tot[q] += t;
    ++cnt[q];
  }
  for (int q = 0; q < nslot; ++q) {
    ms[q] = cnt[q] ? tot[q] / cnt[q] : 0.0;
    count[q] = cnt[q];
  }
}

void build_chunks(edfa_system_s &S, SolveWork &W, hipStream_t s) {
  if (W.nchunk > 0 && W.n == S.n) return;
  std::vector<Chunk> ch;
  std::vector<int> ptr(S.ngrid + 1, 0);
  for (int g = 0; g < S.ngrid; ++g) {
    const GridRange &R = S.ranges_h[g];
    ptr[g] = (int)ch.size();
    for (int a = R.uf0; a < R.uf1; a += CHUNK) ch.push_back(Chunk{a, std::min(a + CHUNK, R.uf1), g});
    for (int a = S.nfu + R.c0; a < S.nfu + R.c1; a += CHUNK)
      ch.push_back(Chunk{a, std::min(a + CHUNK, S.nfu + R.c1), g});
  }
  ptr[S.ngrid] = (int)ch.size();
  W.nchunk = (int)ch.size();
  W.n = S.n;
  W.chunks.ensure(ch.size());
  W.segptr.ensure(ptr.size());
  EDFA_HIP(hipMemcpyAsync(W.chunks.p, ch.data(), sizeof(Chunk) * ch.size(), hipMemcpyHostToDevice, s));
  EDFA_HIP(hipMemcpyAsync(W.segptr.p, ptr.data(), sizeof(int) * ptr.size(), hipMemcpyHostToDevice, s));
  EDFA_HIP(hipStreamSynchronize(s));
}

struct Prof {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  hipEvent_t get() {
    if (used == ev.size()) {
      hipEvent_t e;
      EDFA_HIP(hipEventCreate(&e));
      ev.push_back(e);
    }
    return ev[used++];
  }
  ~Prof() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

// A captured restart cycle and the stream it replays on (released with the solve).
struct GraphCycle {
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~GraphCycle() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev) (void)hipEventDestroy(ev);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

edfa_status gmres(edfa_system_s &S, edfa_precond_s &P, const double *b, double *x,
                  const edfa_solve_params &prm, hipStream_t s, edfa_solve_info *info) {
  const int m = prm.restart;
  if (m < 1 || m > MAXV - 2) fail(EDFA_ERR_ARG, "restart must be in 1..%d", MAXV - 2);
  if (!(prm.rtol > 0.0)) fail(EDFA_ERR_ARG, "rtol must be > 0");
  if (P.prm.precision == 1 && !prm.flexible)
    fail(EDFA_ERR_ARG, "the FP32 preconditioner requires flexible GMRES");
  if (!P.ws) P.ws.reset(new SolveWork());
  SolveWork &W = *P.ws;
  const int n = S.n, nseg = S.ngrid;
  const int tr = prm.transpose ? 1 : 0;
  build_chunks(S, W, s);
  const int nch = W.nchunk;
  const int ld = 2 * m + 4;   // per-chunk / per-segment rows of dot products (2j + 2 used)
  W.V.ensure((size_t)(m + 1) * n);
  if (prm.flexible) {
    W.Z.ensure((size_t)m * n);
    W.Tz.ensure((size_t)nseg * m * m);
  }
  double *Tz = prm.flexible ? W.Tz.p : nullptr;
  W.w.ensure(n);
  W.r.ensure(n);
  W.z.ensure(n);
  W.part.ensure((size_t)nch * ld);
  W.h1.ensure((size_t)nseg * ld);
  W.nrm.ensure((size_t)nseg * ld);
  W.R.ensure((size_t)nseg * m * m);
  W.Hb.ensure((size_t)nseg * m * (m + 1));
  W.coef.ensure((size_t)nseg * (2 * m + 2));
  W.cs.ensure((size_t)nseg * m);
  W.sn.ensure((size_t)nseg * m);
  W.g.ensure((size_t)nseg * (m + 1));
  W.y.ensure((size_t)nseg * m);
  W.scale.ensure(nseg);
  W.ran.ensure(nseg);
  W.st.ensure(nseg);
  std::vector<SegState> hst(nseg);
  for (auto &q : hst) {
    q = SegState{};
    q.rtol = prm.rtol;
  }
  EDFA_HIP(hipMemcpyAsync(W.st.p, hst.data(), sizeof(SegState) * nseg, hipMemcpyHostToDevice, s));
  if (tr && S.AT.rows == 0) csr_transpose(S.A, S.AT, S.tmp, S.tmp2, s);
  if (tr && S.AT_s.rows == 0) build_sell(S.AT, S.AT_s, S.tmp, s);
  apply_tuned(P);
  const Sell<double> &A = tr ? S.AT_s : S.A_s;

  Prof prof;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_spmv, ev_apply;
  EventTimer total;
  total.start(s);

  // profiled system products: the launch records its own events around the kernel
  // Inside the Arnoldi loop of a batch, the products skip the rows of grids that have
  // stopped iterating (every matrix is block-diagonal by grid).
  // One system: every row in grid 0, masked once it has converged (a profiled solve keeps
  // every launch whole, so that its timings are those of real work).
  RowMask live = prm.profile ? RowMask{} : RowMask{nullptr, &W.st.p->active, 0};
  if (nseg > 1) {
    if (S.rowseg.n < (size_t)n) fail(EDFA_ERR_ARG, "batch without its row-to-grid map");
    live = RowMask{S.rowseg.p, &W.st.p->active, (int)(sizeof(SegState) / sizeof(int))};
  }
  // profiling events are recorded on the caller's stream only (never inside a capture)
  auto spmvA = [&](const double *in, double *out, const double *bb, hipStream_t cs,
                   RowMask mk) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prm.profile && cs == s) {
      e0 = prof.get();
      e1 = prof.get();
      ev_spmv.emplace_back(e0, e1);
    }
    spmv_sell<double, double>(A, in, out, bb ? -1.0 : 1.0, bb, 1.0, cs, 0.0, SPMV_OPERATOR, e0, e1,
                              mk);
  };
  ProdProfile pp;
  auto applyP = [&](const double *in, double *out, hipStream_t cs, RowMask mk) {
    const bool pr = prm.profile && cs == s;
    hipEvent_t e0{}, e1{};
    if (pr) {
      e0 = prof.get();
      EDFA_HIP(hipEventRecord(e0, cs));
      if (prm.profile >= 2) P.prof = &pp;
    }
    precond_apply(P, tr, in, out, cs, mk);
    P.prof = nullptr;
    if (pr) {
      e1 = prof.get();
      EDFA_HIP(hipEventRecord(e1, cs));
      ev_apply.emplace_back(e0, e1);
    }
  };
  auto seg_norms = [&](const double *v, double *out, hipStream_t cs) {
    hipLaunchKernelGGL(k_nrm2_part, dim3(nch), dim3(RT), 0, cs, v, W.chunks.p, W.part.p, ld);
    hipLaunchKernelGGL(k_seg_reduce_w, dim3(1, nseg), dim3(256), 0, cs, W.part.p, ld, 1,
                       W.segptr.p, W.st.p, SEG_ALL, out, ld);
    EDFA_CHECK_LAUNCH();
  };
  const int sb = ceil_div(nseg, 64);

  EDFA_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
  EDFA_HIP(hipMemcpyAsync(W.r.p, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
  seg_norms(W.r.p, W.nrm.p, s);
  hipLaunchKernelGGL(k_seg_start, dim3(sb), dim3(64), 0, s, nseg, m, W.st.p, W.nrm.p, ld, W.g.p,
                     W.scale.p, prm.max_iter, 1);
  EDFA_CHECK_LAUNCH();
  int cycles = 0;
  // the least-squares kernel stages the triangle in LDS when it fits (restarts up to 89)
  const int lsq_staged = (size_t)(m + m * m) * sizeof(double) <= 64 * 1024;
  const size_t lsq_lds_bytes = sizeof(double) * (size_t)(lsq_staged ? m + m * m : m);
  // In-loop convergence checks read the states one check late from pinned memory, so the
  // host never drains the device queue: the iterations launched meanwhile run masked (their
  // kernels return at once) when every grid has stopped.  A profiled solve reads them at
  // once (its launches after convergence are then whole iterations, as timed).
  const int check_every = nseg == 1 ? 8 : 16;
  SegState *hpin = W.hst.ensure(nseg);
  hipEvent_t ev_check = nullptr;
  EDFA_HIP(hipEventCreateWithFlags(&ev_check, hipEventDisableTiming));
  struct EventGuard {
    hipEvent_t e;
    ~EventGuard() { (void)hipEventDestroy(e); }
  } ev_guard{ev_check};
  // One restart cycle on stream cs.  With host_checks the host stops early once every
  // segment is inactive; without, converged segments are masked on the device (the
  // form that a graph can hold).
  auto run_cycle = [&](hipStream_t cs, bool host_checks) {
    // q_0 = r / beta
    hipLaunchKernelGGL(k_scale, dim3(nch), dim3(RT), 0, cs, W.r.p, W.V.p, W.chunks.p, W.st.p,
                       W.scale.p);
    EDFA_CHECK_LAUNCH();
    // dots of basis slots [0, j) against u and w, reduced per segment into h1
    auto dots = [&](int j, const double *u, const double *w) {
      launch_dots2(P.cgs2_width, j, nch, cs, W.V.p, (long long)n, u, w, W.chunks.p, W.st.p,
                   W.part.p, ld);
      hipLaunchKernelGGL(k_seg_reduce_w, dim3(ceil_div(2 * j + 2, 4), nseg), dim3(256), 0, cs,
                         W.part.p, ld, 2 * j + 2, W.segptr.p, W.st.p, SEG_ACTIVE, W.h1.p, ld);
    };
    bool pending = false;   // a state copy is in flight behind ev_check
    for (int j = 0; j < m; ++j) {
      double *vj = W.V.p + (size_t)j * n;
      double *zj = prm.flexible ? W.Z.p + (size_t)j * n : W.z.p;
      applyP(vj, zj, cs, live);
      spmvA(zj, W.w.p, nullptr, cs, live);
      dots(j, vj, W.w.p);
      hipLaunchKernelGGL(k_dcgs_step, dim3(nseg), dim3(64), 0, cs, nseg, m, j, 0, W.st.p, W.h1.p,
                         ld, W.Hb.p, W.R.p, W.cs.p, W.sn.p, W.g.p, W.coef.p, W.scale.p,
                         prm.max_iter, Tz);
      hipLaunchKernelGGL(k_dcgs_update, dim3(nch, 2), dim3(RT), 0, cs, W.V.p, (long long)n, j, W.w.p,
                         W.chunks.p, W.st.p, W.coef.p, 2 * m + 2, W.scale.p);
      EDFA_CHECK_LAUNCH();
      if (host_checks && prm.profile && (j + 1) % check_every == 0 && j + 1 < m) {
        EDFA_HIP(hipMemcpyAsync(hpin, W.st.p, sizeof(SegState) * nseg, hipMemcpyDeviceToHost, cs));
        EDFA_HIP(hipStreamSynchronize(cs));
        int a = 0;
        for (int g = 0; g < nseg; ++g) a += hpin[g].active;
        if (!a) break;
      } else if (host_checks && (j + 1) % check_every == 0 && j + 1 < m) {
        if (pending) {
          EDFA_HIP(hipEventSynchronize(ev_check));
          pending = false;
          int a = 0;
          for (int g = 0; g < nseg; ++g) a += hpin[g].active;
          if (!a) break;
        }
        EDFA_HIP(hipMemcpyAsync(hpin, W.st.p, sizeof(SegState) * nseg, hipMemcpyDeviceToHost, cs));
        EDFA_HIP(hipEventRecord(ev_check, cs));
        pending = true;
      }
    }
    // segments whose basis is full: finish the last column with one more pass of dots
    dots(m, W.V.p + (size_t)m * n, W.V.p + (size_t)m * n);
    hipLaunchKernelGGL(k_dcgs_step, dim3(nseg), dim3(64), 0, cs, nseg, m, m, 1, W.st.p, W.h1.p,
                       ld, W.Hb.p, W.R.p, W.cs.p, W.sn.p, W.g.p, W.coef.p, W.scale.p,
                       prm.max_iter, Tz);
    EDFA_CHECK_LAUNCH();
    // end of cycle: y = R^-1 g, x += Z y (flexible) or x += P^-1 (V y)
    hipLaunchKernelGGL(k_record_ran, dim3(sb), dim3(64), 0, cs, nseg, W.st.p, W.ran.p);
    hipLaunchKernelGGL(k_lsq, dim3(nseg), dim3(64), lsq_lds_bytes, cs, nseg, m, W.st.p, W.R.p,
                       W.g.p, W.y.p, W.ran.p, Tz, lsq_staged);
    if (prm.flexible) {
      hipLaunchKernelGGL(k_combine, dim3(nch), dim3(RT), 0, cs, W.Z.p, (long long)n, m, W.chunks.p,
                         W.y.p, W.ran.p, x, 1);
    } else {
      hipLaunchKernelGGL(k_combine, dim3(nch), dim3(RT), 0, cs, W.V.p, (long long)n, m, W.chunks.p,
                         W.y.p, W.ran.p, W.w.p, 0);
      applyP(W.w.p, W.z.p, cs, RowMask{});
      hipLaunchKernelGGL(k_axpy, dim3(ceil_div(n, 256)), dim3(256), 0, cs, (long long)n, W.z.p, x);
    }
    EDFA_CHECK_LAUNCH();
    // true residual r = b - A x and the next cycle's start
    spmvA(x, W.r.p, b, cs, RowMask{});
    seg_norms(W.r.p, W.nrm.p, cs);
    hipLaunchKernelGGL(k_seg_start, dim3(sb), dim3(64), 0, cs, nseg, m, W.st.p, W.nrm.p, ld, W.g.p,
                       W.scale.p, prm.max_iter, 0);
    EDFA_CHECK_LAUNCH();
  };

  // Graph form: the first cycle runs eagerly (every lazy allocation and first-use build
  // happens there), later cycles replay one captured cycle on a stream of the solver's
  // own, ordered after the caller's stream by events.
  GraphCycle gc;
  while (true) {
    // states of every grid through the pinned copy (it also receives the in-cycle reads)
    EDFA_HIP(hipMemcpyAsync(hpin, W.st.p, sizeof(SegState) * nseg, hipMemcpyDeviceToHost, s));
    EDFA_HIP(hipStreamSynchronize(s));
    std::copy(hpin, hpin + nseg, hst.begin());
    if (cycles == 0)
      for (int g = 0; g < nseg; ++g)
        if (!std::isfinite(hst[g].bnorm))
          fail(EDFA_ERR_NAN, "grid %d: the right-hand side has a non-finite entry", g);
    int nact = 0;
    for (auto &q : hst) nact += q.active;
    if (!nact) break;
    ++cycles;
    if (!prm.use_graph || cycles == 1) {
      run_cycle(s, true);
      continue;
    }
    if (!gc.exec) {
      EDFA_HIP(hipStreamCreateWithFlags(&gc.stream, hipStreamNonBlocking));
      EDFA_HIP(hipEventCreateWithFlags(&gc.ev, hipEventDisableTiming));
      EDFA_HIP(hipStreamBeginCapture(gc.stream, hipStreamCaptureModeThreadLocal));
      run_cycle(gc.stream, false);
      EDFA_HIP(hipStreamEndCapture(gc.stream, &gc.graph));
      EDFA_HIP(hipGraphInstantiate(&gc.exec, gc.graph, nullptr, nullptr, 0));
    }
    EDFA_HIP(hipEventRecord(gc.ev, s));
    EDFA_HIP(hipStreamWaitEvent(gc.stream, gc.ev, 0));
    EDFA_HIP(hipGraphLaunch(gc.exec, gc.stream));
    EDFA_HIP(hipEventRecord(gc.ev, gc.stream));
    EDFA_HIP(hipStreamWaitEvent(s, gc.ev, 0));
  }
  total.stop(s);
  const float tms = total.ms();
  int conv = 0, iters = 0;
  double est = 0, rt = 0;
  for (auto &q : hst) {
    conv += q.converged;
    iters = std::max(iters, q.total);
    est = std::max(est, q.bnorm > 0 ? q.est / q.bnorm : 0.0);
    rt = std::max(rt, q.relres);
  }
  if (info) {
    info->iterations = iters;
    info->converged = conv;
    info->cycles = cycles;
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
