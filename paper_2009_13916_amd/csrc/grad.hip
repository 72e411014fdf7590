// Per-cell gradient of a loss with respect to theta_E = ln(multiplier of K^E).
//
// W^E scales as exp(theta_E), so the local fluxes q^E = W^E (p^E 1 - pi^E) of eq.
// fluxes_MHFEM_3 satisfy dq^E/dtheta_E = q^E, and the strong flux of eq.
// fluxes_MHFEM_STRONG, q_i = (W'_ii Lam^E - W_ii Lam^E') / (W_ii + W'_ii), satisfies
// dq_i/dtheta_E = q_i W'_ii / (W_ii + W'_ii) (and the neighbour's flux, -q_i, varies
// oppositely).  With R(u) = A u - b and A^T lambda = dL/du:
//   dL/dtheta_E = -[ sum_{faces i of E, unknown} lambda_pi,i q_i^E
//                  + sum_{interior faces} (lambda_p,E - lambda_p,E') q_i W'_ii/(W_ii + W'_ii)
//                  + sum_{Dirichlet faces} lambda_p,E q_i^E ]
// Neumann faces carry a prescribed flux and contribute nothing.
#include "precond.hpp"

namespace edfa {

__global__ void k_grad_logk(const GridDesc *__restrict__ grids, int ngrid, int ne, int nfu,
                            const double *__restrict__ W, const int8_t *__restrict__ kind,
                            const int *__restrict__ uidx, const double *__restrict__ bcv,
                            const double *__restrict__ u, const double *__restrict__ lam,
                            double *g) {
  const int E = blockIdx.x * blockDim.x + threadIdx.x;
  if (E >= ne) return;
  const GridDesc &G = grids[grid_of(grids, ngrid, E, true)];
  int i, j, k;
  cell_ijk(G, E, i, j, k);
  const double *We = W + 36 * (size_t)E;
  const double pE = u[nfu + E];
  int fc[6];
  double pi[6];
  for (int a = 0; a < 6; ++a) {
    fc[a] = cell_face(G, i, j, k, a);
    const int ui = uidx[fc[a]];
    pi[a] = ui >= 0 ? u[ui] : bcv[fc[a]];
  }
  double acc = 0.0;
  for (int a = 0; a < 6; ++a) {
    double q = 0.0;
    for (int b = 0; b < 6; ++b) q += We[6 * a + b] * (pE - pi[b]);
    const int ui = uidx[fc[a]];
    if (ui >= 0) acc += lam[ui] * q;
    const int8_t kd = kind[fc[a]];
    if (kd == FACE_DIRICHLET) {
      acc += lam[nfu + E] * q;
    } else if (kd == FACE_INTERIOR) {
      const int En = cell_nbr(G, i, j, k, a);
      const int ap = a ^ 1;
      const double *Wn = W + 36 * (size_t)En;
      int ni, nj, nk;
      cell_ijk(G, En, ni, nj, nk);
      const double pn = u[nfu + En];
      double lamE = 0.0, lamN = 0.0;
      for (int b = 0; b < 6; ++b) {
        if (b != a) lamE += We[6 * a + b] * (pE - pi[b]);
        else lamE += We[6 * a + b] * pE;
        const int fb = cell_face(G, ni, nj, nk, b);
        const int ub = uidx[fb];
        const double pib = ub >= 0 ? u[ub] : bcv[fb];
        if (b != ap) lamN += Wn[6 * ap + b] * (pn - pib);
        else lamN += Wn[6 * ap + b] * pn;
      }
      const double w1 = We[7 * a], w2 = Wn[7 * ap];
      const double qs = (w2 * lamE - w1 * lamN) / (w1 + w2);
      acc += (lam[nfu + E] - lam[nfu + En]) * qs * w2 / (w1 + w2);
    }
  }
  g[E] = -acc;
}

void grad_logk(edfa_system_s &S, const double *u, const double *lam, double *g, hipStream_t s) {
  if (S.ne == 0) return;
  hipLaunchKernelGGL(k_grad_logk, dim3(ceil_div(S.ne, 128)), dim3(128), 0, s, S.grids.p, S.ngrid,
                     S.ne, S.nfu, S.W.p, S.kind.p, S.uidx.p, S.bcv.p, u, lam, g);
  EDFA_CHECK_LAUNCH();
}

}  // namespace edfa
