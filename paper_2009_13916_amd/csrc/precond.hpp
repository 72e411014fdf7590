// EDFA preconditioner handle (internal layout of an edfa_precond).
#pragma once

#include <memory>
#include <tuple>
#include <vector>

#include "system.hpp"

namespace edfa {

// Compiled capacities.
constexpr int NCAP = EDFA_NCAP;  // restricted-solve kernels: pattern capacities
constexpr int kCapacities[NCAP] = {16, 32, 40, 44, 48, 64, 128};
constexpr int HMAX = 512;        // max entries of one row of H~ (before filtration)
constexpr int FSAI_MAX = 16;     // max lower-pattern length of a row of A_pipi
constexpr int MAX_COLORS = 512;
constexpr int PATCH_MAX = 256;   // max pattern length of a static patch

// Everything the preconditioner stores, in the working precision T.
template <class T>
struct PrecData {
  // stage 1
  DBuf<int> Q;          // Ne x smax final patterns (base order, then appended)
  DBuf<int> qlen;       // Ne
  DBuf<int> bucket, bcells, bhist;   // capacity bucket of every cell; cells bucket by bucket
  DBuf<T> gbuf, fbuf;   // Ne x smax restricted solutions
  DBuf<int> ell_col;    // A_pipi rows padded to ELL_W entries (column -1 past a row's end)
  DBuf<double> ell_val;
  Csr<T> G;             // G~   (Ne x Nfu)
  Csr<T> FT;            // F~^T (Ne x Nfu): row m = column m of F~
  DBuf<int> ft_ecol;    // F~^T rows padded to ft_w entries (a multiple of 16; column -1 past
  DBuf<T> ft_eval;      //   a row's end), read by the H~ products with vector loads
  int ft_w = 0;
  Csr<T> Fface;         // F~   (Nfu x Ne)
  DBuf<int> Hcol;       // Ne x HMAX raw H~ rows (sorted)
  DBuf<T> Hval;
  DBuf<int> Hlen;
  DBuf<int> hretry;     // cells whose H~ row needs the large hash tables
  Csr<T> Hraw;          // H~ before post-filtration (only when exported)
  Csr<T> H;             // H~ used by stage 2
  Csr<T> GF, GFT;       // FSAI factor of -A_pipi and its transpose
  Csr<double> AppT_unused;
  // stage 2
  Csr<T> S;             // S~ = A_pp - H~ (post-filtered)
  Csr<T> ST;            // pattern of S~^T (colouring)
  DBuf<int> color, perm, iperm;     // perm[new] = old
  DBuf<int> hist, wide;             // colour histograms; wide static patches
  DBuf<int> blocker;                // colouring: the uncoloured neighbour found there (-1: none)
  DBuf<int> jplist;                 // colouring: vertices still uncoloured
  std::vector<int> cstart;          // host: colour c owns new rows [cstart[c], cstart[c+1])
  Csr<T> B;             // P S~ P^T, factored in place into L\U
  DBuf<int> diag;       // Ne: position of the diagonal in B
  Csr<T> L, U;          // strict lower (unit factor) and upper (with diagonal) of B
  Csr<T> ML, MU;        // ISAI of (I + L) and U
  Csr<T> Ln, Un, MLn, MUn;          // L, U, M_L, M_U renumbered to the natural cell order
                                    // (the ISAI application runs on these: its gathers of x
                                    // stay local, no permutation of the vector)
  DBuf<int> scratch_diag;           // unused diagonal positions of the renumbering
  Csr<T> LT, UT, MLT, MUT;          // transposes (built on first transposed apply)
  // SELL-64 copies used by the application
  Sell<T> GF_s, GFT_s, L_s, U_s, ML_s, MU_s, LT_s, UT_s, MLT_s, MUT_s;
  // application scratch (working precision)
  DBuf<T> r, z, t1, t2, y, w, zq, res;
};

// Events around individual sparse products of a profiled solve: rec holds (tuner slot,
// start, stop) per launch; events are created on demand and reused.
struct ProdProfile {
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> rec;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      EDFA_HIP(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[used++];
  }
  ~ProdProfile() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
  // per-slot mean launch time (ms) and launch count
  void summarise(double *ms, int32_t *count, int nslot) const;
};

// GMRES state: chunks of the unknown vector that never straddle a grid of a batch, and
// the per-grid (segment) iteration state.
constexpr int MAXV = 130;        // restart <= MAXV - 2
struct Chunk {
  int start, end, seg;
};
struct SegState {
  double rtol, bnorm, tol, beta, est, relres;
  int active, done, converged, j, total, pad;
};
// Bi-CGStab state of one segment (grid).
struct BiSeg {
  double bnorm, tol, rho, alpha, omega, beta, rnorm, relres;
  int active, done, converged, total, half, first, breakdown, pad;
};
struct SolveWork {
  int nchunk = 0, n = 0;
  DBuf<Chunk> chunks;
  DBuf<int> segptr;
  DBuf<double> V, Z, w, r, z, part, h1, nrm, R, cs, sn, g, y, scale;
  DBuf<double> Hb;     // unrotated Hessenberg columns per segment, m x (m + 1)
  DBuf<double> coef;   // per segment: update coefficients [a | b | c_j] of the current step
  DBuf<double> Tz;     // FGMRES, per segment m x m: column j = [a_j; rho_j], u_j = Q T e_j
  DBuf<int> ran;
  DBuf<SegState> st;
  HBuf<SegState> hst;  // pinned copy of st for the in-loop convergence checks
  // Bi-CGStab vectors and state
  DBuf<double> rhat, p, v, ph, sv, sh, t;
  DBuf<BiSeg> bst;
};
// Chunks of CHUNK unknowns that never straddle a grid (built once per system).
constexpr int SOLVE_CHUNK = 2048;
void build_chunks(edfa_system_s &S, SolveWork &W, hipStream_t s);
// CGS2 dot pass of `j` basis vectors with `width` vectors per block (2, 4 or 8)
void launch_dots2(int width, int j, int nch, hipStream_t s, const double *Q, long long ldq,
                  const double *u, const double *w, const Chunk *ch, const SegState *st,
                  double *part, int ld);

}  // namespace edfa

// A second stream of the handle for setup work that is independent of the main chain (the
// FSAI branch of stage 1), with the events that order it after and join it to the caller's
// stream.  Default priority, like every stream here.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t start = nullptr, done = nullptr;
  SideStream() = default;
  SideStream(const SideStream &) = delete;
  SideStream &operator=(const SideStream &) = delete;
  ~SideStream() {
    if (s) (void)hipStreamSynchronize(s);
    if (start) (void)hipEventDestroy(start);
    if (done) (void)hipEventDestroy(done);
    if (s) (void)hipStreamDestroy(s);
  }
  hipStream_t get() {
    if (!s) {
      EDFA_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      EDFA_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
      EDFA_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    }
    return s;
  }
};

struct edfa_precond_s {
  edfa_system_s *sys = nullptr;
  edfa_params prm{};
  int smax = 0;
  int n_colors = 0;
  int max_pattern = 0;
  int htilde_retry_rows = 0;       // rows of H~ recomputed with the large hash tables
  int bucket_cells[edfa::NCAP] = {};   // cells per capacity bucket at the last stage 1
  int cap_map[edfa::NCAP] = {};        // tuned kernel capacity per bucket (0: its own)
  int cgs2_width = 4;                  // basis vectors per block of the CGS2 dot passes
  // entries of H~ before the post-filtration: copied into pinned memory behind the count
  // (no wait); the setup's later synchronisations complete the copy before it returns
  edfa::HBuf<unsigned long long> nnz_h_raw;
  int color_rounds = 0;            // Jones-Plassmann rounds of the last colouring
  int color_list_rounds = 0;       //   of which over the worklist of uncoloured vertices
  edfa::DBuf<unsigned long long> counter;
  double t_stage1_ms = 0, t_stage2_ms = 0;
  edfa::PrecData<double> d;
  edfa::PrecData<float> f;
  edfa::DBuf<int> flags;           // device error flags: [0] not SPD, [1] capacity, [2], [3]
                                   // scratch values; [4] .. [7] the same for the FSAI branch
  SideStream side;                 // the FSAI branch of stage 1 runs on it
  edfa::DBuf<int> side_tmp, side_tmp2;   // scratch of that branch
  edfa::Csr<float> coupling_f[4];  // FP32 A_ppi, A_pip, A_pip^T, A_ppi^T (FP32 application)
  edfa::Sell<float> coupling_fs[4];
  edfa::DBuf<float> rin_f;         // FP32 copy of the vector being preconditioned
  std::unique_ptr<edfa::SolveWork> ws;
  int tuned[16] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
                                   // autotuned kernel variant of each product (-1: default)
  edfa::ProdProfile *prof = nullptr;   // set while a profiled solve runs eagerly
};

namespace edfa {
void precond_stage1(edfa_precond_s &P, hipStream_t s);
// Times each capacity bucket of the last stage 1 with the larger compiled capacities and
// keeps the fastest per bucket (report may be NULL).
void tune_setup(edfa_precond_s &P, hipStream_t s, edfa_setup_tune *report);
void precond_stage2(edfa_precond_s &P, hipStream_t s);
void precond_apply(edfa_precond_s &P, int transpose, const double *r, double *z, hipStream_t s,
                   RowMask mask = {});
void precond_apply_noalloc(edfa_precond_s &P, int transpose, const double *r, double *z,
                           hipStream_t s);
edfa_status gmres(edfa_system_s &S, edfa_precond_s &P, const double *b, double *x,
                  const edfa_solve_params &prm, hipStream_t s, edfa_solve_info *info);
edfa_status bicgstab(edfa_system_s &S, edfa_precond_s &P, const double *b, double *x,
                     const edfa_solve_params &prm, hipStream_t s, edfa_solve_info *info);
edfa_status transient(edfa_system_s &S, edfa_precond_s &P, const edfa_transient_params &prm,
                      double *u, hipStream_t s, edfa_step_info *steps, int *taken);
template <class T>
void build_hraw(edfa_precond_s &P, PrecData<T> &D, hipStream_t s);
void grad_logk(edfa_system_s &S, const double *u, const double *lam, double *g, hipStream_t s);
void apply_tuned(edfa_precond_s &P);
// True when a matrix's chosen kernel still needs chunk descriptors or a SELL layout built
// on first use.
bool layouts_pending(edfa_precond_s &P);
// slot -1: every slot; variant -1: back to the default choice (at the next setup)
void set_variant(edfa_precond_s &P, int slot, int variant);
int autotune(edfa_precond_s &P, hipStream_t s, edfa_tune_slot *slots = nullptr);
int tune_params(edfa_system_s &S, const edfa_params *cand, int ncand,
                const edfa_solve_params &sp, hipStream_t s, double *times_ms, int *iterations,
                int *status);
// argument checks of a parameter set (EDFA_ERR_ARG on a bad one)
void check_params(const edfa_params &prm);
}  // namespace edfa
