/*
 * edfa.h -- C ABI of the MI355X (gfx950) EDFA-preconditioned GMRES library.
 *
 * Problem: the 2x2 block system of a mixed-hybrid finite element (Darcy) plus
 * finite volume (mass balance) discretisation on logically structured
 * hexahedral grids (Nardean, Ferronato, Abushaikha, "A novel block
 * non-symmetric preconditioner for mixed-hybrid finite-element-based flow
 * simulations", Section 2.3, eq. system):
 *
 *     [ A_pipi  A_pip ] [ pi ]   [ f_pi ]
 *     [ A_ppi   A_pp  ] [ p  ] = [ f_p  ]
 *
 * preconditioned by the Explicit Decoupling Factor Approximation (Section 3,
 * eq. EDFA_prec, Algorithms 1-2) inside restarted right-preconditioned GMRES.
 *
 * Conventions (every entry point):
 *  - All array pointers are DEVICE pointers unless marked (host).
 *  - The caller owns every buffer it passes; the library owns the opaque
 *    handles (create / destroy) and all memory inside them.
 *  - Work is enqueued on the given stream.  Entry points that must learn a
 *    size or a convergence flag synchronise that stream (stated per call).
 *  - Calls on one handle must not overlap in time (no internal locking).
 *  - No exception crosses the ABI.  A negative status is an error, described
 *    by edfa_last_error() (thread-local, valid until the next call on the
 *    same thread); a positive status is a non-fatal outcome.
 *  - Indices are int32, floating point is IEEE binary64 (double) unless a
 *    parameter selects binary32 for the preconditioner.
 *
 * Grid layout (all inputs):
 *  - nodes: (nx+1)(ny+1)(nz+1) x 3, node (i,j,k) at row i + (nx+1)(j + (ny+1)k).
 *  - cells: nx*ny*nz, cell (i,j,k) at i + nx(j + ny k); local nodes a+2b+4c are
 *    nodes (i+a, j+b, k+c); the cell is the trilinear image of the unit cube.
 *  - faces: x-faces (i + (nx+1)(j + ny k)), then y-faces (i + nx(j + (ny+1)k)),
 *    then z-faces (i + nx(j + ny k)).  Local faces of a cell: 0 x-, 1 x+,
 *    2 y-, 3 y+, 4 z-, 5 z+.
 *  - unknowns u = [pi over non-Dirichlet faces, ascending face index;
 *                  p over cells]  (Dirichlet face pressures are eliminated).
 *    For a batch of grids, faces and cells are concatenated grid by grid and
 *    u = [pi of all grids; p of all grids].
 */
#ifndef EDFA_H
#define EDFA_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EDFA_OK = 0,
  EDFA_NOT_CONVERGED = 1,      /* the paper's "NC" (Section 4): x holds the last iterate */
  EDFA_ERR_ARG = -1,           /* invalid argument or inconsistent sizes */
  EDFA_ERR_HIP = -2,           /* a HIP runtime call failed */
  EDFA_ERR_NOMEM = -3,         /* device allocation failed */
  EDFA_ERR_NOT_SPD = -4,       /* a restricted system (or W^E) lost positive definiteness;
                                  the first offending cell index is in edfa_last_error() */
  EDFA_ERR_BREAKDOWN = -5,     /* zero pivot in ILU(0) or a non-finite Krylov quantity */
  EDFA_ERR_NAN = -6,           /* non-finite input */
  EDFA_ERR_CAPACITY = -7       /* a pattern exceeded a compiled maximum (message says which) */
} edfa_status;

typedef struct edfa_system_s *edfa_system;    /* assembled blocks + right-hand side */
typedef struct edfa_precond_s *edfa_precond;  /* EDFA stage-1 and stage-2 data */

/* Boundary condition code per face (ignored on interior faces). */
#define EDFA_BC_NEUMANN   0   /* prescribed outward total face flux (0 = no flow) */
#define EDFA_BC_DIRICHLET 1   /* prescribed face pressure */

/* One grid.  Section 2.1-2.2: Darcy's law with conductivity K and specific
 * weight gamma, mass balance with storage c, backward Euler with step dt.   */
typedef struct {
  int32_t nx, ny, nz;          /* cells per direction, each >= 1 */
  const double *nodes;         /* (nx+1)(ny+1)(nz+1) x 3 coordinates */
  const double *K;             /* N_e x 6 SPD tensor per cell: xx, yy, zz, xy, xz, yz */
  const double *c;             /* N_e storage coefficient, or NULL to use c_scalar */
  double c_scalar;
  double gamma;                /* fluid specific weight (> 0) */
  double dt;                   /* time step (> 0) */
  const int8_t *bc_type;       /* N_f codes EDFA_BC_* */
  const double *bc_value;      /* N_f: p_bar (Dirichlet) or outward total flux (Neumann) */
  const double *p_prev;        /* N_e pressure at the previous step, or NULL for 0 */
  const double *source;        /* N_e cell-mean source density s, or NULL for 0 */
} edfa_problem;

/* Sizes of an assembled system (host struct). */
typedef struct {
  int32_t n_grids;
  int32_t n_cells;             /* N_e */
  int32_t n_faces;             /* N_f (all faces) */
  int32_t n_face_unknowns;     /* N_f^u (non-Dirichlet faces) */
  int32_t n;                   /* N = N_f^u + N_e */
  int32_t axis_structure;      /* 1: every cell of every grid an axis-aligned brick with
                                  diagonal K, so W^E is block-diagonal per direction.  The
                                  smaller structural pattern this allows is chosen grid by
                                  grid: a grid of a batch has the pattern it has alone */
  int64_t nnz;                 /* nnz of the whole matrix */
  int64_t nnz_block[4];        /* A_pipi, A_pip, A_ppi, A_pp */
} edfa_system_info;

/* Assemble the block system (Section 2.2-2.3 and Appendix A).
 *  - Element matrices B^E (eq. B_ij) by 3x3x3 Gauss quadrature of the
 *    Piola-mapped lowest-order Raviart-Thomas basis; W^E = (B^E)^-1.
 *  - Face rows: flux continuity (eq. cont_fluxes); Neumann faces take the
 *    prescribed flux.  Cell rows: FV balance (eq. discr_bal_FV_2) with the
 *    strong inter-element flux (eq. fluxes_MHFEM_STRONG); at a Dirichlet face
 *    the one-sided flux with pi = p_bar, at a Neumann face its prescribed flux.
 *  - Structural patterns (explicit zeros kept): A_pipi couples faces sharing a
 *    cell through a structural entry of W^E; A_ppi row E holds E's own faces and
 *    the faces of each face neighbour coupled to the shared face.
 * count >= 1 grids (a batch is one block-diagonal system).  Input arrays are
 * read during the call only.  Synchronises the stream.
 * Errors: EDFA_ERR_ARG (sizes), EDFA_ERR_NAN (a non-finite entry in nodes, K, c,
 * bc_value, p_prev or source, or a non-finite c_scalar: grid, array and index in the
 * message), EDFA_ERR_NOT_SPD (K or a Jacobian not positive: cell index in the message),
 * EDFA_ERR_NOMEM. */
edfa_status edfa_assemble(const edfa_problem *grids /* (host) array */, int32_t count,
                          hipStream_t stream, edfa_system *out);
void edfa_system_destroy(edfa_system sys);
edfa_status edfa_system_get_info(edfa_system sys, edfa_system_info *info /* (host) */);

/* Replace dt (and optionally p_prev, N_e, NULL keeps it) of every grid: only A_pp's
 * diagonal and f_p change (Appendix A, eq. expr_A_pp).  Asynchronous. */
edfa_status edfa_update_dt(edfa_system sys, double dt, const double *p_prev, hipStream_t stream);

/* Copy out a block: 0 A_pipi, 1 A_pip, 2 A_ppi, 3 A_pp, 4 the whole matrix.
 * Buffers sized from edfa_system_get_info: rowptr rows+1, col/val nnz.
 * Columns are sorted within rows.  Asynchronous. */
edfa_status edfa_export_block(edfa_system sys, int32_t block, int32_t *rowptr, int32_t *col,
                              double *val, hipStream_t stream);
/* Copy out the right-hand side b (N) and the per-cell W^E (N_e x 36, row-major)
 * and volumes (N_e); any pointer may be NULL.  Asynchronous. */
edfa_status edfa_export_rhs(edfa_system sys, double *b, double *W, double *vol,
                            hipStream_t stream);

/* y = A x (transpose = 0) or y = A^T x (transpose = 1), x and y of length N.  FP64. */
edfa_status edfa_spmv(edfa_system sys, int32_t transpose, const double *x, double *y,
                      hipStream_t stream);

/* EDFA parameters (Section 3.1; Algorithm 1 and 2 signatures). */
#define EDFA_STATIC  0
#define EDFA_DYNAMIC 1
#define EDFA_FILT_NONE   0
#define EDFA_FILT_PRE    1   /* filter g~ and f~ before assembling G~, F~ */
#define EDFA_FILT_POST_S 2   /* filter S~ = A_pp - H~ (stage 2) */
#define EDFA_FILT_POST_H 3   /* filter H~ (stage 1) */
#define EDFA_SCHUR_ISAI  0   /* ILU(0) factors applied through sparse approximate inverses */
#define EDFA_SCHUR_EXACT 1   /* ILU(0) factors applied by colour-by-colour substitution */
typedef struct {
  int32_t variant;          /* EDFA_STATIC | EDFA_DYNAMIC */
  int32_t static_level;     /* static: 0 = base pattern Q_0 (pattern of row m of A_ppi);
                               k > 0 adds all faces of cells within k face-neighbour steps */
  int32_t n_add;            /* dynamic: max entries added per sweep */
  int32_t n_ent;            /* dynamic: max entries added in total */
  int32_t it_max;           /* dynamic: max sweeps, <= 0 means n_ent */
  double  tau_filt;         /* relative drop tolerance (Euclidean norm of the row/column) */
  int32_t filt_mode;        /* EDFA_FILT_* */
  int32_t precision;        /* 0: FP64 preconditioner; 1: FP32 setup and application */
  int32_t schur_solver;     /* EDFA_SCHUR_* */
  int32_t isai_steps;       /* ISAI applications per factor (>= 1) */
  int32_t static_axis;      /* static_level k > 0: 0 = the cells within k face steps in every
                               direction; 1/2/3 = only along x/y/z (a strip of 2k + 1 cells);
                               4 = along each cell's axis of largest transmissibility
                               W_(d-,d-) + W_(d+,d+) (ties within 1e-12 to the smaller axis) */
  int32_t htilde_retry;     /* performance knob of the rows of H~ (patterns of up to 64): a
                               row whose support of t = A_pipi R^T g~ exceeds this many faces
                               is recomputed in a second pass with large hash tables (1..256;
                               0: 256, half the small table); results do not depend on it */
} edfa_params;

/* Preconditioner sizes and diagnostics (host struct). */
typedef struct {
  int64_t nnz_G, nnz_F, nnz_H, nnz_S, nnz_GF, nnz_L, nnz_U, nnz_ML, nnz_MU;
  int32_t n_colors;
  int32_t max_pattern;      /* largest |Q^(m)| */
  double  mu;               /* preconditioner density of Section 4, nnz() counting what the
                               application stores and reads: 2 nnz(G_F) for A~_pipi^-1, the
                               coupling blocks, and for S~^-1 nnz(M_L) + nnz(M_U) (plus
                               nnz(L) + nnz(U) when isai_steps > 1) or nnz(L) + nnz(U) with
                               exact substitution */
  double  t_stage1_ms, t_stage2_ms;   /* device time of the last setup */
  int64_t nnz_H_raw;        /* entries of H~ before the post-filtration */
  int32_t htilde_retry_rows;/* rows of H~ whose first pass (small hash tables) overflowed and
                               were recomputed with large tables */
  int32_t color_rounds;     /* parallel colouring rounds of the last stage 2 ... */
  int32_t color_list_rounds;/* ... of which visited only a worklist of the uncoloured cells */
  int32_t cgs2_width;       /* basis vectors per block of the CGS2 dot passes (2, 4 or 8; set
                               by edfa_autotune) */
  int32_t chunks_ML, chunks_MU; /* row chunks (at most 768 entries each, the greedy row-aligned
                               cut of the natural-order rows) of the chunk kernel's descriptors
                               for M_L and M_U; 0 when the matrix has none (short rows) */
} edfa_precond_info;

/* Build the preconditioner: stage 1 (Algorithm 1: restricted SPD solves on static or
 * dynamically grown patterns, pre-filtration, H~ = G~ A_pipi F~, post-filtration on H~,
 * FSAI of -A_pipi) and stage 2 (Algorithm 2: S~ = A_pp - H~, post-filtration on S~,
 * multicolour ILU(0) of S~ and its sparse approximate inverses).  Synchronises the stream.
 * Errors: EDFA_ERR_NOT_SPD (cell index), EDFA_ERR_BREAKDOWN (ILU zero pivot),
 * EDFA_ERR_CAPACITY (pattern or H~ row longer than compiled maxima). */
edfa_status edfa_setup(edfa_system sys, const edfa_params *prm /* (host) */,
                       hipStream_t stream, edfa_precond *out);
/* Re-run stage 2 only, after edfa_update_dt (stage 1 is recycled, Section 3.1). */
edfa_status edfa_setup_stage2(edfa_precond pre, hipStream_t stream);
/* Re-run stage 1 and stage 2 with the same parameters on the same system (whose values may
 * have changed, e.g. after edfa_update_dt), reusing the handle's device memory: no device
 * allocation happens when the new patterns fit the previous ones.  Synchronises the stream. */
edfa_status edfa_resetup(edfa_precond pre, hipStream_t stream);
void edfa_precond_destroy(edfa_precond pre);
edfa_status edfa_precond_get_info(edfa_precond pre, edfa_precond_info *info /* (host) */);

/* Export a stage-1/2 artefact as CSR (rowptr rows+1, col, val; val converted to FP64):
 * 0 G~ (N_e x N_f^u), 1 F~^T (N_e x N_f^u, row m = column m of F~), 2 H~ before
 * post-filtration, 3 H~, 4 S~, 5 G_F (FSAI factor), 6 L (strict lower, colour order),
 * 7 U (colour order), 8 M_L, 9 M_U.  Query sizes with rowptr == NULL: then *nnz (host)
 * and *rows (host) are set and nothing is copied.  perm (N_e, may be NULL) receives
 * perm[new] = old of the colour order when what is 6..9.  Synchronises the stream. */
edfa_status edfa_export_precond(edfa_precond pre, int32_t what, int32_t *rowptr, int32_t *col,
                                double *val, int32_t *perm, int64_t *nnz, int32_t *rows,
                                hipStream_t stream);

/* z = P^-1 r (transpose = 0, eq. EDFA_prec) or z = P^-T r (transpose = 1).  N-vectors.
 * Asynchronous. */
edfa_status edfa_apply(edfa_precond pre, int32_t transpose, const double *r, double *z,
                       hipStream_t stream);

/* edfa_apply without any device allocation, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).  Its workspace
 * -- 2 N_f^u + 5 N_e values in the preconditioner's precision, plus two N-vectors of floats
 * for an FP32 preconditioner, each rounded up to 256 bytes -- lives in one static device
 * array of EDFA_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends; its address is
 * looked up on the first call on each device).  Every call on a GPU shares that array:
 * calls that overlap on one GPU race (serialise them, e.g. on one stream).  Results equal
 * edfa_apply's.  Errors: EDFA_ERR_ARG when the workspace exceeds the array (the message
 * gives both sizes), or when what the application reads does not exist yet and would have
 * to be allocated: the transposed factors (transpose = 1), the FP32 coupling blocks, the
 * descriptors of the 512-entry chunk kernel and the SELL layout of a long-row matrix (when
 * the tuner or edfa_set_variant chose those kernels) are built by a first edfa_apply of the
 * same kind (or a solve); EDFA_ERR_HIP.  Asynchronous. */
#define EDFA_NOALLOC_SCRATCH_BYTES (64u << 20)
edfa_status edfa_apply_noalloc(edfa_precond pre, int32_t transpose, const double *r, double *z,
                               hipStream_t stream);

typedef struct {
  int32_t restart;          /* Krylov dimension per cycle (GMRES(m)), 1..128 */
  int32_t max_iter;         /* total iterations over all cycles */
  int32_t flexible;         /* 1: flexible GMRES (stores Z); required when precision = 1 */
  int32_t transpose;        /* 1: solve A^T x = b with P^-T */
  int32_t use_graph;        /* 1: the first restart cycle runs eagerly; later cycles replay
                               one captured hipGraph of a whole cycle (no host checks inside
                               a cycle; converged grids are masked on the device) on a stream
                               of the solver's own, ordered after `stream` by events.  Same
                               results as use_graph = 0, bit for bit. */
  int32_t profile;          /* 1: time every product with the system matrix and every
                               application with events; 2: also every product inside the
                               applications (the events add a few microseconds per product);
                               eagerly run cycles only */
  double  rtol;             /* stop when ||b - A x|| <= rtol ||b|| (x0 = 0, Section 4) */
  int32_t method;           /* EDFA_GMRES (restart, flexible, use_graph apply) or
                               EDFA_BICGSTAB (the paper's solver, Section 4; restart,
                               flexible ignored, use_graph must be 0) */
} edfa_solve_params;
#define EDFA_GMRES    0
#define EDFA_BICGSTAB 1

typedef struct {
  int32_t iterations;       /* max over grids of the total inner iterations (Bi-CGStab: full
                               iterations, each with two products and two applications) */
  int32_t converged;        /* number of grids converged */
  int32_t cycles;           /* GMRES restart cycles / Bi-CGStab (re)starts */
  double  relres_est;       /* max over grids of the Arnoldi estimate / ||b|| */
  double  relres_true;      /* max over grids of the FP64 ||b - A x|| / ||b|| */
  double  t_solve_ms;       /* device time of the solve */
  double  spmv_avg_ms;      /* profile = 1: mean duration of one SpMV with A */
  int32_t spmv_count;
  double  apply_avg_ms;     /* profile = 1: mean duration of one preconditioner application */
  int32_t apply_count;
  double  slot_ms[16];      /* profile = 2: mean duration of one product with each matrix,
                               numbered as the slots of edfa_tune_slot (0 / 1: the system
                               matrix or its transpose) */
  int32_t slot_launches[16];/* profile = 2: products timed per slot */
} edfa_solve_info;

/* Solve A x = b (or A^T x = b), x0 = 0, each grid of a batch to its own rtol, with
 *  - EDFA_GMRES: restarted right-preconditioned GMRES(restart) (flexible: FGMRES).
 *    Synchronises the stream at the start of every restart cycle.  Inside an eagerly run
 *    cycle the host reads the convergence states every 8 iterations (16 for a batch), one
 *    reading late (it waits for the copy taken 8 iterations earlier while the following
 *    iterations are already queued), and stops the cycle once every grid has converged;
 *    the iterations queued past convergence skip their work.  A graph-replayed cycle
 *    synchronises only at its start.
 *  - EDFA_BICGSTAB: right-preconditioned Bi-CGStab (Section 4: x0 = 0, exit on
 *    ||r_k|| <= rtol ||r_0||).  Synchronises every 4 iterations; when every grid has
 *    stopped, the true residual confirms convergence, and a grid whose recurrence drifted
 *    or broke down restarts from its iterate with the shadow residual r^ = r.
 * b, x: N-vectors (x output only).  Returns EDFA_OK when every grid converged on its
 * true FP64 residual, EDFA_NOT_CONVERGED (the paper's "NC") when max_iter ends a grid
 * first (x = last iterate).  Errors: EDFA_ERR_NAN (b has a non-finite entry: ||b|| is
 * not finite; nothing is iterated), EDFA_ERR_ARG. */
edfa_status edfa_solve(edfa_system sys, edfa_precond pre, const double *b, double *x,
                       const edfa_solve_params *prm /* (host) */, hipStream_t stream,
                       edfa_solve_info *info /* (host), may be NULL */);

/* Transient sequence (Section 4).  Starting from the system's p_prev, each step
 *  - sets dt (edfa_update_dt: A_pp's diagonal and f_p; the previous step's pressure becomes
 *    p_prev), rebuilds stage 2 of `pre` on its recycled stage 1 (stage 1 depends only on
 *    A_pipi, A_pip and A_ppi, which dt does not change; Section 3, implementation details)
 *    and, when stage1_every > 0, stage 1 too on every stage1_every-th step (k = 0, k, 2k..);
 *  - solves from x0 = 0 with `solve` (GMRES or Bi-CGStab);
 *  - measures dp_max = max_E |p^E - p_prev^E| and the largest Courant number of
 *    eq. CFL_number, chi_inf = max_E Q^E dt / (Omega^E porosity), Q^E = sum_i |q_i^E| / 2
 *    with the local fluxes q^E = W^E (p^E 1 - pi^E) (eq. fluxes_MHFEM_3);
 *  - takes the next step dt = min(dt min(dt_mult, dp_target / dp_max), dt_max)
 *    (eq. delta_t_dyn; dp_max = 0 grows dt by dt_mult).
 * The sequence ends after n_steps steps, once the simulated time reaches t_end (> 0), or at
 * the first step that does not converge (its status is returned).  u (N, device) holds the
 * last step's solution; steps (host, n_steps entries, may be NULL) one record per step;
 * *taken (host, may be NULL) the number of steps.  On return the system holds the last
 * step's dt and p_prev, and `pre` the last step's stage 2.  Synchronises every step.
 * Errors: EDFA_ERR_ARG (n_steps < 1, dt0, dt_max, dp_target or porosity not > 0, dt_mult < 1),
 * and those of edfa_solve and edfa_setup_stage2. */
typedef struct {
  int32_t n_steps;          /* largest number of steps */
  double  t_end;            /* stop once the simulated time reaches it (<= 0: no limit) */
  double  dt0;              /* first step */
  double  dt_mult;          /* largest growth factor of dt per step (>= 1) */
  double  dt_max;           /* largest step (> 0; may be +infinity) */
  double  dp_target;        /* pressure change goal Delta p_T (> 0; +infinity: no goal) */
  double  porosity;         /* phi of the Courant number (> 0) */
  int32_t stage1_every;     /* 0: stage 1 built once (by edfa_setup); k > 0: rebuilt every k steps */
  edfa_solve_params solve;  /* per-step solve (rtol, method, restart, ...) */
} edfa_transient_params;

typedef struct {
  double  t;                /* simulated time at the end of the step */
  double  dt;               /* the step */
  double  dp_max;           /* max_E |p^E - p_prev^E| */
  double  chi_inf;          /* max_E chi^E (eq. CFL_number) */
  int32_t iterations;       /* Krylov iterations of the step */
  int32_t converged;        /* 1: the step's solve converged */
  double  t_setup_ms;       /* device time of the step's preconditioner refresh */
  double  t_solve_ms;       /* device time of the step's solve */
} edfa_step_info;

edfa_status edfa_transient(edfa_system sys, edfa_precond pre, const edfa_transient_params *prm,
                           double *u, hipStream_t stream, edfa_step_info *steps /* (host) */,
                           int32_t *taken /* (host) */);

/* Per-cell gradient of a scalar loss L(u) with respect to theta_E = ln(multiplier of K^E),
 * given the forward solution u and the adjoint lambda solving A^T lambda = dL/du:
 *   dL/dtheta_E = -lambda^T dR/dtheta_E,  R(u) = A u - b,
 * where dq^E/dtheta_E = q^E for the local fluxes (eq. fluxes_MHFEM_3) and the strong
 * flux (eq. fluxes_MHFEM_STRONG) varies as q_i W'_ii / (W_ii + W'_ii).  g: N_e.
 * Asynchronous. */
edfa_status edfa_grad_logk(edfa_system sys, const double *u, const double *lambda, double *g,
                           hipStream_t stream);

/* Launch-shape autotuner (not part of the paper's method; its results do not change what
 * is computed, only the rounding order of the sparse products and of the CGS2 dot
 * products).  It times the CGS2 dot pass with 2, 4 and 8 basis vectors per block (24
 * vectors of the system's size, cold cache) and keeps the fastest, and times every sparse matrix
 * that the solve and the application multiply -- the system matrix (and its transpose once
 * built), the FSAI factor and its transpose, the coupling blocks, the ILU(0) factors and
 * their approximate inverses -- with the one-lane-per-row SELL kernel and with the CSR
 * kernel at 2, 4, 8, 16 and 32 lanes per row, each at two load depths, and with the
 * row-chunk kernel, and keeps one of the fastest for each: the default kernel unless another
 * is at least 3% faster, else the first variant in table order within 3% of the fastest
 * (so equivalent kernels do not alternate from run to run); the choice stays with the
 * handle across later setups.  *tuned (host, may be NULL) receives the
 * number of matrices timed; slots (host, may be NULL) the timings of every slot.  Synchronises the stream.  Errors: EDFA_ERR_ARG, EDFA_ERR_HIP. */
#define EDFA_TUNE_SLOTS 16
#define EDFA_TUNE_VARIANTS 14
/* One matrix timed by the autotuner.  Slots: 0 A, 1 A^T, 2 G_F, 3 G_F^T, 4 L, 5 U, 6 M_L,
 * 7 M_U, 8 L^T, 9 U^T, 10 M_L^T, 11 M_U^T, 12 A_ppi, 13 A_pip, 14 A_pip^T, 15 A_ppi^T
 * (the FP32 copies for an FP32 preconditioner).  Variants v = 0..13, as (lanes per row,
 * entries in flight per lane): SELL (1, 4), (1, 8); CSR (2, 2), (2, 4), (4, 2), (4, 4),
 * (8, 2), (8, 4), (16, 2), (16, 4), (32, 2), (32, 4); 12: the chunk kernel (row-aligned
 * chunks of up to 768 entries, one wavefront each, 12 entries in flight per lane); 13: the
 * chunk kernel on chunks of up to 512 entries (8 in flight per lane).  The chunk variants run only on matrices whose mean row exceeds 24 entries
 * (where the first is the default; us[12], us[13] = infinity elsewhere).  us[v]: best of five launches of variant v, in microseconds; when some
 * matrix of the handle exceeds 8 MiB, a 512 MiB read before each timed launch evicts the
 * caches, as a full iteration does in the solve. */
typedef struct {
  int32_t rows, cols;   /* 0 rows: the matrix does not exist (yet); nothing was timed */
  int64_t nnz;
  int32_t variant;      /* the chosen variant */
  int32_t value_bytes;  /* 8 (FP64) or 4 (FP32) */
  int32_t sell_sorted;  /* 1: the SELL copy holds the rows sorted by length in windows */
  float sell_padding;   /* stored SELL entries / nnz */
  float us[EDFA_TUNE_VARIANTS];
} edfa_tune_slot;

edfa_status edfa_autotune(edfa_precond pre, hipStream_t stream, int32_t *tuned /* (host) */,
                          edfa_tune_slot *slots /* (host) EDFA_TUNE_SLOTS entries, may be NULL */);

/* Setup tuner.  Stage 1 sorts the cells into buckets by the capacity their pattern needs
 * (the smallest of the compiled capacities 16, 32, 40, 44, 48, 64, 128 holding the base or
 * static pattern plus n_ent) and runs the restricted solves of each bucket in one launch of
 * the kernel of that capacity (Algorithm 1's loop over the cells).  This call times each
 * non-empty bucket of the last setup with its own capacity and the next two larger ones
 * (best of three launches from scratch copies of the patterns) and keeps the fastest for
 * later setups of the handle (the default unless another is at least 3% faster); larger
 * capacities only change the rounding order of the local solves.  report (host, may be NULL)
 * receives the buckets.  Synchronises the stream.  Errors: EDFA_ERR_ARG, EDFA_ERR_HIP. */
#define EDFA_NCAP 7
typedef struct {
  int32_t buckets;                 /* EDFA_NCAP */
  int32_t capacity[EDFA_NCAP];     /* the bucket's own capacity */
  int32_t cells[EDFA_NCAP];        /* cells in the bucket at the last setup */
  int32_t chosen[EDFA_NCAP];       /* kernel capacity kept for the bucket */
  float   us[EDFA_NCAP][EDFA_NCAP];/* [bucket][capacity]: time of the bucket's launch (0: not timed) */
} edfa_setup_tune;
edfa_status edfa_autotune_setup(edfa_precond pre, hipStream_t stream,
                                edfa_setup_tune *report /* (host), may be NULL */);

/* Choice of the EDFA parameters for a system: the pattern technique and its (n_add, n_ent),
 * the static pattern (level, axis) and the filtration (tau_filt, filt_mode) are the
 * method's main sensitivity axis (Section 4, Tests 1-4, and the Discussion), and the best
 * setting depends on the grid and the conductivity field.  Each of the ncand candidates
 * (host array) is set up on `sys` and solved with `solve` from x0 = 0 against the
 * system's right-hand side; the device time of setup + solve is measured with events on
 * the stream.  *best (host) receives the index of the fastest candidate that converged;
 * times_ms (host, +infinity where a candidate failed or did not converge), iterations
 * (host, -1 where its setup failed) and status (host, its setup or solve status) may be
 * NULL.  A candidate whose setup fails (e.g. EDFA_ERR_CAPACITY) is skipped.  Nothing
 * persists: build the chosen preconditioner with edfa_setup.  Synchronises the stream.
 * Errors: EDFA_ERR_ARG (a bad candidate or solve parameter), EDFA_ERR_BREAKDOWN (no
 * candidate converged). */
edfa_status edfa_tune_params(edfa_system sys, const edfa_params *cand /* (host) */, int32_t ncand,
                             const edfa_solve_params *solve /* (host) */, hipStream_t stream,
                             int32_t *best /* (host) */, double *times_ms /* (host) */,
                             int32_t *iterations /* (host) */, int32_t *status /* (host) */);

/* Pin the sparse-product kernel of one slot (0 .. EDFA_TUNE_SLOTS - 1, numbered as for
 * edfa_tune_slot) or of every slot (slot = -1) to a variant (0 .. EDFA_TUNE_VARIANTS - 1;
 * -1 = the default choice at the next setup), as edfa_autotune would keep it: for callers
 * that want a fixed kernel (and rounding order) instead of a timed choice.  Takes effect
 * at once and survives later setups; the chunk variant applies only to matrices with long
 * rows (the others keep their kernel).  Host only, nothing is launched.
 * Errors: EDFA_ERR_ARG (slot or variant out of range). */
edfa_status edfa_set_variant(edfa_precond pre, int32_t slot, int32_t variant);

const char *edfa_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EDFA_H */
