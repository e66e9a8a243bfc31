/*
 * sdg.h -- C ABI of the MI355X library for the nested viscous-block solve of
 * the block-preconditioned SIP discontinuous Galerkin Stokes solver
 * (Charrier, May & Schnepp, "Symmetric interior penalty discontinuous
 * Galerkin discretisations and block preconditioning for heterogeneous Stokes
 * flow").
 *
 * Problem statement (Sections 2-4): find u in Q_k^2 (discontinuous) and
 * p in Q_{k-1} on a regular Cartesian grid of the rectangle
 * [0, lx] x [0, ly] with element-wise constant viscosity eta_K > 0 and body
 * force f, such that A u + B p = F, B^T u = G (eq. discretestokes), with the
 * SIP form A_h (eq. stiffness_form) and divergence form B_h
 * (eq. divergence_form).  Boundary sides carry Navier (free slip), Neumann
 * or Dirichlet conditions; Dirichlet sides use the symmetric Nitsche/SIP
 * boundary terms with the Navier-face penalty (an addition to the paper, for
 * manufactured solutions).
 *
 * Coefficient layouts (all arrays are dense, row-major, FP64 unless stated):
 *   element e = iy*nx + ix;  basis psi_ij = (2/sqrt(hx hy)) lhat_i(xi)
 *   lhat_j(eta) with lhat_i = sqrt((2i+1)/2) L_i, i.e. L2(K)-orthonormal
 *   tensor Legendre modes (Section 5: orthogonal Legendre basis, orthonormal
 *   pressure basis).
 *   u, f  : [nel][2][k+1][k+1]   (component d, y-mode j, x-mode i)
 *   p     : [nel][k][k]
 *   eta   : [nel]
 *   g     : [2 ny + 2 nx][2][k+1] Dirichlet data per boundary face in the
 *           face-orthonormal basis sqrt(2/|e|) lhat_m; faces ordered left
 *           side (iy = 0..ny-1), right side, bottom side (ix = 0..nx-1), top.
 *   Coarse (continuous Q_1) nodal vectors: [(ny+1)(nx+1)][2], node
 *   jy*(nx+1) + jx, the two velocity components interleaved.
 *
 * Ownership: the caller owns every pointer it passes; the library copies
 * what it keeps.  "_dev" pointers are device (HBM) pointers valid on the
 * problem's stream; the others are host pointers.
 *
 * Errors: functions return SDG_OK (0), a negative error code, or a positive
 * soft outcome (SDG_NOT_CONVERGED: the output holds the last iterate).  No
 * exception crosses this ABI.  sdg_last_error() describes the last failure
 * of the calling thread.
 *
 * Threads: a context and the problems created from it may be used by one
 * thread at a time.
 */
#ifndef SDG_H
#define SDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define SDG_OK 0
#define SDG_ERR_INVALID (-1)     /* bad argument: eta <= 0 or non-finite, k out of range, NULL, n < 1 */
#define SDG_ERR_NOMEM (-2)       /* device allocation failed or over the context's memory budget */
#define SDG_ERR_DEVICE (-3)      /* HIP runtime error */
#define SDG_ERR_UNSUPPORTED (-4) /* e.g. singular all-Neumann viscous problem */
#define SDG_NOT_CONVERGED 1      /* iteration limit reached; last iterate returned */
#define SDG_BREAKDOWN 2          /* Krylov breakdown; last iterate returned */
#define SDG_FLOOR 3              /* the true residual stagnated above rtol within a small factor of
                                    the rounding floor of its evaluation (eps |K||x| / |b|, eps of
                                    FP64, or of the extended residual with opts.refine); the output
                                    is the best iterate and stats.rel_residual the residual reached.
                                    A stagnation above that floor returns SDG_NOT_CONVERGED. */

/* boundary side types, sides ordered left, right, bottom, top */
#define SDG_NAVIER 0
#define SDG_NEUMANN 1
#define SDG_DIRICHLET 2

/* arithmetic of the smoother (block inverses) and the operator apply inside
 * the multigrid cycle */
#define SDG_FP64 0
#define SDG_FP32 1
#define SDG_BF16 2

#define SDG_KMAX 6

typedef struct sdg_mesh {
  int32_t nx, ny;  /* elements per direction, >= 1 */
  double lx, ly;   /* domain size, > 0 */
  int32_t k;       /* velocity order, 1..SDG_KMAX; pressure order k-1 */
  int32_t bc[4];   /* SDG_NAVIER / SDG_NEUMANN / SDG_DIRICHLET per side */
} sdg_mesh;

typedef struct sdg_options {
  double rtol;            /* outer relative residual (2-norm, x0 = 0) */
  double inner_rtol;      /* inner CG tolerance of the Stokes preconditioner (Section 8.1: 1e-3) */
  int32_t max_it;         /* outer iteration limit */
  int32_t inner_max_it;   /* inner iteration limit */
  int32_t restart;        /* FGMRES restart length */
  int32_t smooth_dg;      /* Chebyshev steps before and after on the DG level (Section 8: 2) */
  int32_t smooth_h;       /* Chebyshev steps on each h-level (Section 8: 3) */
  int32_t coarsest_n;     /* h-coarsening stops at <= this many elements per direction (Q_0: node
                             intervals of the element-centre grid, one less than the elements) */
  int32_t eig_steps;      /* Arnoldi steps for lambda* (Section 6: 10) */
  double cheb_lo, cheb_hi;/* Chebyshev bounds as fractions of lambda* (Section 6: 0.1, 1.1) */
  int32_t prec_smoother;  /* SDG_FP64: full block inverses; SDG_FP32 / SDG_BF16: inverse Cholesky
                             factors X = L^{-1} (stored once, packed lower triangle),
                             smoother X^T X */
  int32_t prec_apply;     /* SDG_FP64 / SDG_FP32: operator apply inside the cycle */
  int32_t viscous_krylov; /* viscous solves and the inner solve of the Stokes preconditioner:
                             0: CG (Section 8.1); 1: FGMRES (standalone viscous solves; needed
                             when the cycle is not exactly linear); 2: GCR (Section 8.3) */
  int32_t dedup;          /* 1: share block inverses between elements with equal normalised blocks */
  uint64_t seed;          /* stream of the SplitMix64 start vectors of the eigen-estimates */
  int32_t graphs;         /* 1: each CG iteration after the first replays a captured HIP graph
                             (V-cycle, updates, operator apply, readback of the scalars); the
                             arithmetic is that of the launches it replaces.  Off while tracing. */
  int32_t refine;         /* 0: FP64 iterate and true residual (the residual stops at the FP64
                             rounding floor, about eps |K||x| / |b|).  1: iterative refinement
                             in extended precision (in place of the quadruple-precision Krylov
                             arithmetic of Section 8.3.1): the iterate is a double-FP64 pair and
                             the true residual is evaluated in double-FP64 with operator
                             coefficients exact to long double; FGMRES restarts (Stokes, or
                             viscous_krylov = 1) or CG corrections (viscous, CG) solve for the
                             correction in FP64.  rtol then bounds the residual of the pair. */
  int32_t outer_krylov;   /* Stokes solve: 0: right-preconditioned FGMRES (Section 5, 8.1);
                             1: GCR (Section 8.3, six-inclusion experiment) */
  int32_t coarse_space;   /* p-coarse space of the viscous preconditioner (Section 6): 0: Q_1^2
                             projected to continuous bilinears, with an h-hierarchy on the
                             mesh vertices (A_hp(Q_1), Section 6.1.2); 1: element-wise
                             constants Q_0^2, Galerkin A_0, with an h-hierarchy on the grid
                             of element centres, which coarsens on meshes with an odd
                             number of elements per direction (A_hp(Q_0), Section 6.1.1);
                             on other meshes A_0 is solved directly (A_p(Q_0), at most
                             2048 unknowns) */
} sdg_options;

typedef struct sdg_stats {
  int32_t status;          /* return code of the solve */
  int32_t outer_its;       /* FGMRES (Stokes) or Krylov (viscous) iterations */
  int32_t inner_its_total; /* inner CG iterations summed (Stokes) */
  int32_t inner_its_max;
  double rel_residual;     /* final true relative residual ||b - K x|| / ||b|| in FP64 */
  double setup_ms, solve_ms;
} sdg_stats;

typedef struct sdg_ctx sdg_ctx;
typedef struct sdg_problem sdg_problem;

/* ---- context -------------------------------------------------------------
 * sdg_create: bind the calling thread to HIP device `device` and create a
 * context.  mem_budget (bytes) caps the device memory of all problems of the
 * context (0 = no cap).  */
int sdg_create(int device, size_t mem_budget, sdg_ctx** out);
/* Releases the context; if problems created from it are still alive, the
 * release happens when the last of them is destroyed. */
void sdg_destroy(sdg_ctx* ctx);
/* Message describing the last error on the calling thread ("" if none). */
const char* sdg_last_error(void);
/* Default options: rtol 1e-8, inner_rtol 1e-3 (Section 8.1), restart 30,
 * smooth_dg 2, smooth_h 3 (Section 8), coarsest_n 8, eig_steps 10,
 * cheb 0.1/1.1 (Section 6), FP64 everywhere, CG, dedup on, seed 0, graphs on. */
void sdg_options_default(sdg_options* opts);
/* Device bytes a problem of this size needs at most (deterministic, host
 * only): every element block is counted as distinct, as for a viscosity
 * that varies from element to element; deduplication (opts->dedup) can
 * only lower what is used.  stokes != 0 adds the pressure and FGMRES
 * workspaces.  The request server counts the distinct blocks of each
 * request from its viscosity instead. */
size_t sdg_required_bytes(const sdg_mesh* mesh, const sdg_options* opts, int stokes);
size_t sdg_required_bytes_batch(const sdg_mesh* mesh, const sdg_options* opts, int stokes, int nbatch);

/* ---- problem setup (Sections 4 and 6) ---------------------------------------
 * Copies eta (device pointer, nel values) and performs the setup of the
 * hp-multilevel preconditioner on the device: face penalties
 * (eq. eta_face, eq. const_trace_face, eq. sipg_penalty at its lower bound),
 * element-block Jacobi inverses (eq. smoother; diagonal blocks of A), the
 * Galerkin coarse operators A_1 and A_{1,c} = P_cd^T A_1 P_cd
 * (Section 6.1.2), the Galerkin h-hierarchy, the coarsest dense factor and
 * the Chebyshev bounds (Section 6).  stream is a hipStream_t (NULL = the
 * null stream); every later call on the problem is ordered on it. */
int sdg_problem_create(sdg_ctx* ctx, const sdg_mesh* mesh, const sdg_options* opts,
                       const double* eta_dev, void* stream, sdg_problem** out);
/* Batched form: nbatch (1..4096) independent problems on the same mesh and
 * options, each with its own viscosity (eta_dev: [nbatch][nel]).  Every
 * operator and solve of the problem object then acts on all of them: device
 * arrays are [nbatch][...] (problem after problem), stats/bounds/lambda
 * outputs hold nbatch entries.  Each problem converges on its own test; a
 * problem that has converged keeps its iterate while the others continue.
 * Element blocks are shared across the batch when their normalised blocks
 * coincide (opts.dedup).  sdg_problem_create is the batch of one. */
int sdg_problem_create_batch(sdg_ctx* ctx, const sdg_mesh* mesh, const sdg_options* opts, int nbatch,
                             const double* eta_dev, void* stream, sdg_problem** out);
int sdg_problem_batch(const sdg_problem* prob, int* nbatch);
/* Storage precision of the element-block factors the smoother applies
 * (SDG_FP64: the FP64 inverse; SDG_FP32 or SDG_BF16: the inverse Cholesky
 * factor).  BF16 is asked for with opts.prec_smoother; the setup keeps FP32
 * factors instead when the BF16 ones put the largest eigenvalue of the
 * smoothed DG operator (Arnoldi estimate, Section 6) above 4, against about
 * 2 with exact inverses: blocks whose condition approaches the reciprocal
 * of the BF16 unit (viscosity jumps of 10^6 between neighbours). */
int sdg_problem_smoother_precision(const sdg_problem* prob, int* prec);
void sdg_problem_destroy(sdg_problem* prob);
/* Number of multigrid levels (1 DG level + CG-Q_1 h-levels) and the
 * Chebyshev bounds [lambda_0, lambda_1] per level ([nbatch][nlevels][2];
 * the coarsest CG level is solved directly, its entries are 0 and ignored). */
int sdg_problem_levels(const sdg_problem* prob, int* nlevels);
int sdg_get_bounds(const sdg_problem* prob, double* bounds);
int sdg_set_bounds(sdg_problem* prob, const double* bounds);
/* Largest Ritz value lambda* of eig_steps Arnoldi steps on M^{-1} A at
 * level `level` (0 = DG level), started from the SplitMix64 vector of
 * stream seed + level*2^32 (Section 6: ten GMRES iterations with a random
 * right-hand side).  lambda_out: nbatch values.  hess (may be NULL):
 * [nbatch][steps][steps+1], column j of problem pb holding rows 0..steps of
 * its Hessenberg matrix. */
int sdg_eig_estimate(sdg_problem* prob, int level, double* lambda_out, double* hess);

/* ---- operators on device vectors (for parity and composition) -------------
 * y = A u, A the SIP matrix of eq. (stiffness_form) (FP64). */
int sdg_apply_viscous(sdg_problem* prob, const double* u_dev, double* y_dev);
/* r = b - A u (fused residual). */
int sdg_residual_viscous(sdg_problem* prob, const double* b_dev, const double* u_dev,
                         double* r_dev);
/* y = A u with the FP32 kernel used inside the multigrid cycle (float in/out). */
int sdg_apply_viscous_f32(sdg_problem* prob, const float* u_dev, float* y_dev);
/* q = B^T u (discrete divergence, eq. divergence_form), q: [nel][k][k]. */
int sdg_apply_div(sdg_problem* prob, const double* u_dev, double* q_dev);
/* v = B p (discrete gradient), v: velocity layout. */
int sdg_apply_grad(sdg_problem* prob, const double* p_dev, double* v_dev);
/* z = M_k^{-1} r, M_k the element-block Jacobi operator (eq. smoother),
 * in the precision chosen by opts.prec_smoother (FP64 in/out). */
int sdg_apply_blockjacobi(sdg_problem* prob, const double* r_dev, double* z_dev);
/* Dense diagonal blocks of A: blocks [nel][nb][nb], nb = 2(k+1)^2, row =
 * test mode, column = trial mode (FP64, before inversion). */
int sdg_get_blocks(sdg_problem* prob, double* blocks_dev);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * blocks as sdg_get_blocks, which allocates an element list per call, with
 * that list in a file-scope device array of the library instead (limit:
 * nel * nbatch <= 1048576 elements, else SDG_ERR_INVALID; the array, 4 MiB,
 * is held on each device the library runs on until the process ends).  No
 * hipMalloc, hipFree or allocating call; the work is enqueued on the
 * problem's stream.  All calls on one device share the array: calls that
 * overlap on one device (several streams or threads) race. */
int sdg_get_blocks_noalloc(sdg_problem* prob, double* blocks_dev);
/* rc = P_cd^T R_k^1 r (Section 6: truncation to Q_1 modes, then the
 * transpose of the element-wise nodal-to-modal map, Section 6.1.2). */
int sdg_p_restrict(sdg_problem* prob, const double* r_dev, double* rc_dev);
/* u += P_k^1 P_cd ec (prolongation, P = R^T). */
int sdg_p_prolong_add(sdg_problem* prob, const double* ec_dev, double* u_dev);
/* Stencil of the coarse operator at h-level `level` (0 = A_{1,c} on the
 * finest CG grid): [36][nodes] as [(dy+1)*3+(dx+1)][d][c][node] with
 * (A x)_{node,d} = sum_{dx,dy,c} S[..][d][c][node] x_{node+(dx,dy),c}. */
int sdg_get_coarse_stencil(sdg_problem* prob, int level, double* stencil_dev,
                           int* nx_out, int* ny_out);
/* One application of the hp-multilevel preconditioner (Algorithm 1 with
 * zero initial guess, the h-cycle as coarse solve): x = B_mg b. */
int sdg_vcycle(sdg_problem* prob, const double* b_dev, double* x_dev);
/* Right-hand sides: F = f + Dirichlet lift, G = int q (g.n) on Dirichlet
 * sides (eq. rhs_f plus the Nitsche terms).  g_dev may be NULL. */
int sdg_assemble_rhs(sdg_problem* prob, const double* f_dev, const double* g_dev,
                     double* F_dev, double* G_dev);

/* ---- solves on device arrays ------------------------------------------------
 * Viscous block: u = A^{-1} F with F assembled from f (and g) by the
 * hp-multilevel preconditioned Krylov method of Sections 6 and 8, to
 * opts.rtol.  Blocks the calling thread until done.  stats (may be NULL)
 * receives nbatch entries; the return value is SDG_OK when every problem
 * converged, else the largest soft outcome, or a negative error. */
int sdg_solve_viscous_dev(sdg_problem* prob, const double* f_dev, const double* g_dev,
                          double* u_dev, sdg_stats* stats);
/* Stokes: right-preconditioned FGMRES on eq. (discretestokes) with the
 * upper block-triangular preconditioner of eq. (discretestokespc),
 * S* = diag(1/eta_K) (Section 5) and the inner viscous solve to
 * opts.inner_rtol; the constant-pressure null space is projected out when
 * no side is Neumann and p is returned with zero mean. */
int sdg_solve_stokes_dev(sdg_problem* prob, const double* f_dev, const double* g_dev,
                         double* u_dev, double* p_dev, sdg_stats* stats);

/* Same solves, returning the iterate of opts.refine = 1 as double-FP64 pairs:
 * u = u_hi + u_lo (and p = p_hi + p_lo), u_hi the rounded sum.  The low
 * parts may be NULL; with opts.refine = 0 they are zero. */
int sdg_solve_viscous_ext_dev(sdg_problem* prob, const double* f_dev, const double* g_dev,
                              double* u_hi_dev, double* u_lo_dev, sdg_stats* stats);
int sdg_solve_stokes_ext_dev(sdg_problem* prob, const double* f_dev, const double* g_dev,
                             double* u_hi_dev, double* u_lo_dev, double* p_hi_dev, double* p_lo_dev,
                             sdg_stats* stats);
/* Extended-precision residual (the refinement residual of opts.refine):
 * stokes = 0: r = b - A x;  stokes != 0: [r_u; r_p] = [b_u; b_p] - K [x; p]
 * with K = [A B; B^T 0] (eq. discretestokes), the vectors stacked
 * velocity (all problems) then pressure (all problems) as in the Stokes
 * solves.  x = x_hi + x_lo (x_lo may be NULL), evaluated in double-FP64
 * arithmetic with the unit blocks of eq. stiffness_form and
 * eq. divergence_form integrated in long double, rounded to FP64. */
int sdg_residual_ext(sdg_problem* prob, int stokes, const double* b_dev, const double* x_hi_dev,
                     const double* x_lo_dev, double* r_dev);
/* y = |K| |x| in FP64 (stokes as above): the scale of rounding errors in
 * K x, behind the floor estimate eps |K||x| / |b| of SDG_FLOOR. */
int sdg_abs_apply(sdg_problem* prob, int stokes, const double* x_dev, double* y_dev);

/* ---- one-shot solves on host arrays (copy in, setup, solve, copy out) ------ */
int sdg_solve_viscous(sdg_ctx* ctx, const sdg_mesh* mesh, const sdg_options* opts,
                      const double* eta, const double* f, const double* g, double* u,
                      sdg_stats* stats);
int sdg_solve_stokes(sdg_ctx* ctx, const sdg_mesh* mesh, const sdg_options* opts,
                     const double* eta, const double* f, const double* g, double* u,
                     double* p, sdg_stats* stats);

/* ---- batching form: many viscous solves of different meshes and orders ---
 * n independent viscous solves A_i u_i = F_i (host arrays: eta[i] of nel_i,
 * f[i] and u[i] of nu_i = nel_i 2 (k_i+1)^2 values; u_lo[i] optional, the
 * low parts of the refined iterate; no Dirichlet data) under one set of
 * options.  Requests of identical mesh and order share one batched problem
 * object (their launches cover all of them); with viscous_krylov = 0 (CG,
 * with or without refinement) the CG iterations of all groups run in
 * lockstep and every iteration of every group is one replay of a combined
 * HIP graph with one parallel branch per group, so problems of different
 * sizes and orders overlap on the device in a single launch.  Other Krylov
 * choices solve the groups one after another.  The groups are set up from
 * up to 8 host threads that the call starts and joins (each group on a
 * stream of its own until the solve); an error in one group's setup is
 * returned, with its message, by the call.  stats: n entries, in request
 * order.  Returns SDG_OK when all converged, else the largest soft outcome,
 * or a negative error. */
int sdg_solve_viscous_batch(sdg_ctx* ctx, int n, const sdg_mesh* meshes, const sdg_options* opts,
                            const double* const* eta, const double* const* f, double* const* u,
                            double* const* u_lo, sdg_stats* stats);

/* ---- SplitMix64 (counter form) on the device, for parity of start vectors --
 * out[i] = 2 * (z_i >> 11) * 2^-53 - 1, z_i the i-th SplitMix64 output of
 * state `seed` (Steele, Lea & Flood 2014). */
int sdg_uniform_pm1(sdg_ctx* ctx, uint64_t seed, int64_t n, double* out_dev, void* stream);

/* ---- request server (continuous batching of solves on one GPU) --------------
 * A server owns `slots` worker threads, each with its own HIP stream; while
 * it runs, the CG iterations of all slots are launched together, one
 * combined HIP graph per iteration boundary, so a request admitted into a
 * free slot joins the running launches at its first iteration.
 * sdg_submit copies the request's host inputs (the caller may free them at
 * once) and queues it.  A free slot takes the oldest queued request whose
 * device memory (sdg_required_bytes_batch plus its input and output arrays)
 * fits into what `mem_budget` has left (0 = 90% of the free device memory at
 * creation), together with queued requests of the identical shape (mesh,
 * options, kind, Dirichlet data present or not), up to max_batch, which run
 * as one batched problem.  A request that does not fit may be overtaken by
 * later ones at most `bypass` times.  Each request's solver state stays on
 * the device from setup to the copy of its result; requests on different
 * slots overlap on the device.  Results are those of the same solve alone up
 * to rounding order (a batch shares element blocks scaled by the viscosity
 * ratio).  sdg_wait blocks until the request is done, copies u (and p for
 * Stokes) to the caller's host arrays (either may be NULL) and returns the
 * solve's status.  sdg_req_free releases a request (also one still
 * running: it is then freed when it ends).  sdg_server_destroy finishes every
 * queued request, then stops the workers; requests must be freed by the
 * caller.  A request larger than the budget is rejected with SDG_ERR_NOMEM. */
#define SDG_VISCOUS 0
#define SDG_STOKES 1
typedef struct sdg_server_config {
  int32_t slots;     /* concurrent launch groups, 1..64 (default 4) */
  int32_t max_batch; /* requests per launch group, 1..4096 (default 16) */
  int32_t bypass;    /* overtakes of a waiting head request (default 8) */
  int32_t combine;   /* 1: combine the CG iterations of the slots into one
                        launch per iteration (experimental, off by default:
                        runs with 8 slots and many requests have ended in a
                        host crash whose cause is not known); 0: each slot
                        launches its own iterations */
  size_t mem_budget; /* bytes; 0 = 90% of free device memory */
} sdg_server_config;
typedef struct sdg_req_info {
  double submit_ms, start_ms, end_ms; /* steady-clock times (ms) */
  int32_t batch;                      /* requests in its launch group */
  int32_t pad_;
  size_t bytes;                       /* its admission estimate */
} sdg_req_info;
typedef struct sdg_server sdg_server;
typedef struct sdg_req sdg_req;
void sdg_server_config_default(sdg_server_config* cfg);
int sdg_server_create(sdg_ctx* ctx, const sdg_server_config* cfg, sdg_server** out);
void sdg_server_destroy(sdg_server* srv);
int sdg_submit(sdg_server* srv, const sdg_mesh* mesh, const sdg_options* opts, int kind,
               const double* eta, const double* f, const double* g, sdg_req** out);
int sdg_poll(sdg_req* req, int* done);
int sdg_wait(sdg_req* req, double* u, double* p, sdg_stats* stats, sdg_req_info* info);
void sdg_req_free(sdg_req* req);
int sdg_server_stats(sdg_server* srv, int64_t* completed, size_t* peak_bytes, int* peak_busy,
                     size_t* budget);
/* Iteration-level batching of a server created with combine = 1 (all zero
 * otherwise): CG iterations launched
 * (launches), of which combined launches covering the iterations of several
 * slots at once (combined), the most slots one launch covered, and the
 * combined graphs instantiated (graphs; one per new set of running solves,
 * at most 64 kept).  Any output pointer may be NULL. */
int sdg_server_launch_stats(sdg_server* srv, int64_t* launches, int64_t* combined, int* max_width,
                            int64_t* graphs);
/* Host-only run of the same admission policy on a virtual clock: request i
 * arrives at arrival_ms[i], holds a slot and bytes[i] for service_ms[i];
 * start_ms[i] receives its start.  No GPU is used (capacity planning, tests). */
int sdg_admission_simulate(int n, const double* arrival_ms, const double* service_ms,
                           const size_t* bytes, int slots, size_t budget, int bypass,
                           double* start_ms);

/* ---- tile shapes of the SIP operator kernels and their autotuner -------------
 * The SIP apply/residual kernels work on TX x TY element tiles; each order k
 * has sdg_tile_variants() candidates: variant 0 is the wavefront kernel (one
 * 64-lane wavefront per tile, k+1 lanes per element), variants 1.. the
 * 256-thread LDS tile kernel at several shapes (sdg_tile_shape).  A new
 * problem starts from a measured default per order and precision (or the
 * shape tuned for its size earlier in the process); sdg_get_tile reads and
 * sdg_set_tile picks one for a problem: kernel 0 = apply (y = A u),
 * 1 = residual (r = b - A u); precision SDG_FP64 or SDG_FP32 (the fine-level
 * cycle of the low-precision forms).  sdg_autotune times every candidate on
 * the problem's own shape and stream (reps launches each, HIP events, the
 * problem's Krylov scratch vectors overwritten), keeps the fastest, and
 * records it for every problem later created in this process with the same
 * (k, nx, ny, nbatch).  variants[4] and us[4] (optional) receive the choice
 * and its time per launch for [apply FP64, apply FP32, residual FP64,
 * residual FP32]; FP32 entries are -1 / 0 when the problem has no FP32
 * cycle.  Results are identical up to rounding order for every shape. */
int sdg_tile_variants(int k, int* count);
int sdg_tile_shape(int k, int variant, int* tx, int* ty);
int sdg_get_tile(const sdg_problem* prob, int kernel, int precision, int* variant);
int sdg_set_tile(sdg_problem* prob, int kernel, int precision, int variant);
int sdg_autotune(sdg_problem* prob, int reps, int* variants, double* us);

/* ---- kernel tracing ---------------------------------------------------------
 * While tracing is on, every launch of the traced kernel classes made by
 * problems of this context is bracketed by two HIP events on the problem's
 * stream, and its algorithmic HBM bytes are recorded (vectors read and
 * written once, the viscosity, the smoother's scale and permutation; blocks
 * and stencils that stay cache-resident are not counted).
 * sdg_trace_enable(ctx, 1) clears the counters and starts; (ctx, 0) stops.
 * sdg_trace_read waits for the recorded events and returns, for one class,
 * the number of launches, their summed duration (ms) and summed bytes; any
 * pointer may be NULL.  Tracing adds two event records per traced launch. */
#define SDG_TRACE_SIP_APPLY 0    /* y = A u (FP64 or FP32) */
#define SDG_TRACE_SIP_RESIDUAL 1 /* r = b - A u (FP64 or FP32) */
#define SDG_TRACE_SMOOTHER 2     /* block-Jacobi apply / Chebyshev step */
#define SDG_TRACE_COARSE_TAIL 3  /* small h-levels and coarsest solve (bytes not counted) */
#define SDG_TRACE_CLASSES 4
int sdg_trace_enable(sdg_ctx* ctx, int on);
int sdg_trace_read(sdg_ctx* ctx, int kclass, int64_t* launches, double* total_ms, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* SDG_H */
