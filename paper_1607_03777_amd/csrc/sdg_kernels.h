// Host-side launchers of the device kernels (all enqueue on stream s).
#pragma once

#include "sdg_common.h"

namespace sdg {

// SIP operator (sip_kernels.hip).  Vectors are batched: nbatch problems of
// the same mesh, consecutive in memory; eta is [nbatch][nel].
// var selects the tile shape (sip_tile_variants(k) candidates, 0 = default)
int sip_apply(const MeshDev& M, int k, int nbatch, const double* eta, const double* u, double* y,
              hipStream_t s, int var = 0);
int sip_residual(const MeshDev& M, int k, int nbatch, const double* eta, const double* b,
                 const double* u, double* r, hipStream_t s, int var = 0);
// r = b - A u restricted to its Q1 modes (i, j <= 1), wavefront kernel:
// rq[pb][e][d][j][i], 8 values per element (the layout of a k = 1 vector)
int sip_residual_q1(const MeshDev& M, int k, int nbatch, const double* eta, const double* b,
                    const double* u, double* rq, hipStream_t s);
int sip_residual_q1_f32(const MeshDev& M, int k, int nbatch, const double* eta, const float* b,
                        const float* u, float* rq, hipStream_t s);
int sip_apply_f32(const MeshDev& M, int k, int nbatch, const double* eta, const float* u, float* y,
                  hipStream_t s, int var = 0);
int sip_residual_f32(const MeshDev& M, int k, int nbatch, const double* eta, const float* b,
                     const float* u, float* r, hipStream_t s, int var = 0);
// y = A u with the wavefront kernel, and the partial sums of u.y: one per
// (problem, tile) at part[pb * tiles + tile] (capacity part_cap values);
// reduce_parts then forms u.y per problem.  sip_apply_dot_parts gives the
// number of partials.
int sip_apply_dot(const MeshDev& M, int k, int nbatch, const double* eta, const double* u, double* y,
                  double* part, int part_cap, hipStream_t s);
int sip_apply_dot_parts(const MeshDev& M, int k, int nbatch);
int sip_tile_variants(int k);
int sip_tile_default(int k, bool fp32);
void sip_tile_shape(int k, int var, int* tx, int* ty);
// Diagonal blocks A_KK of the listed elements (one workgroup per listed
// element): blocks[i][a][b] for element elems[i] of problem elems_pb[i].
int sip_block_list(const MeshDev& M, int k, const double* eta, const int* elems, int nlist,
                   double* blocks, hipStream_t s);
// Element-local continuous-Q1 matrices (volume and boundary faces only):
// clocal[pb][e][r][c], r, c = vertex*2 + component.
int sip_coarse_local(const MeshDev& M, int k, int nbatch, const double* eta, double* clocal,
                     hipStream_t s);
int div_apply(const MeshDev& M, int k, int nbatch, const double* u, double* q, hipStream_t s);
int grad_apply(const MeshDev& M, int k, int nbatch, const double* p, double* v, hipStream_t s);
int rhs_assemble(const MeshDev& M, int k, int nbatch, const double* eta, const double* f, const double* g,
                 double* F, double* G, hipStream_t s);

// Block Jacobi (block_kernels.hip)
// In-place inverse of nmat symmetric positive definite n x n matrices
// (Cholesky, triangular inverse, L^-T L^-1).  status[i] = 0 ok, 1 not SPD.
// packed (optional): also store X = L^{-1} as packed lower triangles
int spd_inverse(double* mats, int n, int nmat, int* status, hipStream_t s, double* packed = nullptr);
// Grouped block-Jacobi apply.  Elements perm[start .. start+count) of work
// item w = work[3w .. 3w+2] = (uid, start, count) share block uid; G
// elements per work item at most (bj_group_size).  scale[ge] = eta_rep / eta_ge;
// ab[pb] = Chebyshev coefficients of problem pb = ge / nel.
struct BjPlan {
  int nb, G, nwork, nel;
  const int* perm;
  const int* work;
  const double* scale;
  // blocks that few elements share (k <= 4): stream the quad-packed
  // inverses or factors through LDS, one row per lane, instead of the
  // matrix-core products (the FP64 smoother then takes the packed inverses)
  int stream = 0;
  // inside a batched CG iteration: elements of problems with active[pb] == 0
  // are skipped (null: none)
  const int* active = nullptr;
};
// largest G for an element block of nb unknowns (one wavefront per work item)
int bj_group_size(int nb);
// update flags: d' = b z + a d_old, x' = x + d' (see block_kernels.hip)
enum BjFlags { BJ_READ_X = 1, BJ_READ_D = 2, BJ_FOLD = 4, BJ_WRITE_D = 8, BJ_APPLY = 16 };
int bj_cheb_f64(const BjPlan& P, const double* binv, const double* r, const double* ab, double* d, double* x,
                int flags, hipStream_t s);
int bj_apply_f64(const BjPlan& P, const double* binv, const double* r, double* z, hipStream_t s);
// factored low-precision smoother: z = s_e X^T (X r), X packed lower triangular
int bj_tri_cheb_f32(const BjPlan& P, const float* X, const float* r, const double* ab, float* d, float* x,
                    int flags, hipStream_t s);
int bj_tri_cheb_bf16(const BjPlan& P, const uint16_t* X, const float* r, const double* ab, float* d, float* x,
                     int flags, hipStream_t s);
int bj_tri_apply_f32(const BjPlan& P, const float* X, const float* r, float* z, hipStream_t s);
int bj_tri_apply_bf16(const BjPlan& P, const uint16_t* X, const float* r, float* z, hipStream_t s);
// Convert FP64 inverses to FP32 / BF16 storage.
// packed FP64 factors X -> [nmat][n (n + 2) / 2] lower triangles of 2 x 2
// quads in FP32 / BF16 (tri_quad_size(n) values per block, n even)
int64_t tri_quad_size(int n);
// full symmetric FP64 inverses [nmat][n][n] -> [nmat][n (n + 2) / 2] lower
// triangles of 2 x 2 quads (the streaming FP64 smoother's operand)
int sym_quad_f64(const double* full, int n, int nmat, double* out, hipStream_t s);
int tri_quad_f32(const double* packed, int n, int nmat, float* out, hipStream_t s);
int tri_quad_bf16(const double* packed, int n, int nmat, uint16_t* out, hipStream_t s);

// Transfers and coarse levels (coarse_kernels.hip)
// the first h-level's zero-start Chebyshev step, fused into the kernel that
// restricts its right-hand side: x0 = d0 = cb D^{-1} rc, cb = ab0[2 pb + 1]
struct FirstStep {
  const double* dinv;
  const double* ab0;
  double *x0, *d0;
};
int p_restrict(const MeshDev& M, int k, int nbatch, const double* r, double* rc, hipStream_t s,
               const FirstStep* first = nullptr);
int p_prolong_add(const MeshDev& M, int k, int nbatch, const double* ec, double* u, hipStream_t s);
int p_restrict_f32(const MeshDev& M, int k, int nbatch, const float* r, double* rc, hipStream_t s,
                   const FirstStep* first = nullptr);
int p_prolong_add_f32(const MeshDev& M, int k, int nbatch, const double* ec, float* u, hipStream_t s);
int coarse_stencil_from_local(int nx, int ny, int nbatch, const double* clocal, double* st,
                              hipStream_t s);
int galerkin_coarsen(int nfx, int nfy, int nbatch, const double* stf, double* stc, hipStream_t s);
int stencil_apply(int nx, int ny, int nbatch, const double* st, const double* x, double* y,
                  hipStream_t s);
int stencil_residual(int nx, int ny, int nbatch, const double* st, const double* b,
                     const double* x, double* r, hipStream_t s);
int stencil_diag_inv(int nx, int ny, int nbatch, const double* st, double* dinv, hipStream_t s);
int h_restrict(int ncx, int ncy, int nbatch, const double* rf, double* rc, hipStream_t s);
// the same, with the coarse level's zero-start Chebyshev step fused:
// x0 = d0 = cb D^{-1} rc (ab0: the step's coefficients, [nbatch][2])
int h_restrict_first(int ncx, int ncy, int nbatch, const double* rf, double* rc, const double* dinv,
                     const double* ab0, double* x0, double* d0, hipStream_t s);
int h_prolong_add(int ncx, int ncy, int nbatch, const double* ec, double* xf, hipStream_t s);
// Q_0 coarse space (Section 6.1.1): probe vectors and the gather of A_0's
// stencil from A v (3 x 3 colouring of the elements), and the injection of
// the (0, 0) modes (restriction from the residual's Q_1 modes, 8 per
// element; prolongation into the (0, 0) modes)
int q0_probe_vec(int nx, int ny, int nbatch, int k, int cx, int cy, int d, double* v, hipStream_t s);
int q0_probe_gather(int nx, int ny, int nbatch, int k, int cx, int cy, int d, const double* y, double* st,
                    hipStream_t s);
int q0_restrict(int64_t nel_total, const double* rq1, double* rc, hipStream_t s);
int q0_restrict_f32(int64_t nel_total, const float* rq1, double* rc, hipStream_t s);
int q0_restrict_full(int64_t nel_total, int k, const double* r, double* rc, hipStream_t s);
int q0_prolong_add(int64_t nel_total, int k, const double* ec, double* x, hipStream_t s);
int q0_prolong_add_f32(int64_t nel_total, int k, const double* ec, float* x, hipStream_t s);
int stencil_to_dense(int nx, int ny, int nbatch, const double* st, double* dense, hipStream_t s);
int dense_matvec(int n, int nbatch, const double* A, const double* x, double* y, hipStream_t s);

// Vector kernels (vec_kernels.hip)
int vec_copy(int64_t n, const double* x, double* y, hipStream_t s);
// y[i rep + j] = x[i] for j < rep (rep copies of every value, in place order)
int vec_expand(int64_t n, int rep, const double* x, double* y, hipStream_t s);
int vec_scale_copy(int64_t n, double a, const double* x, double* y, hipStream_t s);  // y = a x
int vec_axpy(int64_t n, double a, const double* x, double* y, hipStream_t s);        // y += a x
int vec_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s);  // y = a x + b y
int vec_mul(int64_t n, const double* d, const double* x, double* y, hipStream_t s);  // y = d .* x
// Chebyshev update. mode 0: d = a d + b z, x += d; mode 1: d = b z, x = d;
// mode 2: d = b z, x += d.
int cheb_update(int64_t n, double a, const double* z, double b, double* d, double* x, int mode,
                hipStream_t s);
int cheb_update_f32(int64_t n, double a, const float* z, double b, float* d, float* x, int mode,
                    hipStream_t s);
// out[j] = <V_j, w> for j < m, V row-major [m][n]; result in device memory
// host_dst[0..n) = src[0..n) (host_dst pinned), then *host_seq = ++*dev_count
int publish_scalars(const double* src, int n, double* host_dst, unsigned* dev_count, unsigned* host_seq,
                    hipStream_t s);
// out[i] = sum over q < nseg of parts[q * n + i], in order of q
int seg_sum(int64_t n, int nseg, const double* parts, double* out, hipStream_t s);
// hs[pb] = done[pb] ? 0 : sqrt(max(sq[pb], 0))
int norm_mask(int nb, const double* sq, const int* done, double* hs, hipStream_t s);
// column j of the batched Arnoldi Hessenberg matrices from two Gram-Schmidt
// passes and ||w||^2, with the stopping test (layout at the kernel)
int arnoldi_col(int nb, int j, int m, const double* h0, const double* h1, const double* hsq, int* stop, int* ms,
                double* H, double* hs, hipStream_t s);
// out[j] = sum of part[j * nparts .. (j + 1) * nparts), in a fixed order
int reduce_parts(int nparts, int nout, const double* part, double* out, hipStream_t s);
int multi_dot(int64_t n, int m, const double* V, int64_t ldv, const double* w, double* out,
              double* scratch, hipStream_t s);
// w -= sum_j h[j] V_j (h in device memory)
int multi_axpy(int64_t n, int m, const double* V, int64_t ldv, const double* h, double* w,
               hipStream_t s);
// y = sum_j h[j] V_j + beta y (h in device memory)
int multi_combine(int64_t n, int m, const double* V, int64_t ldv, const double* h, double* y,
                  hipStream_t s);
int dot(int64_t n, const double* x, const double* y, double* out, double* scratch, hipStream_t s);
// reps consecutive copies of the same n values
int uniform_pm1(uint64_t seed, int64_t n, double* out, hipStream_t s, int reps = 1);
int d2f(int64_t n, const double* x, float* y, hipStream_t s);
int f2d(int64_t n, const float* x, double* y, hipStream_t s);
int pressure_project(int64_t nel, int np, double* p, double* scratch, hipStream_t s);
// Largest real part of the eigenvalues of the m x m upper Hessenberg matrix
// (column-major, leading dimension ld) -> out[0]; one thread.
int hessenberg_max_eig(const double* H, int m, int ld, double* out, hipStream_t s);

// ---- batched variants: vectors [nbatch][n], per-problem scalars in device arrays
int bmulti_dot(int64_t n, int nbatch, int m, const double* V, int64_t ldv, const double* w, double* out,
               double* scratch, hipStream_t s);  // out[pb][j]
int bmulti_axpy(int64_t n, int nbatch, int m, const double* V, int64_t ldv, const double* h, double* w,
                hipStream_t s);  // w[pb] -= sum_j h[pb][j] V_j[pb]
int bmulti_combine(int64_t n, int nbatch, int m, const double* V, int64_t ldv, const double* h, double* y,
                   hipStream_t s);  // y[pb] += sum_j h[pb][j] V_j[pb]
int bscale(int64_t n, int nbatch, const double* a, const double* x, double* y, int invert, hipStream_t s);
int cg_update1(int64_t n, int nbatch, const double* p, const double* q, double* x, double* r,
               const double* rz, const double* pq, const int* active, double* rr, double* scratch,
               hipStream_t s);
int cg_update2(int64_t n, int nbatch, const double* z, double* p, const double* rz_new, const double* rz_old,
               const int* active, hipStream_t s);
// The CG steps with the preceding reduction's second stage folded in (the
// same summation order as reduce_stage2, one launch fewer each):
// partials of <x[pb], y[pb]>, *nparts per problem (first stage only)
int bdot_parts(int64_t n, int nbatch, const double* x, const double* y, double* part, int cap, int* nparts,
               hipStream_t s, const int* active = nullptr);
// rz_new[pb] = sum of rzpart[pb * nparts ..]; then cg_update2
int cg_update2_red(int64_t n, int nbatch, const double* z, double* p, const double* rzpart, int nparts,
                   double* rz_new, const double* rz_old, const int* active, hipStream_t s);
// pq_out[pb] = sum of pqpart[pb * npq ..]; then cg_update1 with the partials
// of ||r||^2 in rrpart (*nrr per problem, at most rr_cap in all)
int cg_update1_red(int64_t n, int nbatch, const double* p, const double* q, double* x, double* r, const double* rz,
                   const double* pqpart, int npq, double* pq_out, const int* active, double* rrpart,
                   int rr_cap, int* nrr, hipStream_t s);
// rr[pb] = sum of rrpart[pb * nrr ..]; then publish_scalars(src, n, ...)
int publish_red(const double* rrpart, int nrr, int nbatch, double* rr, const double* src, int n, double* host_dst,
                unsigned* dev_count, unsigned* host_seq, hipStream_t s);
// ab[pb] = (a, b) Chebyshev coefficients per problem
int bcheb_update(int64_t n, int nbatch, const double* ab, const double* z, double* d, double* x, int mode,
                 hipStream_t s);
int bpressure_project(int64_t nel, int np, int nbatch, int64_t stride, double* p, double* scratch,
                      hipStream_t s);
int bhessenberg_max_eig(int nbatch, const double* H, const int* ms, int ld, int64_t hstride, double* out,
                        hipStream_t s);

int hcheb_step(int nx, int ny, int nbatch, const double* st, const double* dinv, const double* rhs,
               const double* xi, double* xo, double* d, const double* ab, int mode, hipStream_t s);

// coarse tail (the small h-levels in one workgroup per problem)
constexpr int TAIL_MAXLEV = 8;
struct TailLevel {
  int nx, ny;
  const double* st;
  const double* dinv;
  double *b, *x, *r, *d;
  const double* ab;  // [steps][nbatch][2] Chebyshev coefficients
};
struct TailArgs {
  int nlev, nbatch, steps;
  TailLevel lev[TAIL_MAXLEV];
  const double* dense;  // inverse of the last level, [nbatch][n2][n2]
};
int coarse_tail(const TailArgs& A, hipStream_t s);

}  // namespace sdg
