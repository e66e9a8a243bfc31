// Problem setup and solver orchestration behind the C ABI (include/sdg.h).
//
// Setup (Sections 4 and 6): element viscosity -> deduplicated diagonal
// blocks of A (eq. smoother) and their inverses; A_{1,c} = P_cd^T A_1 P_cd
// (Section 6.1.2) from element-local matrices; the Galerkin h-hierarchy;
// the dense inverse of the coarsest operator; Chebyshev bounds
// [cheb_lo, cheb_hi] * lambda* with lambda* the largest Ritz value of
// eig_steps Arnoldi steps on M^{-1} A (Section 6).
//
// Solve: the two-level cycle of Algorithm 1 (Chebyshev with element-block
// Jacobi, 2 steps before and after; the coarse solve is one h-cycle with
// Chebyshev/point-Jacobi smoothing, 3 steps, and the dense coarsest
// inverse), preconditioning CG (Section 8.1) or FGMRES for the viscous
// block, and right-preconditioned FGMRES with the upper block-triangular
// preconditioner for Stokes (Section 5).  The Krylov loops run on the host
// and read one scalar per reduction back; all vector work runs in the
// library's kernels.
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "sdg_common.h"
#include "sdg_kernels.h"

// A context is freed when it has been destroyed and its last problem is
// gone, so problems destroyed after their context stay valid.
struct sdg_ctx {
  int device = 0;
  size_t budget = 0;
  size_t used = 0;
  int live = 0;
  bool closing = false;
};

namespace sdg {
static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }
const char* get_error() { return g_err.c_str(); }
}  // namespace sdg

using namespace sdg;

namespace {

struct CLevel {
  int nx = 0, ny = 0, nn = 0;
  double* st = nullptr;
  double* dinv = nullptr;
  double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *d = nullptr;
  double* dense = nullptr;
  double lmin = 0, lmax = 0;
  bool coarsest = false;
};

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct sdg_problem {
  sdg_ctx* ctx = nullptr;
  sdg_mesh mesh{};
  sdg_options opt{};
  MeshDev M{};
  hipStream_t s = nullptr;
  int k = 0, K1 = 0, NB = 0, NPE = 0;
  int nel = 0;
  int64_t nu = 0, np = 0;
  std::vector<void*> allocs;
  size_t bytes = 0;
  double* eta = nullptr;
  double* etap = nullptr;  // eta expanded over pressure modes (S*^{-1})
  std::vector<double> eta_host;
  // block Jacobi
  int nuniq = 0;
  int* ids = nullptr;
  double* scale = nullptr;
  double* binv = nullptr;
  float* binv32 = nullptr;
  uint16_t* binv16 = nullptr;
  std::vector<int> reps;
  // DG cycle work vectors (FP64 and FP32)
  double *vr = nullptr, *vz = nullptr, *vd = nullptr;
  float *fb = nullptr, *fx = nullptr, *fr = nullptr, *fz = nullptr, *fd = nullptr;
  double lmin0 = 0, lmax0 = 0;
  std::vector<CLevel> lev;
  // Krylov work
  double* red = nullptr;    // reduction scratch
  double* dsc = nullptr;    // device scalars
  double* hsc = nullptr;    // pinned host scalars
  double *cg_r = nullptr, *cg_z = nullptr, *cg_p = nullptr, *cg_q = nullptr;
  // FGMRES (viscous or Stokes): V [(m+1) x n], Z [m x n]
  double *gV = nullptr, *gZ = nullptr, *gw = nullptr, *gt = nullptr;
  int64_t gn = 0;
  // stats of the last solve
  int inner_total = 0, inner_max = 0;
  bool neumann = false;
  double setup_ms = 0;
};

namespace {

constexpr int RED_SCRATCH = 512 * 64;

int palloc(sdg_problem* P, void** out, size_t bytes) {
  *out = nullptr;
  if (bytes == 0) return SDG_OK;
  if (P->ctx->budget && P->ctx->used + bytes > P->ctx->budget) {
    set_error("device memory budget exceeded");
    return SDG_ERR_NOMEM;
  }
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
    *out = nullptr;
    return SDG_ERR_NOMEM;
  }
  P->allocs.push_back(*out);
  P->bytes += bytes;
  P->ctx->used += bytes;
  return SDG_OK;
}

template <typename T>
int palloc_t(sdg_problem* P, T** out, int64_t n) {
  void* p = nullptr;
  int rc = palloc(P, &p, (size_t)n * sizeof(T));
  *out = (T*)p;
  return rc;
}

bool mesh_ok(const sdg_mesh* m) {
  if (!m) return false;
  if (m->nx < 1 || m->ny < 1 || m->k < 1 || m->k > SDG_KMAX) return false;
  if (!(m->lx > 0) || !(m->ly > 0)) return false;
  for (int i = 0; i < 4; ++i)
    if (m->bc[i] < 0 || m->bc[i] > 2) return false;
  return true;
}

// ---------------------------------------------------------------------------
// dedup keys: face kinds and neighbour/self viscosity ratios
// ---------------------------------------------------------------------------
struct BlockKey {
  int kind[4];
  double ratio[4];
  bool operator==(const BlockKey& o) const {
    for (int i = 0; i < 4; ++i)
      if (kind[i] != o.kind[i] || ratio[i] != o.ratio[i]) return false;
    return true;
  }
};
struct BlockKeyHash {
  size_t operator()(const BlockKey& k) const {
    uint64_t h = 1469598103934665603ull;
    for (int i = 0; i < 4; ++i) {
      uint64_t v;
      std::memcpy(&v, &k.ratio[i], 8);
      h = (h ^ (uint64_t)k.kind[i]) * 1099511628211ull;
      h = (h ^ v) * 1099511628211ull;
    }
    return (size_t)h;
  }
};

int setup_blocks(sdg_problem* P) {
  const int nx = P->mesh.nx, ny = P->mesh.ny, nel = P->nel;
  std::vector<int> ids(nel);
  std::vector<double> scale(nel);
  P->reps.clear();
  std::unordered_map<BlockKey, int, BlockKeyHash> map;
  for (int e = 0; e < nel; ++e) {
    const int ix = e % nx, iy = e / nx;
    const double ee = P->eta_host[e];
    BlockKey key;
    const int nbs[4] = {ix > 0 ? e - 1 : -1, ix < nx - 1 ? e + 1 : -1, iy > 0 ? e - nx : -1,
                        iy < ny - 1 ? e + nx : -1};
    for (int f = 0; f < 4; ++f) {
      if (nbs[f] >= 0) {
        key.kind[f] = F_INTERIOR;
        const double r = P->eta_host[nbs[f]] / ee;
        key.ratio[f] = r > 1.0 ? r : 1.0;
      } else {
        key.kind[f] = P->mesh.bc[f];
        key.ratio[f] = 1.0;
      }
    }
    int id;
    if (P->opt.dedup) {
      auto it = map.find(key);
      if (it == map.end()) {
        id = (int)P->reps.size();
        map.emplace(key, id);
        P->reps.push_back(e);
      } else {
        id = it->second;
      }
    } else {
      id = e;
      P->reps.push_back(e);
    }
    ids[e] = id;
    scale[e] = P->eta_host[P->reps[id]] / ee;
  }
  P->nuniq = (int)P->reps.size();
  SDG_TRY(palloc_t(P, &P->ids, nel));
  SDG_TRY(palloc_t(P, &P->scale, nel));
  SDG_HIP(hipMemcpyAsync(P->ids, ids.data(), nel * sizeof(int), hipMemcpyHostToDevice, P->s));
  SDG_HIP(hipMemcpyAsync(P->scale, scale.data(), nel * sizeof(double), hipMemcpyHostToDevice, P->s));
  // blocks of the representatives, then their inverses
  int* dreps = nullptr;
  int* dstat = nullptr;
  SDG_TRY(palloc_t(P, &dreps, P->nuniq));
  SDG_TRY(palloc_t(P, &dstat, P->nuniq));
  SDG_HIP(hipMemcpyAsync(dreps, P->reps.data(), P->nuniq * sizeof(int), hipMemcpyHostToDevice, P->s));
  const int64_t nbb = (int64_t)P->NB * P->NB;
  SDG_TRY(palloc_t(P, &P->binv, (int64_t)P->nuniq * nbb));
  SDG_TRY(sip_block_list(P->M, P->k, P->eta, dreps, P->nuniq, P->binv, P->s));
  SDG_TRY(spd_inverse(P->binv, P->NB, P->nuniq, dstat, P->s));
  std::vector<int> st(P->nuniq);
  SDG_HIP(hipMemcpyAsync(st.data(), dstat, P->nuniq * sizeof(int), hipMemcpyDeviceToHost, P->s));
  SDG_HIP(hipStreamSynchronize(P->s));
  for (int i = 0; i < P->nuniq; ++i)
    if (st[i]) {
      set_error("element block " + std::to_string(P->reps[i]) + " is not positive definite");
      return SDG_ERR_UNSUPPORTED;
    }
  if (P->opt.prec_smoother == SDG_FP32) {
    SDG_TRY(palloc_t(P, &P->binv32, (int64_t)P->nuniq * nbb));
    SDG_TRY(convert_f64_f32(P->binv, P->binv32, (int64_t)P->nuniq * nbb, P->s));
  } else if (P->opt.prec_smoother == SDG_BF16) {
    SDG_TRY(palloc_t(P, &P->binv16, (int64_t)P->nuniq * nbb));
    SDG_TRY(convert_f64_bf16(P->binv, P->binv16, (int64_t)P->nuniq * nbb, P->s));
  }
  return SDG_OK;
}

int setup_coarse(sdg_problem* P) {
  const int nx = P->mesh.nx, ny = P->mesh.ny;
  double* clocal = nullptr;
  SDG_TRY(palloc_t(P, &clocal, (int64_t)P->nel * 64));
  SDG_TRY(sip_coarse_local(P->M, P->k, 1, P->eta, clocal, P->s));
  int cx = nx, cy = ny;
  P->lev.clear();
  while (true) {
    CLevel L;
    L.nx = cx;
    L.ny = cy;
    L.nn = (cx + 1) * (cy + 1);
    SDG_TRY(palloc_t(P, &L.st, (int64_t)36 * L.nn));
    for (double** v : {&L.b, &L.x, &L.r, &L.z, &L.d}) SDG_TRY(palloc_t(P, v, (int64_t)2 * L.nn));
    if (P->lev.empty()) {
      SDG_TRY(coarse_stencil_from_local(cx, cy, 1, clocal, L.st, P->s));
    } else {
      const CLevel& F = P->lev.back();
      SDG_TRY(galerkin_coarsen(F.nx, F.ny, 1, F.st, L.st, P->s));
    }
    const bool more = (cx % 2 == 0) && (cy % 2 == 0) && cx > P->opt.coarsest_n && cy > P->opt.coarsest_n;
    L.coarsest = !more;
    if (L.coarsest) {
      const int n2 = 2 * L.nn;
      if (n2 > 2048) {
        set_error("coarsest level too large for the dense solve (more than 2048 unknowns); use element counts with more factors of two");
        return SDG_ERR_UNSUPPORTED;
      }
      int* dstat = nullptr;
      SDG_TRY(palloc_t(P, &L.dense, (int64_t)n2 * n2));
      SDG_TRY(palloc_t(P, &dstat, 1));
      SDG_TRY(stencil_to_dense(cx, cy, 1, L.st, L.dense, P->s));
      SDG_TRY(spd_inverse(L.dense, n2, 1, dstat, P->s));
      int st = 0;
      SDG_HIP(hipMemcpyAsync(&st, dstat, sizeof(int), hipMemcpyDeviceToHost, P->s));
      SDG_HIP(hipStreamSynchronize(P->s));
      if (st) {
        set_error("coarsest operator is not positive definite (a rigid motion is not restrained)");
        return SDG_ERR_UNSUPPORTED;
      }
    } else {
      SDG_TRY(palloc_t(P, &L.dinv, (int64_t)2 * L.nn));
      SDG_TRY(stencil_diag_inv(cx, cy, 1, L.st, L.dinv, P->s));
    }
    P->lev.push_back(L);
    if (L.coarsest) break;
    cx /= 2;
    cy /= 2;
  }
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// operators used by the cycle and Krylov methods
// ---------------------------------------------------------------------------
int bj64(sdg_problem* P, const double* r, double* z) {
  return blockjacobi_apply_f64(P->NB, P->nel, P->ids, P->scale, P->binv, r, z, P->s);
}
int bj32(sdg_problem* P, const float* r, float* z) {
  if (P->binv16) return blockjacobi_apply_bf16(P->NB, P->nel, P->ids, P->scale, P->binv16, r, z, P->s);
  return blockjacobi_apply_f32(P->NB, P->nel, P->ids, P->scale, P->binv32, r, z, P->s);
}

struct Cheb {
  double theta, delta, sigma;
};
Cheb cheb_params(double lmin, double lmax) {
  Cheb c;
  c.theta = 0.5 * (lmax + lmin);
  c.delta = 0.5 * (lmax - lmin);
  c.sigma = c.theta / c.delta;
  return c;
}

// m Chebyshev steps on the DG level (FP64); zero: x starts at 0
int cheb_dg64(sdg_problem* P, const double* b, double* x, bool zero) {
  const Cheb c = cheb_params(P->lmin0, P->lmax0);
  double rho = 1.0 / c.sigma;
  const int64_t n = P->nu;
  if (zero) {
    SDG_TRY(bj64(P, b, P->vz));
  } else {
    SDG_TRY(sip_residual(P->M, P->k, 1, P->eta, b, x, P->vr, P->s));
    SDG_TRY(bj64(P, P->vr, P->vz));
  }
  SDG_TRY(cheb_update(n, 0.0, P->vz, 1.0 / c.theta, P->vd, x, zero ? 1 : 2, P->s));
  for (int it = 1; it < P->opt.smooth_dg; ++it) {
    SDG_TRY(sip_residual(P->M, P->k, 1, P->eta, b, x, P->vr, P->s));
    SDG_TRY(bj64(P, P->vr, P->vz));
    const double rn = 1.0 / (2.0 * c.sigma - rho);
    SDG_TRY(cheb_update(n, rn * rho, P->vz, 2.0 * rn / c.delta, P->vd, x, 0, P->s));
    rho = rn;
  }
  return SDG_OK;
}

int cheb_dg32(sdg_problem* P, const float* b, float* x, bool zero) {
  const Cheb c = cheb_params(P->lmin0, P->lmax0);
  double rho = 1.0 / c.sigma;
  const int64_t n = P->nu;
  if (zero) {
    SDG_TRY(bj32(P, b, P->fz));
  } else {
    SDG_TRY(sip_residual_f32(P->M, P->k, 1, P->eta, b, x, P->fr, P->s));
    SDG_TRY(bj32(P, P->fr, P->fz));
  }
  SDG_TRY(cheb_update_f32(n, 0.0, P->fz, 1.0 / c.theta, P->fd, x, zero ? 1 : 2, P->s));
  for (int it = 1; it < P->opt.smooth_dg; ++it) {
    SDG_TRY(sip_residual_f32(P->M, P->k, 1, P->eta, b, x, P->fr, P->s));
    SDG_TRY(bj32(P, P->fr, P->fz));
    const double rn = 1.0 / (2.0 * c.sigma - rho);
    SDG_TRY(cheb_update_f32(n, rn * rho, P->fz, 2.0 * rn / c.delta, P->fd, x, 0, P->s));
    rho = rn;
  }
  return SDG_OK;
}

int cheb_h(sdg_problem* P, CLevel& L, bool zero) {
  const Cheb c = cheb_params(L.lmin, L.lmax);
  double rho = 1.0 / c.sigma;
  const int64_t n = 2 * (int64_t)L.nn;
  if (zero) {
    SDG_TRY(vec_mul(n, L.dinv, L.b, L.z, P->s));
  } else {
    SDG_TRY(stencil_residual(L.nx, L.ny, 1, L.st, L.b, L.x, L.r, P->s));
    SDG_TRY(vec_mul(n, L.dinv, L.r, L.z, P->s));
  }
  SDG_TRY(cheb_update(n, 0.0, L.z, 1.0 / c.theta, L.d, L.x, zero ? 1 : 2, P->s));
  for (int it = 1; it < P->opt.smooth_h; ++it) {
    SDG_TRY(stencil_residual(L.nx, L.ny, 1, L.st, L.b, L.x, L.r, P->s));
    SDG_TRY(vec_mul(n, L.dinv, L.r, L.z, P->s));
    const double rn = 1.0 / (2.0 * c.sigma - rho);
    SDG_TRY(cheb_update(n, rn * rho, L.z, 2.0 * rn / c.delta, L.d, L.x, 0, P->s));
    rho = rn;
  }
  return SDG_OK;
}

// h-cycle on level li: L.x = B_h L.b
int hcycle(sdg_problem* P, int li) {
  CLevel& L = P->lev[li];
  if (L.coarsest) return dense_matvec(2 * L.nn, 1, L.dense, L.b, L.x, P->s);
  SDG_TRY(cheb_h(P, L, true));
  SDG_TRY(stencil_residual(L.nx, L.ny, 1, L.st, L.b, L.x, L.r, P->s));
  CLevel& C = P->lev[li + 1];
  SDG_TRY(h_restrict(C.nx, C.ny, 1, L.r, C.b, P->s));
  SDG_TRY(hcycle(P, li + 1));
  SDG_TRY(h_prolong_add(C.nx, C.ny, 1, C.x, L.x, P->s));
  SDG_TRY(cheb_h(P, L, false));
  return SDG_OK;
}

// x = B_mg b in FP64 (Algorithm 1, zero initial guess)
int vcycle64(sdg_problem* P, const double* b, double* x) {
  SDG_TRY(cheb_dg64(P, b, x, true));
  SDG_TRY(sip_residual(P->M, P->k, 1, P->eta, b, x, P->vr, P->s));
  SDG_TRY(p_restrict(P->M, P->k, 1, P->vr, P->lev[0].b, P->s));
  SDG_TRY(hcycle(P, 0));
  SDG_TRY(p_prolong_add(P->M, P->k, 1, P->lev[0].x, x, P->s));
  SDG_TRY(cheb_dg64(P, b, x, false));
  return SDG_OK;
}

// x = B_mg b with the fine level in FP32 (FP64 in and out)
int vcycle32(sdg_problem* P, const double* b, double* x) {
  SDG_TRY(d2f(P->nu, b, P->fb, P->s));
  SDG_TRY(cheb_dg32(P, P->fb, P->fx, true));
  SDG_TRY(sip_residual_f32(P->M, P->k, 1, P->eta, P->fb, P->fx, P->fr, P->s));
  SDG_TRY(p_restrict_f32(P->M, P->k, 1, P->fr, P->lev[0].b, P->s));
  SDG_TRY(hcycle(P, 0));
  SDG_TRY(p_prolong_add_f32(P->M, P->k, 1, P->lev[0].x, P->fx, P->s));
  SDG_TRY(cheb_dg32(P, P->fb, P->fx, false));
  SDG_TRY(f2d(P->nu, P->fx, x, P->s));
  return SDG_OK;
}

int vcycle(sdg_problem* P, const double* b, double* x) {
  if (P->opt.prec_apply == SDG_FP32 || P->opt.prec_smoother != SDG_FP64) return vcycle32(P, b, x);
  return vcycle64(P, b, x);
}

// scalar readback helpers
int read_scalars(sdg_problem* P, int n) {
  SDG_HIP(hipMemcpyAsync(P->hsc, P->dsc, n * sizeof(double), hipMemcpyDeviceToHost, P->s));
  SDG_HIP(hipStreamSynchronize(P->s));
  return SDG_OK;
}
int norm2(sdg_problem* P, int64_t n, const double* x, double* out) {
  SDG_TRY(dot(n, x, x, P->dsc, P->red, P->s));
  SDG_TRY(read_scalars(P, 1));
  *out = std::sqrt(P->hsc[0] > 0 ? P->hsc[0] : 0.0);
  return SDG_OK;
}
int read_device(sdg_problem* P, const double* src, int n) {
  SDG_HIP(hipMemcpyAsync(P->hsc, src, n * sizeof(double), hipMemcpyDeviceToHost, P->s));
  SDG_HIP(hipStreamSynchronize(P->s));
  return SDG_OK;
}
int dot_host(sdg_problem* P, int64_t n, const double* x, const double* y, double* out) {
  SDG_TRY(dot(n, x, y, P->dsc, P->red, P->s));
  SDG_TRY(read_scalars(P, 1));
  *out = P->hsc[0];
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// Chebyshev bounds: Arnoldi (classical Gram-Schmidt twice) on M^{-1} A
// ---------------------------------------------------------------------------
// level -1: DG level; level >= 0: CG level li
int arnoldi(sdg_problem* P, int li, double* lambda, std::vector<double>* hess_out) {
  const int m = P->opt.eig_steps;
  const int64_t n = li < 0 ? P->nu : 2 * (int64_t)P->lev[li].nn;
  double* V = nullptr;
  double* w = nullptr;
  double* dH = nullptr;
  double* hcol = nullptr;
  // temporary workspace, freed at the end
  if (hipMalloc((void**)&V, (size_t)(m + 1) * n * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&w, (size_t)n * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&dH, (size_t)(m + 1) * m * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&hcol, (size_t)(m + 2) * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(V);
    (void)hipFree(w);
    (void)hipFree(dH);
    (void)hipFree(hcol);
    set_error("allocation of the Arnoldi workspace failed");
    return SDG_ERR_NOMEM;
  }
  const uint64_t seed = P->opt.seed + ((uint64_t)(li + 1) << 32);
  int rc = SDG_OK;
  std::vector<double> H((size_t)(m + 1) * m, 0.0);
  int mm = m;
  do {
    if ((rc = uniform_pm1(seed, n, V, P->s)) < 0) break;
    double nv;
    if ((rc = norm2(P, n, V, &nv)) < 0) break;
    if ((rc = vec_scale_copy(n, 1.0 / nv, V, V, P->s)) < 0) break;
    for (int j = 0; j < m; ++j) {
      double* vj = V + (int64_t)j * n;
      if (li < 0) {
        if ((rc = sip_apply(P->M, P->k, 1, P->eta, vj, P->vr, P->s)) < 0) break;
        if ((rc = bj64(P, P->vr, w)) < 0) break;
      } else {
        CLevel& L = P->lev[li];
        if ((rc = stencil_apply(L.nx, L.ny, 1, L.st, vj, L.r, P->s)) < 0) break;
        if ((rc = vec_mul(n, L.dinv, L.r, w, P->s)) < 0) break;
      }
      std::vector<double> h(j + 1, 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        if ((rc = multi_dot(n, j + 1, V, n, w, hcol, P->red, P->s)) < 0) break;
        if ((rc = multi_axpy(n, j + 1, V, n, hcol, w, P->s)) < 0) break;
        if ((rc = read_device(P, hcol, j + 1)) < 0) break;
        for (int i = 0; i <= j; ++i) h[i] += P->hsc[i];
      }
      if (rc < 0) break;
      double hn;
      if ((rc = norm2(P, n, w, &hn)) < 0) break;
      for (int i = 0; i <= j; ++i) H[(size_t)j * (m + 1) + i] = h[i];
      H[(size_t)j * (m + 1) + j + 1] = hn;
      if (hn <= 1e-14 * std::fabs(h[j])) {
        mm = j + 1;
        break;
      }
      if ((rc = vec_scale_copy(n, 1.0 / hn, w, V + (int64_t)(j + 1) * n, P->s)) < 0) break;
    }
    if (rc < 0) break;
    if (hipMemcpyAsync(dH, H.data(), H.size() * sizeof(double), hipMemcpyHostToDevice, P->s) != hipSuccess) {
      set_error("copy of the Hessenberg matrix failed");
      rc = SDG_ERR_DEVICE;
      break;
    }
    if ((rc = hessenberg_max_eig(dH, mm, m + 1, hcol, P->s)) < 0) break;
    if ((rc = read_device(P, hcol, 1)) < 0) break;
  } while (0);
  (void)hipStreamSynchronize(P->s);
  (void)hipFree(V);
  (void)hipFree(w);
  (void)hipFree(dH);
  (void)hipFree(hcol);
  if (rc < 0) return rc;
  *lambda = P->hsc[0];
  if (hess_out) *hess_out = H;
  return SDG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Krylov methods
// ---------------------------------------------------------------------------
namespace {

// Preconditioned CG with x0 = 0; stops when ||r||_2 < rtol ||b||_2 (the
// unpreconditioned, recursively updated residual).
int cg_solve(sdg_problem* P, const double* b, double* x, double rtol, int maxit, int* its,
             double* relres) {
  const int64_t n = P->nu;
  double bn;
  SDG_TRY(norm2(P, n, b, &bn));
  SDG_HIP(hipMemsetAsync(x, 0, n * sizeof(double), P->s));
  *its = 0;
  *relres = 0.0;
  if (bn == 0.0) return SDG_OK;
  if (!std::isfinite(bn)) {
    set_error("right-hand side is not finite");
    return SDG_ERR_INVALID;
  }
  SDG_TRY(vec_copy(n, b, P->cg_r, P->s));
  SDG_TRY(vcycle(P, P->cg_r, P->cg_z));
  SDG_TRY(vec_copy(n, P->cg_z, P->cg_p, P->s));
  double rz;
  SDG_TRY(dot_host(P, n, P->cg_r, P->cg_z, &rz));
  double rel = 1.0;
  int it = 0;
  int status = SDG_NOT_CONVERGED;
  while (it < maxit) {
    SDG_TRY(sip_apply(P->M, P->k, 1, P->eta, P->cg_p, P->cg_q, P->s));
    double pq;
    SDG_TRY(dot_host(P, n, P->cg_p, P->cg_q, &pq));
    if (!(pq > 0.0) || !std::isfinite(pq)) {
      status = SDG_BREAKDOWN;
      break;
    }
    const double alpha = rz / pq;
    SDG_TRY(vec_axpy(n, alpha, P->cg_p, x, P->s));
    SDG_TRY(vec_axpy(n, -alpha, P->cg_q, P->cg_r, P->s));
    ++it;
    double rn;
    SDG_TRY(norm2(P, n, P->cg_r, &rn));
    rel = rn / bn;
    if (!std::isfinite(rel)) {
      status = SDG_BREAKDOWN;
      break;
    }
    if (rel < rtol) {
      status = SDG_OK;
      break;
    }
    SDG_TRY(vcycle(P, P->cg_r, P->cg_z));
    double rz2;
    SDG_TRY(dot_host(P, n, P->cg_r, P->cg_z, &rz2));
    SDG_TRY(vec_axpby(n, 1.0, P->cg_z, rz2 / rz, P->cg_p, P->s));
    rz = rz2;
  }
  *its = it;
  *relres = rel;
  return status;
}

int ensure_gmres(sdg_problem* P, int64_t n) {
  if (P->gV && P->gn >= n) return SDG_OK;
  if (P->gV) {
    set_error("FGMRES workspace size mismatch");
    return SDG_ERR_INVALID;
  }
  const int m = P->opt.restart;
  SDG_TRY(palloc_t(P, &P->gV, (int64_t)(m + 1) * n));
  SDG_TRY(palloc_t(P, &P->gZ, (int64_t)m * n));
  SDG_TRY(palloc_t(P, &P->gw, n));
  SDG_TRY(palloc_t(P, &P->gt, P->nu));
  P->gn = n;
  return SDG_OK;
}

template <typename MV, typename PC, typename PJ>
int fgmres(sdg_problem* P, int64_t n, const double* b_in, double* x, double rtol, int maxit,
           MV matvec, PC prec, PJ project, int* its, double* relres) {
  const int m = P->opt.restart;
  SDG_TRY(ensure_gmres(P, n));
  double* V = P->gV;
  double* Z = P->gZ;
  double* w = P->gw;
  // b lives in V[m] until the first basis vector overwrites it: keep a
  // projected copy in x's place? x is output; use w as the residual vector.
  SDG_TRY(vec_copy(n, b_in, w, P->s));
  SDG_TRY(project(w));
  double bn;
  SDG_TRY(norm2(P, n, w, &bn));
  SDG_HIP(hipMemsetAsync(x, 0, n * sizeof(double), P->s));
  *its = 0;
  *relres = 0.0;
  if (bn == 0.0) return SDG_OK;
  if (!std::isfinite(bn)) {
    set_error("right-hand side is not finite");
    return SDG_ERR_INVALID;
  }
  int total = 0;
  int status = SDG_NOT_CONVERGED;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  double beta = bn;  // residual vector is in w
  while (true) {
    if (beta / bn < rtol) {
      status = SDG_OK;
      break;
    }
    if (total >= maxit) break;
    SDG_TRY(vec_scale_copy(n, 1.0 / beta, w, V, P->s));
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jd = 0;
    bool done = false;
    for (int j = 0; j < m; ++j) {
      double* zj = Z + (int64_t)j * n;
      SDG_TRY(prec(V + (int64_t)j * n, zj));
      SDG_TRY(project(zj));
      SDG_TRY(matvec(zj, w));
      std::vector<double> h(j + 1, 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        SDG_TRY(multi_dot(n, j + 1, V, n, w, P->dsc, P->red, P->s));
        SDG_TRY(multi_axpy(n, j + 1, V, n, P->dsc, w, P->s));
        SDG_TRY(read_scalars(P, j + 1));
        for (int i = 0; i <= j; ++i) h[i] += P->hsc[i];
      }
      double hn;
      SDG_TRY(norm2(P, n, w, &hn));
      for (int i = 0; i <= j; ++i) H[(size_t)j * (m + 1) + i] = h[i];
      H[(size_t)j * (m + 1) + j + 1] = hn;
      if (hn > 0.0 && j + 1 <= m) {
        if (j + 1 < m + 1) SDG_TRY(vec_scale_copy(n, 1.0 / hn, w, V + (int64_t)(j + 1) * n, P->s));
      }
      double* col = &H[(size_t)j * (m + 1)];
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = t;
      }
      const double den = std::hypot(col[j], col[j + 1]);
      if (!(den > 0.0) || !std::isfinite(den)) {
        status = SDG_BREAKDOWN;
        done = true;
        jd = j;
        break;
      }
      cs[j] = col[j] / den;
      sn[j] = col[j + 1] / den;
      col[j] = den;
      col[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++total;
      jd = j + 1;
      const double est = std::fabs(g[j + 1]) / bn;
      if (est < rtol || total >= maxit || hn == 0.0) break;
    }
    // y = H^{-1} g (upper triangular), x += Z y
    for (int i = jd - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < jd; ++l) s -= H[(size_t)l * (m + 1) + i] * y[l];
      y[i] = s / H[(size_t)i * (m + 1) + i];
    }
    if (jd > 0) {
      SDG_HIP(hipMemcpyAsync(P->dsc, y.data(), jd * sizeof(double), hipMemcpyHostToDevice, P->s));
      SDG_TRY(multi_combine(n, jd, Z, n, P->dsc, x, P->s));
    }
    // true residual
    SDG_TRY(matvec(x, w));
    SDG_TRY(vec_axpby(n, 1.0, b_in, -1.0, w, P->s));
    SDG_TRY(project(w));
    SDG_TRY(norm2(P, n, w, &beta));
    if (done) break;
  }
  *its = total;
  *relres = beta / bn;
  if (status != SDG_BREAKDOWN) status = (*relres < rtol) ? SDG_OK : SDG_NOT_CONVERGED;
  return status;
}

// Stokes operator K = [A B; B^T 0] on x = [u; p]
int stokes_matvec(sdg_problem* P, const double* x, double* y) {
  SDG_TRY(sip_apply(P->M, P->k, 1, P->eta, x, y, P->s));
  SDG_TRY(grad_apply(P->M, P->k, 1, x + P->nu, P->gt, P->s));
  SDG_TRY(vec_axpy(P->nu, 1.0, P->gt, y, P->s));
  SDG_TRY(div_apply(P->M, P->k, 1, x, y + P->nu, P->s));
  return SDG_OK;
}

// upper block-triangular preconditioner [A B; 0 S] (eq. discretestokespc)
// with S = -diag(1/eta_K), the viscosity-scaled pressure mass matrix taken
// as an approximation of the (negative definite) Schur complement
// -B^T A^{-1} B:  z_p = S^{-1} v_p = -eta v_p, z_u = (inner CG)(v_u - B z_p)
int stokes_prec(sdg_problem* P, const double* v, double* z) {
  SDG_TRY(vec_mul(P->np, P->etap, v + P->nu, z + P->nu, P->s));
  SDG_TRY(vec_scale_copy(P->np, -1.0, z + P->nu, z + P->nu, P->s));
  SDG_TRY(grad_apply(P->M, P->k, 1, z + P->nu, P->gt, P->s));
  SDG_TRY(vec_axpby(P->nu, 1.0, v, -1.0, P->gt, P->s));
  int its = 0;
  double rel = 0.0;
  int rc = cg_solve(P, P->gt, z, P->opt.inner_rtol, P->opt.inner_max_it, &its, &rel);
  if (rc < 0) return rc;
  P->inner_total += its;
  if (its > P->inner_max) P->inner_max = its;
  return SDG_OK;
}

int stokes_project(sdg_problem* P, double* x) {
  if (P->neumann) return SDG_OK;
  return pressure_project(P->nel, P->NPE, x + P->nu, P->red, P->s);
}

int sync_ms(sdg_problem* P, double t0, double* out) {
  SDG_HIP(hipStreamSynchronize(P->s));
  *out = now_ms() - t0;
  return SDG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* sdg_last_error(void) { return get_error(); }

void sdg_options_default(sdg_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->rtol = 1e-8;
  o->inner_rtol = 1e-3;
  o->max_it = 1000;
  o->inner_max_it = 500;
  o->restart = 30;
  o->smooth_dg = 2;
  o->smooth_h = 3;
  o->coarsest_n = 8;
  o->eig_steps = 10;
  o->cheb_lo = 0.1;
  o->cheb_hi = 1.1;
  o->prec_smoother = SDG_FP64;
  o->prec_apply = SDG_FP64;
  o->viscous_krylov = 0;
  o->dedup = 1;
  o->seed = 0;
}

int sdg_create(int device, size_t mem_budget, sdg_ctx** out) {
  if (!out) {
    set_error("NULL output pointer");
    return SDG_ERR_INVALID;
  }
  *out = nullptr;
  int ndev = 0;
  SDG_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) {
    set_error("device index out of range");
    return SDG_ERR_INVALID;
  }
  SDG_HIP(hipSetDevice(device));
  sdg_ctx* c = new sdg_ctx();
  c->device = device;
  c->budget = mem_budget;
  *out = c;
  return SDG_OK;
}

void sdg_destroy(sdg_ctx* ctx) {
  if (!ctx) return;
  if (ctx->live == 0) delete ctx;
  else ctx->closing = true;
}

static bool opts_ok(const sdg_options* o) {
  if (!o) return false;
  if (!(o->rtol > 0) || !(o->inner_rtol > 0) || o->max_it < 1 || o->inner_max_it < 1) return false;
  if (o->restart < 1 || o->restart > 200 || o->smooth_dg < 1 || o->smooth_h < 1) return false;
  if (o->coarsest_n < 1 || o->eig_steps < 1 || o->eig_steps > 30) return false;
  if (!(o->cheb_lo > 0) || !(o->cheb_hi > o->cheb_lo)) return false;
  if (o->prec_smoother < 0 || o->prec_smoother > 2 || o->prec_apply < 0 || o->prec_apply > 1) return false;
  return true;
}

size_t sdg_required_bytes(const sdg_mesh* mesh, const sdg_options* opts, int stokes) {
  if (!mesh_ok(mesh) || !opts_ok(opts)) return 0;
  const int64_t nel = (int64_t)mesh->nx * mesh->ny;
  const int64_t NB = 2 * (int64_t)(mesh->k + 1) * (mesh->k + 1);
  const int64_t nu = nel * NB, np = nel * mesh->k * mesh->k;
  size_t b = 0;
  b += nel * 8 * 2 + nel * 4 + np * 8;              // eta, scale, ids, etap
  const int64_t nuniq = opts->dedup ? std::min<int64_t>(nel, 4096) : nel;
  b += nuniq * NB * NB * 8;                          // FP64 inverses (dedup: bound)
  if (opts->prec_smoother == SDG_FP32) b += nuniq * NB * NB * 4;
  if (opts->prec_smoother == SDG_BF16) b += nuniq * NB * NB * 2;
  b += nuniq * 8 + nel * 64 * 8;                     // reps/status, coarse local matrices
  int cx = mesh->nx, cy = mesh->ny;
  while (true) {
    const int64_t nn = (int64_t)(cx + 1) * (cy + 1);
    b += nn * (36 + 12) * 8;
    const bool more = cx % 2 == 0 && cy % 2 == 0 && cx > opts->coarsest_n && cy > opts->coarsest_n;
    if (!more) {
      b += 4 * nn * nn * 8 + 8;
      break;
    }
    cx /= 2;
    cy /= 2;
  }
  b += nu * 8 * 3;                                   // DG cycle vectors
  if (opts->prec_apply == SDG_FP32 || opts->prec_smoother != SDG_FP64) b += nu * 4 * 5;
  b += RED_SCRATCH * 8 + 64 * 8 + nu * 8 * 4;        // reductions, CG
  const int64_t n = stokes ? nu + np : nu;
  if (stokes || opts->viscous_krylov == 1) b += ((2 * (int64_t)opts->restart + 2) * n + nu) * 8;
  b += (int64_t)(opts->eig_steps + 2) * std::max<int64_t>(nu, 1) * 8;  // transient Arnoldi
  return b;
}

int sdg_problem_create(sdg_ctx* ctx, const sdg_mesh* mesh, const sdg_options* opts,
                       const double* eta_dev, void* stream, sdg_problem** out) {
  if (!out) {
    set_error("NULL output pointer");
    return SDG_ERR_INVALID;
  }
  *out = nullptr;
  if (!ctx || !eta_dev) {
    set_error("NULL context or viscosity");
    return SDG_ERR_INVALID;
  }
  if (!mesh_ok(mesh)) {
    set_error("invalid mesh (need nx, ny >= 1, 1 <= k <= 6, lx, ly > 0, bc in 0..2)");
    return SDG_ERR_INVALID;
  }
  sdg_options o;
  if (opts) o = *opts;
  else sdg_options_default(&o);
  if (!opts_ok(&o)) {
    set_error("invalid options");
    return SDG_ERR_INVALID;
  }
  bool all_neumann = true;
  bool any_neumann = false;
  for (int i = 0; i < 4; ++i) {
    all_neumann = all_neumann && mesh->bc[i] == SDG_NEUMANN;
    any_neumann = any_neumann || mesh->bc[i] == SDG_NEUMANN;
  }
  if (all_neumann) {
    set_error("all-Neumann viscous problem is singular (rigid motions)");
    return SDG_ERR_UNSUPPORTED;
  }
  SDG_HIP(hipSetDevice(ctx->device));
  const double t0 = now_ms();
  sdg_problem* P = new sdg_problem();
  P->ctx = ctx;
  ctx->live++;
  P->mesh = *mesh;
  P->opt = o;
  P->s = (hipStream_t)stream;
  P->k = mesh->k;
  P->K1 = mesh->k + 1;
  P->NB = 2 * P->K1 * P->K1;
  P->NPE = mesh->k * mesh->k;
  P->nel = mesh->nx * mesh->ny;
  P->nu = (int64_t)P->nel * P->NB;
  P->np = (int64_t)P->nel * P->NPE;
  P->neumann = any_neumann;
  P->M.nx = mesh->nx;
  P->M.ny = mesh->ny;
  P->M.hx = mesh->lx / mesh->nx;
  P->M.hy = mesh->ly / mesh->ny;
  for (int i = 0; i < 4; ++i) P->M.bc[i] = mesh->bc[i];
  auto fail = [&](int rc) {
    sdg_problem_destroy(P);
    return rc;
  };
  int rc;
  if ((rc = palloc_t(P, &P->eta, P->nel)) < 0) return fail(rc);
  P->eta_host.resize(P->nel);
  if (hipMemcpyAsync(P->eta_host.data(), eta_dev, P->nel * sizeof(double), hipMemcpyDeviceToHost, P->s) != hipSuccess ||
      hipStreamSynchronize(P->s) != hipSuccess) {
    set_error("copy of the viscosity failed (device pointer expected)");
    return fail(SDG_ERR_DEVICE);
  }
  for (int e = 0; e < P->nel; ++e)
    if (!(P->eta_host[e] > 0.0) || !std::isfinite(P->eta_host[e])) {
      set_error("viscosity must be positive and finite (element " + std::to_string(e) + ")");
      return fail(SDG_ERR_INVALID);
    }
  if (hipMemcpyAsync(P->eta, P->eta_host.data(), P->nel * sizeof(double), hipMemcpyHostToDevice, P->s) != hipSuccess) {
    set_error("viscosity upload failed");
    return fail(SDG_ERR_DEVICE);
  }
  {
    std::vector<double> ep(P->np);
    for (int e = 0; e < P->nel; ++e)
      for (int m = 0; m < P->NPE; ++m) ep[(size_t)e * P->NPE + m] = P->eta_host[e];
    if ((rc = palloc_t(P, &P->etap, std::max<int64_t>(P->np, 1))) < 0) return fail(rc);
    if (hipMemcpyAsync(P->etap, ep.data(), P->np * sizeof(double), hipMemcpyHostToDevice, P->s) != hipSuccess ||
        hipStreamSynchronize(P->s) != hipSuccess) {
      set_error("upload failed");
      return fail(SDG_ERR_DEVICE);
    }
  }
  if ((rc = setup_blocks(P)) < 0) return fail(rc);
  if ((rc = setup_coarse(P)) < 0) return fail(rc);
  for (double** v : {&P->vr, &P->vz, &P->vd, &P->cg_r, &P->cg_z, &P->cg_p, &P->cg_q})
    if ((rc = palloc_t(P, v, P->nu)) < 0) return fail(rc);
  if (o.prec_apply == SDG_FP32 || o.prec_smoother != SDG_FP64) {
    if (o.prec_smoother == SDG_FP64) {  // FP32 apply with FP32 copies of the inverses
      if ((rc = palloc_t(P, &P->binv32, (int64_t)P->nuniq * P->NB * P->NB)) < 0) return fail(rc);
      if ((rc = convert_f64_f32(P->binv, P->binv32, (int64_t)P->nuniq * P->NB * P->NB, P->s)) < 0) return fail(rc);
    }
    for (float** v : {&P->fb, &P->fx, &P->fr, &P->fz, &P->fd})
      if ((rc = palloc_t(P, v, P->nu)) < 0) return fail(rc);
  }
  if ((rc = palloc_t(P, &P->red, RED_SCRATCH)) < 0) return fail(rc);
  if ((rc = palloc_t(P, &P->dsc, 256)) < 0) return fail(rc);
  if (hipHostMalloc((void**)&P->hsc, 256 * sizeof(double)) != hipSuccess) {
    set_error("pinned allocation failed");
    return fail(SDG_ERR_NOMEM);
  }
  // Chebyshev bounds
  double lam;
  if ((rc = arnoldi(P, -1, &lam, nullptr)) < 0) return fail(rc);
  P->lmin0 = o.cheb_lo * lam;
  P->lmax0 = o.cheb_hi * lam;
  for (size_t li = 0; li < P->lev.size(); ++li) {
    if (P->lev[li].coarsest) continue;
    if ((rc = arnoldi(P, (int)li, &lam, nullptr)) < 0) return fail(rc);
    P->lev[li].lmin = o.cheb_lo * lam;
    P->lev[li].lmax = o.cheb_hi * lam;
  }
  if (hipStreamSynchronize(P->s) != hipSuccess) {
    set_error("setup failed on the device");
    return fail(SDG_ERR_DEVICE);
  }
  P->setup_ms = now_ms() - t0;
  *out = P;
  return SDG_OK;
}

void sdg_problem_destroy(sdg_problem* P) {
  if (!P) return;
  (void)hipStreamSynchronize(P->s);
  for (void* p : P->allocs) (void)hipFree(p);
  if (P->hsc) (void)hipHostFree(P->hsc);
  if (sdg_ctx* c = P->ctx) {
    c->used -= std::min(c->used, P->bytes);
    c->live--;
    if (c->closing && c->live == 0) delete c;
  }
  delete P;
}

int sdg_problem_levels(const sdg_problem* P, int* nlevels) {
  if (!P || !nlevels) {
    set_error("NULL argument");
    return SDG_ERR_INVALID;
  }
  *nlevels = 1 + (int)P->lev.size();
  return SDG_OK;
}

int sdg_get_bounds(const sdg_problem* P, double* b) {
  if (!P || !b) {
    set_error("NULL argument");
    return SDG_ERR_INVALID;
  }
  b[0] = P->lmin0;
  b[1] = P->lmax0;
  for (size_t i = 0; i < P->lev.size(); ++i) {
    b[2 + 2 * i] = P->lev[i].lmin;
    b[3 + 2 * i] = P->lev[i].lmax;
  }
  return SDG_OK;
}

int sdg_set_bounds(sdg_problem* P, const double* b) {
  if (!P || !b) {
    set_error("NULL argument");
    return SDG_ERR_INVALID;
  }
  P->lmin0 = b[0];
  P->lmax0 = b[1];
  for (size_t i = 0; i < P->lev.size(); ++i) {
    P->lev[i].lmin = b[2 + 2 * i];
    P->lev[i].lmax = b[3 + 2 * i];
  }
  return SDG_OK;
}

int sdg_eig_estimate(sdg_problem* P, int level, double* lambda_out, double* hess) {
  if (!P || !lambda_out || level < 0 || level > (int)P->lev.size()) {
    set_error("invalid argument");
    return SDG_ERR_INVALID;
  }
  if (level > 0 && P->lev[level - 1].coarsest) {
    set_error("the coarsest level is solved directly and has no smoother");
    return SDG_ERR_INVALID;
  }
  std::vector<double> H;
  SDG_TRY(arnoldi(P, level - 1, lambda_out, &H));
  if (hess) std::memcpy(hess, H.data(), H.size() * sizeof(double));
  return SDG_OK;
}

#define PCHECK(...)                         \
  do {                                      \
    if (!P) {                               \
      set_error("NULL problem");            \
      return SDG_ERR_INVALID;               \
    }                                       \
    const void* _ptrs[] = {__VA_ARGS__};    \
    for (const void* _p : _ptrs)            \
      if (!_p) {                            \
        set_error("NULL pointer argument"); \
        return SDG_ERR_INVALID;             \
      }                                     \
  } while (0)

int sdg_apply_viscous(sdg_problem* P, const double* u, double* y) {
  PCHECK(u, y);
  return sip_apply(P->M, P->k, 1, P->eta, u, y, P->s);
}
int sdg_residual_viscous(sdg_problem* P, const double* b, const double* u, double* r) {
  PCHECK(b, u, r);
  return sip_residual(P->M, P->k, 1, P->eta, b, u, r, P->s);
}
int sdg_apply_viscous_f32(sdg_problem* P, const float* u, float* y) {
  PCHECK(u, y);
  return sip_apply_f32(P->M, P->k, 1, P->eta, u, y, P->s);
}
int sdg_apply_div(sdg_problem* P, const double* u, double* q) {
  PCHECK(u, q);
  return div_apply(P->M, P->k, 1, u, q, P->s);
}
int sdg_apply_grad(sdg_problem* P, const double* p, double* v) {
  PCHECK(p, v);
  return grad_apply(P->M, P->k, 1, p, v, P->s);
}
int sdg_apply_blockjacobi(sdg_problem* P, const double* r, double* z) {
  PCHECK(r, z);
  if (P->opt.prec_smoother == SDG_FP64) return bj64(P, r, z);
  SDG_TRY(d2f(P->nu, r, P->fr, P->s));
  SDG_TRY(bj32(P, P->fr, P->fz));
  return f2d(P->nu, P->fz, z, P->s);
}
int sdg_get_blocks(sdg_problem* P, double* blocks) {
  PCHECK(blocks);
  std::vector<int> all(P->nel);
  for (int e = 0; e < P->nel; ++e) all[e] = e;
  int* d = nullptr;
  SDG_HIP(hipMalloc((void**)&d, P->nel * sizeof(int)));
  int rc = SDG_OK;
  if (hipMemcpyAsync(d, all.data(), P->nel * sizeof(int), hipMemcpyHostToDevice, P->s) != hipSuccess) rc = SDG_ERR_DEVICE;
  if (rc == SDG_OK) rc = sip_block_list(P->M, P->k, P->eta, d, P->nel, blocks, P->s);
  (void)hipStreamSynchronize(P->s);
  (void)hipFree(d);
  return rc;
}
int sdg_p_restrict(sdg_problem* P, const double* r, double* rc) {
  PCHECK(r, rc);
  return p_restrict(P->M, P->k, 1, r, rc, P->s);
}
int sdg_p_prolong_add(sdg_problem* P, const double* ec, double* u) {
  PCHECK(ec, u);
  return p_prolong_add(P->M, P->k, 1, ec, u, P->s);
}
int sdg_get_coarse_stencil(sdg_problem* P, int level, double* st, int* nx_out, int* ny_out) {
  PCHECK(st);
  if (level < 0 || level >= (int)P->lev.size()) {
    set_error("level out of range");
    return SDG_ERR_INVALID;
  }
  const CLevel& L = P->lev[level];
  SDG_HIP(hipMemcpyAsync(st, L.st, (size_t)36 * L.nn * sizeof(double), hipMemcpyDeviceToDevice, P->s));
  if (nx_out) *nx_out = L.nx;
  if (ny_out) *ny_out = L.ny;
  return SDG_OK;
}
int sdg_vcycle(sdg_problem* P, const double* b, double* x) {
  PCHECK(b, x);
  return vcycle(P, b, x);
}
int sdg_assemble_rhs(sdg_problem* P, const double* f, const double* g, double* F, double* G) {
  PCHECK(f, F, G);
  return rhs_assemble(P->M, P->k, P->eta, f, g, F, G, P->s);
}

int sdg_solve_viscous_dev(sdg_problem* P, const double* f, const double* g, double* u, sdg_stats* st) {
  PCHECK(f, u);
  const double t0 = now_ms();
  double* F = nullptr;
  double* G = nullptr;
  SDG_HIP(hipMalloc((void**)&F, P->nu * sizeof(double)));
  if (hipMalloc((void**)&G, std::max<int64_t>(P->np, 1) * sizeof(double)) != hipSuccess) {
    (void)hipFree(F);
    set_error("allocation failed");
    return SDG_ERR_NOMEM;
  }
  int rc = rhs_assemble(P->M, P->k, P->eta, f, g, F, G, P->s);
  int its = 0;
  double rel = 0.0;
  if (rc >= 0) {
    if (P->opt.viscous_krylov == 1) {
      auto mv = [&](const double* x, double* y) { return sip_apply(P->M, P->k, 1, P->eta, x, y, P->s); };
      auto pc = [&](const double* v, double* z) { return vcycle(P, v, z); };
      auto pj = [&](double*) { return SDG_OK; };
      rc = fgmres(P, P->nu, F, u, P->opt.rtol, P->opt.max_it, mv, pc, pj, &its, &rel);
    } else {
      rc = cg_solve(P, F, u, P->opt.rtol, P->opt.max_it, &its, &rel);
    }
  }
  // true residual ||F - A u|| / ||F||
  double trel = rel;
  if (rc >= 0) {
    double fn, rn;
    int r2 = norm2(P, P->nu, F, &fn);
    if (r2 >= 0) r2 = sip_residual(P->M, P->k, 1, P->eta, F, u, P->vr, P->s);
    if (r2 >= 0) r2 = norm2(P, P->nu, P->vr, &rn);
    if (r2 >= 0) trel = fn > 0 ? rn / fn : 0.0;
    else rc = r2;
  }
  (void)hipStreamSynchronize(P->s);
  (void)hipFree(F);
  (void)hipFree(G);
  if (st) {
    st->status = rc;
    st->outer_its = its;
    st->inner_its_total = 0;
    st->inner_its_max = 0;
    st->rel_residual = trel;
    st->setup_ms = P->setup_ms;
    st->solve_ms = now_ms() - t0;
  }
  return rc;
}

int sdg_solve_stokes_dev(sdg_problem* P, const double* f, const double* g, double* u, double* p,
                         sdg_stats* st) {
  PCHECK(f, u, p);
  const double t0 = now_ms();
  const int64_t n = P->nu + P->np;
  double* b = nullptr;
  double* x = nullptr;
  SDG_HIP(hipMalloc((void**)&b, n * sizeof(double)));
  if (hipMalloc((void**)&x, n * sizeof(double)) != hipSuccess) {
    (void)hipFree(b);
    set_error("allocation failed");
    return SDG_ERR_NOMEM;
  }
  P->inner_total = 0;
  P->inner_max = 0;
  int rc = rhs_assemble(P->M, P->k, P->eta, f, g, b, b + P->nu, P->s);
  int its = 0;
  double rel = 0.0;
  if (rc >= 0) rc = ensure_gmres(P, n);
  if (rc >= 0) {
    auto mv = [&](const double* xx, double* yy) { return stokes_matvec(P, xx, yy); };
    auto pc = [&](const double* v, double* z) { return stokes_prec(P, v, z); };
    auto pj = [&](double* v) { return stokes_project(P, v); };
    rc = fgmres(P, n, b, x, P->opt.rtol, P->opt.max_it, mv, pc, pj, &its, &rel);
  }
  if (rc >= 0) {
    int r2 = stokes_project(P, x);
    if (r2 >= 0 && hipMemcpyAsync(u, x, P->nu * sizeof(double), hipMemcpyDeviceToDevice, P->s) != hipSuccess) r2 = SDG_ERR_DEVICE;
    if (r2 >= 0 && hipMemcpyAsync(p, x + P->nu, P->np * sizeof(double), hipMemcpyDeviceToDevice, P->s) != hipSuccess) r2 = SDG_ERR_DEVICE;
    if (r2 < 0) rc = r2;
  }
  (void)hipStreamSynchronize(P->s);
  (void)hipFree(b);
  (void)hipFree(x);
  if (st) {
    st->status = rc;
    st->outer_its = its;
    st->inner_its_total = P->inner_total;
    st->inner_its_max = P->inner_max;
    st->rel_residual = rel;
    st->setup_ms = P->setup_ms;
    st->solve_ms = now_ms() - t0;
  }
  return rc;
}

static int host_solve(sdg_ctx* ctx, const sdg_mesh* mesh, const sdg_options* opts, const double* eta,
                      const double* f, const double* g, double* u, double* p, sdg_stats* st, bool stokes) {
  if (!ctx || !mesh_ok(mesh) || !eta || !f || !u || (stokes && !p)) {
    set_error("invalid argument");
    return SDG_ERR_INVALID;
  }
  SDG_HIP(hipSetDevice(ctx->device));
  const int64_t nel = (int64_t)mesh->nx * mesh->ny;
  const int64_t NB = 2 * (int64_t)(mesh->k + 1) * (mesh->k + 1);
  const int64_t nu = nel * NB, np = nel * mesh->k * mesh->k;
  const int64_t ng = (int64_t)(2 * mesh->nx + 2 * mesh->ny) * 2 * (mesh->k + 1);
  double *de = nullptr, *df = nullptr, *dg = nullptr, *du = nullptr, *dp = nullptr;
  int rc = SDG_OK;
  auto al = [&](double** q, int64_t n) {
    if (rc < 0) return;
    if (hipMalloc((void**)q, std::max<int64_t>(n, 1) * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      set_error("allocation failed");
      rc = SDG_ERR_NOMEM;
    }
  };
  al(&de, nel);
  al(&df, nu);
  al(&du, nu);
  if (stokes) al(&dp, np);
  if (g) al(&dg, ng);
  if (rc >= 0) {
    if (hipMemcpy(de, eta, nel * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(df, f, nu * 8, hipMemcpyHostToDevice) != hipSuccess ||
        (g && hipMemcpy(dg, g, ng * 8, hipMemcpyHostToDevice) != hipSuccess)) {
      set_error("host to device copy failed");
      rc = SDG_ERR_DEVICE;
    }
  }
  sdg_problem* P = nullptr;
  if (rc >= 0) rc = sdg_problem_create(ctx, mesh, opts, de, nullptr, &P);
  if (rc >= 0) {
    rc = stokes ? sdg_solve_stokes_dev(P, df, dg, du, dp, st) : sdg_solve_viscous_dev(P, df, dg, du, st);
    if (rc >= 0) {
      if (hipMemcpy(u, du, nu * 8, hipMemcpyDeviceToHost) != hipSuccess ||
          (stokes && hipMemcpy(p, dp, np * 8, hipMemcpyDeviceToHost) != hipSuccess)) {
        set_error("device to host copy failed");
        rc = SDG_ERR_DEVICE;
      }
    }
  }
  sdg_problem_destroy(P);
  for (double* q : {de, df, dg, du, dp})
    if (q) (void)hipFree(q);
  return rc;
}

int sdg_solve_viscous(sdg_ctx* ctx, const sdg_mesh* mesh, const sdg_options* opts, const double* eta,
                      const double* f, const double* g, double* u, sdg_stats* st) {
  return host_solve(ctx, mesh, opts, eta, f, g, u, nullptr, st, false);
}
int sdg_solve_stokes(sdg_ctx* ctx, const sdg_mesh* mesh, const sdg_options* opts, const double* eta,
                     const double* f, const double* g, double* u, double* p, sdg_stats* st) {
  return host_solve(ctx, mesh, opts, eta, f, g, u, p, st, true);
}

int sdg_uniform_pm1(sdg_ctx* ctx, uint64_t seed, int64_t n, double* out, void* stream) {
  if (!ctx || !out || n < 0) {
    set_error("invalid argument");
    return SDG_ERR_INVALID;
  }
  return uniform_pm1(seed, n, out, (hipStream_t)stream);
}

}  // extern "C"
