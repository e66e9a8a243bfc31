// p-transfer to the Q_1 coarse space and the continuous-Q_1 h-hierarchy
// (Section 6 and Section 6.1.2).
//
// * R_k^1 keeps the hierarchical modes i, j <= 1; P_k^1 = (R_k^1)^T.
// * P_cd maps nodal values of the continuous bilinear field at the four
//   vertices of an element to its Q_1 modes: with the orthonormal scaling
//   psi_ij = c_ij L_i L_j, c_ij = sqrt((2i+1)(2j+1)/(hx hy)), the vertex
//   (a, b) hat function has mode (i, j) coefficient s_a^i s_b^j / (4 c_ij),
//   s_0 = -1, s_1 = +1.  R_dc = P_cd^T (gather over the <= 4 elements that
//   share a node).
// * A_{1,c} = P_cd^T A_1 P_cd: on continuous bilinear fields the jumps vanish,
//   so every interior-face term of A_1 drops out and A_{1,c} assembles from
//   element-local volume + boundary-face matrices (computed by the SIP tile
//   kernel on the hat functions).  Stored as a 9-point stencil of 2x2 blocks:
//   st[s][d][c][node], s = (dy+1)*3 + (dx+1).
// * h-levels: vertex-centred bilinear interpolation P_h, R_h = P_h^T,
//   A_H = P_h^T A_h P_h computed stencil-wise.
#include "sdg_common.h"
#include "sdg_kernels.h"

namespace sdg {

__device__ __forceinline__ double pcd_coef(int i, int j, int va, int vb, double hx, double hy) {
  const double cij = sqrt((2.0 * i + 1.0) * (2.0 * j + 1.0) / (hx * hy));
  const double si = (i == 0) ? 1.0 : (va ? 1.0 : -1.0);
  const double sj = (j == 0) ? 1.0 : (vb ? 1.0 : -1.0);
  return 0.25 * si * sj / cij;
}

// rc[pb][node][c] = sum over adjacent elements of P_cd^T (Q1 modes of r).
// With x0 non-null, also the first h-level's first Chebyshev step from a
// zero start, fused: x0 = d0 = cb D^{-1} rc (cb = ab0[2 pb + 1]).
template <typename TV>
__global__ void p_restrict_kernel(int nx, int ny, int k1, double hx, double hy, int nbatch,
                                  const TV* __restrict__ r, double* __restrict__ rc,
                                  const double* __restrict__ dinv, const double* __restrict__ ab0,
                                  double* __restrict__ x0, double* __restrict__ d0) {
  const int nn = (nx + 1) * (ny + 1);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nbatch * nn * 2) return;
  const int c = (int)(g & 1);
  const int64_t gn = g >> 1;
  const int64_t pb = gn / nn;
  const int node = (int)(gn - pb * nn);
  const int jx = node % (nx + 1), jy = node / (nx + 1);
  const int KK = k1 * k1, NB = 2 * KK;
  // unconditional loads (an absent element's index clamped to element 0,
  // its terms dropped by select)
  double s = 0.0;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int ex = jx - a, ey = jy - b;  // element whose vertex (a, b) is this node
      const bool in = ex >= 0 && ex < nx && ey >= 0 && ey < ny;
      const TV* re = r + ((pb * ny + (in ? ey : 0)) * (int64_t)nx + (in ? ex : 0)) * NB + c * KK;
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const double t = pcd_coef(i, j, a, b, hx, hy) * double(re[j * k1 + i]);
          s += in ? t : 0.0;
        }
    }
  rc[g] = s;
  if (x0) {
    const double dv = ab0[2 * pb + 1] * (dinv[g] * s);
    d0[g] = dv;
    x0[g] = dv;
  }
}

// u[pb][e][c][j][i] += sum_vertices P_cd ec, i, j <= 1
template <typename TV>
__global__ void p_prolong_kernel(int nx, int ny, int k1, double hx, double hy, int nbatch,
                                 const double* __restrict__ ec, TV* __restrict__ u) {
  const int nel = nx * ny;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nbatch * nel * 8) return;
  const int mode = (int)(g & 3), c = (int)((g >> 2) & 1);
  const int64_t ge = g >> 3;
  const int64_t pb = ge / nel;
  const int e = (int)(ge - pb * nel);
  const int ex = e % nx, ey = e / nx;
  const int i = mode & 1, j = mode >> 1;
  const int nn = (nx + 1) * (ny + 1);
  double s = 0.0;
  for (int b = 0; b < 2; ++b)
    for (int a = 0; a < 2; ++a) {
      const int node = (ey + b) * (nx + 1) + ex + a;
      s += pcd_coef(i, j, a, b, hx, hy) * ec[(pb * nn + node) * 2 + c];
    }
  const int KK = k1 * k1;
  TV* ue = u + ge * 2 * KK + c * KK + j * k1 + i;
  *ue = TV(double(*ue) + s);
}

int p_restrict(const MeshDev& M, int k, int nbatch, const double* r, double* rc, hipStream_t s,
               const FirstStep* first) {
  const int64_t n = (int64_t)nbatch * (M.nx + 1) * (M.ny + 1) * 2;
  hipLaunchKernelGGL(p_restrict_kernel<double>, dim3(ceil_div(n, 256)), dim3(256), 0, s, M.nx, M.ny,
                     k + 1, M.hx, M.hy, nbatch, r, rc, first ? first->dinv : nullptr, first ? first->ab0 : nullptr,
                     first ? first->x0 : nullptr, first ? first->d0 : nullptr);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int p_restrict_f32(const MeshDev& M, int k, int nbatch, const float* r, double* rc, hipStream_t s,
                   const FirstStep* first) {
  const int64_t n = (int64_t)nbatch * (M.nx + 1) * (M.ny + 1) * 2;
  hipLaunchKernelGGL(p_restrict_kernel<float>, dim3(ceil_div(n, 256)), dim3(256), 0, s, M.nx, M.ny,
                     k + 1, M.hx, M.hy, nbatch, r, rc, first ? first->dinv : nullptr, first ? first->ab0 : nullptr,
                     first ? first->x0 : nullptr, first ? first->d0 : nullptr);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int p_prolong_add(const MeshDev& M, int k, int nbatch, const double* ec, double* u, hipStream_t s) {
  const int64_t n = (int64_t)nbatch * M.nx * M.ny * 8;
  hipLaunchKernelGGL(p_prolong_kernel<double>, dim3(ceil_div(n, 256)), dim3(256), 0, s, M.nx, M.ny,
                     k + 1, M.hx, M.hy, nbatch, ec, u);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int p_prolong_add_f32(const MeshDev& M, int k, int nbatch, const double* ec, float* u, hipStream_t s) {
  const int64_t n = (int64_t)nbatch * M.nx * M.ny * 8;
  hipLaunchKernelGGL(p_prolong_kernel<float>, dim3(ceil_div(n, 256)), dim3(256), 0, s, M.nx, M.ny,
                     k + 1, M.hx, M.hy, nbatch, ec, u);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// Q_0 coarse space (Section 6.1.1): the element-wise constants are the (0, 0)
// modes of the hierarchical basis, so P_k^0 injects them and its transpose
// picks them; the coarse unknowns live on the grid of element centres
// (node = element index, two components per node).
// ---------------------------------------------------------------------------
// v = (0, 0) mode of component d set to 1 on the elements of colour
// (cx, cy) = (ix mod 3, iy mod 3), every other entry 0
__global__ void q0_probe_vec_kernel(int nx, int ny, int64_t ntot, int NB, int KK, int cx, int cy, int d,
                                    double* __restrict__ v) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ntot * NB) return;
  const int64_t ge = g / NB;
  const int a = (int)(g - ge * NB);
  const int e = (int)(ge % ((int64_t)nx * ny));
  const int ix = e % nx, iy = e / nx;
  v[g] = (a == d * KK && ix % 3 == cx && iy % 3 == cy) ? 1.0 : 0.0;
}
// A couples an element only with itself and its four face neighbours, and
// those five have five different colours: the (0, 0) response of element g
// to the probe of colour (cx, cy), component d, is the entry of A_0 between
// g and the one element of that colour among them.  Stencil layout as in
// stencil_kernel: st[(s 4 + row 2 + col) NN + g], s = (sy + 1) 3 + (sx + 1).
__global__ void q0_probe_gather_kernel(int nx, int ny, int nbatch, int NB, int KK, int cx, int cy, int d,
                                       const double* __restrict__ y, double* __restrict__ st) {
  const int nel = nx * ny;
  const int64_t NN = (int64_t)nel * nbatch;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= NN) return;
  const int e = (int)(g % nel);
  const int ix = e % nx, iy = e / nx;
  const int off[5][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}};
  for (int o = 0; o < 5; ++o) {
    const int sx = off[o][0], sy = off[o][1];
    const int jx = ix + sx, jy = iy + sy;
    if (jx < 0 || jx >= nx || jy < 0 || jy >= ny || jx % 3 != cx || jy % 3 != cy) continue;
    const int sidx = (sy + 1) * 3 + (sx + 1);
    for (int row = 0; row < 2; ++row) st[(sidx * 4 + row * 2 + d) * NN + g] = y[g * NB + row * KK];
  }
}
int q0_probe_vec(int nx, int ny, int nbatch, int k, int cx, int cy, int d, double* v, hipStream_t s) {
  const int K1 = k + 1, NB = 2 * K1 * K1;
  const int64_t ntot = (int64_t)nx * ny * nbatch;
  hipLaunchKernelGGL(q0_probe_vec_kernel, dim3(ceil_div(ntot * NB, 256)), dim3(256), 0, s, nx, ny, ntot, NB, K1 * K1,
                     cx, cy, d, v);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int q0_probe_gather(int nx, int ny, int nbatch, int k, int cx, int cy, int d, const double* y, double* st,
                    hipStream_t s) {
  const int K1 = k + 1, NB = 2 * K1 * K1;
  const int64_t n = (int64_t)nx * ny * nbatch;
  hipLaunchKernelGGL(q0_probe_gather_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, nx, ny, nbatch, NB, K1 * K1, cx,
                     cy, d, y, st);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
// rc[g][d] = mode (0, 0) of component d of element g of a vector with
// `stride` values per element and `cstride` per component (the residual's
// Q_1 modes: 8 and 4; a full Q_k vector: n_b and (k+1)^2)
template <typename TV>
__global__ void q0_restrict_kernel(int64_t n, int stride, int cstride, const TV* __restrict__ rq,
                                   double* __restrict__ rc) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 2 * n) return;
  rc[g] = double(rq[(g >> 1) * stride + (g & 1) * cstride]);
}
// x[g][d][0][0] += ec[g][d]
template <typename TV>
__global__ void q0_prolong_kernel(int64_t n, int NB, int KK, const double* __restrict__ ec, TV* __restrict__ x) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 2 * n) return;
  TV* p = x + (g >> 1) * NB + (g & 1) * KK;
  *p = TV(double(*p) + ec[g]);
}
int q0_restrict(int64_t nel_total, const double* rq1, double* rc, hipStream_t s) {
  hipLaunchKernelGGL(q0_restrict_kernel<double>, dim3(ceil_div(2 * nel_total, 256)), dim3(256), 0, s, nel_total, 8,
                     4, rq1, rc);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int q0_restrict_f32(int64_t nel_total, const float* rq1, double* rc, hipStream_t s) {
  hipLaunchKernelGGL(q0_restrict_kernel<float>, dim3(ceil_div(2 * nel_total, 256)), dim3(256), 0, s, nel_total, 8, 4,
                     rq1, rc);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int q0_restrict_full(int64_t nel_total, int k, const double* r, double* rc, hipStream_t s) {
  const int K1 = k + 1;
  hipLaunchKernelGGL(q0_restrict_kernel<double>, dim3(ceil_div(2 * nel_total, 256)), dim3(256), 0, s, nel_total,
                     2 * K1 * K1, K1 * K1, r, rc);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int q0_prolong_add(int64_t nel_total, int k, const double* ec, double* x, hipStream_t s) {
  const int K1 = k + 1;
  hipLaunchKernelGGL(q0_prolong_kernel<double>, dim3(ceil_div(2 * nel_total, 256)), dim3(256), 0, s, nel_total,
                     2 * K1 * K1, K1 * K1, ec, x);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int q0_prolong_add_f32(int64_t nel_total, int k, const double* ec, float* x, hipStream_t s) {
  const int K1 = k + 1;
  hipLaunchKernelGGL(q0_prolong_kernel<float>, dim3(ceil_div(2 * nel_total, 256)), dim3(256), 0, s, nel_total,
                     2 * K1 * K1, K1 * K1, ec, x);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// A_{1,c} stencil from element-local 8x8 matrices (rows/cols vertex*2 + comp)
// ---------------------------------------------------------------------------
__global__ void stencil_from_local_kernel(int nx, int ny, int nbatch, const double* __restrict__ cl,
                                          double* __restrict__ st) {
  const int nn = (nx + 1) * (ny + 1);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nbatch * nn) return;
  const int64_t pb = g / nn;
  const int node = (int)(g - pb * nn);
  const int jx = node % (nx + 1), jy = node / (nx + 1);
  const int64_t NNB = (int64_t)nbatch * nn;
  double out[36];
  for (int z = 0; z < 36; ++z) out[z] = 0.0;
  for (int b = 0; b < 2; ++b)
    for (int a = 0; a < 2; ++a) {
      const int ex = jx - a, ey = jy - b;
      if (ex < 0 || ex >= nx || ey < 0 || ey >= ny) continue;
      const double* L = cl + ((pb * ny + ey) * (int64_t)nx + ex) * 64;
      const int vr = b * 2 + a;
      for (int vb = 0; vb < 2; ++vb)
        for (int va = 0; va < 2; ++va) {
          const int vc = vb * 2 + va;
          const int dx = va - a, dy = vb - b;
          const int sidx = (dy + 1) * 3 + (dx + 1);
          for (int d = 0; d < 2; ++d)
            for (int c = 0; c < 2; ++c) out[sidx * 4 + d * 2 + c] += L[(vr * 2 + d) * 8 + vc * 2 + c];
        }
    }
  for (int z = 0; z < 36; ++z) st[z * NNB + g] = out[z];
}

int coarse_stencil_from_local(int nx, int ny, int nbatch, const double* clocal, double* st,
                              hipStream_t s) {
  const int64_t n = (int64_t)nbatch * (nx + 1) * (ny + 1);
  hipLaunchKernelGGL(stencil_from_local_kernel, dim3(ceil_div(n, 128)), dim3(128), 0, s, nx, ny, nbatch,
                     clocal, st);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// Galerkin coarsening A_H = P_h^T A_h P_h on 9-point block stencils
// ---------------------------------------------------------------------------
__device__ __forceinline__ double w1(int o) { return o == 0 ? 1.0 : 0.5; }

__global__ void galerkin_kernel(int nfx, int nfy, int nbatch, const double* __restrict__ stf,
                                double* __restrict__ stc) {
  const int ncx = nfx / 2, ncy = nfy / 2;
  const int nnc = (ncx + 1) * (ncy + 1), nnf = (nfx + 1) * (nfy + 1);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nbatch * nnc) return;
  const int64_t pb = g / nnc;
  const int cn = (int)(g - pb * nnc);
  const int cx = cn % (ncx + 1), cy = cn / (ncx + 1);
  const int64_t NF = (int64_t)nbatch * nnf, NC = (int64_t)nbatch * nnc;
  double out[36];
  for (int z = 0; z < 36; ++z) out[z] = 0.0;
  for (int oy = -1; oy <= 1; ++oy)
    for (int ox = -1; ox <= 1; ++ox) {
      const int fx = 2 * cx + ox, fy = 2 * cy + oy;  // fine node in the support of the coarse node
      if (fx < 0 || fx > nfx || fy < 0 || fy > nfy) continue;
      const double wi = w1(ox) * w1(oy);
      const int64_t fi = pb * nnf + (int64_t)fy * (nfx + 1) + fx;
      for (int sy = -1; sy <= 1; ++sy)
        for (int sx = -1; sx <= 1; ++sx) {
          const int gx = fx + sx, gy = fy + sy;  // fine neighbour j
          if (gx < 0 || gx > nfx || gy < 0 || gy > nfy) continue;
          const int sidx = (sy + 1) * 3 + (sx + 1);
          double a[4];
          for (int z = 0; z < 4; ++z) a[z] = stf[(sidx * 4 + z) * NF + fi];
          // coarse parents of (gx, gy)
          const int px0 = gx >> 1, px1 = (gx + 1) >> 1;
          const int py0 = gy >> 1, py1 = (gy + 1) >> 1;
          for (int py = py0; py <= py1; ++py)
            for (int px = px0; px <= px1; ++px) {
              const double wj = ((gx & 1) ? 0.5 : 1.0) * ((gy & 1) ? 0.5 : 1.0);
              const int ddx = px - cx, ddy = py - cy;
              const int cidx = (ddy + 1) * 3 + (ddx + 1);
              for (int z = 0; z < 4; ++z) out[cidx * 4 + z] += wi * wj * a[z];
            }
        }
    }
  for (int z = 0; z < 36; ++z) stc[z * NC + g] = out[z];
}

int galerkin_coarsen(int nfx, int nfy, int nbatch, const double* stf, double* stc, hipStream_t s) {
  const int64_t n = (int64_t)nbatch * (nfx / 2 + 1) * (nfy / 2 + 1);
  hipLaunchKernelGGL(galerkin_kernel, dim3(ceil_div(n, 128)), dim3(128), 0, s, nfx, nfy, nbatch, stf,
                     stc);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// stencil operators
// ---------------------------------------------------------------------------
template <bool RESID>
__global__ void stencil_kernel(int nx, int ny, int nbatch, const double* __restrict__ st,
                               const double* __restrict__ b, const double* __restrict__ x,
                               double* __restrict__ y) {
  const int nn = (nx + 1) * (ny + 1);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nbatch * nn) return;
  const int64_t pb = g / nn;
  const int node = (int)(g - pb * nn);
  const int jx = node % (nx + 1), jy = node / (nx + 1);
  const int64_t NN = (int64_t)nbatch * nn;
  // unconditional loads (a neighbour index clamped into the grid, the term
  // dropped by select): loads under branches were waited for one by one
  double y0 = 0.0, y1 = 0.0;
#pragma unroll
  for (int sy = -1; sy <= 1; ++sy)
#pragma unroll
    for (int sx = -1; sx <= 1; ++sx) {
      const int gx = jx + sx, gy = jy + sy;
      const bool in = gx >= 0 && gx <= nx && gy >= 0 && gy <= ny;
      const int sidx = (sy + 1) * 3 + (sx + 1);
      const int64_t nb = pb * nn + (in ? (int64_t)gy * (nx + 1) + gx : node);
      const double x0 = x[nb * 2], x1 = x[nb * 2 + 1];
      const double t0 = st[(sidx * 4 + 0) * NN + g] * x0 + st[(sidx * 4 + 1) * NN + g] * x1;
      const double t1 = st[(sidx * 4 + 2) * NN + g] * x0 + st[(sidx * 4 + 3) * NN + g] * x1;
      y0 += in ? t0 : 0.0;
      y1 += in ? t1 : 0.0;
    }
  if (RESID) {
    y[g * 2] = b[g * 2] - y0;
    y[g * 2 + 1] = b[g * 2 + 1] - y1;
  } else {
    y[g * 2] = y0;
    y[g * 2 + 1] = y1;
  }
}

int stencil_apply(int nx, int ny, int nbatch, const double* st, const double* x, double* y,
                  hipStream_t s) {
  const int64_t n = (int64_t)nbatch * (nx + 1) * (ny + 1);
  hipLaunchKernelGGL(stencil_kernel<false>, dim3(ceil_div(n, 256)), dim3(256), 0, s, nx, ny, nbatch, st,
                     nullptr, x, y);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int stencil_residual(int nx, int ny, int nbatch, const double* st, const double* b, const double* x,
                     double* r, hipStream_t s) {
  const int64_t n = (int64_t)nbatch * (nx + 1) * (ny + 1);
  hipLaunchKernelGGL(stencil_kernel<true>, dim3(ceil_div(n, 256)), dim3(256), 0, s, nx, ny, nbatch, st,
                     b, x, r);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

__global__ void diag_inv_kernel(int64_t NN, const double* __restrict__ st, double* __restrict__ dinv) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= NN) return;
  dinv[g * 2] = 1.0 / st[(4 * 4 + 0) * NN + g];
  dinv[g * 2 + 1] = 1.0 / st[(4 * 4 + 3) * NN + g];
}
int stencil_diag_inv(int nx, int ny, int nbatch, const double* st, double* dinv, hipStream_t s) {
  const int64_t n = (int64_t)nbatch * (nx + 1) * (ny + 1);
  hipLaunchKernelGGL(diag_inv_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, st, dinv);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// rc[I] = sum_{i in supp(I)} w_I(i) rf[i]
// rc = R rf (full weighting).  With x0 non-null, also the coarse level's
// first Chebyshev step from a zero start, fused: x0 = d0 = cb D^{-1} rc
// (cb = ab0[2 pb + 1], the step's coefficient), as the zero-start mode of
// hcheb_kernel computes it.
__global__ void h_restrict_kernel(int ncx, int ncy, int nbatch, const double* __restrict__ rf,
                                  double* __restrict__ rc, const double* __restrict__ dinv,
                                  const double* __restrict__ ab0, double* __restrict__ x0,
                                  double* __restrict__ d0) {
  const int nfx = 2 * ncx, nfy = 2 * ncy;
  const int nnc = (ncx + 1) * (ncy + 1), nnf = (nfx + 1) * (nfy + 1);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nbatch * nnc * 2) return;
  const int c = (int)(g & 1);
  const int64_t gn = g >> 1;
  const int64_t pb = gn / nnc;
  const int cn = (int)(gn - pb * nnc);
  const int cx = cn % (ncx + 1), cy = cn / (ncx + 1);
  // unconditional loads (index clamped into the grid, term dropped by select)
  double s = 0.0;
#pragma unroll
  for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
    for (int ox = -1; ox <= 1; ++ox) {
      const int fx = 2 * cx + ox, fy = 2 * cy + oy;
      const bool in = fx >= 0 && fx <= nfx && fy >= 0 && fy <= nfy;
      const int64_t fi = in ? (int64_t)fy * (nfx + 1) + fx : (int64_t)(2 * cy) * (nfx + 1) + 2 * cx;
      const double t = w1(ox) * w1(oy) * rf[(pb * nnf + fi) * 2 + c];
      s += in ? t : 0.0;
    }
  rc[g] = s;
  if (x0) {
    const double dv = ab0[2 * pb + 1] * (dinv[g] * s);
    d0[g] = dv;
    x0[g] = dv;
  }
}
// xf[i] += sum_{parents J} w_J(i) ec[J]
__global__ void h_prolong_kernel(int ncx, int ncy, int nbatch, const double* __restrict__ ec,
                                 double* __restrict__ xf) {
  const int nfx = 2 * ncx, nfy = 2 * ncy;
  const int nnc = (ncx + 1) * (ncy + 1), nnf = (nfx + 1) * (nfy + 1);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nbatch * nnf * 2) return;
  const int c = (int)(g & 1);
  const int64_t gn = g >> 1;
  const int64_t pb = gn / nnf;
  const int fn = (int)(gn - pb * nnf);
  const int fx = fn % (nfx + 1), fy = fn / (nfx + 1);
  const double wx = (fx & 1) ? 0.5 : 1.0, wy = (fy & 1) ? 0.5 : 1.0;
  // parents (fx >> 1 .. (fx + 1) >> 1) x (fy >> 1 .. (fy + 1) >> 1), one or
  // two per direction: four unconditional loads, the repeated parent of an
  // even index dropped by select
  const int px0 = fx >> 1, px1 = (fx + 1) >> 1, py0 = fy >> 1, py1 = (fy + 1) >> 1;
  const double* e = ec + pb * nnc * 2 + c;
  const double e00 = e[((int64_t)py0 * (ncx + 1) + px0) * 2], e01 = e[((int64_t)py0 * (ncx + 1) + px1) * 2];
  const double e10 = e[((int64_t)py1 * (ncx + 1) + px0) * 2], e11 = e[((int64_t)py1 * (ncx + 1) + px1) * 2];
  const bool two_x = px1 != px0, two_y = py1 != py0;
  double s = 0.0;
  s += wx * wy * e00;
  s += two_x ? wx * wy * e01 : 0.0;
  s += two_y ? wx * wy * e10 : 0.0;
  s += (two_x && two_y) ? wx * wy * e11 : 0.0;
  xf[g] += s;
}
int h_restrict(int ncx, int ncy, int nbatch, const double* rf, double* rc, hipStream_t s) {
  return h_restrict_first(ncx, ncy, nbatch, rf, rc, nullptr, nullptr, nullptr, nullptr, s);
}
int h_restrict_first(int ncx, int ncy, int nbatch, const double* rf, double* rc, const double* dinv,
                     const double* ab0, double* x0, double* d0, hipStream_t s) {
  const int64_t n = (int64_t)nbatch * (ncx + 1) * (ncy + 1) * 2;
  hipLaunchKernelGGL(h_restrict_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, ncx, ncy, nbatch, rf,
                     rc, dinv, ab0, x0, d0);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int h_prolong_add(int ncx, int ncy, int nbatch, const double* ec, double* xf, hipStream_t s) {
  const int64_t n = (int64_t)nbatch * (2 * ncx + 1) * (2 * ncy + 1) * 2;
  hipLaunchKernelGGL(h_prolong_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, ncx, ncy, nbatch, ec,
                     xf);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// coarsest level: dense matrix from the stencil; dense matvec with the inverse
// ---------------------------------------------------------------------------
__global__ void stencil_to_dense_kernel(int nx, int ny, int nbatch, const double* __restrict__ st,
                                        double* __restrict__ dense) {
  const int nn = (nx + 1) * (ny + 1), n2 = 2 * nn;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nbatch * nn) return;
  const int64_t pb = g / nn;
  const int node = (int)(g - pb * nn);
  const int jx = node % (nx + 1), jy = node / (nx + 1);
  const int64_t NN = (int64_t)nbatch * nn;
  double* D = dense + pb * (int64_t)n2 * n2;
  for (int c = 0; c < n2; ++c) {
    D[(int64_t)(node * 2) * n2 + c] = 0.0;
    D[(int64_t)(node * 2 + 1) * n2 + c] = 0.0;
  }
  for (int sy = -1; sy <= 1; ++sy)
    for (int sx = -1; sx <= 1; ++sx) {
      const int gx = jx + sx, gy = jy + sy;
      if (gx < 0 || gx > nx || gy < 0 || gy > ny) continue;
      const int sidx = (sy + 1) * 3 + (sx + 1);
      const int nb = gy * (nx + 1) + gx;
      for (int d = 0; d < 2; ++d)
        for (int c = 0; c < 2; ++c)
          D[(int64_t)(node * 2 + d) * n2 + nb * 2 + c] = st[(sidx * 4 + d * 2 + c) * NN + g];
    }
}
int stencil_to_dense(int nx, int ny, int nbatch, const double* st, double* dense, hipStream_t s) {
  const int64_t n = (int64_t)nbatch * (nx + 1) * (ny + 1);
  hipLaunchKernelGGL(stencil_to_dense_kernel, dim3(ceil_div(n, 64)), dim3(64), 0, s, nx, ny, nbatch, st,
                     dense);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// y[pb] = A[pb] x[pb], one workgroup per (problem, 64-row block), wave per row
__global__ __launch_bounds__(256) void dense_matvec_kernel(int n, const double* __restrict__ A,
                                                           const double* __restrict__ x,
                                                           double* __restrict__ y) {
  const int pb = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double* Ap = A + (int64_t)pb * n * n;
  const double* xp = x + (int64_t)pb * n;
  for (int row = blockIdx.x * 4 + wave; row < n; row += gridDim.x * 4) {
    double s = 0.0;
    for (int c = lane; c < n; c += 64) s += Ap[(int64_t)row * n + c] * xp[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) y[(int64_t)pb * n + row] = s;
  }
}
int dense_matvec(int n, int nbatch, const double* A, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(dense_matvec_kernel, dim3(ceil_div(n, 4), nbatch), dim3(256), 0, s, n, A, x, y);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

}  // namespace sdg

namespace sdg {

// ---------------------------------------------------------------------------
// one Chebyshev / point-Jacobi step on an h-level, double-buffered x:
// mode 1: d = b D^-1 rhs, xo = d;  2: d = b D^-1 (rhs - A xi), xo = xi + d;
// mode 0: d = a d + b D^-1 (rhs - A xi), xo = xi + d.  ab[pb] = (a, b).
// ---------------------------------------------------------------------------
__global__ void hcheb_kernel(int nx, int ny, int nbatch, const double* __restrict__ st,
                             const double* __restrict__ dinv, const double* __restrict__ rhs,
                             const double* __restrict__ xi, double* __restrict__ xo, double* __restrict__ d,
                             const double* __restrict__ ab, int mode) {
  const int nn = (nx + 1) * (ny + 1);
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nbatch * nn) return;
  const int64_t pb = g / nn;
  const int node = (int)(g - pb * nn);
  const int jx = node % (nx + 1), jy = node / (nx + 1);
  const int64_t NN = (int64_t)nbatch * nn;
  double r0 = rhs[g * 2], r1 = rhs[g * 2 + 1];
  if (mode != 1) {
    // unconditional loads, as in stencil_kernel
#pragma unroll
    for (int sy = -1; sy <= 1; ++sy)
#pragma unroll
      for (int sx = -1; sx <= 1; ++sx) {
        const int gx = jx + sx, gy = jy + sy;
        const bool in = gx >= 0 && gx <= nx && gy >= 0 && gy <= ny;
        const int sidx = (sy + 1) * 3 + (sx + 1);
        const int64_t nb = pb * nn + (in ? (int64_t)gy * (nx + 1) + gx : node);
        const double x0 = xi[nb * 2], x1 = xi[nb * 2 + 1];
        const double t0 = st[(sidx * 4 + 0) * NN + g] * x0 + st[(sidx * 4 + 1) * NN + g] * x1;
        const double t1 = st[(sidx * 4 + 2) * NN + g] * x0 + st[(sidx * 4 + 3) * NN + g] * x1;
        r0 -= in ? t0 : 0.0;
        r1 -= in ? t1 : 0.0;
      }
  }
  const double ca = ab[2 * pb], cb = ab[2 * pb + 1];
  const double z0 = dinv[g * 2] * r0, z1 = dinv[g * 2 + 1] * r1;
  const double d0 = mode == 0 ? ca * d[g * 2] + cb * z0 : cb * z0;
  const double d1 = mode == 0 ? ca * d[g * 2 + 1] + cb * z1 : cb * z1;
  d[g * 2] = d0;
  d[g * 2 + 1] = d1;
  xo[g * 2] = mode == 1 ? d0 : xi[g * 2] + d0;
  xo[g * 2 + 1] = mode == 1 ? d1 : xi[g * 2 + 1] + d1;
}
int hcheb_step(int nx, int ny, int nbatch, const double* st, const double* dinv, const double* rhs,
               const double* xi, double* xo, double* d, const double* ab, int mode, hipStream_t s) {
  const int64_t n = (int64_t)nbatch * (nx + 1) * (ny + 1);
  hipLaunchKernelGGL(hcheb_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, nx, ny, nbatch, st, dinv, rhs, xi,
                     xo, d, ab, mode);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// coarse tail: the h-cycle below a size threshold in one workgroup per
// problem (levels 0..nlev-1 of the tail, the last one solved with its dense
// inverse); every sweep ends with a workgroup barrier.
// ---------------------------------------------------------------------------
constexpr int TAIL_NT = 1024;

__device__ __forceinline__ void tail_resid(const TailLevel& L, int64_t pb, int nbatch, const double* x,
                                           double* r) {
  const int nn = (L.nx + 1) * (L.ny + 1);
  const int64_t NN = (int64_t)nbatch * nn;
  for (int node = threadIdx.x; node < nn; node += TAIL_NT) {
    const int64_t g = pb * nn + node;
    const int jx = node % (L.nx + 1), jy = node / (L.nx + 1);
    double r0 = L.b[g * 2], r1 = L.b[g * 2 + 1];
    for (int sy = -1; sy <= 1; ++sy)
      for (int sx = -1; sx <= 1; ++sx) {
        const int gx = jx + sx, gy = jy + sy;
        if (gx < 0 || gx > L.nx || gy < 0 || gy > L.ny) continue;
        const int sidx = (sy + 1) * 3 + (sx + 1);
        const int64_t nb = pb * nn + (int64_t)gy * (L.nx + 1) + gx;
        const double x0 = x[nb * 2], x1 = x[nb * 2 + 1];
        r0 -= L.st[(sidx * 4 + 0) * NN + g] * x0 + L.st[(sidx * 4 + 1) * NN + g] * x1;
        r1 -= L.st[(sidx * 4 + 2) * NN + g] * x0 + L.st[(sidx * 4 + 3) * NN + g] * x1;
      }
    r[g * 2] = r0;
    r[g * 2 + 1] = r1;
  }
}

__device__ void tail_cheb(const TailLevel& L, int64_t pb, int nbatch, int steps, bool zero) {
  const int nn = (L.nx + 1) * (L.ny + 1);
  for (int s = 0; s < steps; ++s) {
    const bool first = (s == 0);
    if (!(first && zero)) {
      tail_resid(L, pb, nbatch, L.x, L.r);
      __syncthreads();
    }
    const double ca = L.ab[(int64_t)(s * nbatch + pb) * 2], cb = L.ab[(int64_t)(s * nbatch + pb) * 2 + 1];
    for (int i = threadIdx.x; i < 2 * nn; i += TAIL_NT) {
      const int64_t g = pb * nn * 2 + i;
      const double rv = (first && zero) ? L.b[g] : L.r[g];
      const double z = L.dinv[g] * rv;
      const double dv = first ? cb * z : ca * L.d[g] + cb * z;
      L.d[g] = dv;
      L.x[g] = (first && zero) ? dv : L.x[g] + dv;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(TAIL_NT) void coarse_tail_kernel(TailArgs A) {
  const int64_t pb = blockIdx.x;
  const int nb = A.nbatch;
  // descend
  for (int l = 0; l < A.nlev - 1; ++l) {
    const TailLevel& L = A.lev[l];
    tail_cheb(L, pb, nb, A.steps, true);
    tail_resid(L, pb, nb, L.x, L.r);
    __syncthreads();
    const TailLevel& C = A.lev[l + 1];
    const int ncx = C.nx, ncy = C.ny, nfx = L.nx, nfy = L.ny;
    const int nnc = (ncx + 1) * (ncy + 1), nnf = (nfx + 1) * (nfy + 1);
    for (int i = threadIdx.x; i < 2 * nnc; i += TAIL_NT) {
      const int c = i & 1, cn = i >> 1;
      const int cx = cn % (ncx + 1), cy = cn / (ncx + 1);
      double s = 0.0;
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          const int fx = 2 * cx + ox, fy = 2 * cy + oy;
          if (fx < 0 || fx > nfx || fy < 0 || fy > nfy) continue;
          s += (ox == 0 ? 1.0 : 0.5) * (oy == 0 ? 1.0 : 0.5) *
               L.r[(pb * nnf + (int64_t)fy * (nfx + 1) + fx) * 2 + c];
        }
      C.b[(pb * nnc + cn) * 2 + c] = s;
    }
    __syncthreads();
  }
  // coarsest: x = Dinv b
  {
    const TailLevel& L = A.lev[A.nlev - 1];
    const int nn = (L.nx + 1) * (L.ny + 1), n2 = 2 * nn;
    const double* D = A.dense + pb * (int64_t)n2 * n2;
    const double* b = L.b + pb * n2;
    // one wavefront per row: coalesced row reads, shuffle reduction
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = wave; i < n2; i += TAIL_NT / 64) {
      double s = 0.0;
      for (int j = lane; j < n2; j += 64) s += D[(int64_t)i * n2 + j] * b[j];
      for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
      if (lane == 0) L.x[pb * n2 + i] = s;
    }
    __syncthreads();
  }
  // ascend
  for (int l = A.nlev - 2; l >= 0; --l) {
    const TailLevel& L = A.lev[l];
    const TailLevel& C = A.lev[l + 1];
    const int ncx = C.nx, nfx = L.nx, nfy = L.ny;
    const int nnc = (ncx + 1) * (C.ny + 1), nnf = (nfx + 1) * (nfy + 1);
    for (int i = threadIdx.x; i < 2 * nnf; i += TAIL_NT) {
      const int c = i & 1, fn = i >> 1;
      const int fx = fn % (nfx + 1), fy = fn / (nfx + 1);
      const double wx = (fx & 1) ? 0.5 : 1.0, wy = (fy & 1) ? 0.5 : 1.0;
      double s = 0.0;
      for (int py = fy >> 1; py <= (fy + 1) >> 1; ++py)
        for (int px = fx >> 1; px <= (fx + 1) >> 1; ++px)
          s += wx * wy * C.x[(pb * nnc + (int64_t)py * (ncx + 1) + px) * 2 + c];
      L.x[(pb * nnf + fn) * 2 + c] += s;
    }
    __syncthreads();
    tail_cheb(L, pb, nb, A.steps, false);
  }
}

// The same h-cycle with every operand of the small levels staged in LDS:
// per level the stencil (36 values per node), the inverse diagonal and the
// vectors b, x, r, d; only the restricted right-hand side of the first tail
// level comes from HBM and only its solution goes back; the dense inverse of
// the last level is read from L2.  Each sweep is then LDS traffic only.
__device__ __forceinline__ int tail_nn(const TailLevel& L) { return (L.nx + 1) * (L.ny + 1); }

__global__ __launch_bounds__(TAIL_NT) void coarse_tail_lds_kernel(TailArgs A) {
  extern __shared__ double lds[];
  const int64_t pb = blockIdx.x;
  const int nb = A.nbatch, nl = A.nlev;
  const int t = threadIdx.x;
  // per level: st[36][nn], dinv[2nn], b[2nn], x[2nn], r[2nn], d[2nn]
  double* base[TAIL_MAXLEV];
  {
    int64_t off = 0;
    for (int l = 0; l < nl; ++l) {
      base[l] = lds + off;
      off += 46 * (int64_t)tail_nn(A.lev[l]);
    }
  }
  auto ST = [&](int l) { return base[l]; };
  auto DI = [&](int l) { return base[l] + 36 * tail_nn(A.lev[l]); };
  auto BV = [&](int l) { return base[l] + 38 * tail_nn(A.lev[l]); };
  auto XV = [&](int l) { return base[l] + 40 * tail_nn(A.lev[l]); };
  auto RV = [&](int l) { return base[l] + 42 * tail_nn(A.lev[l]); };
  auto DV = [&](int l) { return base[l] + 44 * tail_nn(A.lev[l]); };
  // this problem's Chebyshev coefficients of every smoothed level (all but
  // the dense coarsest, which has none) and step, after the levels: ab[l][s][2]
  double* sab;
  {
    int64_t off = 0;
    for (int l = 0; l < nl; ++l) off += 46 * (int64_t)tail_nn(A.lev[l]);
    sab = lds + off;
  }
  for (int q = t; q < (nl - 1) * A.steps; q += TAIL_NT) {
    const int l = q / A.steps, st_ = q - l * A.steps;
    sab[2 * q] = A.lev[l].ab[(int64_t)(st_ * nb + pb) * 2];
    sab[2 * q + 1] = A.lev[l].ab[(int64_t)(st_ * nb + pb) * 2 + 1];
  }
  // stage the levels: four loads in flight per thread and round
  for (int l = 0; l < nl; ++l) {
    const TailLevel& L = A.lev[l];
    const int nn = tail_nn(L);
    const int64_t NN = (int64_t)nb * nn;
    if (l < nl - 1) {
      double* st = ST(l);
      for (int q0 = t; q0 < 36 * nn; q0 += 4 * TAIL_NT) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = q0 + u * TAIL_NT;
          const int k = q / nn, node = q - k * nn;
          v[u] = q < 36 * nn ? L.st[(int64_t)k * NN + pb * nn + node] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (q0 + u * TAIL_NT < 36 * nn) st[q0 + u * TAIL_NT] = v[u];
      }
      for (int q = t; q < 2 * nn; q += TAIL_NT) DI(l)[q] = L.dinv[pb * 2 * nn + q];
    }
    if (l == 0)
      for (int q = t; q < 2 * nn; q += TAIL_NT) BV(0)[q] = L.b[pb * 2 * nn + q];
  }
  __syncthreads();
  auto resid = [&](int l) {
    const TailLevel& L = A.lev[l];
    const int nn = tail_nn(L), nxp = L.nx + 1;
    const double *st = ST(l), *b = BV(l), *x = XV(l);
    double* r = RV(l);
    // one thread per unknown (node, component)
    for (int q = t; q < 2 * nn; q += TAIL_NT) {
      const int node = q >> 1, c = q & 1;
      const int jx = node % nxp, jy = node / nxp;
      double rv = b[q];
#pragma unroll
      for (int sy = -1; sy <= 1; ++sy)
#pragma unroll
        for (int sx = -1; sx <= 1; ++sx) {
          const int gx = jx + sx, gy = jy + sy;
          if (gx < 0 || gx > L.nx || gy < 0 || gy > L.ny) continue;
          const int sidx = (sy + 1) * 3 + (sx + 1);
          const int nbn = gy * nxp + gx;
          rv -= st[(sidx * 4 + 2 * c) * nn + node] * x[nbn * 2] + st[(sidx * 4 + 2 * c + 1) * nn + node] * x[nbn * 2 + 1];
        }
      r[q] = rv;
    }
  };
  auto cheb = [&](int l, bool zero) {
    const TailLevel& L = A.lev[l];
    const int nn = tail_nn(L);
    double *b = BV(l), *x = XV(l), *r = RV(l), *d = DV(l);
    const double* di = DI(l);
    for (int s = 0; s < A.steps; ++s) {
      const bool first = (s == 0);
      if (!(first && zero)) {
        resid(l);
        __syncthreads();
      }
      const double ca = sab[2 * (l * A.steps + s)], cb = sab[2 * (l * A.steps + s) + 1];
      for (int i = t; i < 2 * nn; i += TAIL_NT) {
        const double rv = (first && zero) ? b[i] : r[i];
        const double z = di[i] * rv;
        const double dv = first ? cb * z : ca * d[i] + cb * z;
        d[i] = dv;
        x[i] = (first && zero) ? dv : x[i] + dv;
      }
      __syncthreads();
    }
  };
  // descend
  for (int l = 0; l < nl - 1; ++l) {
    cheb(l, true);
    resid(l);
    __syncthreads();
    const TailLevel& L = A.lev[l];
    const TailLevel& C = A.lev[l + 1];
    const int ncx = C.nx, nfx = L.nx, nfy = L.ny;
    const int nnc = tail_nn(C);
    const double* r = RV(l);
    double* bc = BV(l + 1);
    for (int i = t; i < 2 * nnc; i += TAIL_NT) {
      const int c = i & 1, cn = i >> 1;
      const int cx = cn % (ncx + 1), cy = cn / (ncx + 1);
      double sum = 0.0;
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          const int fx = 2 * cx + ox, fy = 2 * cy + oy;
          if (fx < 0 || fx > nfx || fy < 0 || fy > nfy) continue;
          sum += (ox == 0 ? 1.0 : 0.5) * (oy == 0 ? 1.0 : 0.5) * r[(fy * (nfx + 1) + fx) * 2 + c];
        }
      bc[i] = sum;
    }
    __syncthreads();
  }
  // coarsest: x = Dinv b (the inverse from L2)
  {
    const TailLevel& L = A.lev[nl - 1];
    const int n2 = 2 * tail_nn(L);
    const double* D = A.dense + pb * (int64_t)n2 * n2;
    const double* b = BV(nl - 1);
    double* x = XV(nl - 1);
    // each wavefront sums one block of columns for every row (the inverse is
    // stored exactly symmetric, so row i of a column block is read as
    // contiguous column entries across the lanes); partial sums go to the
    // unused stencil space of this level, then one thread per row adds them
    constexpr int NW = TAIL_NT / 64;
    const int wave = t >> 6, lane = t & 63;
    double* part = ST(nl - 1);  // NW * n2 <= 36 nn doubles
    const int cb = (n2 + NW - 1) / NW, c0 = wave * cb, c1 = min(n2, c0 + cb);
    constexpr int CBMAX = 16;  // column blocks up to 16 wide: the loads of a lane are issued together
    for (int i = lane; i < n2; i += 64) {
      double sum = 0.0;
      if (cb <= CBMAX) {
        double dv[CBMAX];
#pragma unroll
        for (int u = 0; u < CBMAX; ++u) dv[u] = (c0 + u < c1) ? D[(int64_t)(c0 + u) * n2 + i] : 0.0;
#pragma unroll
        for (int u = 0; u < CBMAX; ++u)
          if (c0 + u < c1) sum += dv[u] * b[c0 + u];
      } else {
        for (int jj = c0; jj < c1; ++jj) sum += D[(int64_t)jj * n2 + i] * b[jj];
      }
      part[wave * n2 + i] = sum;
    }
    __syncthreads();
    for (int i = t; i < n2; i += TAIL_NT) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) sum += part[w * n2 + i];
      x[i] = sum;
    }
    __syncthreads();
  }
  // ascend
  for (int l = nl - 2; l >= 0; --l) {
    const TailLevel& L = A.lev[l];
    const TailLevel& C = A.lev[l + 1];
    const int ncx = C.nx, nfx = L.nx, nfy = L.ny;
    const int nnf = tail_nn(L);
    const double* xc = XV(l + 1);
    double* x = XV(l);
    for (int i = t; i < 2 * nnf; i += TAIL_NT) {
      const int c = i & 1, fn = i >> 1;
      const int fx = fn % (nfx + 1), fy = fn / (nfx + 1);
      const double wx = (fx & 1) ? 0.5 : 1.0, wy = (fy & 1) ? 0.5 : 1.0;
      double sum = 0.0;
      for (int py = fy >> 1; py <= (fy + 1) >> 1; ++py)
        for (int px = fx >> 1; px <= (fx + 1) >> 1; ++px) sum += wx * wy * xc[(py * (ncx + 1) + px) * 2 + c];
      x[i] += sum;
    }
    __syncthreads();
    cheb(l, false);
  }
  // the first tail level's solution back to HBM
  {
    const TailLevel& L = A.lev[0];
    const int nn = tail_nn(L);
    for (int q = t; q < 2 * nn; q += TAIL_NT) L.x[pb * 2 * nn + q] = XV(0)[q];
  }
}

size_t coarse_tail_lds_bytes(const TailArgs& A) {
  size_t n = 0;
  for (int l = 0; l < A.nlev; ++l) n += 46 * (size_t)(A.lev[l].nx + 1) * (A.lev[l].ny + 1);
  n += 2 * (size_t)A.nlev * A.steps;  // Chebyshev coefficients
  return n * sizeof(double);
}

int coarse_tail(const TailArgs& A, hipStream_t s) {
  const size_t lds = coarse_tail_lds_bytes(A);
  // the LDS form needs the kernel's dynamic LDS limit raised above 64 KB
  static int lds_ok = -1;  // once per process: -1 unknown, 0 no, 1 yes
  if (lds_ok < 0) {
    lds_ok = hipFuncSetAttribute(reinterpret_cast<const void*>(&coarse_tail_lds_kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) == hipSuccess;
    if (!lds_ok) (void)hipGetLastError();
  }
  if (lds_ok == 1 && A.nlev >= 2 && lds <= 150 * 1024) {
    hipLaunchKernelGGL(coarse_tail_lds_kernel, dim3(A.nbatch), dim3(TAIL_NT), lds, s, A);
  } else {
    hipLaunchKernelGGL(coarse_tail_kernel, dim3(A.nbatch), dim3(TAIL_NT), 0, s, A);
  }
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

}  // namespace sdg
