// Vector updates, deterministic two-stage reductions, the SplitMix64 start
// vectors and the small Hessenberg eigenvalue solve behind the Chebyshev
// bounds (Section 6: lambda* from ten GMRES/Arnoldi steps).
#include <algorithm>

#include "sdg_common.h"
#include "sdg_kernels.h"

namespace sdg {

constexpr int VT = 256;
constexpr int RED_BLOCKS = 512;  // fixed partial count: reductions are deterministic

__global__ void copy_kernel(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) y[g] = x[g];
}
__global__ void scale_copy_kernel(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) y[g] = a * x[g];
}
__global__ void axpy_kernel(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) y[g] += a * x[g];
}
__global__ void axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) y[g] = a * x[g] + b * y[g];
}
__global__ void mul_kernel(int64_t n, const double* __restrict__ d, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) y[g] = d[g] * x[g];
}
// mode 0: d = a d + b z, x += d;  mode 1: d = b z, x = d;  mode 2: d = b z, x += d
template <typename T>
__global__ void cheb_kernel(int64_t n, double a, const T* __restrict__ z, double b, T* __restrict__ d,
                            T* __restrict__ x, int mode) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) {
    const T dv = mode == 0 ? T(a * double(d[g]) + b * double(z[g])) : T(b * double(z[g]));
    d[g] = dv;
    x[g] = mode == 1 ? dv : T(x[g] + dv);
  }
}
__global__ void d2f_kernel(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) y[g] = (float)x[g];
}
__global__ void f2d_kernel(int64_t n, const float* __restrict__ x, double* __restrict__ y) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) y[g] = (double)x[g];
}

static inline int grid_for(int64_t n) {
  int64_t b = (n + VT - 1) / VT;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

#define VLAUNCH(kern, n, ...)                                                         \
  do {                                                                               \
    if ((n) > 0) hipLaunchKernelGGL(kern, dim3(grid_for(n)), dim3(VT), 0, s, n, __VA_ARGS__); \
    SDG_CHECK_LAUNCH();                                                              \
  } while (0)

int vec_copy(int64_t n, const double* x, double* y, hipStream_t s) { VLAUNCH(copy_kernel, n, x, y); return SDG_OK; }
// y[i rep + j] = x[i], j < rep
__global__ void expand_kernel(int64_t tot, int rep, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < tot; g += (int64_t)gridDim.x * VT) y[g] = x[g / rep];
}
int vec_expand(int64_t n, int rep, const double* x, double* y, hipStream_t s) {
  const int64_t tot = n * rep;
  VLAUNCH(expand_kernel, tot, rep, x, y);
  return SDG_OK;
}
int vec_scale_copy(int64_t n, double a, const double* x, double* y, hipStream_t s) { VLAUNCH(scale_copy_kernel, n, a, x, y); return SDG_OK; }
int vec_axpy(int64_t n, double a, const double* x, double* y, hipStream_t s) { VLAUNCH(axpy_kernel, n, a, x, y); return SDG_OK; }
int vec_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) { VLAUNCH(axpby_kernel, n, a, x, b, y); return SDG_OK; }
int vec_mul(int64_t n, const double* d, const double* x, double* y, hipStream_t s) { VLAUNCH(mul_kernel, n, d, x, y); return SDG_OK; }
int cheb_update(int64_t n, double a, const double* z, double b, double* d, double* x, int mode, hipStream_t s) {
  VLAUNCH(cheb_kernel<double>, n, a, z, b, d, x, mode);
  return SDG_OK;
}
int cheb_update_f32(int64_t n, double a, const float* z, double b, float* d, float* x, int mode, hipStream_t s) {
  VLAUNCH(cheb_kernel<float>, n, a, z, b, d, x, mode);
  return SDG_OK;
}
int d2f(int64_t n, const double* x, float* y, hipStream_t s) { VLAUNCH(d2f_kernel, n, x, y); return SDG_OK; }
int f2d(int64_t n, const float* x, double* y, hipStream_t s) { VLAUNCH(f2d_kernel, n, x, y); return SDG_OK; }

// ---------------------------------------------------------------------------
// reductions: stage 1 writes RED_BLOCKS partials per output, stage 2 sums
// them in a fixed order
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[VT / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < VT / 64; ++i) t += red[i];
  return t;
}

// partial[j][blk] = sum over the block's slice of V_j . w
__global__ __launch_bounds__(VT) void multidot_stage1(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                      const double* __restrict__ w, double* __restrict__ part) {
  const int j = blockIdx.y;
  const double* v = V + j * ldv;
  double s = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) s += v[g] * w[g];
  s = block_sum(s);
  if (threadIdx.x == 0) part[(int64_t)j * gridDim.x + blockIdx.x] = s;
}
__global__ __launch_bounds__(VT) void reduce_stage2(int nparts, const double* __restrict__ part,
                                                    double* __restrict__ out) {
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += VT) s += part[(int64_t)j * nparts + i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[j] = s;
}

// Copies n scalars into pinned host memory and then, after a system-scope
// fence, bumps a device counter and stores its new value into *host_seq:
// once the host reads the expected sequence number, the scalars are there.
// One thread; the counter makes every replay of a captured graph publish a
// new number.
__global__ void publish_kernel(const double* __restrict__ src, int n, double* host_dst,
                               unsigned* __restrict__ dev_count, volatile unsigned* host_seq) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = 0; i < n; ++i) host_dst[i] = src[i];
  const unsigned v = *dev_count + 1u;
  *dev_count = v;
  __threadfence_system();
  *host_seq = v;
}
int publish_scalars(const double* src, int n, double* host_dst, unsigned* dev_count, unsigned* host_seq,
                    hipStream_t s) {
  hipLaunchKernelGGL(publish_kernel, dim3(1), dim3(64), 0, s, src, n, host_dst, dev_count, host_seq);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// out[i] = sum over q of parts[q * n + i], q in order from 0.0 (the same sum
// the host forms over the segments of a Stokes vector)
__global__ void seg_sum_kernel(int64_t n, int nseg, const double* __restrict__ parts, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int q = 0; q < nseg; ++q) s += parts[q * n + i];
  out[i] = s;
}
int seg_sum(int64_t n, int nseg, const double* parts, double* out, hipStream_t s) {
  if (n <= 0) return SDG_OK;
  hipLaunchKernelGGL(seg_sum_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, n, nseg, parts, out);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
// hs[pb] = done[pb] ? 0 : sqrt(max(sq[pb], 0))
__global__ void norm_mask_kernel(int nb, const double* __restrict__ sq, const int* __restrict__ done,
                                 double* __restrict__ hs) {
  const int pb = blockIdx.x * blockDim.x + threadIdx.x;
  if (pb >= nb) return;
  const double v = sq[pb];
  hs[pb] = done[pb] ? 0.0 : sqrt(v > 0.0 ? v : 0.0);
}
// Column j of every problem's Arnoldi Hessenberg matrix (H: [pb][column]
// [row], leading dimension m + 1), from the two Gram-Schmidt passes'
// coefficients h0, h1 ([pb][i], i <= j) and ||w||^2 after them (hsq): rows
// 0..j take (0 + h0) + h1 and row j + 1 takes ||w||.  A problem stops at the
// first j where ||w|| <= 1e-14 |H[j][j]| (ms[pb] = j + 1, later columns stay
// zero); hs receives the divisor of the next basis vector, 0 for a stopped
// problem (its basis vector becomes zero).
__global__ void arnoldi_col_kernel(int nb, int j, int m, const double* __restrict__ h0,
                                   const double* __restrict__ h1, const double* __restrict__ hsq,
                                   int* __restrict__ stop, int* __restrict__ ms, double* __restrict__ H,
                                   double* __restrict__ hs) {
  const int pb = blockIdx.x * blockDim.x + threadIdx.x;
  if (pb >= nb) return;
  if (stop[pb]) {
    hs[pb] = 0.0;
    return;
  }
  const int mj = j + 1;
  double* col = H + ((int64_t)pb * m + j) * (m + 1);
  for (int i = 0; i <= j; ++i) col[i] = (0.0 + h0[(int64_t)pb * mj + i]) + h1[(int64_t)pb * mj + i];
  const double v = hsq[pb];
  const double hn = sqrt(v > 0.0 ? v : 0.0);
  col[j + 1] = hn;
  if (hn <= 1e-14 * fabs(col[j])) {
    ms[pb] = j + 1;
    stop[pb] = 1;
    hs[pb] = 0.0;
  } else {
    hs[pb] = hn;
  }
}
int arnoldi_col(int nb, int j, int m, const double* h0, const double* h1, const double* hsq, int* stop, int* ms,
                double* H, double* hs, hipStream_t s) {
  hipLaunchKernelGGL(arnoldi_col_kernel, dim3(ceil_div(nb, 256)), dim3(256), 0, s, nb, j, m, h0, h1, hsq, stop, ms,
                     H, hs);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int norm_mask(int nb, const double* sq, const int* done, double* hs, hipStream_t s) {
  hipLaunchKernelGGL(norm_mask_kernel, dim3(ceil_div(nb, 256)), dim3(256), 0, s, nb, sq, done, hs);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

int reduce_parts(int nparts, int nout, const double* part, double* out, hipStream_t s) {
  if (nout <= 0) return SDG_OK;
  hipLaunchKernelGGL(reduce_stage2, dim3(nout), dim3(VT), 0, s, nparts, part, out);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

static inline int red_blocks(int64_t n) {
  int64_t b = (n + VT - 1) / VT;
  return (int)(b < RED_BLOCKS ? (b < 1 ? 1 : b) : RED_BLOCKS);
}
// blocks per problem of the CG kernels that read all partials of a reduction
constexpr int CG_BLOCKS = 128;
static inline int cg_blocks(int64_t n) {
  const int b = red_blocks(n);
  return b < CG_BLOCKS ? b : CG_BLOCKS;
}

int multi_dot(int64_t n, int m, const double* V, int64_t ldv, const double* w, double* out,
              double* scratch, hipStream_t s) {
  if (m <= 0) return SDG_OK;
  const int nb = red_blocks(n);
  hipLaunchKernelGGL(multidot_stage1, dim3(nb, m), dim3(VT), 0, s, n, V, ldv, w, scratch);
  SDG_CHECK_LAUNCH();
  hipLaunchKernelGGL(reduce_stage2, dim3(m), dim3(VT), 0, s, nb, scratch, out);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int dot(int64_t n, const double* x, const double* y, double* out, double* scratch, hipStream_t s) {
  return multi_dot(n, 1, x, 0, y, out, scratch, s);
}

// w -= sum_j h[j] V_j
__global__ void multi_axpy_kernel(int64_t n, int m, const double* __restrict__ V, int64_t ldv,
                                  const double* __restrict__ h, double* __restrict__ w) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) {
    double s = w[g];
    for (int j = 0; j < m; ++j) s -= h[j] * V[j * ldv + g];
    w[g] = s;
  }
}
// y += sum_j h[j] V_j
__global__ void multi_combine_kernel(int64_t n, int m, const double* __restrict__ V, int64_t ldv,
                                     const double* __restrict__ h, double* __restrict__ y) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) {
    double s = y[g];
    for (int j = 0; j < m; ++j) s += h[j] * V[j * ldv + g];
    y[g] = s;
  }
}
int multi_axpy(int64_t n, int m, const double* V, int64_t ldv, const double* h, double* w, hipStream_t s) {
  VLAUNCH(multi_axpy_kernel, n, m, V, ldv, h, w);
  return SDG_OK;
}
int multi_combine(int64_t n, int m, const double* V, int64_t ldv, const double* h, double* y, hipStream_t s) {
  VLAUNCH(multi_combine_kernel, n, m, V, ldv, h, y);
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// SplitMix64 in counter form: z_i = mix(seed + (i+1) * 0x9E3779B97F4A7C15)
// ---------------------------------------------------------------------------
// entry g of the sequence: the g-th output of SplitMix64 started at seed,
// mapped to [-1, 1); out holds reps copies of the first n entries
__global__ void splitmix_kernel(int64_t tot, int64_t n, uint64_t seed, double* __restrict__ out) {
  for (int64_t q = (int64_t)blockIdx.x * VT + threadIdx.x; q < tot; q += (int64_t)gridDim.x * VT) {
    const int64_t g = q % n;
    uint64_t z = seed + (uint64_t)(g + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    out[q] = (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
  }
}
int uniform_pm1(uint64_t seed, int64_t n, double* out, hipStream_t s, int reps) {
  if (n <= 0 || reps <= 0) return SDG_OK;
  const int64_t tot = n * reps;
  VLAUNCH(splitmix_kernel, tot, n, seed, out);
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// pressure mean removal: subtract the mean of the constant modes (uniform
// elements, so c = sqrt|K| on every constant mode)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(VT) void pmean_stage1(int64_t nel, int np, const double* __restrict__ p,
                                                   double* __restrict__ part) {
  double s = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < nel; g += (int64_t)gridDim.x * VT) s += p[g * np];
  s = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ void pmean_sub(int64_t nel, int np, const double* __restrict__ sum, double* __restrict__ p) {
  const double m = sum[0] / (double)nel;
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < nel; g += (int64_t)gridDim.x * VT) p[g * np] -= m;
}
int pressure_project(int64_t nel, int np, double* p, double* scratch, hipStream_t s) {
  const int nb = red_blocks(nel);
  hipLaunchKernelGGL(pmean_stage1, dim3(nb), dim3(VT), 0, s, nel, np, p, scratch);
  SDG_CHECK_LAUNCH();
  hipLaunchKernelGGL(reduce_stage2, dim3(1), dim3(VT), 0, s, nb, scratch, scratch + RED_BLOCKS);
  SDG_CHECK_LAUNCH();
  hipLaunchKernelGGL(pmean_sub, dim3(grid_for(nel)), dim3(VT), 0, s, nel, np, scratch + RED_BLOCKS, p);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// eigenvalues of a small upper Hessenberg matrix: Francis double-shift QR
// with deflation on the active window (Golub & Van Loan, Matrix
// Computations, Sections 7.5.2-7.5.6); returns the largest real part.
// ---------------------------------------------------------------------------
constexpr int HMAX = 32;

__device__ void house3(double x, double y, double z, double* v, double* beta) {
  const double nrm = sqrt(x * x + y * y + z * z);
  if (nrm == 0.0) {
    v[0] = 1.0; v[1] = v[2] = 0.0; *beta = 0.0;
    return;
  }
  const double alpha = x >= 0.0 ? -nrm : nrm;
  v[0] = x - alpha; v[1] = y; v[2] = z;
  const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  *beta = vv > 0.0 ? 2.0 / vv : 0.0;
}

__device__ double hess_max_eig_dev(const double* __restrict__ Hin, int m, int ld) {
  double H[HMAX][HMAX];
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) H[i][j] = (i <= j + 1) ? Hin[(int64_t)j * ld + i] : 0.0;
  double wr[HMAX];
  double gersh = 0.0;
  for (int i = 0; i < m; ++i) {
    double r = 0.0;
    for (int j = 0; j < m; ++j) r += fabs(H[i][j]);
    gersh = r > gersh ? r : gersh;
  }
  const double eps = 2.220446049250313e-16;
  int p = m - 1;
  int its = 0;
  bool ok = true;
  while (p >= 0) {
    // deflation: find the start l of the unreduced active block ending at p
    int l = p;
    while (l > 0) {
      double sc = fabs(H[l - 1][l - 1]) + fabs(H[l][l]);
      if (sc == 0.0) sc = gersh;
      if (fabs(H[l][l - 1]) <= eps * sc) {
        H[l][l - 1] = 0.0;
        break;
      }
      --l;
    }
    if (l == p) {
      wr[p] = H[p][p];
      --p;
      its = 0;
      continue;
    }
    if (l == p - 1) {
      const double a = H[p - 1][p - 1], b = H[p - 1][p], c = H[p][p - 1], d = H[p][p];
      const double half = 0.5 * (a - d), disc = half * half + b * c;
      const double mid = 0.5 * (a + d);
      if (disc >= 0.0) {
        const double r = sqrt(disc);
        wr[p - 1] = mid + r;
        wr[p] = mid - r;
      } else {
        wr[p - 1] = wr[p] = mid;
      }
      p -= 2;
      its = 0;
      continue;
    }
    if (++its > 200) {
      ok = false;
      break;
    }
    // shifts: eigenvalues of the trailing 2x2 (exceptional shift every 11 steps)
    double sh, tt;
    if (its % 11 == 10) {
      const double w = fabs(H[p][p - 1]) + fabs(H[p - 1][p - 2]);
      sh = H[p][p] + 1.5 * w;
      tt = sh * sh / 4.0 + w * w;
    } else {
      sh = H[p - 1][p - 1] + H[p][p];
      tt = H[p - 1][p - 1] * H[p][p] - H[p - 1][p] * H[p][p - 1];
    }
    double x = H[l][l] * H[l][l] + H[l][l + 1] * H[l + 1][l] - sh * H[l][l] + tt;
    double y = H[l + 1][l] * (H[l][l] + H[l + 1][l + 1] - sh);
    double z = H[l + 1][l] * H[l + 2][l + 1];
    for (int k = l; k <= p - 2; ++k) {
      double v[3], beta;
      house3(x, y, z, v, &beta);
      const int c0 = k > l ? k - 1 : l;
      for (int c = c0; c <= p; ++c) {
        const double w = beta * (v[0] * H[k][c] + v[1] * H[k + 1][c] + v[2] * H[k + 2][c]);
        H[k][c] -= w * v[0];
        H[k + 1][c] -= w * v[1];
        H[k + 2][c] -= w * v[2];
      }
      const int r1 = (k + 3 < p) ? k + 3 : p;
      for (int r = l; r <= r1; ++r) {
        const double w = beta * (H[r][k] * v[0] + H[r][k + 1] * v[1] + H[r][k + 2] * v[2]);
        H[r][k] -= w * v[0];
        H[r][k + 1] -= w * v[1];
        H[r][k + 2] -= w * v[2];
      }
      x = H[k + 1][k];
      y = H[k + 2][k];
      if (k < p - 2) z = H[k + 3][k];
    }
    // final Givens rotation on rows/cols p-1, p
    const double rr = sqrt(x * x + y * y);
    if (rr > 0.0) {
      const double cg = x / rr, sg = y / rr;
      for (int c = p - 2; c <= p; ++c) {
        const double a1 = H[p - 1][c], a2 = H[p][c];
        H[p - 1][c] = cg * a1 + sg * a2;
        H[p][c] = -sg * a1 + cg * a2;
      }
      for (int r = l; r <= p; ++r) {
        const double a1 = H[r][p - 1], a2 = H[r][p];
        H[r][p - 1] = cg * a1 + sg * a2;
        H[r][p] = -sg * a1 + cg * a2;
      }
    }
  }
  double best = -1e300;
  if (ok) {
    for (int i = 0; i < m; ++i) best = wr[i] > best ? wr[i] : best;
  } else {
    best = gersh;
  }
  return best;
}

__global__ void hess_eig_kernel(const double* __restrict__ Hin, int m, int ld, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  out[0] = hess_max_eig_dev(Hin, m, ld);
}

int hessenberg_max_eig(const double* H, int m, int ld, double* out, hipStream_t s) {
  if (m < 1 || m > HMAX) {
    set_error("hessenberg size out of range");
    return SDG_ERR_INVALID;
  }
  hipLaunchKernelGGL(hess_eig_kernel, dim3(1), dim3(64), 0, s, H, m, ld, out);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

}  // namespace sdg

// ===========================================================================
// Batched kernels: vectors are [nbatch][n] (problem pb at offset pb * n);
// per-problem scalars are device arrays indexed by pb.
// ===========================================================================
namespace sdg {

// partial[pb][j][blk] = slice of <V_j[pb], w[pb]>; V_j at V + j * ldv.
// PAIRS (n and ldv even, V and w 16-byte aligned): 16-byte loads of value
// pairs, four strides unrolled so that their loads are in flight together
// (each thread has only a few strides), even and odd values summed apart.
template <bool PAIRS>
__global__ __launch_bounds__(VT) void bmultidot_stage1(int64_t n, int m, const double* __restrict__ V,
                                                       int64_t ldv, const double* __restrict__ w,
                                                       double* __restrict__ part, const int* __restrict__ active) {
  const int j = blockIdx.y % m, pb = blockIdx.y / m;
  if (active && !active[pb]) {  // a converged problem of a batched CG iteration (the whole block)
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
  const double* v = V + j * ldv + (int64_t)pb * n;
  const double* ww = w + (int64_t)pb * n;
  const int64_t st = (int64_t)gridDim.x * VT;
  double s = 0.0;
  if constexpr (PAIRS) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2* v2p = reinterpret_cast<const v2*>(v);
    const v2* w2p = reinterpret_cast<const v2*>(ww);
    double s1 = 0.0;
#pragma unroll 4
    for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < (n >> 1); g += st) {
      const v2 a = v2p[g], b = w2p[g];
      s = __builtin_fma(a.x, b.x, s);
      s1 = __builtin_fma(a.y, b.y, s1);
    }
    s += s1;
  } else {
    for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += st) s += v[g] * ww[g];
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}
static void launch_multidot(dim3 grid, int64_t n, int m, const double* V, int64_t ldv, const double* w, double* part,
                            hipStream_t s, const int* active = nullptr) {
  const bool pairs = n % 2 == 0 && (m == 1 || ldv % 2 == 0) && reinterpret_cast<uintptr_t>(V) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(w) % 16 == 0;
  if (pairs)
    hipLaunchKernelGGL(bmultidot_stage1<true>, grid, dim3(VT), 0, s, n, m, V, ldv, w, part, active);
  else
    hipLaunchKernelGGL(bmultidot_stage1<false>, grid, dim3(VT), 0, s, n, m, V, ldv, w, part, active);
}

int bmulti_dot(int64_t n, int nbatch, int m, const double* V, int64_t ldv, const double* w, double* out,
               double* scratch, hipStream_t s) {
  if (m <= 0 || nbatch <= 0) return SDG_OK;
  if ((int64_t)m * nbatch > 512 * 64) {
    set_error("reduction scratch too small for this batch");
    return SDG_ERR_INVALID;
  }
  int nb = red_blocks(n);
  if (nb * m * nbatch > 512 * 64) nb = std::max(1, 512 * 64 / (m * nbatch));
  launch_multidot(dim3(nb, m * nbatch), n, m, V, ldv, w, scratch, s);
  SDG_CHECK_LAUNCH();
  hipLaunchKernelGGL(reduce_stage2, dim3(m * nbatch), dim3(VT), 0, s, nb, scratch, out);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// first stage of <x[pb], y[pb]>: *nparts partials per problem at
// part[pb * nparts + i] (at most cap in all)
int bdot_parts(int64_t n, int nbatch, const double* x, const double* y, double* part, int cap, int* nparts,
               hipStream_t s, const int* active) {
  if (nbatch <= 0 || nbatch > cap) {
    set_error("reduction scratch too small for this batch");
    return SDG_ERR_INVALID;
  }
  int nb = cg_blocks(n);
  if ((int64_t)nb * nbatch > cap) nb = std::max(1, cap / nbatch);
  *nparts = nb;
  launch_multidot(dim3(nb, nbatch), n, 1, x, (int64_t)0, y, part, s, active);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// w[pb] -= sum_j h[pb][j] V_j[pb]
__global__ void bmulti_axpy_kernel(int64_t n, int nbatch, int m, const double* __restrict__ V, int64_t ldv,
                                   const double* __restrict__ h, double* __restrict__ w) {
  const int64_t tot = n * nbatch;
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < tot; g += (int64_t)gridDim.x * VT) {
    const int64_t pb = g / n;
    double s = w[g];
    for (int j = 0; j < m; ++j) s -= h[pb * m + j] * V[j * ldv + g];
    w[g] = s;
  }
}
// y[pb] += sum_j h[pb][j] V_j[pb]
__global__ void bmulti_combine_kernel(int64_t n, int nbatch, int m, const double* __restrict__ V, int64_t ldv,
                                      const double* __restrict__ h, double* __restrict__ y) {
  const int64_t tot = n * nbatch;
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < tot; g += (int64_t)gridDim.x * VT) {
    const int64_t pb = g / n;
    double s = y[g];
    for (int j = 0; j < m; ++j) s += h[pb * m + j] * V[j * ldv + g];
    y[g] = s;
  }
}
int bmulti_axpy(int64_t n, int nbatch, int m, const double* V, int64_t ldv, const double* h, double* w,
                hipStream_t s) {
  const int64_t tot = n * nbatch;
  if (tot > 0) hipLaunchKernelGGL(bmulti_axpy_kernel, dim3(grid_for(tot)), dim3(VT), 0, s, n, nbatch, m, V, ldv, h, w);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int bmulti_combine(int64_t n, int nbatch, int m, const double* V, int64_t ldv, const double* h, double* y,
                   hipStream_t s) {
  const int64_t tot = n * nbatch;
  if (tot > 0) hipLaunchKernelGGL(bmulti_combine_kernel, dim3(grid_for(tot)), dim3(VT), 0, s, n, nbatch, m, V, ldv, h, y);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// y[pb] = a[pb] * x[pb] (a from device memory)
__global__ void bscale_kernel(int64_t n, int64_t tot, const double* __restrict__ a, const double* __restrict__ x,
                              double* __restrict__ y, int invert) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < tot; g += (int64_t)gridDim.x * VT) {
    const double s = a[g / n];
    y[g] = invert ? (s != 0.0 ? x[g] / s : 0.0) : s * x[g];
  }
}
int bscale(int64_t n, int nbatch, const double* a, const double* x, double* y, int invert, hipStream_t s) {
  const int64_t tot = n * nbatch;
  if (tot > 0) hipLaunchKernelGGL(bscale_kernel, dim3(grid_for(tot)), dim3(VT), 0, s, n, tot, a, x, y, invert);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// CG step 1: alpha = active ? rz/pq : 0; x += alpha p; r -= alpha q;
// partial sums of ||r||^2 per problem
__global__ __launch_bounds__(VT) void cg_update1_kernel(int64_t n, const double* __restrict__ p,
                                                        const double* __restrict__ q, double* __restrict__ x,
                                                        double* __restrict__ r, const double* __restrict__ rz,
                                                        const double* __restrict__ pq,
                                                        const int* __restrict__ active,
                                                        double* __restrict__ part) {
  const int pb = blockIdx.y;
  const double a = (active[pb] && pq[pb] > 0.0) ? rz[pb] / pq[pb] : 0.0;
  const int64_t off = (int64_t)pb * n;
  double s = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) {
    const double rv = r[off + g] - a * q[off + g];
    x[off + g] += a * p[off + g];
    r[off + g] = rv;
    s += rv * rv;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) part[(int64_t)pb * gridDim.x + blockIdx.x] = s;
}
int cg_update1(int64_t n, int nbatch, const double* p, const double* q, double* x, double* r,
               const double* rz, const double* pq, const int* active, double* rr, double* scratch,
               hipStream_t s) {
  int nb = red_blocks(n);
  if (nb * nbatch > 512 * 64) nb = std::max(1, 512 * 64 / nbatch);
  hipLaunchKernelGGL(cg_update1_kernel, dim3(nb, nbatch), dim3(VT), 0, s, n, p, q, x, r, rz, pq, active, scratch);
  SDG_CHECK_LAUNCH();
  hipLaunchKernelGGL(reduce_stage2, dim3(nbatch), dim3(VT), 0, s, nb, scratch, rr);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
// CG step 2: p = z + (rz_new / rz_old) p for active problems
__global__ void cg_update2_kernel(int64_t n, int64_t tot, const double* __restrict__ z, double* __restrict__ p,
                                  const double* __restrict__ rz_new, const double* __restrict__ rz_old,
                                  const int* __restrict__ active) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < tot; g += (int64_t)gridDim.x * VT) {
    const int64_t pb = g / n;
    if (!active[pb]) continue;
    p[g] = z[g] + (rz_new[pb] / rz_old[pb]) * p[g];
  }
}
int cg_update2(int64_t n, int nbatch, const double* z, double* p, const double* rz_new, const double* rz_old,
               const int* active, hipStream_t s) {
  const int64_t tot = n * nbatch;
  if (tot > 0) hipLaunchKernelGGL(cg_update2_kernel, dim3(grid_for(tot)), dim3(VT), 0, s, n, tot, z, p, rz_new, rz_old, active);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// mode 0: d = a[pb] d + b[pb] z, x += d; 1: d = b z, x = d; 2: d = b z, x += d
template <typename T>
__global__ void bcheb_kernel(int64_t n, int64_t tot, const double* __restrict__ ab, const T* __restrict__ z,
                             T* __restrict__ d, T* __restrict__ x, int mode) {
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < tot; g += (int64_t)gridDim.x * VT) {
    const int64_t pb = g / n;
    const double a = ab[2 * pb], b = ab[2 * pb + 1];
    const T dv = mode == 0 ? T(a * double(d[g]) + b * double(z[g])) : T(b * double(z[g]));
    d[g] = dv;
    x[g] = mode == 1 ? dv : T(x[g] + dv);
  }
}
int bcheb_update(int64_t n, int nbatch, const double* ab, const double* z, double* d, double* x, int mode,
                 hipStream_t s) {
  const int64_t tot = n * nbatch;
  if (tot > 0) hipLaunchKernelGGL(bcheb_kernel<double>, dim3(grid_for(tot)), dim3(VT), 0, s, n, tot, ab, z, d, x, mode);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// pressure mean removal per problem (constant modes, uniform elements)
__global__ __launch_bounds__(VT) void bpmean_stage1(int64_t nel, int np, int64_t stride, const double* __restrict__ p,
                                                    double* __restrict__ part) {
  const int pb = blockIdx.y;
  double s = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < nel; g += (int64_t)gridDim.x * VT)
    s += p[pb * stride + g * np];
  s = block_sum(s);
  if (threadIdx.x == 0) part[(int64_t)pb * gridDim.x + blockIdx.x] = s;
}
__global__ void bpmean_sub(int64_t nel, int np, int64_t stride, int nbatch, const double* __restrict__ sum,
                           double* __restrict__ p) {
  const int64_t tot = nel * nbatch;
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < tot; g += (int64_t)gridDim.x * VT) {
    const int64_t pb = g / nel, e = g - pb * nel;
    p[pb * stride + e * np] -= sum[pb] / (double)nel;
  }
}
// p[pb] at p + pb * stride (stride >= nel * np)
int bpressure_project(int64_t nel, int np, int nbatch, int64_t stride, double* p, double* scratch,
                      hipStream_t s) {
  int nb = red_blocks(nel);
  if (nb * nbatch > 512 * 32) nb = std::max(1, 512 * 32 / nbatch);
  hipLaunchKernelGGL(bpmean_stage1, dim3(nb, nbatch), dim3(VT), 0, s, nel, np, stride, p, scratch);
  SDG_CHECK_LAUNCH();
  double* sums = scratch + 512 * 32;
  hipLaunchKernelGGL(reduce_stage2, dim3(nbatch), dim3(VT), 0, s, nb, scratch, sums);
  SDG_CHECK_LAUNCH();
  const int64_t tot = nel * nbatch;
  hipLaunchKernelGGL(bpmean_sub, dim3(grid_for(tot)), dim3(VT), 0, s, nel, np, stride, nbatch, sums, p);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// largest eigenvalue for nbatch Hessenberg matrices (one thread each);
// matrix pb at Hin + pb * hstride, order ms[pb]
__global__ void bhess_eig_kernel(int nbatch, const double* __restrict__ Hin, const int* __restrict__ ms, int ld,
                                 int64_t hstride, double* __restrict__ out) {
  const int pb = blockIdx.x * blockDim.x + threadIdx.x;
  if (pb >= nbatch) return;
  out[pb] = hess_max_eig_dev(Hin + pb * hstride, ms[pb], ld);
}
int bhessenberg_max_eig(int nbatch, const double* H, const int* ms, int ld, int64_t hstride, double* out,
                        hipStream_t s) {
  hipLaunchKernelGGL(bhess_eig_kernel, dim3(ceil_div(nbatch, 64)), dim3(64), 0, s, nbatch, H, ms, ld, hstride, out);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}


// ---------------------------------------------------------------------------
// CG steps with the preceding reduction's second stage folded in.  Every
// block first sums its problem's partials with the loop and block_sum of
// reduce_stage2 (the same order, so the same value in every block), then
// does its slice of the update; block 0 of each problem stores the sum.  As
// every block reads all partials, these kernels and the first stage that
// feeds them use at most CG_BLOCKS blocks per problem.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_total(int nparts, const double* __restrict__ part) {
  __shared__ double tot;
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += VT) s += part[i];
  s = block_sum(s);
  if (threadIdx.x == 0) tot = s;
  __syncthreads();
  const double t = tot;
  __syncthreads();
  return t;
}

// rz_new[pb] = sum of rzpart[pb][0 .. nparts); p = z + (rz_new / rz_old) p
__global__ __launch_bounds__(VT) void cg_update2_red_kernel(int64_t n, const double* __restrict__ z,
                                                            double* __restrict__ p,
                                                            const double* __restrict__ rzpart, int nparts,
                                                            double* __restrict__ rz_new,
                                                            const double* __restrict__ rz_old,
                                                            const int* __restrict__ active) {
  const int pb = blockIdx.y;
  const double rz = block_total(nparts, rzpart + (int64_t)pb * nparts);
  if (blockIdx.x == 0 && threadIdx.x == 0) rz_new[pb] = rz;
  if (!active[pb]) return;
  const double beta = rz / rz_old[pb];
  const int64_t off = (int64_t)pb * n;
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT)
    p[off + g] = z[off + g] + beta * p[off + g];
}
int cg_update2_red(int64_t n, int nbatch, const double* z, double* p, const double* rzpart, int nparts,
                   double* rz_new, const double* rz_old, const int* active, hipStream_t s) {
  if (n <= 0 || nbatch <= 0) return SDG_OK;
  hipLaunchKernelGGL(cg_update2_red_kernel, dim3(cg_blocks(n), nbatch), dim3(VT), 0, s, n, z, p, rzpart, nparts,
                     rz_new, rz_old, active);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// pq[pb] = sum of pqpart[pb][0 .. npq); alpha = active ? rz/pq : 0;
// x += alpha p; r -= alpha q; partial sums of ||r||^2 into rrpart[pb][blk]
__global__ __launch_bounds__(VT) void cg_update1_red_kernel(int64_t n, const double* __restrict__ p,
                                                            const double* __restrict__ q, double* __restrict__ x,
                                                            double* __restrict__ r, const double* __restrict__ rz,
                                                            const double* __restrict__ pqpart, int npq,
                                                            double* __restrict__ pq_out,
                                                            const int* __restrict__ active,
                                                            double* __restrict__ rrpart) {
  const int pb = blockIdx.y;
  const double pq = block_total(npq, pqpart + (int64_t)pb * npq);
  if (blockIdx.x == 0 && threadIdx.x == 0) pq_out[pb] = pq;
  if (!active[pb]) {  // converged: x and r stay as they are (the whole block)
    if (threadIdx.x == 0) rrpart[(int64_t)pb * gridDim.x + blockIdx.x] = 0.0;
    return;
  }
  const double a = pq > 0.0 ? rz[pb] / pq : 0.0;
  const int64_t off = (int64_t)pb * n;
  double s = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * VT + threadIdx.x; g < n; g += (int64_t)gridDim.x * VT) {
    const double rv = r[off + g] - a * q[off + g];
    x[off + g] += a * p[off + g];
    r[off + g] = rv;
    s += rv * rv;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) rrpart[(int64_t)pb * gridDim.x + blockIdx.x] = s;
}
int cg_update1_red(int64_t n, int nbatch, const double* p, const double* q, double* x, double* r, const double* rz,
                   const double* pqpart, int npq, double* pq_out, const int* active, double* rrpart,
                   int rr_cap, int* nrr, hipStream_t s) {
  if (n <= 0 || nbatch <= 0) return SDG_OK;
  int nb = cg_blocks(n);
  if ((int64_t)nb * nbatch > rr_cap) nb = std::max(1, rr_cap / nbatch);
  if ((int64_t)nb * nbatch > rr_cap) {
    set_error("reduction scratch too small for this batch");
    return SDG_ERR_INVALID;
  }
  *nrr = nb;
  hipLaunchKernelGGL(cg_update1_red_kernel, dim3(nb, nbatch), dim3(VT), 0, s, n, p, q, x, r, rz, pqpart, npq, pq_out,
                     active, rrpart);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// rr[pb] = sum of rrpart[pb][0 .. nrr) for every problem, then the
// publication of publish_kernel: src[0 .. n) to pinned host memory, a system
// fence, the device counter and its new value to *host_seq.  One block: a
// group of tp lanes (a power of two, at most a wavefront) per problem, each
// lane summing every tp-th partial, then the group's lanes in xor order.
__global__ __launch_bounds__(VT) void publish_red_kernel(const double* __restrict__ rrpart, int nrr, int nbatch,
                                                         double* rr, const double* src, int n, double* host_dst,
                                                         unsigned* __restrict__ dev_count,
                                                         volatile unsigned* host_seq) {
  int tp = 64;
  while (tp > 1 && tp * nbatch > VT) tp >>= 1;
  const int groups = VT / tp, g = threadIdx.x / tp, l = threadIdx.x % tp;
  for (int pb0 = 0; pb0 < nbatch; pb0 += groups) {
    const int pb = pb0 + g;
    double s = 0.0;
    if (pb < nbatch)
      for (int i = l; i < nrr; i += tp) s += rrpart[(int64_t)pb * nrr + i];
    for (int off = tp / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (pb < nbatch && l == 0) rr[pb] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int i = 0; i < n; ++i) host_dst[i] = src[i];
  const unsigned v = *dev_count + 1u;
  *dev_count = v;
  __threadfence_system();
  *host_seq = v;
}
int publish_red(const double* rrpart, int nrr, int nbatch, double* rr, const double* src, int n, double* host_dst,
                unsigned* dev_count, unsigned* host_seq, hipStream_t s) {
  hipLaunchKernelGGL(publish_red_kernel, dim3(1), dim3(VT), 0, s, rrpart, nrr, nbatch, rr, src, n, host_dst,
                     dev_count, host_seq);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

}  // namespace sdg
