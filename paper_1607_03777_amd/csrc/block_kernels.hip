// Element-block Jacobi smoother (eq. smoother: the diagonal blocks of A).
//
// Setup inverts each (deduplicated) diagonal block in place: Cholesky
// factor L (right-looking), in-place triangular inverse X = L^{-1}, then
// B^{-1} = X^T X.  One workgroup per matrix; the matrices stay in global
// memory (L2-resident during the factorisation), so the same kernel serves
// element blocks (n <= 98) and the dense coarsest-level operator.
//
// The apply is z_e = s_e * Binv[id_e] r_e, where id_e is the element's
// unique block and s_e = eta_rep / eta_e rescales a shared block to the
// element (blocks with equal face kinds and neighbour viscosity ratios are
// equal up to the factor eta_K).
#include "sdg_common.h"
#include "sdg_kernels.h"

namespace sdg {

constexpr int INV_NT = 256;

// packed (optional): receives X = L^{-1} as a packed lower triangle
// (row a holds X[a][0..a] at offset a(a+1)/2), n(n+1)/2 entries per matrix.
__global__ __launch_bounds__(INV_NT) void spd_inverse_kernel(double* __restrict__ mats, int n,
                                                             int* __restrict__ status,
                                                             double* __restrict__ packed) {
  double* A = mats + (int64_t)blockIdx.x * n * n;
  extern __shared__ double tmp[];  // n doubles
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  // Cholesky, lower triangle, in place
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      const double d = A[(int64_t)k * n + k];
      if (!(d > 0.0) || !isfinite(d)) bad = 1;
      A[(int64_t)k * n + k] = sqrt(d > 0.0 ? d : 1e-300);
    }
    __syncthreads();
    const double lkk = A[(int64_t)k * n + k];
    for (int i = k + 1 + tid; i < n; i += INV_NT) A[(int64_t)i * n + k] /= lkk;
    __syncthreads();
    const int m = n - k - 1;
    for (int idx = tid; idx < m * m; idx += INV_NT) {
      const int i = k + 1 + idx / m, j = k + 1 + idx % m;
      if (j <= i) A[(int64_t)i * n + j] -= A[(int64_t)i * n + k] * A[(int64_t)j * n + k];
    }
    __syncthreads();
  }
  // X = L^{-1} in place, columns from the last to the first
  for (int j = n - 1; j >= 0; --j) {
    if (tid == 0) A[(int64_t)j * n + j] = 1.0 / A[(int64_t)j * n + j];
    __syncthreads();
    for (int i = j + 1 + tid; i < n; i += INV_NT) {
      double s = 0.0;
      for (int m = j + 1; m <= i; ++m) s += A[(int64_t)i * n + m] * A[(int64_t)m * n + j];
      tmp[i] = s;
    }
    __syncthreads();
    const double xjj = A[(int64_t)j * n + j];
    for (int i = j + 1 + tid; i < n; i += INV_NT) A[(int64_t)i * n + j] = -tmp[i] * xjj;
    __syncthreads();
  }
  if (packed) {
    double* pk = packed + (int64_t)blockIdx.x * n * (n + 1) / 2;
    for (int idx = tid; idx < n * n; idx += INV_NT) {
      const int a = idx / n, b = idx % n;
      if (b <= a) pk[a * (a + 1) / 2 + b] = A[(int64_t)a * n + b];
    }
    __syncthreads();
  }
  // B^{-1} = X^T X: upper triangle written directly, diagonal staged
  for (int idx = tid; idx < n * n; idx += INV_NT) {
    const int a = idx / n, b = idx % n;
    if (b < a) continue;
    double s = 0.0;
    for (int m = b; m < n; ++m) s += A[(int64_t)m * n + a] * A[(int64_t)m * n + b];
    if (a == b) tmp[a] = s;
    else A[(int64_t)a * n + b] = s;
  }
  __syncthreads();
  for (int a = tid; a < n; a += INV_NT) A[(int64_t)a * n + a] = tmp[a];
  __syncthreads();
  for (int idx = tid; idx < n * n; idx += INV_NT) {
    const int a = idx / n, b = idx % n;
    if (b < a) A[(int64_t)a * n + b] = A[(int64_t)b * n + a];
  }
  if (tid == 0 && status) status[blockIdx.x] = bad;
}

int spd_inverse(double* mats, int n, int nmat, int* status, hipStream_t s, double* packed) {
  if (nmat <= 0) return SDG_OK;
  hipLaunchKernelGGL(spd_inverse_kernel, dim3(nmat), dim3(INV_NT), n * sizeof(double), s, mats, n,
                     status, packed);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

// ---------------------------------------------------------------------------
// apply
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_to_f32(uint16_t v) {
  return __uint_as_float(((uint32_t)v) << 16);
}

template <typename TM, typename TV>
__global__ __launch_bounds__(256) void bj_apply_kernel(int nb, int64_t nel_total,
                                                       const int* __restrict__ ids,
                                                       const double* __restrict__ scale,
                                                       const TM* __restrict__ binv,
                                                       const TV* __restrict__ r, TV* __restrict__ z) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nel_total * nb) return;
  const int64_t e = g / nb;
  const int a = (int)(g - e * nb);
  const TM* row = binv + ((int64_t)ids[e] * nb + a) * nb;
  const TV* re = r + e * nb;
  if constexpr (sizeof(TM) == 8) {
    double acc = 0.0;
#pragma unroll 4
    for (int b = 0; b < nb; ++b) acc += row[b] * double(re[b]);
    z[g] = TV(acc * scale[e]);
  } else if constexpr (sizeof(TM) == 4) {
    float acc = 0.f;
#pragma unroll 4
    for (int b = 0; b < nb; ++b) acc += row[b] * float(re[b]);
    z[g] = TV(acc * float(scale[e]));
  } else {
    float acc = 0.f;
#pragma unroll 4
    for (int b = 0; b < nb; ++b) acc += bf16_to_f32(row[b]) * float(re[b]);
    z[g] = TV(acc * float(scale[e]));
  }
}

int blockjacobi_apply_f64(int nb, int64_t nel_total, const int* ids, const double* scale,
                          const double* binv, const double* r, double* z, hipStream_t s) {
  const int64_t n = nel_total * nb;
  hipLaunchKernelGGL((bj_apply_kernel<double, double>), dim3(ceil_div(n, 256)), dim3(256), 0, s,
                     nb, nel_total, ids, scale, binv, r, z);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int blockjacobi_apply_f32(int nb, int64_t nel_total, const int* ids, const double* scale,
                          const float* binv, const float* r, float* z, hipStream_t s) {
  const int64_t n = nel_total * nb;
  hipLaunchKernelGGL((bj_apply_kernel<float, float>), dim3(ceil_div(n, 256)), dim3(256), 0, s, nb,
                     nel_total, ids, scale, binv, r, z);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int blockjacobi_apply_bf16(int nb, int64_t nel_total, const int* ids, const double* scale,
                           const uint16_t* binv, const float* r, float* z, hipStream_t s) {
  const int64_t n = nel_total * nb;
  hipLaunchKernelGGL((bj_apply_kernel<uint16_t, float>), dim3(ceil_div(n, 256)), dim3(256), 0, s,
                     nb, nel_total, ids, scale, binv, r, z);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

__global__ void f64_to_f32_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) out[g] = (float)in[g];
}
__global__ void f64_to_bf16_kernel(const double* __restrict__ in, uint16_t* __restrict__ out,
                                   int64_t n) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  // round to nearest even from the FP32 value
  const uint32_t u = __float_as_uint((float)in[g]);
  const uint32_t lsb = (u >> 16) & 1u;
  out[g] = (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}
int convert_f64_f32(const double* in, float* out, int64_t n, hipStream_t s) {
  if (n <= 0) return SDG_OK;
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, in, out, n);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int convert_f64_bf16(const double* in, uint16_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return SDG_OK;
  hipLaunchKernelGGL(f64_to_bf16_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, s, in, out, n);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

}  // namespace sdg

namespace sdg {

// Fused smoother step on the DG level: z_e = s_e Binv[id_e] r_e, then the
// Chebyshev recurrence with per-problem coefficients ab[pb] = (a, b):
// mode 0: d = a d + b z, x += d;  1: d = b z, x = d;  2: d = b z, x += d.
template <typename TM, typename TV>
__global__ __launch_bounds__(256) void bj_cheb_kernel(int nb, int64_t nel_total, int nel,
                                                      const int* __restrict__ ids,
                                                      const double* __restrict__ scale,
                                                      const TM* __restrict__ binv,
                                                      const TV* __restrict__ r,
                                                      const double* __restrict__ ab,
                                                      TV* __restrict__ d, TV* __restrict__ x, int mode) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nel_total * nb) return;
  const int64_t e = g / nb;
  const int a = (int)(g - e * nb);
  const int64_t pb = e / nel;
  const TM* row = binv + ((int64_t)ids[e] * nb + a) * nb;
  const TV* re = r + e * nb;
  double z;
  if constexpr (sizeof(TM) == 8) {
    double acc = 0.0;
#pragma unroll 4
    for (int b = 0; b < nb; ++b) acc += row[b] * double(re[b]);
    z = acc * scale[e];
  } else if constexpr (sizeof(TM) == 4) {
    float acc = 0.f;
#pragma unroll 4
    for (int b = 0; b < nb; ++b) acc += row[b] * float(re[b]);
    z = double(acc * float(scale[e]));
  } else {
    float acc = 0.f;
#pragma unroll 4
    for (int b = 0; b < nb; ++b) acc += bf16_to_f32(row[b]) * float(re[b]);
    z = double(acc * float(scale[e]));
  }
  const double ca = ab[2 * pb], cb = ab[2 * pb + 1];
  const double dv = mode == 0 ? ca * double(d[g]) + cb * z : cb * z;
  d[g] = TV(dv);
  x[g] = mode == 1 ? TV(dv) : TV(double(x[g]) + dv);
}

int bj_cheb_f64(int nb, int64_t nel_total, int nel, const int* ids, const double* scale, const double* binv,
                const double* r, const double* ab, double* d, double* x, int mode, hipStream_t s) {
  const int64_t n = nel_total * nb;
  hipLaunchKernelGGL((bj_cheb_kernel<double, double>), dim3(ceil_div(n, 256)), dim3(256), 0, s, nb,
                     nel_total, nel, ids, scale, binv, r, ab, d, x, mode);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int bj_cheb_f32(int nb, int64_t nel_total, int nel, const int* ids, const double* scale, const float* binv,
                const float* r, const double* ab, float* d, float* x, int mode, hipStream_t s) {
  const int64_t n = nel_total * nb;
  hipLaunchKernelGGL((bj_cheb_kernel<float, float>), dim3(ceil_div(n, 256)), dim3(256), 0, s, nb,
                     nel_total, nel, ids, scale, binv, r, ab, d, x, mode);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int bj_cheb_bf16(int nb, int64_t nel_total, int nel, const int* ids, const double* scale, const uint16_t* binv,
                 const float* r, const double* ab, float* d, float* x, int mode, hipStream_t s) {
  const int64_t n = nel_total * nb;
  hipLaunchKernelGGL((bj_cheb_kernel<uint16_t, float>), dim3(ceil_div(n, 256)), dim3(256), 0, s, nb,
                     nel_total, nel, ids, scale, binv, r, ab, d, x, mode);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

}  // namespace sdg

namespace sdg {

// ---------------------------------------------------------------------------
// Low-precision smoother through the inverse Cholesky factor: with
// A_KK = L L^T and X = L^{-1} stored as a packed lower triangle in FP32 or
// BF16, z_e = s_e X^T (X r_e).  Rounding X keeps the smoother symmetric
// positive definite (X^T X with X nonsingular), which rounding the entries of
// the full inverse does not when the block is ill conditioned, and the
// triangle is half the bytes.  One workgroup handles EPB = 256 / nb elements.
// ---------------------------------------------------------------------------
template <typename TM>
__device__ __forceinline__ float ldx(const TM* p) {
  if constexpr (sizeof(TM) == 2) return bf16_to_f32(*p);
  else return float(*p);
}

template <typename TM, typename TV>
__global__ __launch_bounds__(256) void bj_tri_kernel(int nb, int64_t nel_total, int nel,
                                                     const int* __restrict__ ids,
                                                     const double* __restrict__ scale,
                                                     const TM* __restrict__ X, const TV* __restrict__ r,
                                                     const double* __restrict__ ab, TV* __restrict__ d,
                                                     TV* __restrict__ x, TV* __restrict__ z_out, int mode) {
  __shared__ float sr[256];
  __shared__ float sy[256];
  const int epb = 256 / nb;
  const int t = threadIdx.x;
  const int le = t / nb, a = t - le * nb;
  const int64_t e = (int64_t)blockIdx.x * epb + le;
  const bool live = le < epb && e < nel_total;
  const int64_t npk = (int64_t)nb * (nb + 1) / 2;
  const TM* Xe = live ? X + (int64_t)ids[e] * npk : X;
  if (live) sr[t] = float(r[e * nb + a]);
  __syncthreads();
  if (live) {
    const TM* row = Xe + (int64_t)a * (a + 1) / 2;
    const float* re = sr + le * nb;
    float acc = 0.f;
    for (int b = 0; b <= a; ++b) acc += ldx(row + b) * re[b];
    sy[t] = acc;
  }
  __syncthreads();
  if (!live) return;
  const float* ye = sy + le * nb;
  float acc = 0.f;
  for (int c = a; c < nb; ++c) acc += ldx(Xe + (int64_t)c * (c + 1) / 2 + a) * ye[c];
  const double zv = double(acc) * scale[e];
  const int64_t g = e * nb + a;
  if (z_out) {
    z_out[g] = TV(zv);
    return;
  }
  const int64_t pb = e / nel;
  const double ca = ab[2 * pb], cb = ab[2 * pb + 1];
  const double dv = mode == 0 ? ca * double(d[g]) + cb * zv : cb * zv;
  d[g] = TV(dv);
  x[g] = mode == 1 ? TV(dv) : TV(double(x[g]) + dv);
}

template <typename TM>
static int launch_tri(int nb, int64_t nel_total, int nel, const int* ids, const double* scale, const TM* X,
                      const float* r, const double* ab, float* d, float* x, float* z, int mode, hipStream_t s) {
  if (nb > 256) {
    set_error("element block larger than 256 for the factored smoother");
    return SDG_ERR_UNSUPPORTED;
  }
  const int epb = 256 / nb;
  hipLaunchKernelGGL((bj_tri_kernel<TM, float>), dim3(ceil_div(nel_total, epb)), dim3(256), 0, s, nb, nel_total,
                     nel, ids, scale, X, r, ab, d, x, z, mode);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

int bj_tri_cheb_f32(int nb, int64_t nel_total, int nel, const int* ids, const double* scale, const float* X,
                    const float* r, const double* ab, float* d, float* x, int mode, hipStream_t s) {
  return launch_tri<float>(nb, nel_total, nel, ids, scale, X, r, ab, d, x, nullptr, mode, s);
}
int bj_tri_cheb_bf16(int nb, int64_t nel_total, int nel, const int* ids, const double* scale, const uint16_t* X,
                     const float* r, const double* ab, float* d, float* x, int mode, hipStream_t s) {
  return launch_tri<uint16_t>(nb, nel_total, nel, ids, scale, X, r, ab, d, x, nullptr, mode, s);
}
int bj_tri_apply_f32(int nb, int64_t nel_total, const int* ids, const double* scale, const float* X,
                     const float* r, float* z, hipStream_t s) {
  return launch_tri<float>(nb, nel_total, 1, ids, scale, X, r, nullptr, nullptr, nullptr, z, 0, s);
}
int bj_tri_apply_bf16(int nb, int64_t nel_total, const int* ids, const double* scale, const uint16_t* X,
                      const float* r, float* z, hipStream_t s) {
  return launch_tri<uint16_t>(nb, nel_total, 1, ids, scale, X, r, nullptr, nullptr, nullptr, z, 0, s);
}

}  // namespace sdg
