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
// equal up to the factor eta_K).  Elements are grouped by id_e, so the apply
// is a small dense product Binv * [r_e1 ... r_eG] per group.  FP64: one
// wavefront per group of 16 on the matrix cores (FP64 MFMA), fragments read
// straight from L1/L2 and HBM.  Factored FP32/BF16: one workgroup stages the
// factor and the residual columns in LDS, 4 x 4 register tiles per thread.
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


// ---------------------------------------------------------------------------
// grouped apply
//
// Work item w = (uid, start, count): elements perm[start .. start+count) all
// use block uid.  The kernel is specialised on K1 = k + 1, so the block size
// NB = 2 K1^2, the padded row length NBP (NB rounded up to 4) and the
// largest group GMAX are compile-time constants and every staging loop
// unrolls into independent loads.  LDS holds the matrix as [b][a] rows
// (FP64 inverse: Binv, symmetric; factored: X^T and X, zero outside the
// triangle) and the residual columns as R[b][e].  Thread t owns rows
// a0 .. a0+3 (a0 = 4 (t mod NAG)) of elements e0 .. e0+3 (e0 = 4 (t div NAG)).
// The operands of the Chebyshev update are fetched before the product, so
// their latency hides behind it.
//
// Update (z = s_e Binv r_e, per-problem coefficients ab[pb] = (a, b)):
// d' = b z + a d_old, x' = x + d', where d_old is d (BJ_READ_D) or x itself
// (BJ_FOLD: the step after a start from zero, whose direction equals x);
// without BJ_READ_X the old x is zero; d' is stored only with BJ_WRITE_D;
// BJ_APPLY stores z in x instead.
// ---------------------------------------------------------------------------
template <typename TM, typename TV>
struct BjArgs {
  int G, nel;
  const int* perm;
  const int* work;
  const double* scale;
  const TM* mat;
  const TV* r;
  const double* ab;
  TV* d;
  TV* x;
  int flags;
};

template <typename TM>
__device__ __forceinline__ float ld_f32(const TM* p) {
  if constexpr (sizeof(TM) == 2) return __uint_as_float(((uint32_t)*p) << 16);
  else return float(*p);
}

template <int K1>
struct BjShape {
  static constexpr int NB = 2 * K1 * K1;
  static constexpr int NBP = (NB + 3) & ~3;
  static constexpr int NAG = NBP / 4;
  static constexpr int GMAX = 4 * (256 / NAG);
};

template <typename TC>
__device__ __forceinline__ void tile_fma(TC (&acc)[4][4], const TC* __restrict__ mrow,
                                         const TC* __restrict__ rrow) {
  TC m[4], v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    m[i] = mrow[i];
    v[i] = rrow[i];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = fma(m[i], v[j], acc[i][j]);
}

template <typename TV>
struct Pair {
  TV v[2];
};
template <typename TV>
__device__ __forceinline__ Pair<TV> ld2(const TV* p) {
  if constexpr (sizeof(TV) == 8) {
    const double2 q = *reinterpret_cast<const double2*>(p);
    return Pair<TV>{{q.x, q.y}};
  } else {
    const float2 q = *reinterpret_cast<const float2*>(p);
    return Pair<TV>{{q.x, q.y}};
  }
}
template <typename TV>
__device__ __forceinline__ void st2(TV* p, TV a, TV b) {
  if constexpr (sizeof(TV) == 8) *reinterpret_cast<double2*>(p) = make_double2(a, b);
  else *reinterpret_cast<float2*>(p) = make_float2(a, b);
}

template <int K1, typename TM, typename TV, bool TRI>
__global__ __launch_bounds__(256) void bj_group_kernel(BjArgs<TM, TV> A) {
  using TC = TV;  // FP64 vectors accumulate in FP64, FP32 vectors in FP32
  using S = BjShape<K1>;
  constexpr int NB = S::NB, NBP = S::NBP, NAG = S::NAG, GMAX = S::GMAX;
  __shared__ __align__(16) TC M0[NB * NBP];
  __shared__ __align__(16) TC M1[TRI ? NB * NBP : 4];
  __shared__ __align__(16) TC R[NB * GMAX];
  __shared__ __align__(16) TC Y[TRI ? NB * GMAX : 4];
  __shared__ int sperm[GMAX];
  const int G = A.G;
  const int t = threadIdx.x;
  const int uid = A.work[3 * blockIdx.x], start = A.work[3 * blockIdx.x + 1],
            cnt = A.work[3 * blockIdx.x + 2];
  for (int q = t; q < cnt; q += 256) sperm[q] = A.perm[start + q];

  if constexpr (!TRI) {
    const TM* B = A.mat + (int64_t)uid * NB * NB;
#pragma unroll
    for (int i0 = 0; i0 < NB * NBP; i0 += 256) {
      const int i = i0 + t;
      if (i < NB * NBP) {
        const int b = i / NBP, a = i - b * NBP;
        M0[i] = a < NB ? TC(B[b * NB + a]) : TC(0);
      }
    }
  } else {
    // packed lower triangle: X[a][b] (b <= a) at a(a+1)/2 + b
    const TM* X = A.mat + (int64_t)uid * NB * (NB + 1) / 2;
#pragma unroll
    for (int i0 = 0; i0 < NB * NBP; i0 += 256) {
      const int i = i0 + t;
      if (i < NB * NBP) {
        const int b = i / NBP, a = i - b * NBP;
        M0[i] = (a < NB && b <= a) ? TC(ld_f32(X + a * (a + 1) / 2 + b)) : TC(0);  // X^T[b][a]
        M1[i] = (a <= b) ? TC(ld_f32(X + b * (b + 1) / 2 + a)) : TC(0);            // X[b][a]
      }
    }
  }
  __syncthreads();  // sperm
  {
    constexpr int NLD = (NB * GMAX + 255) / 256;
    TV v[NLD];
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int i = q * 256 + t;
      const int e = i / NB, b = i - e * NB;
      v[q] = e < cnt ? A.r[(int64_t)sperm[e] * NB + b] : TV(0);
    }
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int i = q * 256 + t;
      const int e = i / NB, b = i - e * NB;
      if (e < G) R[b * G + e] = TC(v[q]);
    }
  }

  const int ag = t % NAG, eg = t / NAG;
  const int a0 = 4 * ag, e0 = 4 * eg;
  const bool act = e0 < cnt;  // e0 < cnt <= G
  const bool hi = a0 + 2 < NB;  // rows a0+2, a0+3 exist (NB is even)
  const int flags = A.flags;
  // operands of the update, fetched ahead of the product
  int64_t ge[4];
  TV xo[4][4], dold[4][4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ge[j] = -1;
#pragma unroll
    for (int i = 0; i < 4; ++i) xo[j][i] = dold[j][i] = TV(0);
  }
  if (act) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (e0 + j >= cnt) break;
      ge[j] = sperm[e0 + j];
      const TV* xx = A.x + ge[j] * NB + a0;
      const TV* dd = A.d + ge[j] * NB + a0;
      if (flags & BJ_READ_X) {
        Pair<TV> p = ld2(xx);
        xo[j][0] = p.v[0];
        xo[j][1] = p.v[1];
        if (hi) {
          p = ld2(xx + 2);
          xo[j][2] = p.v[0];
          xo[j][3] = p.v[1];
        }
      }
      if (flags & BJ_READ_D) {
        Pair<TV> p = ld2(dd);
        dold[j][0] = p.v[0];
        dold[j][1] = p.v[1];
        if (hi) {
          p = ld2(dd + 2);
          dold[j][2] = p.v[0];
          dold[j][3] = p.v[1];
        }
      }
    }
  }
  __syncthreads();  // R, M0, M1

  TC acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = TC(0);
  if constexpr (!TRI) {
    if (act)
#pragma unroll 2
      for (int b = 0; b < NB; ++b) tile_fma(acc, M0 + b * NBP + a0, R + b * G + e0);
  } else {
    // y = X r (rows a0..a0+3 need b <= a0+3), then z = X^T y (c >= a0)
    if (act) {
      const int bend = min(a0 + 4, NB);
      for (int b = 0; b < bend; ++b) tile_fma(acc, M0 + b * NBP + a0, R + b * G + e0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (a0 + i < NB)
#pragma unroll
          for (int j = 0; j < 4; ++j) Y[(a0 + i) * G + e0 + j] = acc[i][j];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = TC(0);
    if (act)
      for (int c = a0; c < NB; ++c) tile_fma(acc, M1 + c * NBP + a0, Y + c * G + e0);
  }
  if (!act) return;

#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (ge[j] < 0) break;
    const double sc = A.scale[ge[j]];
    TV* xx = A.x + ge[j] * NB + a0;
    TV* dd = A.d + ge[j] * NB + a0;
    TV xn[4], dn[4];
    if (flags & BJ_APPLY) {
#pragma unroll
      for (int i = 0; i < 4; ++i) xn[i] = TV(double(acc[i][j]) * sc);
    } else {
      const int64_t pb = ge[j] / A.nel;
      const double ca = A.ab[2 * pb], cb = A.ab[2 * pb + 1];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double z = double(acc[i][j]) * sc;
        double dv = cb * z;
        if (flags & BJ_READ_D) dv += ca * double(dold[j][i]);
        if (flags & BJ_FOLD) dv += ca * double(xo[j][i]);
        dn[i] = TV(dv);
        xn[i] = TV((flags & BJ_READ_X) ? double(xo[j][i]) + dv : dv);
      }
      if (flags & BJ_WRITE_D) {
        st2(dd, dn[0], dn[1]);
        if (hi) st2(dd + 2, dn[2], dn[3]);
      }
    }
    st2(xx, xn[0], xn[1]);
    if (hi) st2(xx + 2, xn[2], xn[3]);
  }
}

int bj_group_size(int nb, bool full_f64) {
  if (full_f64) return 16;  // one wavefront's matrix-core columns
  const int nag = ((nb + 3) & ~3) / 4;
  return 4 * (256 / nag);
}

typedef double v4d __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// FP64 full inverse, one wavefront per work item of up to 16 NG elements, no
// LDS and no barriers.  Lane (c, kq) = (lane % 16, lane / 16) gathers the
// residual fragments of elements c + 16 g (rows 4s + kq: 32 contiguous bytes
// per element across the four lane groups); each block fragment, read from
// L1/L2 (a block is shared by many work items), feeds NG products; the update
// reads and writes the rows of the accumulator fragments
// (D[16t + 4r + kq][c]).  Waves are independent, so the latency of one hides
// behind the others.
// ---------------------------------------------------------------------------
template <int K1, int NG>
__global__ __launch_bounds__(256) void bj_wave_kernel(BjArgs<double, double> A, int nwork) {
  constexpr int NB = 2 * K1 * K1, KP = (NB + 3) & ~3, NT = (NB + 15) / 16;
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= nwork) return;
  const int uid = A.work[3 * w], start = A.work[3 * w + 1], cnt = A.work[3 * w + 2];
  const int c = lane & 15, kq = lane >> 4;
  int64_t ge[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) ge[g] = (c + 16 * g < cnt) ? A.perm[start + c + 16 * g] : -1;
  const double* B = A.mat + (int64_t)uid * NB * NB;
  const int flags = A.flags;
  // operands of the update, fetched ahead of the product
  double xo[NG][NT][4], dold[NG][NT][4];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * tt + 4 * r + kq;
        const bool ok = ge[g] >= 0 && i < NB;
        xo[g][tt][r] = (ok && (flags & (BJ_READ_X | BJ_FOLD))) ? A.x[ge[g] * NB + i] : 0.0;
        dold[g][tt][r] = (ok && (flags & BJ_READ_D)) ? A.d[ge[g] * NB + i] : 0.0;
      }
  v4d acc[NG][NT];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) acc[g][tt] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
  for (int s4 = 0; s4 < KP; s4 += 4) {
    const int k = s4 + kq;
    double bv[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) bv[g] = (ge[g] >= 0 && k < NB) ? A.r[ge[g] * NB + k] : 0.0;
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      const int i = 16 * tt + c;
      // A[i][k] = B[k][i] (the block is symmetric)
      const double a = (k < NB && i < NB) ? B[k * NB + i] : 0.0;
#pragma unroll
      for (int g = 0; g < NG; ++g) acc[g][tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[g], acc[g][tt], 0, 0, 0);
    }
  }
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    if (ge[g] < 0) continue;
    const double sc = A.scale[ge[g]];
    double* xx = A.x + ge[g] * NB;
    double* dd = A.d + ge[g] * NB;
    double ca = 0.0, cb = 1.0;
    if (!(flags & BJ_APPLY)) {
      const int64_t pb = ge[g] / A.nel;
      ca = A.ab[2 * pb];
      cb = A.ab[2 * pb + 1];
    }
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * tt + 4 * r + kq;
        if (i >= NB) continue;
        const double z = acc[g][tt][r] * sc;
        if (flags & BJ_APPLY) {
          xx[i] = z;
          continue;
        }
        double dv = cb * z;
        if (flags & BJ_READ_D) dv += ca * dold[g][tt][r];
        if (flags & BJ_FOLD) dv += ca * xo[g][tt][r];
        if (flags & BJ_WRITE_D) dd[i] = dv;
        xx[i] = (flags & BJ_READ_X) ? xo[g][tt][r] + dv : dv;
      }
  }
}

template <int K1, typename TM, typename TV, bool TRI>
static void launch_k(const BjPlan& P, const TM* mat, const TV* r, const double* ab, TV* d, TV* x, int flags,
                     hipStream_t s) {
  BjArgs<TM, TV> A{P.G, P.nel, P.perm, P.work, P.scale, mat, r, ab, d, x, flags};
  if constexpr (!TRI && sizeof(TM) == 8 && sizeof(TV) == 8)
    hipLaunchKernelGGL((bj_wave_kernel<K1, 1>), dim3((P.nwork + 3) / 4), dim3(256), 0, s, A, P.nwork);
  else
    hipLaunchKernelGGL((bj_group_kernel<K1, TM, TV, TRI>), dim3(P.nwork), dim3(256), 0, s, A);
}

template <typename TM, typename TV, bool TRI>
static int launch_group(const BjPlan& P, const TM* mat, const TV* r, const double* ab, TV* d, TV* x, int flags,
                        hipStream_t s) {
  if (P.nwork <= 0) return SDG_OK;
  if (P.G < 4 || P.G % 4 || P.G > bj_group_size(P.nb, !TRI && sizeof(TM) == 8 && sizeof(TV) == 8)) {
    set_error("block smoother: group size does not fit one workgroup");
    return SDG_ERR_INVALID;
  }
  // the update moves pairs of values: x and d must be aligned to two values
  const uintptr_t al = 2 * sizeof(TV);
  if (reinterpret_cast<uintptr_t>(x) % al || reinterpret_cast<uintptr_t>(d) % al) {
    set_error("block smoother: vectors must be aligned to two values");
    return SDG_ERR_INVALID;
  }
  switch (P.nb) {
    case 8: launch_k<2, TM, TV, TRI>(P, mat, r, ab, d, x, flags, s); break;
    case 18: launch_k<3, TM, TV, TRI>(P, mat, r, ab, d, x, flags, s); break;
    case 32: launch_k<4, TM, TV, TRI>(P, mat, r, ab, d, x, flags, s); break;
    case 50: launch_k<5, TM, TV, TRI>(P, mat, r, ab, d, x, flags, s); break;
    case 72: launch_k<6, TM, TV, TRI>(P, mat, r, ab, d, x, flags, s); break;
    case 98: launch_k<7, TM, TV, TRI>(P, mat, r, ab, d, x, flags, s); break;
    default:
      set_error("block smoother: unsupported element block size");
      return SDG_ERR_UNSUPPORTED;
  }
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

int bj_cheb_f64(const BjPlan& P, const double* binv, const double* r, const double* ab, double* d, double* x,
                int flags, hipStream_t s) {
  return launch_group<double, double, false>(P, binv, r, ab, d, x, flags, s);
}
int bj_apply_f64(const BjPlan& P, const double* binv, const double* r, double* z, hipStream_t s) {
  return launch_group<double, double, false>(P, binv, r, nullptr, nullptr, z, BJ_APPLY, s);
}
int bj_tri_cheb_f32(const BjPlan& P, const float* X, const float* r, const double* ab, float* d, float* x,
                    int flags, hipStream_t s) {
  return launch_group<float, float, true>(P, X, r, ab, d, x, flags, s);
}
int bj_tri_cheb_bf16(const BjPlan& P, const uint16_t* X, const float* r, const double* ab, float* d, float* x,
                     int flags, hipStream_t s) {
  return launch_group<uint16_t, float, true>(P, X, r, ab, d, x, flags, s);
}
int bj_tri_apply_f32(const BjPlan& P, const float* X, const float* r, float* z, hipStream_t s) {
  return launch_group<float, float, true>(P, X, r, nullptr, nullptr, z, BJ_APPLY, s);
}
int bj_tri_apply_bf16(const BjPlan& P, const uint16_t* X, const float* r, float* z, hipStream_t s) {
  return launch_group<uint16_t, float, true>(P, X, r, nullptr, nullptr, z, BJ_APPLY, s);
}

}  // namespace sdg
