// Element-block Jacobi smoother (eq. smoother: the diagonal blocks of A).
//
// Setup inverts each (deduplicated) diagonal block in place: Cholesky
// factor L (right-looking), in-place triangular inverse X = L^{-1}, then
// B^{-1} = X^T X.  One workgroup per matrix; element blocks (n <= 98) are
// factored in LDS, the larger dense coarsest-level operator in global
// memory (L2-resident during the factorisation), by the same kernel.
//
// The apply is z_e = s_e * Binv[id_e] r_e, where id_e is the element's
// unique block and s_e = eta_rep / eta_e rescales a shared block to the
// element (blocks with equal face kinds and neighbour viscosity ratios are
// equal up to the factor eta_K).  Elements are grouped by id_e, so the apply
// is a small dense product Binv * [r_e1 ... r_eG] per group: one wavefront
// per group of 16 on the matrix cores (FP64 MFMA), fragments read straight
// from L1/L2 and HBM, for the FP64 inverse and for the factored FP32/BF16
// form (FP64 and FP32 matrix cores respectively) alike.
#include "sdg_common.h"
#include "sdg_kernels.h"

namespace sdg {

constexpr int INV_NT = 256;

// packed (optional): receives X = L^{-1} as a packed lower triangle
// (row a holds X[a][0..a] at offset a(a+1)/2), n(n+1)/2 entries per matrix.
// in_lds: the matrix is staged in LDS for the factorisation (element blocks,
// n <= SPD_LDS_MAX); otherwise it is worked on in global memory.
__global__ __launch_bounds__(INV_NT) void spd_inverse_kernel(double* __restrict__ mats, int n,
                                                             int* __restrict__ status,
                                                             double* __restrict__ packed, int in_lds) {
  double* const G = mats + (int64_t)blockIdx.x * n * n;
  extern __shared__ double smem[];  // tmp[n], then the matrix [n][n] when in_lds
  double* const tmp = smem;
  double* const A = in_lds ? smem + n : G;
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  if (in_lds)
    for (int idx = tid; idx < n * n; idx += INV_NT) A[idx] = G[idx];
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
  if (in_lds) {
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += INV_NT) G[idx] = A[idx];
  }
  if (tid == 0 && status) status[blockIdx.x] = bad;
}

// element blocks up to k = 6 (98 x 98, 77 KB) are factored in LDS: every
// step of the factorisation then waits on LDS instead of L2 (many small
// matrices, as with a viscosity that varies per element)
constexpr int SPD_LDS_MAX = 98;
int spd_inverse(double* mats, int n, int nmat, int* status, hipStream_t s, double* packed) {
  if (nmat <= 0) return SDG_OK;
  // the LDS form above 64 KB needs the kernel's dynamic LDS limit raised
  static int lds_ok = -1;  // once per process: -1 unknown, 0 no, 1 yes
  if (lds_ok < 0) {
    lds_ok = hipFuncSetAttribute(reinterpret_cast<const void*>(&spd_inverse_kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) == hipSuccess;
    if (!lds_ok) (void)hipGetLastError();
  }
  const size_t lds_bytes = ((size_t)n * n + n) * sizeof(double);
  const int in_lds = n <= SPD_LDS_MAX && (lds_bytes <= 64 * 1024 || lds_ok == 1);
  hipLaunchKernelGGL(spd_inverse_kernel, dim3(nmat), dim3(INV_NT), in_lds ? lds_bytes : n * sizeof(double), s,
                     mats, n, status, packed, in_lds);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}


// Low-precision factors: from the packed FP64 X = L^{-1} (row a holds
// X[a][0..a] at offset a(a+1)/2) to the storage type, once, as the lower
// triangle of 2 x 2 quads: quad (m, p), p <= m < NB/2, holds
// X[2m][2p], X[2m][2p+1], X[2m+1][2p], X[2m+1][2p+1] at offset
// 4 (m(m+1)/2 + p), NB(NB+2)/2 values per block (X[2m][2m+1] is a stored
// zero).  The product y = X r reads a quad's row pair (contiguous), the
// product z = X^T y its column pair (the whole quad, then a select).
__device__ __forceinline__ uint16_t to_bf16(double v) {
  // round to nearest even from the FP32 value
  const uint32_t u = __float_as_uint((float)v);
  const uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}
int64_t tri_quad_size(int n) { return (int64_t)n * (n + 2) / 2; }
template <typename TM>
__global__ void tri_quad_kernel(const double* __restrict__ packed, int n, int64_t nmat, TM* __restrict__ out) {
  const int64_t per = (int64_t)n * (n + 2) / 2;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nmat * per) return;
  const int64_t u = g / per;
  const int e = (int)(g - u * per), qd = e >> 2, ab = e & 3;
  int m = 0;  // quad (m, p) with m(m+1)/2 <= qd < (m+1)(m+2)/2
  while ((m + 1) * (m + 2) / 2 <= qd) ++m;
  const int p = qd - m * (m + 1) / 2;
  const int a = 2 * m + (ab >> 1), b = 2 * p + (ab & 1);
  const double* pk = packed + u * ((int64_t)n * (n + 1) / 2);
  const double x = b <= a ? pk[(int64_t)a * (a + 1) / 2 + b] : 0.0;  // X[a][b]
  if constexpr (sizeof(TM) == 2)
    out[g] = to_bf16(x);
  else
    out[g] = TM(x);
}
int tri_quad_f32(const double* packed, int n, int nmat, float* out, hipStream_t s) {
  const int64_t tot = (int64_t)nmat * tri_quad_size(n);
  if (tot <= 0) return SDG_OK;
  if (n % 2) {
    set_error("low-precision factors: odd block size");
    return SDG_ERR_INVALID;
  }
  hipLaunchKernelGGL(tri_quad_kernel<float>, dim3(ceil_div(tot, 256)), dim3(256), 0, s, packed, n, (int64_t)nmat,
                     out);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int tri_quad_bf16(const double* packed, int n, int nmat, uint16_t* out, hipStream_t s) {
  const int64_t tot = (int64_t)nmat * tri_quad_size(n);
  if (tot <= 0) return SDG_OK;
  if (n % 2) {
    set_error("low-precision factors: odd block size");
    return SDG_ERR_INVALID;
  }
  hipLaunchKernelGGL(tri_quad_kernel<uint16_t>, dim3(ceil_div(tot, 256)), dim3(256), 0, s, packed, n,
                     (int64_t)nmat, out);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}


// FP64 block inverses for the streaming smoother: the symmetric B^{-1} once,
// as the lower triangle of 2 x 2 quads in the layout above (quad (m, p),
// p <= m, rows 2m, 2m+1 and columns 2p, 2p+1; the diagonal quads whole).
__global__ void sym_quad_kernel(const double* __restrict__ full, int n, int64_t nmat, double* __restrict__ out) {
  const int64_t per = (int64_t)n * (n + 2) / 2;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nmat * per) return;
  const int64_t u = g / per;
  const int e = (int)(g - u * per), qd = e >> 2, ab = e & 3;
  int m = 0;
  while ((m + 1) * (m + 2) / 2 <= qd) ++m;
  const int p = qd - m * (m + 1) / 2;
  out[g] = full[u * n * n + (int64_t)(2 * m + (ab >> 1)) * n + 2 * p + (ab & 1)];
}
int sym_quad_f64(const double* full, int n, int nmat, double* out, hipStream_t s) {
  const int64_t tot = (int64_t)nmat * tri_quad_size(n);
  if (tot <= 0) return SDG_OK;
  if (n % 2) {
    set_error("packed block inverses: odd block size");
    return SDG_ERR_INVALID;
  }
  hipLaunchKernelGGL(sym_quad_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, s, full, n, (int64_t)nmat, out);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}


// ---------------------------------------------------------------------------
// grouped apply
//
// Work item w = (uid, start, count): elements perm[start .. start+count) all
// use block uid.  Update (z = s_e Binv r_e, per-problem coefficients
// ab[pb] = (a, b)): d' = b z + a d_old, x' = x + d', where d_old is d
// (BJ_READ_D) or x itself (BJ_FOLD: the step after a start from zero, whose
// direction equals x); without BJ_READ_X the old x is zero; d' is stored
// only with BJ_WRITE_D; BJ_APPLY stores z in x instead.
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
  const int* active;  // null, or per problem: 0 = skip its elements
};
// element ge of the plan, or -1 for a converged problem of a batched CG
// iteration (active[pb] == 0)
__device__ __forceinline__ int64_t bj_elem(const int* active, int nel, int64_t ge) {
  return ge >= 0 && active && !active[ge / nel] ? -1 : ge;
}

int bj_group_size(int nb) {
  (void)nb;
  return 16;  // one wavefront's matrix-core columns
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

// Row order of the FP64 kernel.  Within every 16-row group the lane group q
// (= lane / 16) holds rows 8h + 2q + s, h, s in {0, 1}: two adjacent pairs,
// so vectors move as 16-byte pairs and each element's 128-byte stretch of a
// group is read by one instruction pair.  The matrix-core products follow
// that order: k-step (g, h, s) contracts rows 16g + 8h + 2q + s, and block
// row 16t + perm16(i) feeds accumulator row i, where
// perm16(4r + q) = 8(r >> 1) + 2q + (r & 1); accumulator component r of
// lane group q then holds output row 16t + 8(r >> 1) + 2q + (r & 1), the
// same pair layout as the inputs.
__device__ __forceinline__ int perm16(int i) { return 8 * (i >> 3) + 2 * (i & 3) + ((i >> 2) & 1); }

// ---------------------------------------------------------------------------
// FP64 full inverse, one wavefront per work item of up to 16 elements.  Lane
// (c, q) = (lane % 16, lane / 16) works on element c; its residual, x and d
// rows come in 16-byte pairs (row order above), and each block fragment pair
// feeds two products.  Work items are sorted by block, so the four
// wavefronts of a workgroup nearly always share one: the workgroup stages
// the block of its first work item in LDS once (rows padded to NB + 2
// values) and a wavefront with that block reads its fragments from there;
// any other wavefront reads them from L1/L2.  Blocks above 72 x 72 (k = 6)
// stay in L1/L2, and so do the 50 x 50 blocks of k = 4, where the staging
// barrier measured slower than the fragment loads it saves (k = 2, 3, 5 run
// 4-14% faster staged).  The update operands are fetched first.  For k >= 4
// the product is software-pipelined: the fragments of the next k-step are
// requested before the products of the current one.
// ---------------------------------------------------------------------------
template <int K1>
__global__ __launch_bounds__(256, (K1 == 5 ? 4 : K1 == 6 ? 3 : K1 == 7 ? 2 : 1)) void bj_wave_kernel(BjArgs<double, double> A, int nwork) {
  constexpr int NB = 2 * K1 * K1, NT = (NB + 15) / 16;
  constexpr bool STAGE = NB <= 72 && K1 != 5;
  // software-pipelined product from k = 4 on (plain apply at 64 x 64 x 16:
  // k = 4 19.3 -> 17.5 us, k = 5 39.7 -> 30.8 us, k = 6 55.3 -> 44.6 us);
  // below, the plain loop is as fast.  The update operands are requested
  // after the product and the launch bounds ask for one wavefront per SIMD
  // more than the product would leave: held through it, the operands and
  // the double buffers cost one (k = 4: 21.7 us)
  constexpr bool PIPE = K1 >= 5;
  constexpr bool LATE_OPS = K1 >= 5;
  constexpr int LDB = NB + 2;
  __shared__ double sB[STAGE ? NB * LDB : 2];
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  const bool wvalid = w < nwork;
  const int uid = wvalid ? A.work[3 * w] : -1;
  const int start = wvalid ? A.work[3 * w + 1] : 0, cnt = wvalid ? A.work[3 * w + 2] : 0;
  const int c = lane & 15, q = lane >> 4;
  const int64_t ge = bj_elem(A.active, A.nel, (c < cnt) ? A.perm[start + c] : -1);
  const int flags = A.flags;
  // operands of the update (rows 16t + 8h + 2q, +1): requested first, or,
  // with the pipelined product, right after its first k-step's loads
  v2d xo[NT][2], dold[NT][2];
  auto load_ops = [&]() {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = 16 * t + 8 * h + 2 * q;
        const bool ok = ge >= 0 && i < NB;
        xo[t][h] = (ok && (flags & (BJ_READ_X | BJ_FOLD))) ? *reinterpret_cast<const v2d*>(A.x + ge * NB + i)
                                                            : v2d{0.0, 0.0};
        dold[t][h] = (ok && (flags & BJ_READ_D)) ? *reinterpret_cast<const v2d*>(A.d + ge * NB + i) : v2d{0.0, 0.0};
      }
  };
  if constexpr (!PIPE) load_ops();
  // blockIdx.x * 4 < nwork: the grid has ceil(nwork / 4) workgroups
  const int uid0 = A.work[3 * (blockIdx.x * 4)];
  if constexpr (STAGE) {
    const double* B0 = A.mat + (int64_t)uid0 * NB * NB;
    for (int e2 = threadIdx.x; e2 < NB * NB / 2; e2 += 256) {
      const int row = (2 * e2) / NB, col = 2 * e2 - row * NB;  // NB is even: pairs stay in a row
      *reinterpret_cast<v2d*>(sB + row * LDB + col) = *reinterpret_cast<const v2d*>(B0 + 2 * e2);
    }
    __syncthreads();
  }
  if (!wvalid) return;
  if (__ballot(ge >= 0) == 0) return;  // every element skipped (after the barrier)
  const double* B = A.mat + (int64_t)uid * NB * NB;
  const bool from_lds = STAGE && uid == uid0;
  const int prow = perm16(c);
  v4d acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
  if constexpr (!PIPE) {
#pragma unroll
    for (int g = 0; g < NT; ++g)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (16 * g + 8 * h >= NB) continue;
        const int k0 = 16 * g + 8 * h + 2 * q;
        const v2d rb = (ge >= 0 && k0 < NB) ? *reinterpret_cast<const v2d*>(A.r + ge * NB + k0) : v2d{0.0, 0.0};
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int arow = 16 * t + prow;
          // A[i][k] = Binv[arow][k] (the block is symmetric either way)
          v2d a = v2d{0.0, 0.0};
          if (arow < NB && k0 < NB)
            a = from_lds ? *reinterpret_cast<const v2d*>(sB + arow * LDB + k0)
                         : *reinterpret_cast<const v2d*>(B + arow * NB + k0);
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, rb.x, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, rb.y, acc[t], 0, 0, 0);
        }
      }
  } else {
    // Every load of the product is unconditional (an address clamped into the
    // block or the vector, the value zeroed by a select where it lies outside),
    // and the loads of k-step s + 1 are issued before the products of k-step
    // s, so a wavefront waits for one L2 round trip at a time while the matrix
    // cores work, not for one per k-step after they finish.  Idle lanes read
    // element 0.  k-step s contracts rows 8 s + 2 q, + 1 (s = 2 g + h).
    const int64_t gsafe = ge >= 0 ? ge : 0;
    constexpr int NS = (NB + 7) / 8;
    auto load_step = [&](int st, v2d& rb, v2d (&a)[NT]) {
      const int k0 = 8 * st + 2 * q;
      const bool kin = k0 < NB;  // k0 is even and NB even: the pair is inside
      rb = *reinterpret_cast<const v2d*>(A.r + gsafe * NB + (kin ? k0 : 0));
      if (!(ge >= 0 && kin)) rb = v2d{0.0, 0.0};
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int arow = 16 * t + prow;
        const bool ok = arow < NB && kin;
        // A[i][k] = Binv[arow][k] (the block is symmetric either way)
        a[t] = from_lds ? *reinterpret_cast<const v2d*>(sB + (ok ? arow * LDB + k0 : 0))
                        : *reinterpret_cast<const v2d*>(B + (ok ? arow * NB + k0 : 0));
        if (!ok) a[t] = v2d{0.0, 0.0};
      }
    };
    v2d rbuf[2], abuf[2][NT];
    load_step(0, rbuf[0], abuf[0]);
    if constexpr (!LATE_OPS) load_ops();
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const int cu = st & 1;
      if (st + 1 < NS) load_step(st + 1, rbuf[cu ^ 1], abuf[cu ^ 1]);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(abuf[cu][t].x, rbuf[cu].x, acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(abuf[cu][t].y, rbuf[cu].y, acc[t], 0, 0, 0);
      }
    }
    if constexpr (LATE_OPS) load_ops();
  }
  if (ge < 0) return;
  const double sc = A.scale[ge];
  double* xx = A.x + ge * NB;
  double* dd = A.d + ge * NB;
  double ca = 0.0, cb = 1.0;
  if (!(flags & BJ_APPLY)) {
    const int64_t pb = ge / A.nel;
    ca = A.ab[2 * pb];
    cb = A.ab[2 * pb + 1];
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = 16 * t + 8 * h + 2 * q;
      if (i >= NB) continue;
      const v2d z = v2d{acc[t][2 * h], acc[t][2 * h + 1]} * sc;
      if (flags & BJ_APPLY) {
        *reinterpret_cast<v2d*>(xx + i) = z;
        continue;
      }
      v2d dv = cb * z;
      if (flags & BJ_READ_D) dv += ca * dold[t][h];
      if (flags & BJ_FOLD) dv += ca * xo[t][h];
      if (flags & BJ_WRITE_D) *reinterpret_cast<v2d*>(dd + i) = dv;
      *reinterpret_cast<v2d*>(xx + i) = (flags & BJ_READ_X) ? xo[t][h] + dv : dv;
    }
}

// ---------------------------------------------------------------------------
// Factored low-precision smoother, one wavefront per work item of up to 16
// elements: y = X r, then z = X^T y, on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32), X = L^{-1} stored once as the lower triangle of
// 2 x 2 quads in FP32 or BF16 (layout at tri_quad_kernel), vectors in FP32.  The rows follow the pair order of the
// FP64 kernel (lane group q holds rows 16g + 8h + 2q + s), so vectors and
// factor rows move as pairs.  The FP32 product puts D row 4q + r in
// component r of lane group q (checked on the GPU), so block row
// 16t + permf(i) feeds accumulator row i with
// permf(4q + r) = 8(r >> 1) + 2q + (r & 1): component r then holds output
// row 16t + 8(r >> 1) + 2q + (r & 1), and the accumulator of y is exactly
// the operand the second product needs for its k-steps.  Zero blocks of
// the triangles (row group below or above the column group) are skipped at
// compile time.
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int permf(int i) { return 8 * ((i & 3) >> 1) + 2 * (i >> 2) + (i & 1); }
// row pair (q[2s], q[2s + 1]) and column pair (q[s], q[2 + s]) of the quad q
template <typename TM>
__device__ __forceinline__ v2f ld_row_pair(const TM* q, int s) {
  if constexpr (sizeof(TM) == 2) {
    const uint32_t w = *reinterpret_cast<const uint32_t*>(q + 2 * s);
    return v2f{__uint_as_float(w << 16), __uint_as_float(w & 0xFFFF0000u)};
  } else {
    return *reinterpret_cast<const v2f*>(q + 2 * s);
  }
}
template <typename TM>
__device__ __forceinline__ v2f ld_col_pair(const TM* q, int s) {
  if constexpr (sizeof(TM) == 2) {
    const uint2 w = *reinterpret_cast<const uint2*>(q);
    return s ? v2f{__uint_as_float(w.x & 0xFFFF0000u), __uint_as_float(w.y & 0xFFFF0000u)}
             : v2f{__uint_as_float(w.x << 16), __uint_as_float(w.y << 16)};
  } else {
    const v4f v = *reinterpret_cast<const v4f*>(q);
    return s ? v2f{v.y, v.w} : v2f{v.x, v.z};
  }
}

template <int K1, typename TM>
__global__ __launch_bounds__(256) void bj_wave_lp_kernel(BjArgs<TM, float> A, int nwork) {
  constexpr int NB = 2 * K1 * K1, NT = (NB + 15) / 16;
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= nwork) return;
  const int uid = A.work[3 * w], start = A.work[3 * w + 1], cnt = A.work[3 * w + 2];
  const int c = lane & 15, q = lane >> 4;
  const int64_t ge = bj_elem(A.active, A.nel, (c < cnt) ? A.perm[start + c] : -1);
  if (__ballot(ge >= 0) == 0) return;  // every element skipped
  constexpr int QS = NB * (NB + 2) / 2;
  const TM* X = A.mat + (int64_t)uid * QS;
  const int prow = permf(c);
  const int flags = A.flags;
  // y = X r, then z = X^T y; the k-step (g, h, s) of z = X^T y takes
  // component 2h + s of y[g].  Both products run as one sequence of 2 NS
  // k-steps whose loads are unconditional (clamped addresses, zeroed by
  // select) and issued one k-step ahead of the products, so the factor
  // fragments of the next k-step (and X^T's first ones, during the last
  // steps of y = X r) are in flight while the matrix cores work.
  constexpr int NS = (NB + 7) / 8;
  const int64_t gsafe = ge >= 0 ? ge : 0;
  auto load_step = [&](int u, v2f& rb, v2f (&a)[NT]) {
    const bool second = u >= NS;
    const int st = second ? u - NS : u, g = st >> 1, k0 = 8 * st + 2 * q;
    const bool kin = k0 < NB;  // k0 is even and NB even: the pair is inside
    if (!second) {
      rb = *reinterpret_cast<const v2f*>(A.r + gsafe * NB + (kin ? k0 : 0));
      if (!(ge >= 0 && kin)) rb = v2f{0.f, 0.f};
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (second ? g < t : g > t) continue;  // X is zero above, X^T below the diagonal
      const int arow = 16 * t + prow;
      // X[arow][k0, k0 + 1]: row pair arow & 1 of quad (arow / 2, k0 / 2);
      // X^T[arow][k0, k0 + 1] = X[k0, k0 + 1][arow]: column pair arow & 1 of
      // quad (k0 / 2, arow / 2); quads above the diagonal are not stored
      const int qm = second ? k0 >> 1 : arow >> 1, qp = second ? arow >> 1 : k0 >> 1;
      const bool ok = arow < NB && kin && qp <= qm;
      const TM* qa = X + (ok ? 4 * (qm * (qm + 1) / 2 + qp) : 0);
      a[t] = second ? ld_col_pair(qa, arow & 1) : ld_row_pair(qa, arow & 1);
      if (!ok) a[t] = v2f{0.f, 0.f};
    }
  };
  v4f y[NT], z[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) y[t] = z[t] = v4f{0.f, 0.f, 0.f, 0.f};
  v2f rbuf[2], abuf[2][NT];
  load_step(0, rbuf[0], abuf[0]);
#pragma unroll
  for (int u = 0; u < 2 * NS; ++u) {
    const int cu = u & 1;
    if (u + 1 < 2 * NS) load_step(u + 1, rbuf[cu ^ 1], abuf[cu ^ 1]);
    if (u < NS) {
      const int g = u >> 1;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (g > t) continue;
        y[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(abuf[cu][t].x, rbuf[cu].x, y[t], 0, 0, 0);
        y[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(abuf[cu][t].y, rbuf[cu].y, y[t], 0, 0, 0);
      }
    } else {
      const int st = u - NS, g = st >> 1, h = st & 1;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (g < t) continue;
        z[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(abuf[cu][t].x, y[g][2 * h], z[t], 0, 0, 0);
        z[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(abuf[cu][t].y, y[g][2 * h + 1], z[t], 0, 0, 0);
      }
    }
  }
  // operands of the update (rows 16t + 8h + 2q, +1), requested after the
  // products so that they stay out of their register peak
  v2f xo[NT][2], dold[NT][2];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = 16 * t + 8 * h + 2 * q;
      const bool ok = ge >= 0 && i < NB;
      xo[t][h] = (ok && (flags & (BJ_READ_X | BJ_FOLD))) ? *reinterpret_cast<const v2f*>(A.x + ge * NB + i)
                                                          : v2f{0.f, 0.f};
      dold[t][h] = (ok && (flags & BJ_READ_D)) ? *reinterpret_cast<const v2f*>(A.d + ge * NB + i) : v2f{0.f, 0.f};
    }
  if (ge < 0) return;
  const double sc = A.scale[ge];
  float* xx = A.x + ge * NB;
  float* dd = A.d + ge * NB;
  double ca = 0.0, cb = 1.0;
  if (!(flags & BJ_APPLY)) {
    const int64_t pb = ge / A.nel;
    ca = A.ab[2 * pb];
    cb = A.ab[2 * pb + 1];
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = 16 * t + 8 * h + 2 * q;
      if (i >= NB) continue;
      const double z0 = double(z[t][2 * h]) * sc, z1 = double(z[t][2 * h + 1]) * sc;
      if (flags & BJ_APPLY) {
        *reinterpret_cast<v2f*>(xx + i) = v2f{float(z0), float(z1)};
        continue;
      }
      double d0 = cb * z0, d1 = cb * z1;
      if (flags & BJ_READ_D) {
        d0 += ca * double(dold[t][h].x);
        d1 += ca * double(dold[t][h].y);
      }
      if (flags & BJ_FOLD) {
        d0 += ca * double(xo[t][h].x);
        d1 += ca * double(xo[t][h].y);
      }
      if (flags & BJ_WRITE_D) *reinterpret_cast<v2f*>(dd + i) = v2f{float(d0), float(d1)};
      if (flags & BJ_READ_X)
        *reinterpret_cast<v2f*>(xx + i) = v2f{float(double(xo[t][h].x) + d0), float(double(xo[t][h].y) + d1)};
      else
        *reinterpret_cast<v2f*>(xx + i) = v2f{float(d0), float(d1)};
    }
}

// ---------------------------------------------------------------------------
// Factored low-precision smoother for blocks that few elements share (a
// viscosity that varies per element, where every element has a block of its
// own and reading the factors is the whole cost): one wavefront per work
// item copies the item's quad-packed factor X into LDS once, with coalesced
// 16-byte (FP32) or 8-byte (BF16) loads, widened to FP32; then, for each
// element of the item, lane i forms row i of y = X r and of z = X^T y from
// LDS (quad row pairs for X, quad column pairs for X^T), accumulating in
// FP32 (even and odd terms apart, then added), and applies the same update
// as the matrix-core kernel.  Used up to k = 4 (at k = 5, 6 the per-lane
// triangular loops and the LDS per wavefront made it slower than the
// matrix-core kernel on distinct blocks: 253 vs 245, 305 vs 243 us for
// 65536 and 32768 elements).
// ---------------------------------------------------------------------------
template <int K1, typename TM>
__global__ __launch_bounds__(64) void bj_stream_lp_kernel(BjArgs<TM, float> A, int nwork) {
  constexpr int NB = 2 * K1 * K1, NP = NB / 2, QS = NB * (NB + 2) / 2, NQ = QS / 4;
  constexpr int RJ = (NB + 63) / 64;  // rows per lane (one up to k = 4)
  __shared__ __align__(16) float sq[QS];
  __shared__ __align__(16) float sr[NB];
  __shared__ __align__(16) float sy[NB];
  const int lane = threadIdx.x;
  const int w = blockIdx.x;
  if (w >= nwork) return;  // the grid has exactly nwork workgroups
  const int uid = A.work[3 * w], start = A.work[3 * w + 1], cnt = A.work[3 * w + 2];
  if (A.active) {  // every element skipped: not even the factor is read
    bool any = false;
    for (int c = 0; c < cnt; ++c) any = any || bj_elem(A.active, A.nel, A.perm[start + c]) >= 0;
    if (!any) return;
  }
  const TM* X = A.mat + (int64_t)uid * QS;
  for (int e = lane; e < NQ; e += 64) {
    v4f v;
    if constexpr (sizeof(TM) == 2) {
      const uint2 u = *reinterpret_cast<const uint2*>(X + 4 * e);
      v = v4f{__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xFFFF0000u), __uint_as_float(u.y << 16),
              __uint_as_float(u.y & 0xFFFF0000u)};
    } else {
      v = *reinterpret_cast<const v4f*>(X + 4 * e);
    }
    *reinterpret_cast<v4f*>(sq + 4 * e) = v;
  }
  const int flags = A.flags;
  for (int c = 0; c < cnt; ++c) {
    const int64_t ge = A.perm[start + c];
    if (bj_elem(A.active, A.nel, ge) < 0) continue;  // the same for the whole workgroup
    const float* rr = A.r + ge * NB;
#pragma unroll
    for (int j = 0; j < RJ; ++j) {
      const int i = lane + 64 * j;
      if (i < NB) sr[i] = rr[i];
    }
    __syncthreads();  // one wavefront: orders the LDS writes before the reads
#pragma unroll
    for (int j = 0; j < RJ; ++j) {
      const int i = lane + 64 * j;
      if (i < NB) {
        // y_i = sum_{p <= m} X[i][2p, 2p + 1] . r[2p, 2p + 1], m = i / 2
        const int m = i >> 1;
        const float* qr = sq + 2 * m * (m + 1) + 2 * (i & 1);
        float a0 = 0.f, a1 = 0.f;  // even and odd columns
#pragma unroll 4
        for (int p = 0; p <= m; ++p) {
          const v2f xv = *reinterpret_cast<const v2f*>(qr + 4 * p);
          const v2f rv = *reinterpret_cast<const v2f*>(sr + 2 * p);
          a0 = __builtin_fmaf(xv.x, rv.x, a0);
          a1 = __builtin_fmaf(xv.y, rv.y, a1);
        }
        sy[i] = a0 + a1;
      }
    }
    __syncthreads();
    float zr[RJ];
#pragma unroll
    for (int j = 0; j < RJ; ++j) {
      const int i = lane + 64 * j;
      zr[j] = 0.f;
      if (i < NB) {
        // z_i = sum_{m >= p} X[2m, 2m + 1][i] . y[2m, 2m + 1], p = i / 2
        const int p = i >> 1, b = i & 1;
        float a0 = 0.f, a1 = 0.f;  // even and odd rows of X
#pragma unroll 4
        for (int m = p; m < NP; ++m) {
          const float* qq = sq + 2 * m * (m + 1) + 4 * p + b;
          const v2f yv = *reinterpret_cast<const v2f*>(sy + 2 * m);
          a0 = __builtin_fmaf(qq[0], yv.x, a0);
          a1 = __builtin_fmaf(qq[2], yv.y, a1);
        }
        zr[j] = a0 + a1;
      }
    }
    const double sc = A.scale[ge];
    float* xx = A.x + ge * NB;
    float* dd = A.d + ge * NB;
    double ca = 0.0, cb = 1.0;
    if (!(flags & BJ_APPLY)) {
      const int64_t pb = ge / A.nel;
      ca = A.ab[2 * pb];
      cb = A.ab[2 * pb + 1];
    }
#pragma unroll
    for (int j = 0; j < RJ; ++j) {
      const int i = lane + 64 * j;
      if (i >= NB) continue;
      const double z = double(zr[j]) * sc;
      if (flags & BJ_APPLY) {
        xx[i] = float(z);
        continue;
      }
      double dv = cb * z;
      if (flags & BJ_READ_D) dv += ca * double(dd[i]);
      const double xo = (flags & (BJ_READ_X | BJ_FOLD)) ? double(xx[i]) : 0.0;
      if (flags & BJ_FOLD) dv += ca * xo;
      if (flags & BJ_WRITE_D) dd[i] = float(dv);
      xx[i] = (flags & BJ_READ_X) ? float(xo + dv) : float(dv);
    }
    // the next element's r and y reuse the LDS rows: all lanes are done
    // with this element's (one wavefront; the barrier orders LDS access)
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// FP64 smoother for blocks that few elements share (k <= 4): as the
// streaming factored kernel above, with the symmetric inverse B^{-1} stored
// once as lower-triangle quads (half the bytes of the full square) and one
// product per element: lane i forms row i of z = B^{-1} r from quad row pairs
// (columns up to its own row pair) and quad column pairs (the transposes of
// the quads below), in FP64 with two accumulators.
// ---------------------------------------------------------------------------
template <int K1>
__global__ __launch_bounds__(64) void bj_stream_f64_kernel(BjArgs<double, double> A, int nwork) {
  constexpr int NB = 2 * K1 * K1, NP = NB / 2, QS = NB * (NB + 2) / 2;
  static_assert(NB <= 64, "one row per lane");
  __shared__ __align__(16) double sq[QS];
  __shared__ __align__(16) double sr[NB];
  const int lane = threadIdx.x;
  const int w = blockIdx.x;
  if (w >= nwork) return;  // the grid has exactly nwork workgroups
  const int uid = A.work[3 * w], start = A.work[3 * w + 1], cnt = A.work[3 * w + 2];
  if (A.active) {  // every element skipped: not even the inverse is read
    bool any = false;
    for (int c = 0; c < cnt; ++c) any = any || bj_elem(A.active, A.nel, A.perm[start + c]) >= 0;
    if (!any) return;
  }
  const double* B = A.mat + (int64_t)uid * QS;
  for (int e = lane; e < QS / 2; e += 64)
    *reinterpret_cast<v2d*>(sq + 2 * e) = *reinterpret_cast<const v2d*>(B + 2 * e);
  const int flags = A.flags;
  const int m = lane >> 1, a = lane & 1;
  for (int c = 0; c < cnt; ++c) {
    const int64_t ge = A.perm[start + c];
    if (bj_elem(A.active, A.nel, ge) < 0) continue;  // the same for the whole workgroup
    if (lane < NB) sr[lane] = A.r[ge * NB + lane];
    __syncthreads();  // one wavefront: orders the LDS writes before the reads
    double z = 0.0;
    if (lane < NB) {
      double a0 = 0.0, a1 = 0.0;  // even and odd columns
      const double* qr = sq + 2 * m * (m + 1) + 2 * a;
#pragma unroll 4
      for (int p = 0; p <= m; ++p) {  // B[i][2p, 2p + 1]: row pair a of quad (m, p)
        const v2d xv = *reinterpret_cast<const v2d*>(qr + 4 * p);
        const v2d rv = *reinterpret_cast<const v2d*>(sr + 2 * p);
        a0 = __builtin_fma(xv.x, rv.x, a0);
        a1 = __builtin_fma(xv.y, rv.y, a1);
      }
#pragma unroll 4
      for (int p = m + 1; p < NP; ++p) {  // B[2p, 2p + 1][i]: column pair a of quad (p, m)
        const double* qq = sq + 2 * p * (p + 1) + 4 * m + a;
        const v2d rv = *reinterpret_cast<const v2d*>(sr + 2 * p);
        a0 = __builtin_fma(qq[0], rv.x, a0);
        a1 = __builtin_fma(qq[2], rv.y, a1);
      }
      z = (a0 + a1) * A.scale[ge];
    }
    if (lane < NB) {
      double* xx = A.x + ge * NB;
      if (flags & BJ_APPLY) {
        xx[lane] = z;
      } else {
        const int64_t pb = ge / A.nel;
        const double ca = A.ab[2 * pb], cb = A.ab[2 * pb + 1];
        double* dd = A.d + ge * NB;
        double dv = cb * z;
        if (flags & BJ_READ_D) dv += ca * dd[lane];
        const double xo = (flags & (BJ_READ_X | BJ_FOLD)) ? xx[lane] : 0.0;
        if (flags & BJ_FOLD) dv += ca * xo;
        if (flags & BJ_WRITE_D) dd[lane] = dv;
        xx[lane] = (flags & BJ_READ_X) ? xo + dv : dv;
      }
    }
    __syncthreads();  // the next element's r reuses the LDS row
  }
}

template <int K1, typename TM, typename TV, bool TRI>
static void launch_k(const BjPlan& P, const TM* mat, const TV* r, const double* ab, TV* d, TV* x, int flags,
                     hipStream_t s) {
  BjArgs<TM, TV> A{P.G, P.nel, P.perm, P.work, P.scale, mat, r, ab, d, x, flags, P.active};
  if constexpr (!TRI && sizeof(TM) == 8 && sizeof(TV) == 8) {
    bool streamed = false;
    if constexpr (K1 <= 5)
      if (P.stream) {  // mat: the quad-packed inverses (sym_quad_f64)
        hipLaunchKernelGGL((bj_stream_f64_kernel<K1>), dim3(P.nwork), dim3(64), 0, s, A, P.nwork);
        streamed = true;
      }
    if (!streamed)
      hipLaunchKernelGGL((bj_wave_kernel<K1>), dim3((P.nwork + 3) / 4), dim3(256), 0, s, A, P.nwork);
  } else {
    bool streamed = false;
    if constexpr (K1 <= 5)
      if (P.stream) {
        hipLaunchKernelGGL((bj_stream_lp_kernel<K1, TM>), dim3(P.nwork), dim3(64), 0, s, A, P.nwork);
        streamed = true;
      }
    if (!streamed)
      hipLaunchKernelGGL((bj_wave_lp_kernel<K1, TM>), dim3((P.nwork + 3) / 4), dim3(256), 0, s, A, P.nwork);
  }
}

template <typename TM, typename TV, bool TRI>
static int launch_group(const BjPlan& P, const TM* mat, const TV* r, const double* ab, TV* d, TV* x, int flags,
                        hipStream_t s) {
  if (P.nwork <= 0) return SDG_OK;
  if (P.G < 4 || P.G % 4 || P.G > 16) {  // one wavefront's 16 matrix-core columns
    set_error("block smoother: group size does not fit one workgroup");
    return SDG_ERR_INVALID;
  }
  // vectors move in pairs of values: r, x and d must be aligned to two values
  const uintptr_t al = 2 * sizeof(TV);
  if (reinterpret_cast<uintptr_t>(x) % al || reinterpret_cast<uintptr_t>(d) % al ||
      reinterpret_cast<uintptr_t>(r) % al || reinterpret_cast<uintptr_t>(mat) % 16) {
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
