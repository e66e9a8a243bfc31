// Shared device helpers of the SIP-DG library: 1D Legendre constants in the
// L2(-1,1)-orthonormal scaling lhat_i = sqrt((2i+1)/2) L_i, error plumbing,
// launch helpers.
//
// Every table entry is a function of compile-time indices: kernels unroll
// their mode loops over the template parameter K1 = k+1, so the constants
// fold into instruction immediates and the structural zeros of the
// derivative matrix drop out at compile time.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/sdg.h"

namespace sdg {

// ---------------------------------------------------------------------------
// 1D constants (Legendre end values and derivatives)
// ---------------------------------------------------------------------------
// lhat_i(+1) = sqrt((2i+1)/2), lhat_i(-1) = (-1)^i sqrt((2i+1)/2)
// lhat_i'(+1) = sqrt((2i+1)/2) i(i+1)/2, lhat_i'(-1) = (-1)^(i+1) of that.
__host__ __device__ __forceinline__ double onb(int i) { return sqrt((2.0 * i + 1.0) * 0.5); }
__host__ __device__ __forceinline__ double e_end(int i, int plus) {
  return (plus || !(i & 1)) ? onb(i) : -onb(i);
}
__host__ __device__ __forceinline__ double d_end(int i, int plus) {
  const double v = onb(i) * 0.5 * i * (i + 1);
  return (plus || (i & 1)) ? v : -v;
}
// Derivative matrix: lhat_i' = sum_m D(m, i) lhat_m, nonzero only for m < i
// with m + i odd, where it equals sqrt((2m+1)(2i+1)).
__host__ __device__ __forceinline__ constexpr bool d_nz(int m, int i) { return m < i && ((m + i) & 1); }
__host__ __device__ __forceinline__ double d_val(int m, int i) {
  return sqrt((2.0 * m + 1.0) * (2.0 * i + 1.0));
}
// Workgroups of one launch are handed to the eight XCDs of the chip in turn
// (linear id modulo 8), and each XCD has its own L2.  xcd_order maps the
// linear id to a logical index such that every XCD receives one contiguous
// range of logical indices: neighbouring tiles then share an L2.  It is a
// bijection on [0, total).
__device__ __forceinline__ uint32_t xcd_order(uint32_t lid, uint32_t total) {
  const uint32_t q = total >> 3, r = total & 7, x = lid & 7, k = lid >> 3;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}
// 1D stiffness S = D^T D: int lhat_i' lhat_l' = sqrt((2i+1)(2l+1))/2 *
// min(i,l)(min(i,l)+1) when i + l is even, else 0.
__host__ __device__ __forceinline__ constexpr bool s_nz(int i, int l) {
  return ((i + l) & 1) == 0 && i > 0 && l > 0;
}
__host__ __device__ __forceinline__ double s_val(int i, int l) {
  const int m = i < l ? i : l;
  return sqrt((2.0 * i + 1.0) * (2.0 * l + 1.0)) * 0.5 * m * (m + 1);
}

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
const char* get_error();

#define SDG_HIP(call)                                                                \
  do {                                                                               \
    hipError_t _e = (call);                                                          \
    if (_e != hipSuccess) {                                                          \
      ::sdg::set_error(std::string(#call) + ": " + hipGetErrorString(_e) + " at " + \
                       __FILE__ + ":" + std::to_string(__LINE__));                  \
      return SDG_ERR_DEVICE;                                                         \
    }                                                                                \
  } while (0)

#define SDG_TRY(call)              \
  do {                             \
    int _rc = (call);              \
    if (_rc < 0) return _rc;       \
  } while (0)

#define SDG_CHECK_LAUNCH() SDG_HIP(hipGetLastError())

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Face kinds used by the kernels.
enum FaceKind : int { F_NAVIER = SDG_NAVIER, F_NEUMANN = SDG_NEUMANN, F_DIRICHLET = SDG_DIRICHLET, F_INTERIOR = 3 };

// Geometry/boundary description passed by value to kernels.
struct MeshDev {
  int nx, ny;
  double hx, hy;
  int bc[4];  // left, right, bottom, top
  // inside a batched CG iteration: problems with active[pb] == 0 have
  // converged, and the operator kernels skip them (null: none skipped)
  const int* active = nullptr;
};

}  // namespace sdg
