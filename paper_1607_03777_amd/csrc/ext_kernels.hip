// Extended-precision residual of the viscous and Stokes systems, for
// iterative refinement below the FP64 rounding floor.
//
// The paper meets orthogonalisation breakdown of the FP64 Krylov methods at
// viscosity contrasts beyond 10^3 and switches to quadruple precision
// arithmetic (Section 8.3.1).  Here the Krylov iterations stay in FP64 and
// the accuracy that FP64 cannot represent is recovered by refinement
// (restarted FGMRES or CG corrections): the iterate is carried as a
// double-FP64 pair x = x_hi + x_lo and the residual b - K x is evaluated in
// double-FP64 arithmetic with operator coefficients that are exact to the
// 64-bit mantissa of the host's long double.  Two floors are removed that
// way: rounding in the evaluation of K x (about eps |K||x| / |b|) and the
// FP64 representation of the coefficients and of x itself, both of which
// are larger than 1e-8 at a viscosity contrast of 10^4 on a 64 x 64 mesh of
// Q_4 elements.
//
// Operator form.  Every block of A (eq. stiffness_form) and B
// (eq. divergence_form) between an element and itself or a face neighbour is
// a fixed "unit" matrix times one scalar: eta_K for the volume term
// (2 eta eps(u):eps(v)), eta of the trial or test side for the two
// consistency terms of a face, the face penalty sigma_F = gamma_F C_F
// (eq. sipg_penalty at its lower bound, eq. const_trace_face) for the jump
// term, and 1 for B.  The unit matrices depend only on (k, h_x, h_y) and on
// the side and boundary kind; they are integrated once on the host in long
// double by Gauss-Legendre quadrature with k+2 points (exact for these
// polynomial integrands) and stored as double-FP64 pairs.  The residual
// kernels then form, per element row, the sum of the unit rows against the
// element's and its neighbours' coefficients, every product and sum in
// double-FP64 (TwoSum / FMA-based TwoProd).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "sdg_common.h"
#include "ext_kernels.h"

// elements per workgroup of the velocity-row kernel (k <= 4, k >= 5) and the
// unroll depth of its column loop
// (measured at 64 x 64 x 16, k = 4, and 256 x 256, k = 3..6: two elements
// per workgroup were fastest at every order, 1.2-3.4x faster than one, and
// 8 the slowest; the unroll depth made no difference)
#ifndef EXT_G_LOW
#define EXT_G_LOW 2
#endif
#ifndef EXT_G_HIGH
#define EXT_G_HIGH 2
#endif
#ifndef EXT_UNROLL
#define EXT_UNROLL 4
#endif

namespace sdg {

// ---------------------------------------------------------------------------
// host: unit blocks in long double
// ---------------------------------------------------------------------------
namespace {

typedef long double LD;

void gauss_ld(int n, std::vector<LD>& x, std::vector<LD>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    LD t = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
    LD dp = 1;
    for (int it = 0; it < 60; ++it) {
      LD p0 = 1, p1 = t;
      for (int m = 1; m < n; ++m) {
        const LD p2 = ((2 * m + 1) * t * p1 - m * p0) / (m + 1);
        p0 = p1;
        p1 = p2;
      }
      // P_n' = n (t P_n - P_{n-1}) / (t^2 - 1)
      dp = n * (t * p1 - p0) / (t * t - 1);
      const LD dt = p1 / dp;
      t -= dt;
      if (fabsl(dt) <= 1e-21L * (1 + fabsl(t))) {
        if (it > 1) break;
      }
    }
    LD p0 = 1, p1 = t;
    for (int m = 1; m < n; ++m) {
      const LD p2 = ((2 * m + 1) * t * p1 - m * p0) / (m + 1);
      p0 = p1;
      p1 = p2;
    }
    dp = n * (t * p1 - p0) / (t * t - 1);
    x[i] = t;
    w[i] = 2 / ((1 - t * t) * dp * dp);
  }
}

// orthonormal Legendre values and derivatives lhat_0..lhat_k at t
void onb_ld(int k, LD t, LD* v, LD* d) {
  LD P[16], D[16];
  P[0] = 1;
  D[0] = 0;
  if (k >= 1) {
    P[1] = t;
    D[1] = 1;
  }
  for (int n = 1; n < k; ++n) {
    P[n + 1] = ((2 * n + 1) * t * P[n] - n * P[n - 1]) / (n + 1);
    D[n + 1] = D[n - 1] + (2 * n + 1) * P[n];
  }
  for (int i = 0; i <= k; ++i) {
    const LD sc = sqrtl((2 * i + 1) / (LD)2);
    v[i] = sc * P[i];
    d[i] = sc * D[i];
  }
}

// velocity basis at reference point (xi, et): val[a][c], eps[a][c][r]
// (strain of phi_a), div[a]; a = (d (k+1) + j)(k+1) + i
struct VPoint {
  std::vector<LD> val, eps, div;
};
VPoint vbasis(int k, LD hx, LD hy, LD xi, LD et) {
  const int K1 = k + 1, NB = 2 * K1 * K1;
  LD lx[16], dlx[16], ly[16], dly[16];
  onb_ld(k, xi, lx, dlx);
  onb_ld(k, et, ly, dly);
  const LD c = 2 / sqrtl(hx * hy);
  VPoint P;
  P.val.assign(NB * 2, 0);
  P.eps.assign(NB * 4, 0);
  P.div.assign(NB, 0);
  for (int d = 0; d < 2; ++d)
    for (int j = 0; j < K1; ++j)
      for (int i = 0; i < K1; ++i) {
        const int a = (d * K1 + j) * K1 + i;
        LD g[2][2] = {{0, 0}, {0, 0}};
        P.val[a * 2 + d] = c * lx[i] * ly[j];
        g[d][0] = c * (2 / hx) * dlx[i] * ly[j];
        g[d][1] = c * (2 / hy) * lx[i] * dly[j];
        for (int cc = 0; cc < 2; ++cc)
          for (int r = 0; r < 2; ++r) P.eps[(a * 2 + cc) * 2 + r] = (g[cc][r] + g[r][cc]) / 2;
        P.div[a] = g[0][0] + g[1][1];
      }
  return P;
}
// pressure basis chi_m, m = j k + i (i, j < k)
std::vector<LD> pbasis(int k, LD hx, LD hy, LD xi, LD et) {
  std::vector<LD> out(k * k, 0);
  if (k < 1) return out;
  LD lx[16], dlx[16], ly[16], dly[16];
  onb_ld(k - 1, xi, lx, dlx);
  onb_ld(k - 1, et, ly, dly);
  const LD c = 2 / sqrtl(hx * hy);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < k; ++i) out[j * k + i] = c * lx[i] * ly[j];
  return out;
}

// side S (0 left, 1 right, 2 bottom, 3 top): reference point of Gauss node
// g, outward normal, line-weight factor
void side_point(int S, LD g, LD hx, LD hy, LD* xi, LD* et, LD n[2], LD* jac) {
  n[0] = n[1] = 0;
  if (S < 2) {
    *xi = S == 0 ? -1 : 1;
    *et = g;
    n[0] = S == 0 ? -1 : 1;
    *jac = hy / 2;
  } else {
    *xi = g;
    *et = S == 2 ? -1 : 1;
    n[1] = S == 2 ? -1 : 1;
    *jac = hx / 2;
  }
}

void put(std::vector<double2>& T, size_t off, LD v) {
  const double hi = (double)v;
  T[off] = make_double2(hi, (double)(v - (LD)hi));
}

}  // namespace

void ext_unit_blocks(int k, double lx, double ly, int nx, int ny, const int bc[4], std::vector<double2>& TA,
                     std::vector<double2>& TBu, std::vector<double2>& TBp, double2 cpen[2]) {
  const int K1 = k + 1, NB = 2 * K1 * K1, NP = k * k;
  const LD hx = (LD)lx / nx, hy = (LD)ly / ny;
  std::vector<LD> g, w;
  gauss_ld(k + 2, g, w);
  const int nq = k + 2;
  std::vector<LD> A((size_t)EXT_NA * NB * NB, 0), B((size_t)EXT_NBLK_B * NB * std::max(NP, 1), 0);
  auto a_at = [&](int blk, int a, int b) -> LD& { return A[((size_t)blk * NB + a) * NB + b]; };
  auto b_at = [&](int blk, int a, int m) -> LD& { return B[((size_t)blk * NB + a) * std::max(NP, 1) + m]; };
  // volume: 2 eps(phi_a):eps(phi_b) and -div(phi_a) chi_m
  for (int qy = 0; qy < nq; ++qy)
    for (int qx = 0; qx < nq; ++qx) {
      const LD wq = w[qx] * w[qy] * hx * hy / 4;
      const VPoint P = vbasis(k, hx, hy, g[qx], g[qy]);
      const std::vector<LD> ch = pbasis(k, hx, hy, g[qx], g[qy]);
      for (int a = 0; a < NB; ++a) {
        for (int b = 0; b < NB; ++b) {
          LD s = 0;
          for (int cr = 0; cr < 4; ++cr) s += P.eps[a * 4 + cr] * P.eps[b * 4 + cr];
          a_at(EXT_V, a, b) += 2 * wq * s;
        }
        for (int m = 0; m < NP; ++m) b_at(EXT_BVOL, a, m) -= wq * P.div[a] * ch[m];
      }
    }
  // interior faces: direction 0 (x-normal) pairs the right side of the
  // minus element with the left side of the plus element; direction 1 the
  // top of the minus with the bottom of the plus.  Side index 0 = minus.
  for (int dir = 0; dir < 2; ++dir) {
    const int Sside[2] = {dir == 0 ? 1 : 3, dir == 0 ? 0 : 2};
    for (int q = 0; q < nq; ++q) {
      VPoint P[2];
      std::vector<LD> ch[2];
      LD n[2][2], wl = 0;
      for (int sd = 0; sd < 2; ++sd) {
        LD xi, et, jac;
        side_point(Sside[sd], g[q], hx, hy, &xi, &et, n[sd], &jac);
        P[sd] = vbasis(k, hx, hy, xi, et);
        ch[sd] = pbasis(k, hx, hy, xi, et);
        wl = w[q] * jac;
      }
      for (int t = 0; t < 2; ++t) {  // test side (the element whose rows these are)
        const int s = 1 - t;
        const int base = ext_face_base(dir, t);
        for (int a = 0; a < NB; ++a) {
          for (int b = 0; b < NB; ++b) {
            // trial on side s' in {t, s}; T1 ~ eta of the trial side,
            // T2 ~ eta of the test side, T3 ~ sigma_F
            for (int which = 0; which < 2; ++which) {
              const int sp = which == 0 ? t : s;
              LD t1 = 0, t2 = 0, t3 = 0;
              for (int c = 0; c < 2; ++c)
                for (int r = 0; r < 2; ++r) {
                  const LD vt = P[t].val[a * 2 + c] * n[t][r];
                  const LD vs = P[sp].val[b * 2 + c] * n[sp][r];
                  t1 -= P[sp].eps[(b * 2 + c) * 2 + r] * vt;
                  t2 -= P[t].eps[(a * 2 + c) * 2 + r] * vs;
                  t3 += vs * vt;
                }
              if (which == 0) {
                a_at(base + EXT_SELF12, a, b) += wl * (t1 + t2);
                a_at(base + EXT_SELF3, a, b) += wl * t3;
              } else {
                a_at(base + EXT_NB1, a, b) += wl * t1;
                a_at(base + EXT_NB2, a, b) += wl * t2;
                a_at(base + EXT_NB3, a, b) += wl * t3;
              }
            }
          }
          // {q}[[v.n]] = 1/2 q^s' (v^t . n^t): self (pressure side t) and
          // neighbour (pressure side s)
          LD vn = P[t].val[a * 2] * n[t][0] + P[t].val[a * 2 + 1] * n[t][1];
          for (int m = 0; m < NP; ++m) {
            b_at(ext_bface(dir, t) + 0, a, m) += wl * vn * ch[t][m] / 2;
            b_at(ext_bface(dir, t) + 1, a, m) += wl * vn * ch[s][m] / 2;
          }
        }
      }
    }
  }
  // boundary sides: Navier (normal components) and Dirichlet (full vector)
  // Nitsche terms; Neumann sides contribute nothing
  for (int S = 0; S < 4; ++S) {
    if (bc[S] == SDG_NEUMANN) continue;
    for (int q = 0; q < nq; ++q) {
      LD xi, et, n[2], jac;
      side_point(S, g[q], hx, hy, &xi, &et, n, &jac);
      const LD wl = w[q] * jac;
      const VPoint P = vbasis(k, hx, hy, xi, et);
      const std::vector<LD> ch = pbasis(k, hx, hy, xi, et);
      for (int a = 0; a < NB; ++a) {
        const LD vna = P.val[a * 2] * n[0] + P.val[a * 2 + 1] * n[1];
        LD sna[2];  // 2 eps(phi_a) n
        for (int c = 0; c < 2; ++c) sna[c] = 2 * (P.eps[(a * 2 + c) * 2] * n[0] + P.eps[(a * 2 + c) * 2 + 1] * n[1]);
        for (int b = 0; b < NB; ++b) {
          const LD vnb = P.val[b * 2] * n[0] + P.val[b * 2 + 1] * n[1];
          LD snb[2];
          for (int c = 0; c < 2; ++c)
            snb[c] = 2 * (P.eps[(b * 2 + c) * 2] * n[0] + P.eps[(b * 2 + c) * 2 + 1] * n[1]);
          LD b12, b3;
          if (bc[S] == SDG_NAVIER) {
            const LD nsna = sna[0] * n[0] + sna[1] * n[1], nsnb = snb[0] * n[0] + snb[1] * n[1];
            b12 = -nsnb * vna - nsna * vnb;
            b3 = vnb * vna;
          } else {
            b12 = -(snb[0] * P.val[a * 2] + snb[1] * P.val[a * 2 + 1]) -
                  (sna[0] * P.val[b * 2] + sna[1] * P.val[b * 2 + 1]);
            b3 = P.val[b * 2] * P.val[a * 2] + P.val[b * 2 + 1] * P.val[a * 2 + 1];
          }
          a_at(EXT_BND + 2 * S, a, b) += wl * b12;
          a_at(EXT_BND + 2 * S + 1, a, b) += wl * b3;
        }
        for (int m = 0; m < NP; ++m) b_at(EXT_BBND + S, a, m) += wl * vna * ch[m];
      }
    }
  }
  // device layouts: A blocks column-major ([b][a]: rows a of one column
  // consecutive, so the threads of a row-parallel kernel read coalesced),
  // B blocks column-major for the velocity rows and row-major for the
  // pressure rows
  TA.assign((size_t)EXT_NA * NB * NB, make_double2(0, 0));
  for (int blk = 0; blk < EXT_NA; ++blk)
    for (int a = 0; a < NB; ++a)
      for (int b = 0; b < NB; ++b) put(TA, ((size_t)blk * NB + b) * NB + a, a_at(blk, a, b));
  const int NPm = std::max(NP, 1);
  TBu.assign((size_t)EXT_NBLK_B * NB * NPm, make_double2(0, 0));
  TBp.assign((size_t)EXT_NBLK_B * NB * NPm, make_double2(0, 0));
  for (int blk = 0; blk < EXT_NBLK_B; ++blk)
    for (int a = 0; a < NB; ++a)
      for (int m = 0; m < NP; ++m) {
        put(TBu, ((size_t)blk * NPm + m) * NB + a, b_at(blk, a, m));
        put(TBp, ((size_t)blk * NB + a) * NPm + m, b_at(blk, a, m));
      }
  // C_F = (k+1)^2 |e| / |K| = (k+1)^2 / h_n (x-normal faces: h_x)
  const LD cx = (LD)(K1 * K1) / hx, cy = (LD)(K1 * K1) / hy;
  const double hxd = (double)cx, hyd = (double)cy;
  cpen[0] = make_double2(hxd, (double)(cx - (LD)hxd));
  cpen[1] = make_double2(hyd, (double)(cy - (LD)hyd));
}

// ---------------------------------------------------------------------------
// device: double-FP64 arithmetic (error-free transformations)
// ---------------------------------------------------------------------------
struct dd {
  double hi, lo;
};
// Knuth's TwoSum: s + e = a + b exactly
__device__ __forceinline__ dd two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
// |a| >= |b| (or a = 0)
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  return {s, b - (s - a)};
}
// p + e = a b exactly (FMA)
__device__ __forceinline__ dd two_prod(double a, double b) {
  const double p = a * b;
  return {p, __builtin_fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_add(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  const dd t = two_sum(x.lo, y.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_mul(dd x, dd y) {
  dd p = two_prod(x.hi, y.hi);
  p.lo = __builtin_fma(x.hi, y.lo, __builtin_fma(x.lo, y.hi, p.lo));
  return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_neg(dd x) { return {-x.hi, -x.lo}; }
__device__ __forceinline__ dd mk(double2 v) { return {v.x, v.y}; }

// sum_b T[b*ld + row] x[b] in double-FP64 (ABS: sum |T_hi| |x_hi| in FP64)
template <int N, bool ABS>
__device__ __forceinline__ dd col_dot(const double2* __restrict__ T, int row, int ld, const double2* x) {
  dd s = {0.0, 0.0};
  for (int b = 0; b < N; ++b) {
    const double2 c = T[(size_t)b * ld + row];
    if (ABS) {
      s.hi += fabs(c.x) * fabs(x[b].x);
    } else if (c.x != 0.0) {
      s = dd_add(s, dd_mul(mk(c), mk(x[b])));
    }
  }
  return s;
}
template <bool ABS>
__device__ __forceinline__ dd acc_sub(dd acc, dd scal, dd v) {
  if (ABS) return {acc.hi + fabs(scal.hi) * v.hi, 0.0};
  return dd_add(acc, dd_neg(dd_mul(scal, v)));
}

// neighbour of element (ix, iy) across side S, -1 on the boundary
__device__ __forceinline__ int nbr(int S, int ix, int iy, int nx, int ny) {
  switch (S) {
    case 0: return ix > 0 ? iy * nx + ix - 1 : -1;
    case 1: return ix < nx - 1 ? iy * nx + ix + 1 : -1;
    case 2: return iy > 0 ? (iy - 1) * nx + ix : -1;
    default: return iy < ny - 1 ? (iy + 1) * nx + ix : -1;
  }
}

// Velocity rows: r = F - A x - B p (ABS: |A||x| + |B||p|), x = xh + xl.
// One workgroup per row of G consecutive elements of one problem (the last
// group of a mesh row may be partial), thread a = row a of every element of
// the group: each entry of a unit block is read once and applied to all
// elements that use that block, with their own scalars.  The vectors of the
// group, its two x-neighbours outside it and the elements above and below it
// are staged in LDS as (hi, lo) pairs.
//
// The sum over a block's columns is formed by Dot2 (Ogita, Rump and Oishi,
// "Accurate sum and dot product", 2005), adapted to operands given as
// double-FP64 pairs: the product of the high parts is split exactly by an
// FMA (TwoProduct), the running sum by TwoSum, and the two cross products
// with the low parts (whose own rounding is far below the result's
// accuracy) go into the low word with the error terms.  The block's sum is
// then scaled by its scalar and subtracted from the row in full double-FP64.
// Sums of one block's row a against the vectors VS(e) of the group members
// in mask, into (sh, sl) per member; then acc -= SC(e) * sum per member.
template <int N, int G, bool ABS, typename VS, typename SC>
__device__ __forceinline__ void blk_apply(const double2* __restrict__ T, int a, int ld, unsigned mask, VS vs, SC sc,
                                          dd (&acc)[G]) {
  double sh[G], sl[G];
#pragma unroll
  for (int e = 0; e < G; ++e) sh[e] = sl[e] = 0.0;
  // unrolled EXT_UNROLL columns deep: the loads of the next columns are in
  // flight while the current ones are summed
#pragma unroll EXT_UNROLL
  for (int b = 0; b < N; ++b) {
    const double2 c = T[(size_t)b * ld + a];
    // every member is summed (slots of absent elements hold zeros): no
    // branch in the loop; the mask applies when the sums are used
#pragma unroll
    for (int e = 0; e < G; ++e) {
      const double2 x = vs(e)[b];
      if (ABS) {
        sh[e] += fabs(c.x) * fabs(x.x);
      } else {
        const double p = c.x * x.x;
        const double pe = __builtin_fma(c.x, x.x, -p);
        const double cross = __builtin_fma(c.x, x.y, c.y * x.x);
        const dd s = two_sum(sh[e], p);
        sh[e] = s.hi;
        sl[e] += s.lo + (pe + cross);
      }
    }
  }
#pragma unroll
  for (int e = 0; e < G; ++e) {
    if (!(mask & (1u << e))) continue;
    const dd scal = sc(e);
    if (ABS) {
      acc[e].hi += fabs(scal.hi) * sh[e];
    } else {
      acc[e] = dd_add(acc[e], dd_neg(dd_mul(scal, two_sum(sh[e], sl[e]))));
    }
  }
}

template <int K1> struct ExtGroup { static constexpr int G = K1 <= 5 ? EXT_G_LOW : EXT_G_HIGH; };

template <int K1, bool ABS>
__global__ __launch_bounds__(128) void ext_u_kernel(MeshDev M, const double* __restrict__ eta,
                                                     const double* __restrict__ F, const double* __restrict__ xh,
                                                     const double* __restrict__ xl, const double* __restrict__ ph,
                                                     const double* __restrict__ pl, const double2* __restrict__ TA,
                                                     const double2* __restrict__ TB, double2 cx, double2 cy,
                                                     double* __restrict__ r) {
  constexpr int NB = 2 * K1 * K1, NP = (K1 - 1) * (K1 - 1), NPm = NP > 0 ? NP : 1;
  constexpr int G = ExtGroup<K1>::G;
  // slots: 0..G-1 the group, G left of it, G+1 right of it, G+2.. below, 2G+2.. above
  constexpr int NSLOT = 3 * G + 2;
  __shared__ double2 xs[NSLOT][NB];
  __shared__ double2 ps[NSLOT][NPm];
  __shared__ double es[NSLOT];
  const int nx = M.nx, ny = M.ny, nel = nx * ny;
  const int ngx = (nx + G - 1) / G;
  const int iy = blockIdx.x / ngx, ix0 = (blockIdx.x - iy * ngx) * G;
  const int pb = blockIdx.y;
  const int64_t off = (int64_t)pb * nel;
  const int ng = nx - ix0 < G ? nx - ix0 : G;  // elements in this group
  // element of slot q, or -1
  auto slot_el = [&](int q) -> int {
    if (q < G) return q < ng ? iy * nx + ix0 + q : -1;
    if (q == G) return ix0 > 0 ? iy * nx + ix0 - 1 : -1;
    if (q == G + 1) return ix0 + G < nx ? iy * nx + ix0 + G : -1;
    const int i = (q - G - 2) % G, above = (q - G - 2) / G;
    if (i >= ng) return -1;
    const int jy = above ? iy + 1 : iy - 1;
    return (jy >= 0 && jy < ny) ? jy * nx + ix0 + i : -1;
  };
  for (int q = threadIdx.x; q < NSLOT * NB; q += blockDim.x) {
    const int slot = q / NB, a = q - slot * NB;
    const int el = slot_el(slot);
    double2 v = make_double2(0.0, 0.0);
    if (el >= 0) {
      const int64_t g = (off + el) * NB + a;
      v = make_double2(xh[g], xl ? xl[g] : 0.0);
    }
    xs[slot][a] = v;
  }
  if (ph && NP > 0)
    for (int q = threadIdx.x; q < NSLOT * NP; q += blockDim.x) {
      const int slot = q / NP, m = q - slot * NP;
      const int el = slot_el(slot);
      double2 v = make_double2(0.0, 0.0);
      if (el >= 0) {
        const int64_t g = (off + el) * NP + m;
        v = make_double2(ph[g], pl ? pl[g] : 0.0);
      }
      ps[slot][m] = v;
    }
  for (int q = threadIdx.x; q < NSLOT; q += blockDim.x) {
    const int el = slot_el(q);
    es[q] = el >= 0 ? eta[off + el] : 0.0;
  }
  __syncthreads();
  const int a = threadIdx.x;
  if (a >= NB) return;
  unsigned own = 0;  // elements of the group
#pragma unroll
  for (int e = 0; e < G; ++e)
    if (e < ng) own |= 1u << e;
  dd acc[G];
#pragma unroll
  for (int e = 0; e < G; ++e) {
    const double F0 = (!ABS && e < ng) ? F[(off + iy * nx + ix0 + e) * NB + a] : 0.0;
    acc[e] = {F0, 0.0};
  }
  auto self = [&](int e) -> const double2* { return xs[e]; };
  auto selfp = [&](int e) -> const double2* { return ps[e]; };
  auto de = [&](int e) -> dd { return {es[e], 0.0}; };
  auto one = [&](int) -> dd { return {1.0, 0.0}; };
  blk_apply<NB, G, ABS>(TA + (size_t)EXT_V * NB * NB, a, NB, own, self, de, acc);
  for (int S = 0; S < 4; ++S) {
    const int dir = S >> 1;
    const dd cpen = mk(dir == 0 ? cx : cy);
    // the neighbour's slot of member e across side S
    auto nslot = [&](int e) -> int {
      return S == 0 ? (e > 0 ? e - 1 : G) : S == 1 ? (e + 1 < ng ? e + 1 : G + 1) : S == 2 ? G + 2 + e : 2 * G + 2 + e;
    };
    unsigned inner = 0;
#pragma unroll
    for (int e = 0; e < G; ++e) {
      const int ixe = ix0 + e;
      const bool has = e < ng && (S == 0 ? ixe > 0 : S == 1 ? ixe + 1 < nx : S == 2 ? iy > 0 : iy + 1 < ny);
      if (has) inner |= 1u << e;
    }
    const unsigned bnd = (M.bc[S] != SDG_NEUMANN) ? (own & ~inner) : 0u;
    auto nbv = [&](int e) -> const double2* { return xs[nslot(e)]; };
    auto nbp = [&](int e) -> const double2* { return ps[nslot(e)]; };
    auto en = [&](int e) -> dd { return {es[nslot(e)], 0.0}; };
    auto sig = [&](int e) -> dd {
      const double ee = es[e], enb = es[nslot(e)];
      return dd_mul({4.0 * (ee > enb ? ee : enb), 0.0}, cpen);
    };
    auto sigb = [&](int e) -> dd { return dd_mul({8.0 * es[e], 0.0}, cpen); };
    if (inner) {
      const int t = (S & 1) ? 0 : 1;  // right/top side: the element is the minus side
      const double2* base = TA + (size_t)ext_face_base(dir, t) * NB * NB;
      blk_apply<NB, G, ABS>(base + (size_t)EXT_SELF12 * NB * NB, a, NB, inner, self, de, acc);
      blk_apply<NB, G, ABS>(base + (size_t)EXT_SELF3 * NB * NB, a, NB, inner, self, sig, acc);
      blk_apply<NB, G, ABS>(base + (size_t)EXT_NB1 * NB * NB, a, NB, inner, nbv, en, acc);
      blk_apply<NB, G, ABS>(base + (size_t)EXT_NB2 * NB * NB, a, NB, inner, nbv, de, acc);
      blk_apply<NB, G, ABS>(base + (size_t)EXT_NB3 * NB * NB, a, NB, inner, nbv, sig, acc);
      if (ph && NP > 0) {
        const double2* bb = TB + (size_t)ext_bface(dir, t) * NB * NPm;
        blk_apply<NP, G, ABS>(bb, a, NB, inner, selfp, one, acc);
        blk_apply<NP, G, ABS>(bb + (size_t)NB * NPm, a, NB, inner, nbp, one, acc);
      }
    }
    if (bnd) {
      blk_apply<NB, G, ABS>(TA + (size_t)(EXT_BND + 2 * S) * NB * NB, a, NB, bnd, self, de, acc);
      blk_apply<NB, G, ABS>(TA + (size_t)(EXT_BND + 2 * S + 1) * NB * NB, a, NB, bnd, self, sigb, acc);
      if (ph && NP > 0) blk_apply<NP, G, ABS>(TB + (size_t)(EXT_BBND + S) * NB * NPm, a, NB, bnd, selfp, one, acc);
    }
  }
  if (ph && NP > 0) blk_apply<NP, G, ABS>(TB + (size_t)EXT_BVOL * NB * NPm, a, NB, own, selfp, one, acc);
#pragma unroll
  for (int e = 0; e < G; ++e)
    if (e < ng) r[(off + iy * nx + ix0 + e) * NB + a] = acc[e].hi + acc[e].lo;
}

// Pressure rows: r = G - B^T u (ABS: |B^T||u|).  One 64-lane workgroup per
// (element, problem); every pressure row m has L = 64 / NP lanes (a power of
// two) that share its columns: lane (m, l) sums the columns b = l mod L of
// all of the row's blocks by Dot2 (the blocks' scalars are all 1), and the
// L partial sums are combined in double-FP64 through lane shuffles.
// Row-major B blocks: entry (a, m) at a * NP + m.
template <int NP>
struct PRowLanes {
  static constexpr int L = NP <= 1 ? 64 : NP <= 2 ? 32 : NP <= 4 ? 16 : NP <= 8 ? 8 : NP <= 16 ? 4 : NP <= 32 ? 2 : 1;
};
template <int K1, bool ABS>
__global__ __launch_bounds__(64) void ext_p_kernel(MeshDev M, const double* __restrict__ G,
                                                    const double* __restrict__ uh, const double* __restrict__ ul,
                                                    const double2* __restrict__ TBp, double* __restrict__ r) {
  constexpr int NB = 2 * K1 * K1, NP = (K1 - 1) * (K1 - 1), NPm = NP > 0 ? NP : 1;
  constexpr int L = PRowLanes<NPm>::L;
  __shared__ double2 us[5][NB];
  const int nel = M.nx * M.ny;
  const int e = blockIdx.x, pb = blockIdx.y;
  const int ix = e % M.nx, iy = e / M.nx;
  const int64_t off = (int64_t)pb * nel;
  int nbs[4];
  for (int S = 0; S < 4; ++S) nbs[S] = nbr(S, ix, iy, M.nx, M.ny);
  for (int i = threadIdx.x; i < 5 * NB; i += blockDim.x) {
    const int slot = i / NB, a = i - slot * NB;
    const int el = slot == 0 ? e : nbs[slot - 1];
    double2 v = make_double2(0.0, 0.0);
    if (el >= 0) {
      const int64_t g = (off + el) * NB + a;
      v = make_double2(uh[g], ul ? ul[g] : 0.0);
    }
    us[slot][a] = v;
  }
  __syncthreads();
  const int m = threadIdx.x / L, l = threadIdx.x - m * L;
  const bool row = m < NP;
  double sh = 0.0, sl = 0.0;
  // columns l, l + L, ... of block blk against slot vector u
  auto blk = [&](int bi, const double2* u) {
    const double2* T = TBp + (size_t)bi * NB * NPm;
    for (int b = l; b < NB; b += L) {
      const double2 c = T[(size_t)b * NPm + (row ? m : 0)];
      const double2 x = u[b];
      if (ABS) {
        sh += fabs(c.x) * fabs(x.x);
      } else {
        const double p = c.x * x.x;
        const double pe = __builtin_fma(c.x, x.x, -p);
        const double cross = __builtin_fma(c.x, x.y, c.y * x.x);
        const dd s2 = two_sum(sh, p);
        sh = s2.hi;
        sl += s2.lo + (pe + cross);
      }
    }
  };
  blk(EXT_BVOL, us[0]);
  for (int S = 0; S < 4; ++S) {
    const int dir = S >> 1;
    if (nbs[S] >= 0) {
      const int s = (S & 1) ? 0 : 1;  // the element's side of the face
      // self: pressure side s, velocity side s; neighbour: velocity side 1 - s
      blk(ext_bface(dir, s), us[0]);
      blk(ext_bface(dir, 1 - s) + 1, us[1 + S]);
    } else if (M.bc[S] != SDG_NEUMANN) {
      blk(EXT_BBND + S, us[0]);
    }
  }
  // combine the row's L lanes (adjacent lanes) in double-FP64
  dd t = ABS ? dd{sh, 0.0} : two_sum(sh, sl);
#pragma unroll
  for (int o = L / 2; o > 0; o >>= 1) {
    const double oh = __shfl_xor(t.hi, o, 64), ol = __shfl_xor(t.lo, o, 64);
    t = ABS ? dd{t.hi + oh, 0.0} : dd_add(t, {oh, ol});
  }
  if (!row || l != 0) return;
  dd acc = ABS ? dd{0.0, 0.0} : dd{G[(off + e) * NP + m], 0.0};
  acc = ABS ? dd{t.hi, 0.0} : dd_add(acc, dd_neg(t));
  r[(off + e) * NP + m] = acc.hi + acc.lo;
}

// (xh, xl) += d in double-FP64; xh then holds the rounded sum
__global__ void dd_accumulate_kernel(int64_t n, const double* __restrict__ d, double* __restrict__ xh,
                                     double* __restrict__ xl) {
  for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < n; g += (int64_t)gridDim.x * 256) {
    const dd s = two_sum(xh[g], d[g]);
    const dd t = fast_two_sum(s.hi, s.lo + xl[g]);
    xh[g] = t.hi;
    xl[g] = t.lo;
  }
}

template <int K1>
int ext_launch(const MeshDev& M, int nbatch, bool abs_mode, const double* eta, const double* F, const double* xh,
               const double* xl, const double* ph, const double* pl, const double* G, const ExtTables& T,
               double* r_u, double* r_p, hipStream_t s) {
  constexpr int GE = ExtGroup<K1>::G;
  constexpr int NTU = (2 * K1 * K1 + 63) / 64 * 64;  // one thread per row, whole wavefronts
  const dim3 grid_u(((M.nx + GE - 1) / GE) * M.ny, nbatch);
  if (abs_mode)
    hipLaunchKernelGGL((ext_u_kernel<K1, true>), grid_u, dim3(NTU), 0, s, M, eta, F, xh, xl, ph, pl, T.A, T.Bu,
                       T.cpen[0], T.cpen[1], r_u);
  else
    hipLaunchKernelGGL((ext_u_kernel<K1, false>), grid_u, dim3(NTU), 0, s, M, eta, F, xh, xl, ph, pl, T.A, T.Bu,
                       T.cpen[0], T.cpen[1], r_u);
  SDG_CHECK_LAUNCH();
  const dim3 grid(M.nx * M.ny, nbatch);
  if (r_p && K1 > 1) {
    if (abs_mode)
      hipLaunchKernelGGL((ext_p_kernel<K1, true>), grid, dim3(64), 0, s, M, G, xh, xl, T.Bp, r_p);
    else
      hipLaunchKernelGGL((ext_p_kernel<K1, false>), grid, dim3(64), 0, s, M, G, xh, xl, T.Bp, r_p);
    SDG_CHECK_LAUNCH();
  }
  return SDG_OK;
}

int ext_residual(const MeshDev& M, int k, int nbatch, bool abs_mode, const double* eta, const double* F,
                 const double* xh, const double* xl, const double* ph, const double* pl, const double* G,
                 const ExtTables& T, double* r_u, double* r_p, hipStream_t s) {
  if (M.nx * M.ny == 0 || nbatch == 0) return SDG_OK;
  switch (k) {
    case 1: return ext_launch<2>(M, nbatch, abs_mode, eta, F, xh, xl, ph, pl, G, T, r_u, r_p, s);
    case 2: return ext_launch<3>(M, nbatch, abs_mode, eta, F, xh, xl, ph, pl, G, T, r_u, r_p, s);
    case 3: return ext_launch<4>(M, nbatch, abs_mode, eta, F, xh, xl, ph, pl, G, T, r_u, r_p, s);
    case 4: return ext_launch<5>(M, nbatch, abs_mode, eta, F, xh, xl, ph, pl, G, T, r_u, r_p, s);
    case 5: return ext_launch<6>(M, nbatch, abs_mode, eta, F, xh, xl, ph, pl, G, T, r_u, r_p, s);
    case 6: return ext_launch<7>(M, nbatch, abs_mode, eta, F, xh, xl, ph, pl, G, T, r_u, r_p, s);
    default:
      set_error("order k out of range");
      return SDG_ERR_INVALID;
  }
}

int dd_accumulate(int64_t n, const double* d, double* xh, double* xl, hipStream_t s) {
  if (n <= 0) return SDG_OK;
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  hipLaunchKernelGGL(dd_accumulate_kernel, dim3((int)b), dim3(256), 0, s, n, d, xh, xl);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

}  // namespace sdg
