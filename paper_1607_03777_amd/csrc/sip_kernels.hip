// SIP viscous operator A (eq. stiffness_form) on the hierarchical Legendre
// basis, matrix-free, plus the divergence/gradient operators B^T, B
// (eq. divergence_form) and the right-hand-side assembly.
//
// Modal closed forms used here (orthonormal basis, c = 2/sqrt(hx hy)):
//  * volume: with D the 1D derivative matrix and S = D^T D,
//      y0 = eta [2(2/hx)^2 S_x u0 + (2/hy)^2 S_y u0 + (2/hx)(2/hy) D_y^T D_x u1]
//      y1 = eta [2(2/hy)^2 S_y u1 + (2/hx)^2 S_x u1 + (2/hx)(2/hy) D_x^T D_y u0]
//    (the strain terms 2 eta eps(u):eps(v) are Euclidean products of modal
//    derivative coefficients because the mass matrix is the identity);
//  * faces: every face function is a 1D Legendre series; a face with normal
//    direction n (hn = h_n, ht = the other) contributes to the adjacent
//    element y_d[..] += a_d e_end(.) + b_d d_end(.), where (a, b) come from
//    the traces t (values) and g (normal derivatives) of both sides:
//      J = t^- - t^+, sigma = {2 eta eps(u)} n^-, Q = -sigma + alpha J,
//    alpha = gamma_F C_F with gamma_F = 4 eta_F (interior, eta_F = max of
//    the neighbours, eq. eta_face) or 8 eta_K (Navier/Dirichlet), and
//    C_F = (k+1)^2/hn (discrete trace lemma).  Navier faces keep only the
//    normal component; a Dirichlet face is an interior face whose outer
//    trace is zero and whose inner viscosity counts twice (full, not
//    averaged, flux).
//
// The tile kernel stages a TX x TY block of elements in LDS, computes face
// traces from row/column pencils (halo neighbours read from HBM/L2), turns
// each face into coefficients with one thread per face, then applies the
// volume and face terms in a row pass and a column pass; all mode loops are
// unrolled over K1 = k+1 so the Legendre constants are immediates.
#include "sdg_common.h"
#include "sdg_kernels.h"

namespace sdg {

// Shapes of the 256-thread tile kernel (TX x TY elements per workgroup) per
// K1.  The operator's variant 0 is the wavefront kernel; variants 1..4 are
// these tile shapes (candidates for the autotuner), the first of which also
// serves the block and coarse-column modes.
constexpr int TILE_NV[8] = {0, 0, 4, 4, 4, 4, 4, 4};
constexpr int TILE_TX[8][4] = {{0}, {0}, {8, 16, 8, 16}, {8, 8, 16, 4}, {4, 8, 8, 4},
                               {4, 8, 8, 4}, {4, 4, 8, 2}, {4, 4, 2, 2}};
constexpr int TILE_TY[8][4] = {{0}, {0}, {8, 4, 4, 8}, {4, 8, 4, 4}, {4, 4, 2, 2},
                               {4, 2, 4, 2}, {2, 4, 2, 2}, {2, 4, 2, 4}};
template <int K1> struct Tile {
  static constexpr int TX = TILE_TX[K1][0], TY = TILE_TY[K1][0];
};

constexpr int NT = 256;  // threads per tile workgroup

// ---------------------------------------------------------------------------
// face coefficients from traces
// tr layout per face: [side s][comp d][w][m], w = 0 trace value, 1 normal
// derivative; the output uses the same slots with w = 0 -> a, 1 -> b.
// ---------------------------------------------------------------------------
// Coefficients of one interior face, stored mode by mode into the face
// record f (sides in `sides`: bit 0 the minus side, bit 1 the plus side), so
// that only the traces stay live in registers.
template <int K1, int DIR, typename T>
__device__ __forceinline__ void interior_coefs(const T (&tm)[2][K1], const T (&gm)[2][K1],
                                               const T (&tp)[2][K1], const T (&gp)[2][K1],
                                               T etam, T etap, T alpha, T hn, T ht, T* f, int sides) {
  constexpr int N = DIR, TT = 1 - DIR;
  const T c2n = T(2) / hn, c2t = T(2) / ht;
#pragma unroll
  for (int m = 0; m < K1; ++m) {
    T dtm = 0, dtp = 0, dtj = 0;
#pragma unroll
    for (int j = 0; j < K1; ++j) {
      if (d_nz(m, j)) {
        dtm += T(d_val(m, j)) * tm[N][j];
        dtp += T(d_val(m, j)) * tp[N][j];
      }
      if (d_nz(j, m)) dtj += T(d_val(j, m)) * (tm[TT][j] - tp[TT][j]);
    }
    const T jn = tm[N][m] - tp[N][m];
    const T jt = tm[TT][m] - tp[TT][m];
    const T sn = c2n * (etam * gm[N][m] + etap * gp[N][m]);
    const T st = T(0.5) * (c2t * (etam * dtm + etap * dtp) + c2n * (etam * gm[TT][m] + etap * gp[TT][m]));
    const T qn = -sn + alpha * jn;
    const T qt = -st + alpha * jt;
    if (sides & 1) {
      f[((0 * 2 + N) * 2 + 0) * K1 + m] = c2n * (qn - etam / ht * dtj);
      f[((0 * 2 + N) * 2 + 1) * K1 + m] = -c2n * c2n * etam * jn;
      f[((0 * 2 + TT) * 2 + 0) * K1 + m] = c2n * qt;
      f[((0 * 2 + TT) * 2 + 1) * K1 + m] = -c2n / hn * etam * jt;
    }
    if (sides & 2) {
      f[((1 * 2 + N) * 2 + 0) * K1 + m] = -c2n * (qn + etap / ht * dtj);
      f[((1 * 2 + N) * 2 + 1) * K1 + m] = -c2n * c2n * etap * jn;
      f[((1 * 2 + TT) * 2 + 0) * K1 + m] = -c2n * qt;
      f[((1 * 2 + TT) * 2 + 1) * K1 + m] = -c2n / hn * etap * jt;
    }
  }
}

template <int K1, typename T>
__device__ __forceinline__ void zero_sides(T* f, int sides) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
    if (sides & (1 << s))
#pragma unroll
      for (int z = 0; z < 4 * K1; ++z) f[s * 4 * K1 + z] = T(0);
}

// Turns the traces of face record f into its coefficients, in place (the
// traces are read into registers first).
// kind: F_INTERIOR, or the boundary kind with `side` the present side.
// isolate: each side sees a zero neighbour (diagonal blocks).
// skip_interior: interior faces contribute nothing (continuous Q1 fields).
template <int K1, int DIR, typename T>
__device__ void face_coefs(T* f, int kind, int side, T etam, T etap, T hn, T ht, bool isolate,
                           bool skip_interior) {
  T tm[2][K1], gm[2][K1], tp[2][K1], gp[2][K1];
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int m = 0; m < K1; ++m) {
      tm[d][m] = f[((0 * 2 + d) * 2 + 0) * K1 + m];
      gm[d][m] = f[((0 * 2 + d) * 2 + 1) * K1 + m];
      tp[d][m] = f[((1 * 2 + d) * 2 + 0) * K1 + m];
      gp[d][m] = f[((1 * 2 + d) * 2 + 1) * K1 + m];
    }
  const T kk = T(K1 * K1);
  if (kind == F_INTERIOR) {
    if (skip_interior) {
      zero_sides<K1, T>(f, 3);
    } else {
      const T alpha = T(4) * (etam > etap ? etam : etap) * kk / hn;
      if (!isolate) {
        interior_coefs<K1, DIR, T>(tm, gm, tp, gp, etam, etap, alpha, hn, ht, f, 3);
      } else {
        T z[2][K1];
#pragma unroll
        for (int d = 0; d < 2; ++d)
#pragma unroll
          for (int m = 0; m < K1; ++m) z[d][m] = T(0);
        interior_coefs<K1, DIR, T>(tm, gm, z, z, etam, etap, alpha, hn, ht, f, 1);
        interior_coefs<K1, DIR, T>(z, z, tp, gp, etam, etap, alpha, hn, ht, f, 2);
      }
    }
  } else if (kind == F_NAVIER) {
    constexpr int N = DIR;
    const T eta = side == 0 ? etam : etap;
    const T alpha = T(8) * eta * kk / hn;
    const T sgn = side == 0 ? T(1) : T(-1);
    const T c2n = T(2) / hn;
    const T w = T(4) * eta / hn;
    zero_sides<K1, T>(f, 3);
#pragma unroll
    for (int m = 0; m < K1; ++m) {
      const T t = side == 0 ? tm[N][m] : tp[N][m];
      const T g = side == 0 ? gm[N][m] : gp[N][m];
      f[((side * 2 + N) * 2 + 0) * K1 + m] = c2n * (alpha * t - sgn * w * g);
      f[((side * 2 + N) * 2 + 1) * K1 + m] = -c2n * sgn * w * t;
    }
  } else if (kind == F_DIRICHLET) {
    T z[2][K1];
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int m = 0; m < K1; ++m) z[d][m] = T(0);
    const T eta2 = T(2) * (side == 0 ? etam : etap);
    const T alpha = T(4) * eta2 * kk / hn;
    zero_sides<K1, T>(f, side == 0 ? 2 : 1);
    if (side == 0)
      interior_coefs<K1, DIR, T>(tm, gm, z, z, eta2, T(0), alpha, hn, ht, f, 1);
    else
      interior_coefs<K1, DIR, T>(z, z, tp, gp, T(0), eta2, alpha, hn, ht, f, 2);
  } else {
    zero_sides<K1, T>(f, 3);
  }
}

// Coefficients of mode m of one face (the tile kernel's face phase: one
// thread per face and mode).  f holds the face's traces; sdm the derivative
// matrix D(m, i) (zero off its pattern).  o[(s * 2 + d) * 2 + w] receives
// a (w = 0) and b (w = 1) of side s, component d; the same formulas as
// face_coefs, written for a runtime mode index.
template <int K1, int DIR, typename T>
__device__ __forceinline__ void face_mode(const T* __restrict__ f, int m, int kind, int side, T etam, T etap,
                                          T hn, T ht, bool isolate, bool skip_interior,
                                          const T* __restrict__ sdm, T (&o)[8]) {
  constexpr int N = DIR, TT = 1 - DIR;
#pragma unroll
  for (int z = 0; z < 8; ++z) o[z] = T(0);
  if (kind < 0 || kind == F_NEUMANN || (kind == F_INTERIOR && skip_interior)) return;
  const T kk = T(K1 * K1);
  const T c2n = T(2) / hn, c2t = T(2) / ht;
  auto at = [&](int s, int d, int w, int j) { return f[((s * 2 + d) * 2 + w) * K1 + j]; };
  if (kind == F_NAVIER) {
    const T eta = side == 0 ? etam : etap;
    const T alpha = T(8) * eta * kk / hn;
    const T sgn = side == 0 ? T(1) : T(-1);
    const T w = T(4) * eta / hn;
    const T t = at(side, N, 0, m), g = at(side, N, 1, m);
    o[(side * 2 + N) * 2 + 0] = c2n * (alpha * t - sgn * w * g);
    o[(side * 2 + N) * 2 + 1] = -c2n * sgn * w * t;
    return;
  }
  // interior-type face: mm/mp switch the minus/plus traces on or off,
  // `sides` selects the outputs kept
  auto core = [&](T mm, T mp, T em, T ep, T alpha, int sides) {
    T dtm = 0, dtp = 0, dtj = 0;
    for (int j = m + 1; j < K1; j += 2) {
      const T c = sdm[m * K1 + j];
      dtm += c * (mm * at(0, N, 0, j));
      dtp += c * (mp * at(1, N, 0, j));
    }
    for (int j = (m & 1) ^ 1; j < m; j += 2)
      dtj += sdm[j * K1 + m] * (mm * at(0, TT, 0, j) - mp * at(1, TT, 0, j));
    const T jn = mm * at(0, N, 0, m) - mp * at(1, N, 0, m);
    const T jt = mm * at(0, TT, 0, m) - mp * at(1, TT, 0, m);
    const T sn = c2n * (em * (mm * at(0, N, 1, m)) + ep * (mp * at(1, N, 1, m)));
    const T st = T(0.5) * (c2t * (em * dtm + ep * dtp) +
                           c2n * (em * (mm * at(0, TT, 1, m)) + ep * (mp * at(1, TT, 1, m))));
    const T qn = -sn + alpha * jn;
    const T qt = -st + alpha * jt;
    if (sides & 1) {
      o[(0 * 2 + N) * 2 + 0] = c2n * (qn - em / ht * dtj);
      o[(0 * 2 + N) * 2 + 1] = -c2n * c2n * em * jn;
      o[(0 * 2 + TT) * 2 + 0] = c2n * qt;
      o[(0 * 2 + TT) * 2 + 1] = -c2n / hn * em * jt;
    }
    if (sides & 2) {
      o[(1 * 2 + N) * 2 + 0] = -c2n * (qn + ep / ht * dtj);
      o[(1 * 2 + N) * 2 + 1] = -c2n * c2n * ep * jn;
      o[(1 * 2 + TT) * 2 + 0] = -c2n * qt;
      o[(1 * 2 + TT) * 2 + 1] = -c2n / hn * ep * jt;
    }
  };
  if (kind == F_INTERIOR) {
    const T alpha = T(4) * (etam > etap ? etam : etap) * kk / hn;
    if (!isolate) {
      core(T(1), T(1), etam, etap, alpha, 3);
    } else {
      core(T(1), T(0), etam, etap, alpha, 1);
      core(T(0), T(1), etam, etap, alpha, 2);
    }
  } else {  // Dirichlet: zero outer trace, the present side's viscosity counted twice
    const T eta2 = T(2) * (side == 0 ? etam : etap);
    const T alpha = T(4) * eta2 * kk / hn;
    if (side == 0) core(T(1), T(0), eta2, T(0), alpha, 1);
    else core(T(0), T(1), T(0), eta2, alpha, 2);
  }
}

// ---------------------------------------------------------------------------
// tile kernel
// ---------------------------------------------------------------------------
enum ApplyMode { M_APPLY = 0, M_RESID = 1, M_BLOCKCOL = 2, M_COARSECOL = 3, M_RESQ1 = 4 };

// MODE M_APPLY / M_RESID: tile grid over the mesh (blockIdx.y = problem).
// MODE M_BLOCKCOL: TX = TY = 1, blockIdx.x indexes `elems` (global element
//   ids pb*nel + e); loops over the NB unit columns, writes out_mat[list][a][col].
// MODE M_COARSECOL: tile grid; loops over the 8 hat columns, writes
//   out_mat[pb*nel + e][r][col].
template <int K1, int MODE, typename T, int TX, int TY>
__global__ __launch_bounds__(NT, (K1 >= 7 ? 3 : 1)) void sip_tile_kernel(MeshDev M, const T* __restrict__ u,
                                                      const T* __restrict__ bvec, T* __restrict__ y,
                                                      const double* __restrict__ eta_all,
                                                      double* __restrict__ out_mat,
                                                      const int* __restrict__ elems,
                                                      int64_t vec_stride) {
  constexpr int KK = K1 * K1, NB = 2 * KK, E = TX * TY;
  constexpr int NFV = (TX + 1) * TY, NFH = TX * (TY + 1);
  constexpr int FW = 8 * K1;
  constexpr int FS = FW + 1;  // face record stride: odd, so one-thread-per-face access avoids bank conflicts
  constexpr int EW = TX + 2;
  __shared__ T su[E * NB];
  __shared__ T sdm[K1 * K1];  // derivative matrix D(m, i) (zero off its pattern)
  __shared__ T sy[E * NB];
  __shared__ T sf[(NFV + NFH) * FS];
  __shared__ T seta[(TY + 2) * EW];

  const int tid = threadIdx.x;
  const int nx = M.nx, ny = M.ny;
  int ix0, iy0;
  int64_t pb;
  if (MODE == M_BLOCKCOL) {
    const int g = elems[blockIdx.x];
    pb = g / (nx * ny);
    const int e = g - (int)pb * nx * ny;
    ix0 = e % nx;
    iy0 = e / nx;
  } else {
    const int ntx = (nx + TX - 1) / TX;
    ix0 = (blockIdx.x % ntx) * TX;
    iy0 = (blockIdx.x / ntx) * TY;
    pb = blockIdx.y;
    // a converged problem of a batched CG iteration (the whole block)
    if ((MODE == M_APPLY || MODE == M_RESID) && M.active && !M.active[pb]) return;
  }
  const double* eta = eta_all + pb * (int64_t)nx * ny;
  if (MODE == M_APPLY || MODE == M_RESID) {
    u += pb * vec_stride;
    y += pb * vec_stride;
    if (MODE == M_RESID) bvec += pb * vec_stride;
  }
  const T hx = T(M.hx), hy = T(M.hy);

  // ---- S0: load viscosity (tile + halo ring) and the tile's coefficients
  for (int q = tid; q < (TY + 2) * EW; q += NT) {
    const int ix = ix0 - 1 + q % EW, iy = iy0 - 1 + q / EW;
    seta[q] = (ix >= 0 && ix < nx && iy >= 0 && iy < ny) ? T(eta[(int64_t)iy * nx + ix]) : T(0);
  }
  for (int q = tid; q < K1 * K1; q += NT) {
    const int m = q / K1, i = q % K1;
    sdm[q] = d_nz(m, i) ? T(d_val(m, i)) : T(0);
  }
  constexpr int NCOLS = (MODE == M_BLOCKCOL) ? NB : (MODE == M_COARSECOL ? 8 : 1);
  for (int col = 0; col < NCOLS; ++col) {
  for (int q = tid; q < E * NB; q += NT) {
    const int ty = q / (TX * NB), rem = q - ty * TX * NB, tx = rem / NB, a = rem - tx * NB;
    const int ix = ix0 + tx, iy = iy0 + ty;
    T v = T(0);
    if (ix < nx && iy < ny) {
      if (MODE == M_APPLY || MODE == M_RESID) {
        v = u[((int64_t)iy * nx + ix0) * NB + rem];
      } else if (MODE == M_BLOCKCOL) {
        v = (a == col) ? T(1) : T(0);
      } else {  // hat function (vertex va, vb; component cc) as modal Q1 coefficients
        const int vtx = col >> 1, cc = col & 1, va = vtx & 1, vb = vtx >> 1;
        const int d = a / KK, j = (a % KK) / K1, i = a % K1;
        if (d == cc && i <= 1 && j <= 1) {
          const double cij = sqrt((2.0 * i + 1.0) * (2.0 * j + 1.0) / (M.hx * M.hy));
          const double si = (i == 0) ? 1.0 : (va ? 1.0 : -1.0);
          const double sj = (j == 0) ? 1.0 : (vb ? 1.0 : -1.0);
          v = T(0.25 * si * sj / cij);
        }
      }
    }
    su[q] = v;
  }
  __syncthreads();

  // ---- S1: traces of rows (x-faces) and columns (y-faces), derivatives for
  // the mixed terms.  Row items: tx in [-1, TX], ty in [0, TY), d, j.
  {
    constexpr int NROW = (TX + 2) * TY * 2 * K1;
    constexpr int NCOL = TX * (TY + 2) * 2 * K1;
    const bool halo_ok = (MODE == M_APPLY || MODE == M_RESID);
    for (int q = tid; q < NROW + NCOL; q += NT) {
      if (q < NROW) {
        const int j = q % K1, d = (q / K1) & 1, r = q / (2 * K1);
        const int tx = r % (TX + 2) - 1, ty = r / (TX + 2);
        const int ix = ix0 + tx, iy = iy0 + ty;
        T row[K1];
        const bool inside = (tx >= 0 && tx < TX);
        const bool exists = (ix >= 0 && ix < nx && iy < ny);
        if (inside) {
          const T* p = su + (ty * TX + tx) * NB + d * KK + j * K1;
#pragma unroll
          for (int i = 0; i < K1; ++i) row[i] = p[i];
        } else if (exists && halo_ok) {
          const T* p = u + ((int64_t)iy * nx + ix) * NB + d * KK + j * K1;
#pragma unroll
          for (int i = 0; i < K1; ++i) row[i] = p[i];
        } else {
#pragma unroll
          for (int i = 0; i < K1; ++i) row[i] = T(0);
        }
        T tl = 0, gl = 0, tr = 0, gr = 0;
#pragma unroll
        for (int i = 0; i < K1; ++i) {
          tl += T(e_end(i, 0)) * row[i];
          gl += T(d_end(i, 0)) * row[i];
          tr += T(e_end(i, 1)) * row[i];
          gr += T(d_end(i, 1)) * row[i];
        }
        // left end belongs to face fx = tx (plus side), right end to fx = tx+1 (minus side)
        if (tx >= 0) {
          T* f = sf + (ty * (TX + 1) + tx) * FS;
          f[((1 * 2 + d) * 2 + 0) * K1 + j] = tl;
          f[((1 * 2 + d) * 2 + 1) * K1 + j] = gl;
        }
        if (tx < TX) {
          T* f = sf + (ty * (TX + 1) + tx + 1) * FS;
          f[((0 * 2 + d) * 2 + 0) * K1 + j] = tr;
          f[((0 * 2 + d) * 2 + 1) * K1 + j] = gr;
        }
      } else {
        const int qq = q - NROW;
        const int i = qq % K1, d = (qq / K1) & 1, r = qq / (2 * K1);
        const int tx = r % TX, ty = r / TX - 1;
        const int ix = ix0 + tx, iy = iy0 + ty;
        T cl[K1];
        const bool inside = (ty >= 0 && ty < TY);
        const bool exists = (iy >= 0 && iy < ny && ix < nx);
        if (inside) {
          const T* p = su + (ty * TX + tx) * NB + d * KK + i;
#pragma unroll
          for (int jj = 0; jj < K1; ++jj) cl[jj] = p[jj * K1];
        } else if (exists && halo_ok) {
          const T* p = u + ((int64_t)iy * nx + ix) * NB + d * KK + i;
#pragma unroll
          for (int jj = 0; jj < K1; ++jj) cl[jj] = p[jj * K1];
        } else {
#pragma unroll
          for (int jj = 0; jj < K1; ++jj) cl[jj] = T(0);
        }
        T tb = 0, gb = 0, tt = 0, gt = 0;
#pragma unroll
        for (int jj = 0; jj < K1; ++jj) {
          tb += T(e_end(jj, 0)) * cl[jj];
          gb += T(d_end(jj, 0)) * cl[jj];
          tt += T(e_end(jj, 1)) * cl[jj];
          gt += T(d_end(jj, 1)) * cl[jj];
        }
        if (ty >= 0) {
          T* f = sf + (NFV + ty * TX + tx) * FS;
          f[((1 * 2 + d) * 2 + 0) * K1 + i] = tb;
          f[((1 * 2 + d) * 2 + 1) * K1 + i] = gb;
        }
        if (ty < TY) {
          T* f = sf + (NFV + (ty + 1) * TX + tx) * FS;
          f[((0 * 2 + d) * 2 + 0) * K1 + i] = tt;
          f[((0 * 2 + d) * 2 + 1) * K1 + i] = gt;
        }
      }
    }
  }
  __syncthreads();

  // ---- S2: one thread per face and mode: traces -> coefficients.  All
  // items read their traces before any item overwrites them in place.
  {
    constexpr int NF = NFV + NFH, NITEM = NF * K1, NIT = (NITEM + NT - 1) / NT;
    T ov[NIT][8];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int q = it * NT + tid;
#pragma unroll
      for (int z = 0; z < 8; ++z) ov[it][z] = T(0);
      if (q >= NITEM) continue;
      const int fq = q / K1, m = q - fq * K1;
      const T* f = sf + fq * FS;
      if (fq < NFV) {
        const int ty = fq / (TX + 1), fx = fq - ty * (TX + 1);
        const int iy = iy0 + ty, ixm = ix0 + fx - 1, ixp = ix0 + fx;
        const bool pm = (ixm >= 0 && ixm < nx), pp = (ixp < nx);
        int kind = -1, side = 0;
        if (iy < ny) {
          if (pm && pp) kind = F_INTERIOR;
          else if (!pm && pp) { kind = M.bc[0]; side = 1; }
          else if (pm && ixp == nx) { kind = M.bc[1]; side = 0; }
        }
        const T em = seta[(ty + 1) * EW + fx], ep = seta[(ty + 1) * EW + fx + 1];
        face_mode<K1, 0, T>(f, m, kind, side, em, ep, hx, hy, MODE == M_BLOCKCOL, MODE == M_COARSECOL, sdm,
                            ov[it]);
      } else {
        const int qq = fq - NFV;
        const int fy = qq / TX, tx = qq - fy * TX;
        const int ix = ix0 + tx, iym = iy0 + fy - 1, iyp = iy0 + fy;
        const bool pm = (iym >= 0 && iym < ny), pp = (iyp < ny);
        int kind = -1, side = 0;
        if (ix < nx) {
          if (pm && pp) kind = F_INTERIOR;
          else if (!pm && pp) { kind = M.bc[2]; side = 1; }
          else if (pm && iyp == ny) { kind = M.bc[3]; side = 0; }
        }
        const T em = seta[fy * EW + tx + 1], ep = seta[(fy + 1) * EW + tx + 1];
        face_mode<K1, 1, T>(f, m, kind, side, em, ep, hy, hx, MODE == M_BLOCKCOL, MODE == M_COARSECOL, sdm,
                            ov[it]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int q = it * NT + tid;
      if (q >= NITEM) continue;
      const int fq = q / K1, m = q - fq * K1;
      T* f = sf + fq * FS;
#pragma unroll
      for (int z = 0; z < 8; ++z) f[z * K1 + m] = ov[it][z];
    }
  }
  __syncthreads();

  // ---- S3: row pass (x-direction volume terms, x-faces, mixed term of y1)
  const T cxx = T(4) / (hx * hx), cyy = T(4) / (hy * hy), cxy = T(4) / (hx * hy);
  for (int q = tid; q < E * 2 * K1; q += NT) {
    const int j = q % K1, d = (q / K1) & 1, el = q / (2 * K1);
    const int tx = el % TX, ty = el / TX;
    const T et = seta[(ty + 1) * EW + tx + 1];
    const T* rp = su + el * NB + d * KK + j * K1;
    T row[K1], out[K1];
#pragma unroll
    for (int i = 0; i < K1; ++i) row[i] = rp[i];
    const T cx = (d == 0 ? T(2) : T(1)) * et * cxx;
#pragma unroll
    for (int i = 0; i < K1; ++i) {
      T s = 0;
#pragma unroll
      for (int l = 0; l < K1; ++l)
        if (s_nz(i, l)) s += T(s_val(i, l)) * row[l];
      out[i] = cx * s;
    }
    if (d == 1) {  // D_x^T (D_y u0), row j; (D_y u0)[j][m] = sum_{l > j} D(j, l) u0[l][m]
      const T* u0 = su + el * NB;
      T r0[K1];
#pragma unroll
      for (int m = 0; m < K1; ++m) r0[m] = T(0);
      for (int l = j + 1; l < K1; l += 2) {
        const T c = sdm[j * K1 + l];
#pragma unroll
        for (int m = 0; m < K1; ++m) r0[m] += c * u0[l * K1 + m];
      }
#pragma unroll
      for (int i = 0; i < K1; ++i) {
        T s = 0;
#pragma unroll
        for (int m = 0; m < K1; ++m)
          if (d_nz(m, i)) s += T(d_val(m, i)) * r0[m];
        out[i] += et * cxy * s;
      }
    }
    const T* fl = sf + (ty * (TX + 1) + tx) * FS;      // plus side of left face
    const T* fr = sf + (ty * (TX + 1) + tx + 1) * FS;  // minus side of right face
    const T al = fl[((1 * 2 + d) * 2 + 0) * K1 + j], bl = fl[((1 * 2 + d) * 2 + 1) * K1 + j];
    const T ar = fr[((0 * 2 + d) * 2 + 0) * K1 + j], br = fr[((0 * 2 + d) * 2 + 1) * K1 + j];
    T* op = sy + el * NB + d * KK + j * K1;
#pragma unroll
    for (int i = 0; i < K1; ++i)
      op[i] = out[i] + al * T(e_end(i, 0)) + bl * T(d_end(i, 0)) + ar * T(e_end(i, 1)) +
              br * T(d_end(i, 1));
  }
  __syncthreads();

  // ---- S4: column pass (y-direction volume terms, y-faces, mixed term of y0)
  for (int q = tid; q < E * 2 * K1; q += NT) {
    const int i = q % K1, d = (q / K1) & 1, el = q / (2 * K1);
    const int tx = el % TX, ty = el / TX;
    const T et = seta[(ty + 1) * EW + tx + 1];
    const T* cp = su + el * NB + d * KK + i;
    T cl[K1], out[K1];
#pragma unroll
    for (int jj = 0; jj < K1; ++jj) cl[jj] = cp[jj * K1];
    const T cy = (d == 1 ? T(2) : T(1)) * et * cyy;
#pragma unroll
    for (int jj = 0; jj < K1; ++jj) {
      T s = 0;
#pragma unroll
      for (int l = 0; l < K1; ++l)
        if (s_nz(jj, l)) s += T(s_val(jj, l)) * cl[l];
      out[jj] = cy * s;
    }
    if (d == 0) {  // D_y^T (D_x u1), column i; (D_x u1)[m][i] = sum_{l > i} D(i, l) u1[m][l]
      const T* u1 = su + el * NB + KK;
      T c1[K1];
#pragma unroll
      for (int m = 0; m < K1; ++m) c1[m] = T(0);
      for (int l = i + 1; l < K1; l += 2) {
        const T c = sdm[i * K1 + l];
#pragma unroll
        for (int m = 0; m < K1; ++m) c1[m] += c * u1[m * K1 + l];
      }
#pragma unroll
      for (int jj = 0; jj < K1; ++jj) {
        T s = 0;
#pragma unroll
        for (int m = 0; m < K1; ++m)
          if (d_nz(m, jj)) s += T(d_val(m, jj)) * c1[m];
        out[jj] += et * cxy * s;
      }
    }
    const T* fb = sf + (NFV + ty * TX + tx) * FS;        // plus side of bottom face
    const T* ft = sf + (NFV + (ty + 1) * TX + tx) * FS;  // minus side of top face
    const T ab = fb[((1 * 2 + d) * 2 + 0) * K1 + i], bb = fb[((1 * 2 + d) * 2 + 1) * K1 + i];
    const T at = ft[((0 * 2 + d) * 2 + 0) * K1 + i], bt = ft[((0 * 2 + d) * 2 + 1) * K1 + i];
    // the result goes to sy (this thread's own column): su stays intact for
    // the other columns' mixed terms
    T* sp = sy + el * NB + d * KK + i;
#pragma unroll
    for (int jj = 0; jj < K1; ++jj)
      sp[jj * K1] = sp[jj * K1] + out[jj] + ab * T(e_end(jj, 0)) + bb * T(d_end(jj, 0)) +
                    at * T(e_end(jj, 1)) + bt * T(d_end(jj, 1));
  }
  __syncthreads();

  // ---- S5: write out
  if (MODE == M_APPLY || MODE == M_RESID) {
    for (int q = tid; q < E * NB; q += NT) {
      const int ty = q / (TX * NB), rem = q - ty * TX * NB, tx = rem / NB;
      const int ix = ix0 + tx, iy = iy0 + ty;
      if (ix < nx && iy < ny) {
        const int64_t g = ((int64_t)iy * nx + ix0) * NB + rem;
        y[g] = (MODE == M_RESID) ? bvec[g] - sy[q] : sy[q];
      }
    }
  } else if (MODE == M_BLOCKCOL) {
    for (int a = tid; a < NB; a += NT) out_mat[((int64_t)blockIdx.x * NB + a) * NB + col] = double(sy[a]);
  } else {  // M_COARSECOL: project the Q1 modes with P_cd^T -> local nodal row (vtx', comp')
    for (int q = tid; q < E * 8; q += NT) {
      const int el = q / 8, r = q % 8, vtx = r >> 1, cc = r & 1, va = vtx & 1, vb = vtx >> 1;
      const int tx = el % TX, ty = el / TX;
      const int ix = ix0 + tx, iy = iy0 + ty;
      if (ix < nx && iy < ny) {
        double s = 0;
        for (int j = 0; j < 2; ++j)
          for (int i = 0; i < 2; ++i) {
            const double cij = sqrt((2.0 * i + 1.0) * (2.0 * j + 1.0) / (M.hx * M.hy));
            const double si = (i == 0) ? 1.0 : (va ? 1.0 : -1.0);
            const double sj = (j == 0) ? 1.0 : (vb ? 1.0 : -1.0);
            s += 0.25 * si * sj / cij * double(sy[el * NB + cc * KK + j * K1 + i]);
          }
        const int64_t e = (int64_t)iy * nx + ix + pb * (int64_t)nx * ny;
        out_mat[(e * 8 + r) * 8 + col] = s;
      }
    }
  }
  __syncthreads();
  }  // column loop
}

// ---------------------------------------------------------------------------
// Wavefront kernel (apply / residual): one 64-lane wavefront per tile of
// WT::TX x WT::TY elements, K1 lanes per element.  Lane (el, j) first holds
// row j of both components of its element (x-direction work: x-face traces,
// S_x), then mode j of its element's two x-faces (face coefficients applied
// to its own row); then, through the element staged in LDS, column j
// (y-direction work: y-face traces, S_y, the mixed term of y0), then mode j
// of the two y-faces (applied to its own column) and the mixed term of y1;
// the column results come back to the row lanes through LDS.  The x-faces
// and the y-faces take turns in one face buffer, so a wavefront holds about
// 10 KB of LDS at k = 4 in FP64 and sixteen of them fit a compute unit.
// Traces of neighbours outside the tile are formed by the edge lanes from
// their rows/columns in HBM/L2, requested together with the tile's own rows
// so that their latency overlaps; every face slot is written in each phase
// (zeros where the mesh ends).  The few entries of the derivative matrix D a
// lane needs (row and column of its mode j) are held in registers.
// ---------------------------------------------------------------------------
template <int K1> struct WaveTile;
template <> struct WaveTile<2> { static constexpr int TX = 8, TY = 4; };
template <> struct WaveTile<3> { static constexpr int TX = 7, TY = 3; };
template <> struct WaveTile<4> { static constexpr int TX = 4, TY = 4; };
template <> struct WaveTile<5> { static constexpr int TX = 4, TY = 3; };
template <> struct WaveTile<6> { static constexpr int TX = 5, TY = 2; };
template <> struct WaveTile<7> { static constexpr int TX = 3, TY = 3; };

// LDS layout of the wavefront kernel.  The staged element is stored
// transposed, su[(d K1 + col) S + el K1 + row], so that the row pass (lane
// (el, j) touching row j) addresses consecutive words and the column pass
// (lane (el, i) touching column i) addresses el K1 + i S; a face record is
// split by slot, sf[slot Q + face K1 + mode], so that the lanes of adjacent
// elements touch consecutive words.  S and Q are the strides with the fewest
// LDS bank conflicts (32 and 64 banks of 4 bytes) among those that keep the
// workgroups per compute unit of the element-major layout.
template <int K1, typename T> struct WaveLds;
template <> struct WaveLds<2, double> { static constexpr int S = 65, Q = 80; };
template <> struct WaveLds<3, double> { static constexpr int S = 65, Q = 84; };
template <> struct WaveLds<4, double> { static constexpr int S = 65, Q = 80; };
template <> struct WaveLds<5, double> { static constexpr int S = 63, Q = 80; };
template <> struct WaveLds<6, double> { static constexpr int S = 65, Q = 90; };
template <> struct WaveLds<7, double> { static constexpr int S = 63, Q = 84; };
template <> struct WaveLds<2, float> { static constexpr int S = 65, Q = 80; };
template <> struct WaveLds<3, float> { static constexpr int S = 65, Q = 84; };
template <> struct WaveLds<4, float> { static constexpr int S = 65, Q = 80; };
template <> struct WaveLds<5, float> { static constexpr int S = 62, Q = 80; };
template <> struct WaveLds<6, float> { static constexpr int S = 65, Q = 90; };
template <> struct WaveLds<7, float> { static constexpr int S = 63, Q = 84; };

// Face coefficients at mode m (the formulas of face_mode above), with the
// record's slots QS apart and the derivative entries taken from registers:
// up[t] = D(m, m+1+2t),
// dn[t] = D(m-1-2t, m); ihn = 1/hn and iht = 1/ht are passed in, so the
// coefficients take no divisions.
template <int K1, int DIR, int QS, typename T>
__device__ __forceinline__ void face_mode_w(const T* __restrict__ f, int m, int kind, int side, T etam, T etap,
                                            T ihn, T iht, const T (&up)[K1 / 2], const T (&dn)[K1 / 2],
                                            T (&o)[8]) {
  constexpr int N = DIR, TT = 1 - DIR;
#pragma unroll
  for (int z = 0; z < 8; ++z) o[z] = T(0);
  if (kind < 0 || kind == F_NEUMANN) return;
  const T kk = T(K1 * K1);
  const T c2n = T(2) * ihn, c2t = T(2) * iht;
  auto at = [&](int s, int d, int w, int j) { return f[((s * 2 + d) * 2 + w) * QS + j]; };
  if (kind == F_NAVIER) {
    const T eta = side == 0 ? etam : etap;
    const T alpha = T(8) * eta * kk * ihn;
    const T sgn = side == 0 ? T(1) : T(-1);
    const T w = T(4) * eta * ihn;
    const T t = at(side, N, 0, m), g = at(side, N, 1, m);
    o[(side * 2 + N) * 2 + 0] = c2n * (alpha * t - sgn * w * g);
    o[(side * 2 + N) * 2 + 1] = -c2n * sgn * w * t;
    return;
  }
  // interior face; a Dirichlet face switches the outer trace off and counts
  // the present side's viscosity twice
  T mm = T(1), mp = T(1), em = etam, ep = etap, alpha;
  int sides = 3;
  if (kind == F_INTERIOR) {
    alpha = T(4) * (etam > etap ? etam : etap) * kk * ihn;
  } else {
    const T eta2 = T(2) * (side == 0 ? etam : etap);
    alpha = T(4) * eta2 * kk * ihn;
    if (side == 0) {
      mp = T(0);
      em = eta2;
      ep = T(0);
      sides = 1;
    } else {
      mm = T(0);
      em = T(0);
      ep = eta2;
      sides = 2;
    }
  }
  T dtm = 0, dtp = 0, dtj = 0;
#pragma unroll
  for (int t = 0; t < K1 / 2; ++t) {
    const int jp = m + 1 + 2 * t, jn = m - 1 - 2 * t;
    if (jp < K1) {
      dtm += up[t] * (mm * at(0, N, 0, jp));
      dtp += up[t] * (mp * at(1, N, 0, jp));
    }
    if (jn >= 0) dtj += dn[t] * (mm * at(0, TT, 0, jn) - mp * at(1, TT, 0, jn));
  }
  const T jn = mm * at(0, N, 0, m) - mp * at(1, N, 0, m);
  const T jt = mm * at(0, TT, 0, m) - mp * at(1, TT, 0, m);
  const T sn = c2n * (em * (mm * at(0, N, 1, m)) + ep * (mp * at(1, N, 1, m)));
  const T st = T(0.5) * (c2t * (em * dtm + ep * dtp) +
                         c2n * (em * (mm * at(0, TT, 1, m)) + ep * (mp * at(1, TT, 1, m))));
  const T qn = -sn + alpha * jn;
  const T qt = -st + alpha * jt;
  if (sides & 1) {
    o[(0 * 2 + N) * 2 + 0] = c2n * (qn - em * iht * dtj);
    o[(0 * 2 + N) * 2 + 1] = -c2n * c2n * em * jn;
    o[(0 * 2 + TT) * 2 + 0] = c2n * qt;
    o[(0 * 2 + TT) * 2 + 1] = -c2n * ihn * em * jt;
  }
  if (sides & 2) {
    o[(1 * 2 + N) * 2 + 0] = -c2n * (qn + ep * iht * dtj);
    o[(1 * 2 + N) * 2 + 1] = -c2n * c2n * ep * jn;
    o[(1 * 2 + TT) * 2 + 0] = -c2n * qt;
    o[(1 * 2 + TT) * 2 + 1] = -c2n * ihn * ep * jt;
  }
}

// dotp (apply only, may be null): receives u.y over the tile, one partial per
// (problem, tile) at dotp[pb * tiles + tile], summed in a fixed order.
// Up to k = 4 the launch bounds ask for four wavefronts per SIMD (the
// unconditional loads would otherwise take the residual to 132 VGPRs).
template <int K1, int MODE, typename T>
__global__ __launch_bounds__(64, (K1 <= 5 ? 4 : 1)) void sip_wave_kernel(MeshDev M, const T* __restrict__ u,
                                                      const T* __restrict__ bvec, T* __restrict__ y,
                                                      const double* __restrict__ eta_all, int64_t vec_stride,
                                                      double* __restrict__ dotp) {
  constexpr int TX = WaveTile<K1>::TX, TY = WaveTile<K1>::TY;
  constexpr int KK = K1 * K1, NB = 2 * KK, E = TX * TY, NH = K1 / 2;
  static_assert(E * K1 <= 64, "tile does not fit a wavefront");
  constexpr int NFV = (TX + 1) * TY, NFH = TX * (TY + 1), NF = NFV > NFH ? NFV : NFH;
  constexpr int S = WaveLds<K1, T>::S, Q = WaveLds<K1, T>::Q;
  static_assert(S >= E * K1 && Q >= NF * K1, "LDS strides too small");
  __shared__ T su[(2 * K1 - 1) * S + E * K1];  // [d][col][el][row]; later the column results
  __shared__ T sf[7 * Q + NF * K1];  // face records: slots (s, d, w) of [face][m]; x-faces, then y-faces
  // element e's entry (row, col) of component d
  auto SU = [&](int e, int d, int row, int col) -> T& { return su[(d * K1 + col) * S + e * K1 + row]; };
  // slot (s, d, w) of the face record at fp, mode m
  auto FA = [&](T* fp, int sd, int d, int w, int m) -> T& { return fp[((sd * 2 + d) * 2 + w) * Q + m]; };
  const int lane = threadIdx.x;
  const int nx = M.nx, ny = M.ny;
  const int ntx = (nx + TX - 1) / TX;
  // tiles in XCD-contiguous order (the grid is tiles x problems)
  const uint32_t lt = xcd_order(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int tile = (int)(lt % gridDim.x);
  const int ix0 = (tile % ntx) * TX, iy0 = (tile / ntx) * TY;
  const int64_t pb = lt / gridDim.x;
  if (M.active && !M.active[pb]) {  // a converged problem of a batched CG iteration
    if (MODE == M_APPLY && dotp && lane == 0) dotp[pb * gridDim.x + tile] = 0.0;
    return;
  }
  const double* eta = eta_all + pb * (int64_t)nx * ny;
  constexpr bool RES = MODE == M_RESID || MODE == M_RESQ1;
  u += pb * vec_stride;
  // M_RESQ1 writes the residual's Q1 modes only: [pb][e][d][j][i], i, j <= 1
  y += MODE == M_RESQ1 ? pb * (int64_t)nx * ny * 8 : pb * vec_stride;
  if (RES) bvec += pb * vec_stride;
  const T ihx = T(1.0 / M.hx), ihy = T(1.0 / M.hy);

  const int el = lane / K1, j = lane - el * K1;  // j: row, then face mode and column
  const bool act = el < E;
  const int tx = el % TX, ty = el / TX;
  const int ix = ix0 + tx, iy = iy0 + ty;
  const bool valid = act && ix < nx && iy < ny;
  const int64_t ge = (int64_t)iy * nx + ix;

  // Every global load below is unconditional: lanes outside the mesh (and
  // lanes without a neighbour to read) load from an element of the mesh and
  // discard the value by a select.  Loads under branches made the compiler
  // wait for earlier loads between the branches, several HBM round trips per
  // wavefront instead of one.
  const int64_t gs = valid ? ge : 0;
  // viscosity of the element and of its neighbours (the element's own where
  // the mesh ends: boundary faces read only the present side)
  T et, eL, eR, eB, eT;
  {
    const double v0 = eta[gs];
    const double vl = eta[valid && ix > 0 ? gs - 1 : gs];
    const double vr = eta[valid && ix + 1 < nx ? gs + 1 : gs];
    const double vb = eta[valid && iy > 0 ? gs - nx : gs];
    const double vt = eta[valid && iy + 1 < ny ? gs + nx : gs];
    et = valid ? T(v0) : T(0);
    eL = valid ? T(vl) : T(0);
    eR = valid ? T(vr) : T(0);
    eB = valid ? T(vb) : T(0);
    eT = valid ? T(vt) : T(0);
  }
  T up[NH], dn[NH];
#pragma unroll
  for (int t = 0; t < NH; ++t) {
    T a = T(0), b = T(0);
#pragma unroll
    for (int q = 0; q < K1; ++q)
      if (j == q) {
        if (q + 1 + 2 * t < K1) a = T(d_val(q, q + 1 + 2 * t));
        if (q - 1 - 2 * t >= 0) b = T(d_val(q - 1 - 2 * t, q));
      }
    up[t] = a;
    dn[t] = b;
  }

  const T cxx = T(4) * ihx * ihx, cyy = T(4) * ihy * ihy, cxy = T(4) * ihx * ihy;
  auto trace4 = [](const T (&v)[K1], T& tl, T& gl, T& tr, T& gr) {
    tl = gl = tr = gr = T(0);
#pragma unroll
    for (int i = 0; i < K1; ++i) {
      tl += T(e_end(i, 0)) * v[i];
      gl += T(d_end(i, 0)) * v[i];
      tr += T(e_end(i, 1)) * v[i];
      gr += T(d_end(i, 1)) * v[i];
    }
  };

  // neighbour data outside the tile, requested up front with the element's
  // own rows: edge lanes in x take row j of the left/right neighbour, edge
  // lanes in y column j of the bottom/top neighbour (tiles are at least two
  // elements wide and tall, so a lane needs at most one of each)
  const int64_t gx = (tx == 0 && ix > 0) ? ge - 1 : (tx == TX - 1 && ix + 1 < nx) ? ge + 1 : -1;
  const int64_t gy = (ty == 0 && iy > 0) ? ge - nx : (ty == TY - 1 && iy + 1 < ny) ? ge + nx : -1;
  const bool hx = valid && gx >= 0, hy = valid && gy >= 0;
  const int64_t gxs = hx ? gx : gs, gys = hy ? gy : gs;
  T hxr[2][K1], hyc[2][K1];
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int i = 0; i < K1; ++i) {
      hxr[d][i] = u[gxs * NB + d * KK + j * K1 + i];
      hyc[d][i] = u[gys * NB + d * KK + i * K1 + j];
    }
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int i = 0; i < K1; ++i) {
      if (!hx) hxr[d][i] = T(0);
      if (!hy) hyc[d][i] = T(0);
    }

  // ---- rows: stage the element, x-face traces, S_x
  T yr[2][K1];
  T* fl = sf + (ty * (TX + 1) + tx) * K1;  // left x-face, this element on the plus side
  T* fr = fl + K1;                          // right x-face, minus side
  if (act) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      T r[K1];
#pragma unroll
      for (int i = 0; i < K1; ++i) r[i] = u[gs * NB + d * KK + j * K1 + i];
#pragma unroll
      for (int i = 0; i < K1; ++i)
        if (!valid) r[i] = T(0);
#pragma unroll
      for (int i = 0; i < K1; ++i) SU(el, d, j, i) = r[i];
      T tl, gl, tr, gr;
      trace4(r, tl, gl, tr, gr);
      FA(fl, 1, d, 0, j) = tl;
      FA(fl, 1, d, 1, j) = gl;
      FA(fr, 0, d, 0, j) = tr;
      FA(fr, 0, d, 1, j) = gr;
      // the outer sides of the tile's left and right faces (zero where the
      // mesh ends: hxr is zero there)
      if (tx == 0 || tx == TX - 1) {
        T a0, a1, a2, a3;
        trace4(hxr[d], a0, a1, a2, a3);
        if (tx == 0) {
          FA(fl, 0, d, 0, j) = a2;
          FA(fl, 0, d, 1, j) = a3;
        } else {
          FA(fr, 1, d, 0, j) = a0;
          FA(fr, 1, d, 1, j) = a1;
        }
      }
      const T cx = (d == 0 ? T(2) : T(1)) * et * cxx;
#pragma unroll
      for (int i = 0; i < K1; ++i) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < K1; ++l)
          if (s_nz(i, l)) acc += T(s_val(i, l)) * r[l];
        yr[d][i] = cx * acc;
      }
    }
  }
  __syncthreads();

  // ---- x-faces at mode m = j, applied to row j
  if (act) {
    T o[8];
    {
      const int kind = ix > 0 ? F_INTERIOR : M.bc[0];
      face_mode_w<K1, 0, Q, T>(fl, j, valid ? kind : -1, 1, eL, et, ihx, ihy, up, dn, o);
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const T a = o[(1 * 2 + d) * 2 + 0], b = o[(1 * 2 + d) * 2 + 1];
#pragma unroll
        for (int i = 0; i < K1; ++i) yr[d][i] += a * T(e_end(i, 0)) + b * T(d_end(i, 0));
      }
    }
    {
      const int kind = ix + 1 < nx ? F_INTERIOR : M.bc[1];
      face_mode_w<K1, 0, Q, T>(fr, j, valid ? kind : -1, 0, et, eR, ihx, ihy, up, dn, o);
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const T a = o[(0 * 2 + d) * 2 + 0], b = o[(0 * 2 + d) * 2 + 1];
#pragma unroll
        for (int i = 0; i < K1; ++i) yr[d][i] += a * T(e_end(i, 1)) + b * T(d_end(i, 1));
      }
    }
  }
  __syncthreads();  // the face buffer is free again

  // the residual's right-hand side, requested before the column work
  T bres[2][K1];
  if constexpr (RES) {
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int i = 0; i < K1; ++i) {
        const bool need = MODE == M_RESID || (j < 2 && i < 2);
        bres[d][i] = (MODE == M_RESID || i < 2) ? bvec[gs * NB + d * KK + j * K1 + i] : T(0);
        if (!(valid && need)) bres[d][i] = T(0);
      }
  }

  // ---- columns (lane column ic = j): y-face traces, S_y, mixed term of y0
  T yc[2][K1];
  const int ic = j;
  T* fb = sf + (ty * TX + tx) * K1;        // bottom y-face, this element on the plus side
  T* ft = sf + ((ty + 1) * TX + tx) * K1;  // top y-face, minus side
  if (act) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      T c[K1];
#pragma unroll
      for (int jj = 0; jj < K1; ++jj) c[jj] = SU(el, d, jj, ic);
      T tb, gb, tt, gt;
      trace4(c, tb, gb, tt, gt);
      FA(fb, 1, d, 0, ic) = tb;
      FA(fb, 1, d, 1, ic) = gb;
      FA(ft, 0, d, 0, ic) = tt;
      FA(ft, 0, d, 1, ic) = gt;
      if (ty == 0 || ty == TY - 1) {
        T a0, a1, a2, a3;
        trace4(hyc[d], a0, a1, a2, a3);
        if (ty == 0) {
          FA(fb, 0, d, 0, ic) = a2;
          FA(fb, 0, d, 1, ic) = a3;
        } else {
          FA(ft, 1, d, 0, ic) = a0;
          FA(ft, 1, d, 1, ic) = a1;
        }
      }
      const T cy = (d == 1 ? T(2) : T(1)) * et * cyy;
#pragma unroll
      for (int jj = 0; jj < K1; ++jj) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < K1; ++l)
          if (s_nz(jj, l)) acc += T(s_val(jj, l)) * c[l];
        yc[d][jj] = cy * acc;
      }
    }
    // D_y^T (D_x u1) on column ic: (D_x u1)[m][ic] = sum_{l > ic} D(ic, l) u1[m][l]
    T w[K1];
#pragma unroll
    for (int m = 0; m < K1; ++m) w[m] = T(0);
#pragma unroll
    for (int t = 0; t < NH; ++t) {
      const int l = ic + 1 + 2 * t;
      if (l < K1) {
#pragma unroll
        for (int m = 0; m < K1; ++m) w[m] += up[t] * SU(el, 1, m, l);
      }
    }
#pragma unroll
    for (int jj = 0; jj < K1; ++jj) {
      T acc = T(0);
#pragma unroll
      for (int m = 0; m < K1; ++m)
        if (d_nz(m, jj)) acc += T(d_val(m, jj)) * w[m];
      yc[0][jj] += et * cxy * acc;
    }
  }
  __syncthreads();

  // ---- y-faces at mode m = j, applied to column j; mixed term of y1
  if (act) {
    T o[8];
    {
      const int kind = iy > 0 ? F_INTERIOR : M.bc[2];
      face_mode_w<K1, 1, Q, T>(fb, j, valid ? kind : -1, 1, eB, et, ihy, ihx, up, dn, o);
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const T a = o[(1 * 2 + d) * 2 + 0], b = o[(1 * 2 + d) * 2 + 1];
#pragma unroll
        for (int jj = 0; jj < K1; ++jj) yc[d][jj] += a * T(e_end(jj, 0)) + b * T(d_end(jj, 0));
      }
    }
    {
      const int kind = iy + 1 < ny ? F_INTERIOR : M.bc[3];
      face_mode_w<K1, 1, Q, T>(ft, j, valid ? kind : -1, 0, et, eT, ihy, ihx, up, dn, o);
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const T a = o[(0 * 2 + d) * 2 + 0], b = o[(0 * 2 + d) * 2 + 1];
#pragma unroll
        for (int jj = 0; jj < K1; ++jj) yc[d][jj] += a * T(e_end(jj, 1)) + b * T(d_end(jj, 1));
      }
    }
    // D_x^T (D_y u0) on row j: (D_y u0)[j][m'] = sum_{l > j} D(j, l) u0[l][m']
    T r0[K1];
#pragma unroll
    for (int mm = 0; mm < K1; ++mm) r0[mm] = T(0);
#pragma unroll
    for (int t = 0; t < NH; ++t) {
      const int l = j + 1 + 2 * t;
      if (l < K1) {
#pragma unroll
        for (int mm = 0; mm < K1; ++mm) r0[mm] += up[t] * SU(el, 0, l, mm);
      }
    }
#pragma unroll
    for (int i = 0; i < K1; ++i) {
      T acc = T(0);
#pragma unroll
      for (int mm = 0; mm < K1; ++mm)
        if (d_nz(mm, i)) acc += T(d_val(mm, i)) * r0[mm];
      yr[1][i] += et * cxy * acc;
    }
  }
  // u.y = u.(row part) + u.(column part), with u still staged in LDS
  double dot = 0.0;
  if (MODE == M_APPLY && dotp && valid) {
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int i = 0; i < K1; ++i)
        dot += double(SU(el, d, j, i)) * double(yr[d][i]) + double(SU(el, d, i, ic)) * double(yc[d][i]);
  }
  __syncthreads();
  // column results back to rows
  if (act) {
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int jj = 0; jj < K1; ++jj) SU(el, d, jj, ic) = yc[d][jj];
  }
  __syncthreads();
  if constexpr (MODE == M_RESQ1) {
    if (valid && j < 2) {
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const T v = yr[d][i] + SU(el, d, j, i);
          y[ge * 8 + d * 4 + j * 2 + i] = bres[d][i] - v;
        }
    }
  } else if (valid) {
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int i = 0; i < K1; ++i) {
        const int64_t g = ge * NB + d * KK + j * K1 + i;
        const T v = yr[d][i] + SU(el, d, j, i);
        if constexpr (MODE == M_RESID) y[g] = bres[d][i] - v;
        else y[g] = v;
      }
  }
  if (MODE == M_APPLY && dotp) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) dot += __shfl_xor(dot, off, 64);
    if (lane == 0) dotp[pb * gridDim.x + tile] = dot;
  }
}

// ---------------------------------------------------------------------------
// B^T u (divergence) and B p (gradient): one thread per element (and
// component for B p); neighbour traces are read directly.
// ---------------------------------------------------------------------------
template <int K1>
__device__ __forceinline__ double trace_row(const double* ue, int d, int j, int plus) {
  // value trace of component d at mode j on the x-face (plus: xi = +1)
  double s = 0;
  const double* p = ue + d * K1 * K1 + j * K1;
#pragma unroll
  for (int i = 0; i < K1; ++i) s += e_end(i, plus) * p[i];
  return s;
}
template <int K1>
__device__ __forceinline__ double trace_col(const double* ue, int d, int i, int plus) {
  double s = 0;
  const double* p = ue + d * K1 * K1 + i;
#pragma unroll
  for (int j = 0; j < K1; ++j) s += e_end(j, plus) * p[j * K1];
  return s;
}

template <int K1>
__global__ __launch_bounds__(256) void div_kernel(MeshDev M, const double* __restrict__ u,
                                                  double* __restrict__ q, int64_t nel_total) {
  constexpr int K = K1 - 1, KK = K1 * K1, NB = 2 * KK;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nel_total) return;
  const int nel = M.nx * M.ny;
  const int64_t pb = g / nel;
  const int e = (int)(g - pb * nel);
  const int ix = e % M.nx, iy = e / M.nx;
  const double* ue = u + g * NB;
  const double hx = M.hx, hy = M.hy;
  double out[K][K];
#pragma unroll
  for (int b = 0; b < K; ++b)
#pragma unroll
    for (int a = 0; a < K; ++a) {
      double s = 0;
#pragma unroll
      for (int i = 0; i < K1; ++i)
        if (d_nz(a, i)) s += d_val(a, i) * ue[0 * KK + b * K1 + i];
      double s2 = 0;
#pragma unroll
      for (int j = 0; j < K1; ++j)
        if (d_nz(b, j)) s2 += d_val(b, j) * ue[1 * KK + j * K1 + a];
      out[b][a] = -(2.0 / hx) * s - (2.0 / hy) * s2;
    }
  // x-faces: mode b along the face
#pragma unroll
  for (int side = 0; side < 2; ++side) {  // 0 left face (element = plus side), 1 right face (minus side)
    const int nbx = side == 0 ? ix - 1 : ix + 1;
    const bool interior = nbx >= 0 && nbx < M.nx;
    const int kind = interior ? F_INTERIOR : M.bc[side];
    if (kind == F_NEUMANN) continue;
    const double* un = ue + (int64_t)(nbx - ix) * NB;
#pragma unroll
    for (int b = 0; b < K; ++b) {
      const double tself = trace_row<K1>(ue, 0, b, side == 1);
      double c;
      if (interior) {
        const double tn = trace_row<K1>(un, 0, b, side == 0);
        const double jm = side == 1 ? tself - tn : tn - tself;  // t^- - t^+
        c = (1.0 / hx) * jm;
      } else {
        c = (side == 1 ? 1.0 : -1.0) * (2.0 / hx) * tself;
      }
#pragma unroll
      for (int a = 0; a < K; ++a) out[b][a] += c * e_end(a, side == 1);
    }
  }
#pragma unroll
  for (int side = 0; side < 2; ++side) {  // 0 bottom, 1 top
    const int nby = side == 0 ? iy - 1 : iy + 1;
    const bool interior = nby >= 0 && nby < M.ny;
    const int kind = interior ? F_INTERIOR : M.bc[2 + side];
    if (kind == F_NEUMANN) continue;
    const double* un = ue + (int64_t)(nby - iy) * M.nx * NB;
#pragma unroll
    for (int a = 0; a < K; ++a) {
      const double tself = trace_col<K1>(ue, 1, a, side == 1);
      double c;
      if (interior) {
        const double tn = trace_col<K1>(un, 1, a, side == 0);
        const double jm = side == 1 ? tself - tn : tn - tself;
        c = (1.0 / hy) * jm;
      } else {
        c = (side == 1 ? 1.0 : -1.0) * (2.0 / hy) * tself;
      }
#pragma unroll
      for (int b = 0; b < K; ++b) out[b][a] += c * e_end(b, side == 1);
    }
  }
  double* qe = q + g * (K * K);
#pragma unroll
  for (int b = 0; b < K; ++b)
#pragma unroll
    for (int a = 0; a < K; ++a) qe[b * K + a] = out[b][a];
}

template <int K1>
__device__ __forceinline__ double ptrace_x(const double* qe, int j, int plus) {
  constexpr int K = K1 - 1;
  double s = 0;
#pragma unroll
  for (int a = 0; a < K; ++a) s += e_end(a, plus) * qe[j * K + a];
  return s;
}
template <int K1>
__device__ __forceinline__ double ptrace_y(const double* qe, int i, int plus) {
  constexpr int K = K1 - 1;
  double s = 0;
#pragma unroll
  for (int b = 0; b < K; ++b) s += e_end(b, plus) * qe[b * K + i];
  return s;
}

template <int K1>
__global__ __launch_bounds__(256) void grad_kernel(MeshDev M, const double* __restrict__ p,
                                                   double* __restrict__ v, int64_t nel_total) {
  constexpr int K = K1 - 1, KK = K1 * K1, NB = 2 * KK, NP = K * K;
  const int64_t g2 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g2 >= 2 * nel_total) return;
  const int64_t g = g2 >> 1;
  const int d = (int)(g2 & 1);
  const int nel = M.nx * M.ny;
  const int64_t pb = g / nel;
  const int e = (int)(g - pb * nel);
  const int ix = e % M.nx, iy = e / M.nx;
  const double* qe = p + g * NP;
  const double hx = M.hx, hy = M.hy;
  double out[K1][K1];
  if (d == 0) {
#pragma unroll
    for (int j = 0; j < K1; ++j)
#pragma unroll
      for (int i = 0; i < K1; ++i) {
        double s = 0;
        if (j < K) {
#pragma unroll
          for (int m = 0; m < K; ++m)
            if (d_nz(m, i)) s += d_val(m, i) * qe[j * K + m];
        }
        out[j][i] = -(2.0 / hx) * s;
      }
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int nbx = side == 0 ? ix - 1 : ix + 1;
      const bool interior = nbx >= 0 && nbx < M.nx;
      const int kind = interior ? F_INTERIOR : M.bc[side];
      if (kind == F_NEUMANN) continue;
      const double* qn = qe + (int64_t)(nbx - ix) * NP;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        const double qs = ptrace_x<K1>(qe, j, side == 1);
        double c;
        if (interior) {
          const double qa = 0.5 * (qs + ptrace_x<K1>(qn, j, side == 0));
          c = (side == 1 ? 1.0 : -1.0) * (2.0 / hx) * qa;
        } else {
          c = (side == 1 ? 1.0 : -1.0) * (2.0 / hx) * qs;
        }
#pragma unroll
        for (int i = 0; i < K1; ++i) out[j][i] += c * e_end(i, side == 1);
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < K1; ++j)
#pragma unroll
      for (int i = 0; i < K1; ++i) {
        double s = 0;
        if (i < K) {
#pragma unroll
          for (int m = 0; m < K; ++m)
            if (d_nz(m, j)) s += d_val(m, j) * qe[m * K + i];
        }
        out[j][i] = -(2.0 / hy) * s;
      }
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const int nby = side == 0 ? iy - 1 : iy + 1;
      const bool interior = nby >= 0 && nby < M.ny;
      const int kind = interior ? F_INTERIOR : M.bc[2 + side];
      if (kind == F_NEUMANN) continue;
      const double* qn = qe + (int64_t)(nby - iy) * M.nx * NP;
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const double qs = ptrace_y<K1>(qe, i, side == 1);
        double c;
        if (interior) {
          const double qa = 0.5 * (qs + ptrace_y<K1>(qn, i, side == 0));
          c = (side == 1 ? 1.0 : -1.0) * (2.0 / hy) * qa;
        } else {
          c = (side == 1 ? 1.0 : -1.0) * (2.0 / hy) * qs;
        }
#pragma unroll
        for (int j = 0; j < K1; ++j) out[j][i] += c * e_end(j, side == 1);
      }
    }
  }
  double* ve = v + g * NB + d * KK;
#pragma unroll
  for (int j = 0; j < K1; ++j)
#pragma unroll
    for (int i = 0; i < K1; ++i) ve[j * K1 + i] = out[j][i];
}

// ---------------------------------------------------------------------------
// right-hand sides: F = f + Dirichlet lift, G = int q (g.n) on Dirichlet sides
// ---------------------------------------------------------------------------
template <int K1>
__global__ __launch_bounds__(256) void rhs_kernel(MeshDev M, int nbatch, const double* __restrict__ eta_all,
                                                  const double* __restrict__ f,
                                                  const double* __restrict__ gdir_all,
                                                  double* __restrict__ F, double* __restrict__ G) {
  constexpr int K = K1 - 1, KK = K1 * K1, NB = 2 * KK;
  const int64_t ge = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nel = M.nx * M.ny;
  if (ge >= (int64_t)nel * nbatch) return;
  const int64_t pb = ge / nel;
  const int e = (int)(ge - pb * nel);
  const int ix = e % M.nx, iy = e / M.nx;
  const double* eta = eta_all + pb * nel;
  double* Fe = F + ge * NB;
  for (int a = 0; a < NB; ++a) Fe[a] = f[ge * NB + a];
  double* Ge = G + ge * K * K;
  for (int a = 0; a < K * K; ++a) Ge[a] = 0.0;
  if (gdir_all == nullptr) return;
  const double* gdir = gdir_all + pb * (int64_t)(2 * M.nx + 2 * M.ny) * 2 * K1;
  // sides of this element on the boundary: 0 left, 1 right, 2 bottom, 3 top
  for (int side = 0; side < 4; ++side) {
    bool on = (side == 0 && ix == 0) || (side == 1 && ix == M.nx - 1) || (side == 2 && iy == 0) ||
              (side == 3 && iy == M.ny - 1);
    if (!on || M.bc[side] != F_DIRICHLET) continue;
    const int fi = side == 0 ? iy : side == 1 ? M.ny + iy : side == 2 ? 2 * M.ny + ix : 2 * M.ny + M.nx + ix;
    const int dir = side < 2 ? 0 : 1;
    const double hn = dir == 0 ? M.hx : M.hy, ht = dir == 0 ? M.hy : M.hx;
    const double sc = sqrt(hn / 2.0);
    // face coefficients with the inner trace zero and the outer trace g
    double tr[8 * K1];
    for (int z = 0; z < 8 * K1; ++z) tr[z] = 0.0;
    const int present = (side == 1 || side == 3) ? 0 : 1;  // right/top: element is minus side
    const int absent = 1 - present;
    for (int d = 0; d < 2; ++d)
      for (int m = 0; m < K1; ++m) tr[((absent * 2 + d) * 2 + 0) * K1 + m] = sc * gdir[((int64_t)fi * 2 + d) * K1 + m];
    const double e2 = 2.0 * eta[e];
    if (dir == 0)
      face_coefs<K1, 0, double>(tr, F_INTERIOR, 0, present == 0 ? e2 : 0.0, present == 1 ? e2 : 0.0, hn, ht, false, false);
    else
      face_coefs<K1, 1, double>(tr, F_INTERIOR, 0, present == 0 ? e2 : 0.0, present == 1 ? e2 : 0.0, hn, ht, false, false);
    // face_coefs used alpha = 4 max(eta^-, eta^+) K1^2/hn = 8 eta K1^2 / hn
    const int plus_end = present == 0;  // the element's end at this face
    for (int d = 0; d < 2; ++d)
      for (int m = 0; m < K1; ++m) {
        const double av = tr[((present * 2 + d) * 2 + 0) * K1 + m];
        const double bv = tr[((present * 2 + d) * 2 + 1) * K1 + m];
        for (int o = 0; o < K1; ++o) {
          const double add = av * e_end(o, plus_end) + bv * d_end(o, plus_end);
          if (dir == 0) Fe[d * KK + m * K1 + o] -= add;  // mode m along y, o along x
          else Fe[d * KK + o * K1 + m] -= add;           // mode m along x, o along y
        }
      }
    // G: int q (g.n)
    const double sgn = present == 0 ? 1.0 : -1.0;
    const int dn = dir;  // normal component
    for (int m = 0; m < K; ++m) {
      const double gn = sc * gdir[((int64_t)fi * 2 + dn) * K1 + m];
      for (int o = 0; o < K; ++o) {
        const double add = sgn * (2.0 / hn) * e_end(o, plus_end) * gn;
        if (dir == 0) Ge[m * K + o] += add;
        else Ge[o * K + m] += add;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <int K1, int MODE, typename T, int V>
static void launch_var(const MeshDev& M, int nbatch, const T* u, const T* b, T* y, const double* eta,
                       double* out_mat, hipStream_t s) {
  constexpr int TX = TILE_TX[K1][V], TY = TILE_TY[K1][V];
  const int ntiles = ceil_div(M.nx, TX) * ceil_div(M.ny, TY);
  const int64_t stride = (int64_t)M.nx * M.ny * 2 * K1 * K1;
  hipLaunchKernelGGL((sip_tile_kernel<K1, MODE, T, TX, TY>), dim3(ntiles, nbatch), dim3(NT), 0, s,
                     M, u, b, y, eta, out_mat, nullptr, stride);
}

template <int K1>
static int wave_tiles(const MeshDev& M) {
  return ceil_div(M.nx, WaveTile<K1>::TX) * ceil_div(M.ny, WaveTile<K1>::TY);
}
template <int K1, int MODE, typename T>
static void launch_wave(const MeshDev& M, int nbatch, const T* u, const T* b, T* y, const double* eta,
                        hipStream_t s, double* dotp = nullptr) {
  const int ntiles = wave_tiles<K1>(M);
  const int64_t stride = (int64_t)M.nx * M.ny * 2 * K1 * K1;
  hipLaunchKernelGGL((sip_wave_kernel<K1, MODE, T>), dim3(ntiles, nbatch), dim3(64), 0, s, M, u, b, y, eta, stride,
                     dotp);
}

// var: 0 = wavefront kernel, 1..TILE_NV = tile kernel shapes (apply/residual)
template <int K1, int MODE, typename T>
static int launch_tile(const MeshDev& M, int nbatch, const T* u, const T* b, T* y, const double* eta,
                       double* out_mat, hipStream_t s, int var = 0) {
  if (var < 0 || var > TILE_NV[K1]) {
    set_error("tile variant out of range");
    return SDG_ERR_INVALID;
  }
  if constexpr (MODE == M_APPLY || MODE == M_RESID) {
    switch (var) {
      case 0: launch_wave<K1, MODE, T>(M, nbatch, u, b, y, eta, s); break;
      case 1: launch_var<K1, MODE, T, 0>(M, nbatch, u, b, y, eta, out_mat, s); break;
      case 2: launch_var<K1, MODE, T, 1>(M, nbatch, u, b, y, eta, out_mat, s); break;
      case 3: launch_var<K1, MODE, T, 2>(M, nbatch, u, b, y, eta, out_mat, s); break;
      default:
        if constexpr (TILE_NV[K1] > 3) launch_var<K1, MODE, T, 3>(M, nbatch, u, b, y, eta, out_mat, s);
        break;
    }
  } else {
    launch_var<K1, MODE, T, 0>(M, nbatch, u, b, y, eta, out_mat, s);
  }
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

int sip_tile_variants(int k) { return (k >= 1 && k <= 6) ? TILE_NV[k + 1] + 1 : 0; }
// default kernel form per order and precision, from sweeps at 64 x 64 x 16
// (k = 4) and 64 x 64 x 8 problems: the wavefront kernel for every order
int sip_tile_default(int k, bool fp32) {
  (void)k;
  (void)fp32;
  return 0;
}
void sip_tile_shape(int k, int var, int* tx, int* ty) {
  const bool ok = k >= 1 && k <= 6 && var >= 0 && var <= TILE_NV[k + 1];
  *tx = *ty = 0;
  if (!ok) return;
  if (var > 0) {
    *tx = TILE_TX[k + 1][var - 1];
    *ty = TILE_TY[k + 1][var - 1];
    return;
  }
  switch (k + 1) {
    case 2: *tx = WaveTile<2>::TX; *ty = WaveTile<2>::TY; break;
    case 3: *tx = WaveTile<3>::TX; *ty = WaveTile<3>::TY; break;
    case 4: *tx = WaveTile<4>::TX; *ty = WaveTile<4>::TY; break;
    case 5: *tx = WaveTile<5>::TX; *ty = WaveTile<5>::TY; break;
    case 6: *tx = WaveTile<6>::TX; *ty = WaveTile<6>::TY; break;
    default: *tx = WaveTile<7>::TX; *ty = WaveTile<7>::TY; break;
  }
}
template <int K1>
static int launch_block_list(const MeshDev& M, const double* eta, const int* elems, int nlist,
                             double* blocks, hipStream_t s) {
  if (nlist <= 0) return SDG_OK;
  hipLaunchKernelGGL((sip_tile_kernel<K1, M_BLOCKCOL, double, 1, 1>), dim3(nlist, 1), dim3(NT), 0,
                     s, M, nullptr, nullptr, nullptr, eta, blocks, elems, (int64_t)0);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

#define SDG_K1_SWITCH(k1, CALL)                 \
  switch (k1) {                                 \
    case 2: { constexpr int KK1 = 2; CALL; } break; \
    case 3: { constexpr int KK1 = 3; CALL; } break; \
    case 4: { constexpr int KK1 = 4; CALL; } break; \
    case 5: { constexpr int KK1 = 5; CALL; } break; \
    case 6: { constexpr int KK1 = 6; CALL; } break; \
    case 7: { constexpr int KK1 = 7; CALL; } break; \
    default: set_error("order k out of range"); return SDG_ERR_INVALID; \
  }

int sip_apply(const MeshDev& M, int k, int nbatch, const double* eta, const double* u, double* y,
              hipStream_t s, int var) {
  SDG_K1_SWITCH(k + 1, return (launch_tile<KK1, M_APPLY, double>(M, nbatch, u, nullptr, y, eta, nullptr, s, var)));
  return SDG_OK;
}
template <int K1>
static int launch_apply_dot(const MeshDev& M, int nbatch, const double* eta, const double* u, double* y,
                            double* part, int part_cap, hipStream_t s) {
  const int ntiles = wave_tiles<K1>(M);
  if ((int64_t)ntiles * nbatch > part_cap) {
    set_error("apply with dot: too many tiles for the partial-sum buffer");
    return SDG_ERR_INVALID;
  }
  launch_wave<K1, M_APPLY, double>(M, nbatch, u, nullptr, y, eta, s, part);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int sip_apply_dot(const MeshDev& M, int k, int nbatch, const double* eta, const double* u, double* y,
                  double* part, int part_cap, hipStream_t s) {
  SDG_K1_SWITCH(k + 1, return (launch_apply_dot<KK1>(M, nbatch, eta, u, y, part, part_cap, s)));
  return SDG_OK;
}
int sip_apply_dot_parts(const MeshDev& M, int k, int nbatch) {
  switch (k + 1) {
    case 2: return wave_tiles<2>(M) * nbatch;
    case 3: return wave_tiles<3>(M) * nbatch;
    case 4: return wave_tiles<4>(M) * nbatch;
    case 5: return wave_tiles<5>(M) * nbatch;
    case 6: return wave_tiles<6>(M) * nbatch;
    case 7: return wave_tiles<7>(M) * nbatch;
    default: return 0;
  }
}
template <int K1, typename T>
static int launch_resq1(const MeshDev& M, int nbatch, const double* eta, const T* b, const T* u, T* rq,
                        hipStream_t s) {
  launch_wave<K1, M_RESQ1, T>(M, nbatch, u, b, rq, eta, s);
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int sip_residual_q1(const MeshDev& M, int k, int nbatch, const double* eta, const double* b,
                    const double* u, double* rq, hipStream_t s) {
  SDG_K1_SWITCH(k + 1, return (launch_resq1<KK1, double>(M, nbatch, eta, b, u, rq, s)));
  return SDG_OK;
}
int sip_residual_q1_f32(const MeshDev& M, int k, int nbatch, const double* eta, const float* b,
                        const float* u, float* rq, hipStream_t s) {
  SDG_K1_SWITCH(k + 1, return (launch_resq1<KK1, float>(M, nbatch, eta, b, u, rq, s)));
  return SDG_OK;
}
int sip_residual(const MeshDev& M, int k, int nbatch, const double* eta, const double* b,
                 const double* u, double* r, hipStream_t s, int var) {
  SDG_K1_SWITCH(k + 1, return (launch_tile<KK1, M_RESID, double>(M, nbatch, u, b, r, eta, nullptr, s, var)));
  return SDG_OK;
}
int sip_apply_f32(const MeshDev& M, int k, int nbatch, const double* eta, const float* u, float* y,
                  hipStream_t s, int var) {
  SDG_K1_SWITCH(k + 1, return (launch_tile<KK1, M_APPLY, float>(M, nbatch, u, nullptr, y, eta, nullptr, s, var)));
  return SDG_OK;
}
int sip_residual_f32(const MeshDev& M, int k, int nbatch, const double* eta, const float* b,
                     const float* u, float* r, hipStream_t s, int var) {
  SDG_K1_SWITCH(k + 1, return (launch_tile<KK1, M_RESID, float>(M, nbatch, u, b, r, eta, nullptr, s, var)));
  return SDG_OK;
}
int sip_block_list(const MeshDev& M, int k, const double* eta, const int* elems, int nlist,
                   double* blocks, hipStream_t s) {
  SDG_K1_SWITCH(k + 1, return (launch_block_list<KK1>(M, eta, elems, nlist, blocks, s)));
  return SDG_OK;
}
int sip_coarse_local(const MeshDev& M, int k, int nbatch, const double* eta, double* clocal,
                     hipStream_t s) {
  SDG_K1_SWITCH(k + 1, return (launch_tile<KK1, M_COARSECOL, double>(M, nbatch, nullptr, nullptr, nullptr, eta, clocal, s)));
  return SDG_OK;
}
int div_apply(const MeshDev& M, int k, int nbatch, const double* u, double* q, hipStream_t s) {
  const int64_t n = (int64_t)M.nx * M.ny * nbatch;
  SDG_K1_SWITCH(k + 1, hipLaunchKernelGGL((div_kernel<KK1>), dim3(ceil_div(n, 256)), dim3(256), 0, s, M, u, q, n));
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int grad_apply(const MeshDev& M, int k, int nbatch, const double* p, double* v, hipStream_t s) {
  const int64_t n = (int64_t)M.nx * M.ny * nbatch;
  SDG_K1_SWITCH(k + 1, hipLaunchKernelGGL((grad_kernel<KK1>), dim3(ceil_div(2 * n, 256)), dim3(256), 0, s, M, p, v, n));
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}
int rhs_assemble(const MeshDev& M, int k, int nbatch, const double* eta, const double* f, const double* g,
                 double* F, double* G, hipStream_t s) {
  const int64_t n = (int64_t)M.nx * M.ny * nbatch;
  SDG_K1_SWITCH(k + 1, hipLaunchKernelGGL((rhs_kernel<KK1>), dim3(ceil_div(n, 256)), dim3(256), 0, s, M, nbatch, eta, f, g, F, G));
  SDG_CHECK_LAUNCH();
  return SDG_OK;
}

}  // namespace sdg
