// Extended-precision residual (ext_kernels.hip): unit-block tables and
// launchers.
#pragma once

#include <vector>

#include "sdg_common.h"

namespace sdg {

// A tables (n_b x n_b unit blocks, column-major): the volume block; per face
// direction dir (0: x-normal, 1: y-normal) and test side t (0: the minus
// element, whose right/top side the face is; 1: the plus element) the two
// self blocks ((T1 + T2), coefficient eta_K; T3, coefficient sigma_F) and
// the three neighbour blocks (T1, eta of the neighbour; T2, eta_K; T3,
// sigma_F); per boundary side S (left, right, bottom, top) the blocks of
// coefficients eta_K and sigma_F (zero on Neumann sides).
constexpr int EXT_V = 0;
constexpr int EXT_SELF12 = 0, EXT_SELF3 = 1, EXT_NB1 = 2, EXT_NB2 = 3, EXT_NB3 = 4;
__host__ __device__ constexpr int ext_face_base(int dir, int t) { return 1 + (dir * 2 + t) * 5; }
constexpr int EXT_BND = 21;
constexpr int EXT_NA = 29;
// B tables (n_b x k^2): the volume block; per direction and velocity side t
// the block with the pressure of the same side, then of the other side; per
// boundary side one block.
constexpr int EXT_BVOL = 0;
__host__ __device__ constexpr int ext_bface(int dir, int t) { return 1 + (dir * 2 + t) * 2; }
constexpr int EXT_BBND = 9;
constexpr int EXT_NBLK_B = 13;

struct ExtTables {
  const double2* A = nullptr;   // [EXT_NA][n_b][n_b], entry (a, b) at b n_b + a
  const double2* Bu = nullptr;  // [EXT_NBLK_B][k^2][n_b], entry (a, m) at m n_b + a
  const double2* Bp = nullptr;  // [EXT_NBLK_B][n_b][k^2], entry (a, m) at a k^2 + m
  double2 cpen[2];              // (k+1)^2 / h_x, (k+1)^2 / h_y as double-FP64 pairs
};

// Host: the unit blocks of a mesh (k, element size lx/nx by ly/ny, side
// kinds bc) integrated in long double, as double-FP64 pairs in the device
// layouts above.
void ext_unit_blocks(int k, double lx, double ly, int nx, int ny, const int bc[4], std::vector<double2>& TA,
                     std::vector<double2>& TBu, std::vector<double2>& TBp, double2 cpen[2]);

// r_u = F - A x - B p and (r_p != nullptr) r_p = G - B^T x, with
// x = xh + xl and p = ph + pl (xl, pl, ph may be null: zero), evaluated in
// double-FP64 and rounded to FP64.  abs_mode: r_u = |A||xh| + |B||ph|,
// r_p = |B^T||xh| in FP64 (F and G unused).  Batched over nbatch problems.
int ext_residual(const MeshDev& M, int k, int nbatch, bool abs_mode, const double* eta, const double* F,
                 const double* xh, const double* xl, const double* ph, const double* pl, const double* G,
                 const ExtTables& T, double* r_u, double* r_p, hipStream_t s);
// (xh, xl) += d in double-FP64
int dd_accumulate(int64_t n, const double* d, double* xh, double* xl, hipStream_t s);

}  // namespace sdg
