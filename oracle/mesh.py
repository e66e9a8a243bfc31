"""Cartesian grid, DoF numbering and face enumeration (oracle).

Grid: n_x by n_y affine rectangles on [0, l_x] x [0, l_y] (Section 3, regular
Cartesian grid).  Element e = iy*n_x + ix.  Boundary sides are ordered
(left, right, bottom, top) with codes NAVIER, NEUMANN, DIRICHLET.  Navier and
Neumann are the paper's boundary conditions (Section 2); Dirichlet
(Nitsche-type SIP boundary terms) is a reading added for manufactured
solutions, see the notes in the oracle's assembly module.

Canonical coefficient layout (shared I/O convention with the GPU library):
  u[e][d][j][i]  d = component, j = y-mode, i = x-mode, 0 <= i, j <= k
  p[e][j][i]     0 <= i, j <= k-1
  g[f][d][m]     Dirichlet data on boundary face f, face-orthonormal modes
                 m = 0..k; boundary faces ordered left side (iy = 0..n_y-1),
                 right side, bottom side (ix = 0..n_x-1), top side.
"""
from dataclasses import dataclass, field

import numpy as np

NAVIER, NEUMANN, DIRICHLET = 0, 1, 2
LEFT, RIGHT, BOTTOM, TOP = 0, 1, 2, 3


@dataclass
class Mesh:
    nx: int
    ny: int
    k: int
    lx: float = 1.0
    ly: float = 1.0
    bc: tuple = field(default=(NAVIER, NAVIER, NAVIER, NAVIER))

    @property
    def hx(self):
        return self.lx / self.nx

    @property
    def hy(self):
        return self.ly / self.ny

    @property
    def nel(self):
        return self.nx * self.ny

    @property
    def k1(self):
        return self.k + 1

    @property
    def nbu(self):
        """velocity DoF per element, 2 (k+1)^2"""
        return 2 * self.k1 * self.k1

    @property
    def nbp(self):
        """pressure DoF per element, k^2"""
        return self.k * self.k

    @property
    def nu(self):
        return self.nel * self.nbu

    @property
    def np_(self):
        return self.nel * self.nbp

    def elem(self, ix, iy):
        return iy * self.nx + ix

    def elem_origin(self, e):
        iy, ix = divmod(e, self.nx)
        return ix * self.hx, iy * self.hy

    def nbfaces(self):
        return 2 * self.ny + 2 * self.nx

    def boundary_faces(self):
        """List of (side, element, face_index) in the canonical order."""
        out = []
        fi = 0
        for side in (LEFT, RIGHT, BOTTOM, TOP):
            rng = range(self.ny) if side in (LEFT, RIGHT) else range(self.nx)
            for t in rng:
                if side == LEFT:
                    e = self.elem(0, t)
                elif side == RIGHT:
                    e = self.elem(self.nx - 1, t)
                elif side == BOTTOM:
                    e = self.elem(t, 0)
                else:
                    e = self.elem(t, self.ny - 1)
                out.append((side, e, fi))
                fi += 1
        return out

    def interior_faces(self):
        """(minus element, plus element, direction) with direction 0 for a
        face normal to x (minus = left) and 1 for a face normal to y
        (minus = below)."""
        out = []
        for iy in range(self.ny):
            for ix in range(self.nx - 1):
                out.append((self.elem(ix, iy), self.elem(ix + 1, iy), 0))
        for iy in range(self.ny - 1):
            for ix in range(self.nx):
                out.append((self.elem(ix, iy), self.elem(ix, iy + 1), 1))
        return out

    def no_neumann(self):
        return all(b != NEUMANN for b in self.bc)
