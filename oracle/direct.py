"""Direct solves of the discrete systems (oracle; test infrastructure only).

The hp-multilevel Krylov method of Sections 5-6 converges to the unique
solution of the discrete system: u = A^{-1} F for the viscous block (A is
SPD by the discrete coercivity lemma), and the solution of the saddle point
system eq. (discretestokes) with the pressure normalised to zero mean when
there is no Neumann boundary (eq. governing_equations:pressure).  These
routines compute that solution by sparse LU (scipy's SuperLU) or, for tiny
meshes, dense numpy solves.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import (assemble_A, assemble_B, assemble_rhs,
                       pressure_mean_vector)
from .mesh import Mesh


def solve_viscous(mesh: Mesh, eta, f, g=None, dense=False):
    A = assemble_A(mesh, eta)
    F, _ = assemble_rhs(mesh, eta, f, g)
    if dense:
        return np.linalg.solve(A.toarray(), F)
    return spla.splu(A.tocsc()).solve(F)


def stokes_matrix(mesh: Mesh, eta):
    """[[A, B], [B^T, 0]] plus, when no side is Neumann, one bordering row and
    column c (c.p = int p) that removes the constant-pressure null space."""
    A = assemble_A(mesh, eta).tocsr()
    B = assemble_B(mesh).tocsr()
    blocks = [[A, B], [B.T, None]]
    K = sp.bmat(blocks, format="csr")
    if mesh.no_neumann():
        c = pressure_mean_vector(mesh)
        col = sp.csr_matrix(np.concatenate([np.zeros(mesh.nu), c])[:, None])
        K = sp.bmat([[K, col], [col.T, None]], format="csr")
    return K


def solve_stokes(mesh: Mesh, eta, f, g=None, dense=False):
    """Returns (u, p); p has zero mean when there is no Neumann side."""
    K = stokes_matrix(mesh, eta)
    F, G = assemble_rhs(mesh, eta, f, g)
    rhs = np.concatenate([F, G])
    if mesh.no_neumann():
        rhs = np.concatenate([rhs, [0.0]])
    if dense:
        x = np.linalg.solve(K.toarray(), rhs)
    else:
        x = spla.splu(K.tocsc()).solve(rhs)
    u = x[:mesh.nu]
    p = x[mesh.nu:mesh.nu + mesh.np_]
    return u, p
