"""Extended-precision references (oracle; test infrastructure only).

At high viscosity contrast the FP64 rounding floor of the true residual,
about eps |K||x| / |b|, lies above the tolerances the solves are asked for
(at 64 x 64 Q_4 elements and contrast 10^4 it is several 1e-8; the paper
meets the same limit in its Krylov orthogonalisation and moves to quadruple
precision, Section 8.3.1).  A residual below that floor only has a meaning
against an operator and an iterate carried in more than FP64.  This module
provides both, in numpy.longdouble (64-bit mantissa on x86):

  * the matrices assembled in long double (assembly routines with
    dtype=longdouble), residuals b - K x of iterates given as FP64 pairs
    x_hi + x_lo;
  * reference solutions by classical iterative refinement (Wilkinson): the
    residual in long double, the correction from an FP64 solver, the
    iterate accumulated in long double.  The FP64 corrector is a sparse LU
    (SuperLU) of the viscous or bordered Stokes matrix, or, where the Stokes
    LU does not fit, FGMRES preconditioned by the upper block-triangular
    preconditioner of eq. (discretestokespc) with the viscous block solved
    by its LU.

The limit of the refinement is the long-double floor, about
2^-64 |K||x| / |b|.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import assemble_A, assemble_B, assemble_rhs, pressure_mean_vector
from .mesh import Mesh
from .multigrid import fgmres

LD = np.longdouble


def _pair(hi, lo):
    x = np.asarray(hi, dtype=np.float64).astype(LD)
    if lo is not None:
        x = x + np.asarray(lo, dtype=np.float64).astype(LD)
    return x


def viscous_system(mesh: Mesh, eta, f, g=None):
    """(A, F) in long double."""
    A = assemble_A(mesh, eta, dtype=LD).tocsr()
    F, _ = assemble_rhs(mesh, eta, f, g, dtype=LD)
    return A, F


def stokes_system(mesh: Mesh, eta, f, g=None):
    """(K, b) in long double, K = [A B; B^T 0] (eq. discretestokes)."""
    A = assemble_A(mesh, eta, dtype=LD).tocsr()
    B = assemble_B(mesh, dtype=LD).tocsr()
    K = sp.bmat([[A, B], [B.T, None]], format="csr")
    F, G = assemble_rhs(mesh, eta, f, g, dtype=LD)
    return K, np.concatenate([F, G])


def rel_residual(K, b, x):
    """||b - K x|| / ||b|| evaluated in long double."""
    r = b - K @ x
    return float(np.sqrt(np.sum(r * r)) / np.sqrt(np.sum(b * b)))


def viscous_residual(mesh: Mesh, eta, f, u_hi, u_lo=None, g=None):
    A, F = viscous_system(mesh, eta, f, g)
    return rel_residual(A, F, _pair(u_hi, u_lo))


def stokes_residual(mesh: Mesh, eta, f, u_hi, p_hi, u_lo=None, p_lo=None, g=None):
    K, b = stokes_system(mesh, eta, f, g)
    return rel_residual(K, b, np.concatenate([_pair(u_hi, u_lo), _pair(p_hi, p_lo)]))


def refine(apply_ld, b, correct, tol=None, maxit=30):
    """Iterative refinement: x = 0; repeat r = b - K x (long double),
    x += correct(r in FP64) until ||r|| stops decreasing by 2x or falls
    below tol ||b||.  Returns (x, history of ||r|| / ||b||)."""
    x = np.zeros(len(b), dtype=LD)
    bn = np.sqrt(np.sum(b * b))
    hist = []
    r = b.copy()
    for _ in range(maxit):
        rn = float(np.sqrt(np.sum(r * r)) / bn)
        hist.append(rn)
        if tol is not None and rn <= tol:
            break
        if len(hist) >= 3 and hist[-1] > 0.5 * hist[-2] and hist[-2] > 0.5 * hist[-3]:
            break
        x = x + np.asarray(correct(np.asarray(r, dtype=np.float64)), dtype=np.float64).astype(LD)
        r = b - apply_ld(x)
    return x, hist


def solve_viscous_ext(mesh: Mesh, eta, f, g=None):
    """u = A^{-1} F in long double (returned as long double)."""
    A, F = viscous_system(mesh, eta, f, g)
    lu = spla.splu(assemble_A(mesh, eta).tocsc())
    x, _ = refine(lambda v: A @ v, F, lu.solve)
    return x


def _mean_zero(mesh: Mesh, p):
    c = pressure_mean_vector(mesh).astype(p.dtype)
    return p - (c @ p) / (c @ c) * c


def solve_stokes_ext(mesh: Mesh, eta, f, g=None, method="lu"):
    """(u, p) of eq. (discretestokes) in long double, p with zero mean when
    no side is Neumann.  method 'lu': corrections from a SuperLU
    factorisation of the (bordered) Stokes matrix; 'block': from FGMRES with
    the block preconditioner and the viscous LU (for meshes whose Stokes LU
    does not fit)."""
    K, b = stokes_system(mesh, eta, f, g)
    nu, npr = mesh.nu, mesh.np_
    border = mesh.no_neumann()
    if method == "lu":
        A64 = assemble_A(mesh, eta).tocsr()
        B64 = assemble_B(mesh).tocsr()
        K64 = sp.bmat([[A64, B64], [B64.T, None]], format="csr")
        if border:
            c = np.concatenate([np.zeros(nu), pressure_mean_vector(mesh)])[:, None]
            K64 = sp.bmat([[K64, sp.csr_matrix(c)], [sp.csr_matrix(c.T), None]], format="csc")
        lu = spla.splu(K64.tocsc())

        def correct(r):
            if border:
                return lu.solve(np.concatenate([r, [0.0]]))[: nu + npr]
            return lu.solve(r)
    else:
        A64 = assemble_A(mesh, eta).tocsc()
        B64 = assemble_B(mesh).tocsr()
        lu = spla.splu(A64)
        etap = np.repeat(np.asarray(eta, dtype=np.float64), mesh.nbp)
        cm = pressure_mean_vector(mesh)

        def project(v):
            if not border:
                return v
            out = v.copy()
            out[nu:] -= (cm @ v[nu:]) / (cm @ cm) * cm
            return out

        def matvec(v):
            return np.concatenate([A64 @ v[:nu] + B64 @ v[nu:], B64.T @ v[:nu]])

        def prec(v):
            yp = -etap * v[nu:]
            return np.concatenate([lu.solve(v[:nu] - B64 @ yp), yp])

        def correct(r):
            y, _, _ = fgmres(matvec, r, prec, 1e-11, restart=60, maxit=600, project=project)
            return y

    x, _ = refine(lambda v: K @ v, b, correct)
    u, p = x[:nu], x[nu:]
    if border:
        p = _mean_zero(mesh, p)
    return u, p


def stokes_error_estimate(mesh: Mesh, eta, f, u_hi, p_hi, u_lo=None, p_lo=None, rtol=1e-8, maxit=60, **mg):
    """Relative velocity and pressure error of an FP64-pair Stokes iterate,
    for meshes where a refined reference is too costly: the error e solves
    K e = r with r = b - K x formed in long double, and e is obtained by the
    paper's own iteration (FGMRES with the block preconditioner and the
    hp-multigrid inner solve, StokesSolver) to rtol relative to ||r||.  A
    residual reduction of 1e-8 fixes e to about a percent (a loose one does
    not: the error of a random perturbation needs it).  Returns
    (|e_u| / |u|, |e_p| / |p|, ||r|| / ||b||)."""
    from .multigrid import StokesSolver
    K, b = stokes_system(mesh, eta, f)
    x = np.concatenate([_pair(u_hi, u_lo), _pair(p_hi, p_lo)])
    r = b - K @ x
    rel = float(np.sqrt(np.sum(r * r)) / np.sqrt(np.sum(b * b)))
    r64 = np.asarray(r, dtype=np.float64)
    nu = mesh.nu
    S = StokesSolver(mesh, eta, **mg)
    eu, ep, _, _ = S.solve(r64[:nu], r64[nu:], rtol=rtol, maxit=maxit)
    xu = np.asarray(x[:nu], dtype=np.float64)
    xp = np.asarray(x[nu:], dtype=np.float64)
    if mesh.no_neumann():
        xp = np.asarray(_mean_zero(mesh, xp), dtype=np.float64)
    return (float(np.linalg.norm(eu) / np.linalg.norm(xu)), float(np.linalg.norm(ep) / np.linalg.norm(xp)), rel)
