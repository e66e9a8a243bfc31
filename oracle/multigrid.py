"""The paper's iterative solver, in plain FP64 numpy/scipy (oracle; test
infrastructure only).

Components (Sections 5, 6, 8):
  * element-block Jacobi M_k = diagonal blocks of A (eq. smoother), applied
    through per-block Cholesky factors;
  * Chebyshev smoothing preconditioned by M_k with bounds
    [0.1 lambda*, 1.1 lambda*], lambda* the largest Ritz value of ten
    Arnoldi (GMRES) steps on M^{-1} A from a random vector (Section 6);
  * aggressive p-coarsening Q_k -> Q_1 by truncation of the hierarchical
    modes (restriction R), prolongation P = R^T, Galerkin A_1 = P^T A P;
  * the DG -> CG projection A_{1,c} = P_cd^T A_1 P_cd with P_cd the
    element-wise nodal-to-modal map (Section 6.1.2), computed here by L2
    projection of the bilinear hat functions with Gauss quadrature;
  * a vertex-centred h-hierarchy with bilinear interpolation P_h,
    R_h = P_h^T, Galerkin A_H = P_h^T A_h P_h, Chebyshev smoothing with point
    Jacobi and a dense Cholesky solve on the coarsest level (Section 6.1.1-2);
  * the two-level cycle of Algorithm 1 with the h-cycle as the coarse solve;
  * CG on A preconditioned by one cycle (Section 8: the preconditioner is
    linear, so CG is admissible) and right-preconditioned FGMRES on the
    Stokes system with the upper block-triangular preconditioner of eq.
    (discretestokespc) and S = -diag(1/eta_K), the viscosity-scaled pressure
    mass matrix standing in for the Schur complement -B^T A^{-1} B (Section 5).

Readings where the paper is silent (listed in the design notes too):
  * 2 Chebyshev steps before and 2 after on the DG level, 3 and 3 on every
    h-level (Section 8: "up and down smoothing each");
  * h-levels: coarsen while the element count per direction is even and
    larger than `coarsest_n`;
  * the coarse "solve" of Algorithm 1 is one h-cycle, which keeps the
    preconditioner linear;
  * lambda* is taken for the preconditioned operator M^{-1} A.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .assemble import (assemble_A, assemble_B, assemble_rhs,
                       pressure_mean_vector, schur_diag)
from .legendre import gauss
from .mesh import Mesh
from .rng import level_stream, uniform_pm1


# ----------------------------------------------------------------------------
# transfers
# ----------------------------------------------------------------------------
def q1_mode_indices(mesh: Mesh):
    """Fine DoF indices of the modes i, j <= 1 (hierarchical truncation to
    Q_1^2), ordered e, d, j, i with 8 entries per element."""
    k1 = mesh.k1
    loc = [(d * k1 + j) * k1 + i for d in range(2) for j in range(2)
           for i in range(2)]
    loc = np.array(loc)
    return (np.arange(mesh.nel)[:, None] * mesh.nbu + loc[None, :]).ravel()


def p_prolongation(mesh: Mesh):
    """P_k^1: zero-padding of the Q_1 modes into Q_k (sparse, nu x 8 nel)."""
    idx = q1_mode_indices(mesh)
    n1 = len(idx)
    return sp.csr_matrix((np.ones(n1), (idx, np.arange(n1))),
                         shape=(mesh.nu, n1))


def cg_node(nx, jx, jy):
    return jy * (nx + 1) + jx


def p_cd(mesh: Mesh):
    """P_cd: continuous nodal Q_1 (nodes (nx+1)(ny+1), unknown = 2*node + d)
    -> discontinuous modal Q_1 (8 per element), by L2 projection of each hat
    function onto the element's orthonormal Legendre modes."""
    hx, hy = mesh.hx, mesh.hy
    g, w = gauss(4)
    X, Y = np.meshgrid(g, g, indexing="xy")
    W = np.outer(w, w).ravel() * hx * hy / 4.0
    X, Y = X.ravel(), Y.ravel()
    c = 2.0 / np.sqrt(hx * hy)
    lhat = [np.full_like(X, np.sqrt(0.5)), np.sqrt(1.5) * X]
    lhaty = [np.full_like(Y, np.sqrt(0.5)), np.sqrt(1.5) * Y]
    hat_x = [(1 - X) / 2, (1 + X) / 2]
    hat_y = [(1 - Y) / 2, (1 + Y) / 2]
    # local[m, v]: mode m = j*2+i of the hat of vertex v = b*2+a
    local = np.zeros((4, 4))
    for j in range(2):
        for i in range(2):
            psi = c * lhat[i] * lhaty[j]
            for b in range(2):
                for a in range(2):
                    local[j * 2 + i, b * 2 + a] = np.sum(W * psi * hat_x[a] * hat_y[b])
    rows, cols, vals = [], [], []
    for iy in range(mesh.ny):
        for ix in range(mesh.nx):
            e = mesh.elem(ix, iy)
            for d in range(2):
                for m in range(4):
                    for v in range(4):
                        a, b = v % 2, v // 2
                        node = cg_node(mesh.nx, ix + a, iy + b)
                        rows.append(e * 8 + d * 4 + m)
                        cols.append(2 * node + d)
                        vals.append(local[m, v])
    nn = (mesh.nx + 1) * (mesh.ny + 1)
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.nel * 8, 2 * nn))


def p_q0(mesh: Mesh):
    """P_k^0: the element-wise constants (Section 6, p-coarse space Q_0^2)
    in the hierarchical orthonormal basis are the (0, 0) modes, so the
    prolongation is their injection (nu x 2 nel; coarse unknown 2 e + d,
    the element index e = iy nx + ix read as a node of the nx x ny grid of
    element centres)."""
    k1 = mesh.k1
    rows = [e * mesh.nbu + d * k1 * k1 for e in range(mesh.nel) for d in range(2)]
    cols = [2 * e + d for e in range(mesh.nel) for d in range(2)]
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(mesh.nu, 2 * mesh.nel))


def h_prolongation(ncx, ncy):
    """Bilinear interpolation from the (ncx+1)(ncy+1) coarse nodes to the
    (2ncx+1)(2ncy+1) fine nodes, two interleaved components."""
    nfx, nfy = 2 * ncx, 2 * ncy

    def w1(jf, nc):
        if jf % 2 == 0:
            return [(jf // 2, 1.0)]
        return [((jf - 1) // 2, 0.5), ((jf + 1) // 2, 0.5)]

    rows, cols, vals = [], [], []
    for jy in range(nfy + 1):
        for jx in range(nfx + 1):
            for cy, wy in w1(jy, ncy):
                for cx, wx in w1(jx, ncx):
                    for d in range(2):
                        rows.append(2 * cg_node(nfx, jx, jy) + d)
                        cols.append(2 * cg_node(ncx, cx, cy) + d)
                        vals.append(wx * wy)
    return sp.csr_matrix((vals, (rows, cols)),
                         shape=(2 * (nfx + 1) * (nfy + 1),
                                2 * (ncx + 1) * (ncy + 1)))


# ----------------------------------------------------------------------------
# smoothers and eigenvalue estimate
# ----------------------------------------------------------------------------
class BlockJacobi:
    """M_k^{-1} from the diagonal blocks of A via Cholesky."""

    def __init__(self, A: sp.bsr_matrix, nb):
        nel = A.shape[0] // nb
        A = sp.bsr_matrix(A, blocksize=(nb, nb))
        blocks = np.zeros((nel, nb, nb))
        for r in range(nel):
            for p in range(A.indptr[r], A.indptr[r + 1]):
                if A.indices[p] == r:
                    blocks[r] = A.data[p]
        self.blocks = blocks
        L = np.linalg.cholesky(blocks)
        Linv = np.linalg.inv(L)
        self.inv = np.einsum("eba,ebc->eac", Linv, Linv)  # L^-T L^-1
        self.nb = nb

    def __call__(self, r):
        R = r.reshape(-1, self.nb)
        return np.einsum("eab,eb->ea", self.inv, R).ravel()


class PointJacobi:
    def __init__(self, A):
        self.dinv = 1.0 / A.diagonal()

    def __call__(self, r):
        return self.dinv * r


def arnoldi_lambda_max(A, Minv, seed, level, steps=10):
    """Largest real part of the eigenvalues of the Arnoldi Hessenberg matrix
    of M^{-1} A after `steps` steps (modified Gram-Schmidt), started from the
    SplitMix64 vector of stream (seed, level)."""
    n = A.shape[0]
    v = uniform_pm1(level_stream(seed, level), n)
    V = [v / np.linalg.norm(v)]
    H = np.zeros((steps + 1, steps))
    m = steps
    for j in range(steps):
        w = Minv(A @ V[j])
        for i in range(j + 1):
            H[i, j] = np.dot(w, V[i])
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] <= 1e-14 * abs(H[j, j]):
            m = j + 1
            break
        V.append(w / H[j + 1, j])
    ev = np.linalg.eigvals(H[:m, :m])
    return float(np.max(ev.real)), H[:m + 1, :m]


def chebyshev(A, Minv, b, x, lmin, lmax, m, x_is_zero=False):
    """m steps of Chebyshev iteration on A x = b preconditioned by M
    (three-term recurrence with theta, delta, sigma = theta/delta)."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = b.copy() if x_is_zero else b - A @ x
    d = Minv(r) / theta
    x = x.copy()
    for it in range(m):
        x = x + d
        if it == m - 1:
            break
        r = b - A @ x
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * Minv(r)
        rho = rho_new
    return x


# ----------------------------------------------------------------------------
# hierarchy and cycle
# ----------------------------------------------------------------------------
class Level:
    pass


class Hierarchy:
    """hp-multilevel preconditioner for the viscous block: A_hp(Q_1)
    (coarse_space 'q1', Section 6.1.2) or A_hp(Q_0) (coarse_space 'q0',
    Section 6.1.1: Galerkin A_0 = (P_k^0)^T A P_k^0 on the element-wise
    constants, an h-hierarchy on the grid of element centres, which
    coarsens while its node count per direction is odd, i.e. on meshes
    with an odd number of elements; on other meshes A_0 is the coarsest
    level and is solved directly, the variant A_p(Q_0))."""

    def __init__(self, mesh: Mesh, eta, smooth_dg=2, smooth_h=3, coarsest_n=8,
                 seed=0, eig_steps=10, lo=0.1, hi=1.1, bounds=None, A=None, coarse_space="q1"):
        self.mesh = mesh
        self.smooth_dg, self.smooth_h = smooth_dg, smooth_h
        self.A = A if A is not None else assemble_A(mesh, eta)
        self.Acsr = self.A.tocsr()
        self.M = BlockJacobi(self.A, mesh.nbu)
        if coarse_space == "q0":
            self.Pfull = p_q0(mesh)  # element constants -> DG-Q_k
            Ac = (self.Pfull.T @ self.Acsr @ self.Pfull).tocsr()
            # the centres form a grid of nx x ny nodes: nx - 1 intervals
            nx, ny = mesh.nx - 1, mesh.ny - 1
        else:
            self.Pp = p_prolongation(mesh)
            self.Pcd = p_cd(mesh)
            self.Pfull = (self.Pp @ self.Pcd).tocsr()  # CG-Q1 nodal -> DG-Q_k
            A1 = (self.Pp.T @ self.Acsr @ self.Pp).tocsr()
            self.A1 = A1
            Ac = (self.Pcd.T @ A1 @ self.Pcd).tocsr()
            nx, ny = mesh.nx, mesh.ny
        self.levels = []
        Al = Ac
        while True:
            lev = Level()
            lev.A, lev.nx, lev.ny = Al, nx, ny
            lev.J = PointJacobi(Al)
            self.levels.append(lev)
            if nx % 2 == 0 and ny % 2 == 0 and nx > coarsest_n and ny > coarsest_n:
                lev.P = h_prolongation(nx // 2, ny // 2)
                Al = (lev.P.T @ Al @ lev.P).tocsr()
                nx, ny = nx // 2, ny // 2
            else:
                lev.P = None
                lev.chol = sla.cho_factor(Al.toarray(), lower=True)
                break
        # Chebyshev bounds: level 0 = DG level, level l >= 1 = h-levels
        if bounds is not None:
            self.bounds = list(bounds)
        else:
            self.bounds = []
            lam, _ = arnoldi_lambda_max(self.Acsr, self.M, seed, 0, eig_steps)
            self.bounds.append((lo * lam, hi * lam))
            for li, lev in enumerate(self.levels[:-1]):
                lam, _ = arnoldi_lambda_max(lev.A, lev.J, seed, li + 1, eig_steps)
                self.bounds.append((lo * lam, hi * lam))

    def h_cycle(self, li, b):
        lev = self.levels[li]
        if lev.P is None:
            return sla.cho_solve(lev.chol, b)
        lmin, lmax = self.bounds[li + 1]
        x = chebyshev(lev.A, lev.J, b, np.zeros_like(b), lmin, lmax,
                      self.smooth_h, x_is_zero=True)
        r = b - lev.A @ x
        e = self.h_cycle(li + 1, lev.P.T @ r)
        x = x + lev.P @ e
        return chebyshev(lev.A, lev.J, b, x, lmin, lmax, self.smooth_h)

    def vcycle(self, b):
        """One cycle of Algorithm 1 on the DG level with zero initial guess."""
        lmin, lmax = self.bounds[0]
        x = chebyshev(self.Acsr, self.M, b, np.zeros_like(b), lmin, lmax,
                      self.smooth_dg, x_is_zero=True)
        r = b - self.Acsr @ x
        e = self.h_cycle(0, self.Pfull.T @ r)
        x = x + self.Pfull @ e
        return chebyshev(self.Acsr, self.M, b, x, lmin, lmax, self.smooth_dg)


# ----------------------------------------------------------------------------
# Krylov drivers
# ----------------------------------------------------------------------------
def pcg(A, b, prec, rtol, maxit=500, x0=None):
    """Preconditioned CG; stops when the unpreconditioned residual 2-norm
    drops below rtol * ||b||.  Returns (x, iterations, history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A @ x
    bn = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bn if bn > 0 else 0.0]
    if bn == 0:
        return x, 0, hist
    z = prec(r)
    p = z.copy()
    rz = np.dot(r, z)
    it = 0
    while it < maxit and hist[-1] >= rtol:
        q = A @ p
        alpha = rz / np.dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        hist.append(np.linalg.norm(r) / bn)
        if hist[-1] < rtol:
            break
        z = prec(r)
        rz_new = np.dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, hist


def fgmres(matvec, b, prec, rtol, restart=30, maxit=500, project=None):
    """Right-preconditioned flexible GMRES(restart) with classical
    Gram-Schmidt applied twice; stops on the residual 2-norm relative to the
    initial one (x0 = 0).  `project` (optional) is applied to b and to every
    preconditioned vector.  Returns (x, iterations, history)."""
    if project is not None:
        b = project(b)
    n = len(b)
    x = np.zeros(n)
    bn = np.linalg.norm(b)
    hist = [1.0]
    if bn == 0:
        return x, 0, hist
    total = 0
    r = b.copy()
    while total < maxit:
        beta = np.linalg.norm(r)
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        gvec = np.zeros(restart + 1)
        gvec[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(restart):
            z = prec(V[j])
            if project is not None:
                z = project(z)
            Z[j] = z
            w = matvec(z)
            for _ in range(2):
                h = V[:j + 1] @ w
                w = w - V[:j + 1].T @ h
                H[:j + 1, j] += h
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            total += 1
            j_done = j + 1
            hist.append(abs(gvec[j + 1]) / bn)
            if hist[-1] < rtol or total >= maxit:
                break
        y = sla.solve_triangular(H[:j_done, :j_done], gvec[:j_done])
        x = x + Z[:j_done].T @ y
        r = b - matvec(x)
        if np.linalg.norm(r) / bn < rtol or total >= maxit:
            break
    return x, total, hist


class ViscousSolver:
    """Viscous block: CG preconditioned by one hp-cycle."""

    def __init__(self, mesh: Mesh, eta, **kw):
        self.h = Hierarchy(mesh, eta, **kw)

    def solve(self, F, rtol=1e-8, maxit=500):
        return pcg(self.h.Acsr, F, self.h.vcycle, rtol, maxit)


class StokesSolver:
    """Right-preconditioned FGMRES on [A B; B^T 0] with the upper
    block-triangular preconditioner [A B; 0 S] of eq. (discretestokespc):
    P^{-1} x: y_p = S^{-1} x_p, y_u = (inner CG, rtol_inner)(x_u - B y_p).

    S approximates the pressure Schur complement of the saddle matrix,
    0 - B^T A^{-1} B, which is negative definite; the approximation of
    Section 5 (pressure mass matrix scaled by 1/eta_K, diagonal in the
    orthonormal basis) therefore enters as S = -diag(1/eta_K).  The text
    writes the Schur complement without the minus sign; with exact blocks
    either sign converges in two iterations, but with the inexact inner solve
    only the negative one keeps the preconditioned spectrum on one side of
    the origin."""

    def __init__(self, mesh: Mesh, eta, inner_rtol=1e-3, inner_maxit=200, **kw):
        self.mesh = mesh
        self.h = Hierarchy(mesh, eta, **kw)
        self.B = assemble_B(mesh).tocsr()
        self.sinv = 1.0 / schur_diag(mesh, eta)  # = eta_K per mode
        self.inner_rtol = inner_rtol
        self.inner_maxit = inner_maxit
        self.inner_its = []
        self.cmean = pressure_mean_vector(mesh) if mesh.no_neumann() else None

    def matvec(self, x):
        nu = self.mesh.nu
        u, p = x[:nu], x[nu:]
        return np.concatenate([self.h.Acsr @ u + self.B @ p, self.B.T @ u])

    def project(self, x):
        if self.cmean is None:
            return x
        nu = self.mesh.nu
        c = self.cmean
        out = x.copy()
        out[nu:] -= (np.dot(c, x[nu:]) / np.dot(c, c)) * c
        return out

    def prec(self, x):
        nu = self.mesh.nu
        xu, xp = x[:nu], x[nu:]
        yp = -self.sinv * xp
        yu, it, _ = pcg(self.h.Acsr, xu - self.B @ yp, self.h.vcycle,
                        self.inner_rtol, self.inner_maxit)
        self.inner_its.append(it)
        return np.concatenate([yu, yp])

    def solve(self, F, G, rtol=1e-8, restart=30, maxit=500):
        b = np.concatenate([F, G])
        x, its, hist = fgmres(self.matvec, b, self.prec, rtol, restart, maxit,
                              project=self.project)
        nu = self.mesh.nu
        u, p = x[:nu], x[nu:]
        if self.cmean is not None:
            p = p - (np.dot(self.cmean, p) / np.dot(self.cmean, self.cmean)) * self.cmean
        return u, p, its, hist
