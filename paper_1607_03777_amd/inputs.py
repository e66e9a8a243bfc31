"""Seeded synthetic inputs (mesh, per-element viscosity, modal body force,
Dirichlet data) for the SIP-DG viscous and Stokes solves.

This module holds input generation only, none of the solver's arithmetic.
Both the GPU library's tests/benchmark and the CPU oracle receive the arrays it
produces.  Coefficient layout (the library's canonical I/O):

  eta[e]            e = iy*nx + ix, element-wise constant viscosity
  f[e][d][j][i]     L2(K)-orthonormal tensor-Legendre modes of the body force
  g[face][d][m]     Dirichlet data on boundary faces (left side iy = 0..ny-1,
                    right side, bottom side ix = 0..nx-1, top side), in the
                    face-orthonormal basis sqrt(2/|e|) lhat_m

The basis is psi_ij = (2/sqrt(hx hy)) lhat_i(xi) lhat_j(eta),
lhat_i = sqrt((2i+1)/2) L_i on the reference square [-1, 1]^2.

Workloads follow the paper's shapes: unit square, element-wise constant
viscosity with jumps aligned to inclusions, element viscosity = max over the
closed element and buoyancy only on elements fully inside an inclusion
(Section 8.3: element-wise maximum viscosity and minimum density).
"""
from dataclasses import dataclass, field

import numpy as np

NAVIER, NEUMANN, DIRICHLET = 0, 1, 2


@dataclass
class Problem:
    nx: int
    ny: int
    k: int
    eta: np.ndarray
    f: np.ndarray
    g: np.ndarray = None
    bc: tuple = (NAVIER, NAVIER, NAVIER, NAVIER)
    lx: float = 1.0
    ly: float = 1.0
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nel(self):
        return self.nx * self.ny

    @property
    def nu(self):
        return self.nel * 2 * (self.k + 1) ** 2

    @property
    def np_(self):
        return self.nel * self.k * self.k


# ----------------------------------------------------------------------------
# projections of given functions onto the modal basis (input preparation)
# ----------------------------------------------------------------------------
def _onb(k, x):
    out = np.zeros((k + 1, len(x)))
    for i in range(k + 1):
        c = np.zeros(i + 1)
        c[i] = 1.0
        out[i] = np.sqrt((2 * i + 1) / 2.0) * np.polynomial.legendre.legval(x, c)
    return out


def project_modal(func, nx, ny, k, lx=1.0, ly=1.0, nq=None):
    """L2 projection of a vector field func(x, y) -> (fx, fy) onto
    Q_k^2 per element; returns (nel, 2, k+1, k+1)."""
    nq = nq or k + 6
    g, w = np.polynomial.legendre.leggauss(nq)
    hx, hy = lx / nx, ly / ny
    B = _onb(k, g)  # (k+1, nq)
    c = 2.0 / np.sqrt(hx * hy)
    ix = np.arange(nx)
    iy = np.arange(ny)
    # physical quadrature coordinates for every element
    X = (ix[None, :, None, None] * hx + (g[None, None, None, :] + 1) * hx / 2)
    Y = (iy[:, None, None, None] * hy + (g[None, None, :, None] + 1) * hy / 2)
    X, Y = np.broadcast_arrays(X, Y)  # (ny, nx, nq_y, nq_x)
    fx, fy = func(X, Y)
    fx = np.broadcast_to(fx, X.shape)
    fy = np.broadcast_to(fy, X.shape)
    jac = hx * hy / 4.0
    out = np.zeros((ny, nx, 2, k + 1, k + 1))
    for d, fv in enumerate((fx, fy)):
        # int f psi_ij = jac * c * sum_q w_qx w_qy f B_i(x_q) B_j(y_q)
        out[:, :, d] = jac * c * np.einsum("yxba,b,a,jb,ia->yxji",
                                          fv, w, w, B, B)
    return out.reshape(nx * ny, 2, k + 1, k + 1)


def project_scalar(func, nx, ny, k, lx=1.0, ly=1.0, nq=None):
    """L2 projection of a scalar onto Q_{k-1} per element: (nel, k, k)."""
    v = project_modal(lambda x, y: (func(x, y), 0.0 * x), nx, ny, k - 1, lx,
                      ly, nq)
    return v[:, 0]


def project_boundary(func, nx, ny, k, lx=1.0, ly=1.0, nq=None):
    """Face-orthonormal modal coefficients of func on every boundary face."""
    nq = nq or k + 6
    g, w = np.polynomial.legendre.leggauss(nq)
    hx, hy = lx / nx, ly / ny
    B = _onb(k, g)
    out = []
    for side in range(4):
        n = ny if side < 2 else nx
        for t in range(n):
            if side < 2:
                y = t * hy + (g + 1) * hy / 2
                x = np.full_like(y, 0.0 if side == 0 else lx)
                length = hy
            else:
                x = t * hx + (g + 1) * hx / 2
                y = np.full_like(x, 0.0 if side == 2 else ly)
                length = hx
            fx, fy = func(x, y)
            fx = np.broadcast_to(fx, x.shape)
            fy = np.broadcast_to(fy, x.shape)
            # int_e f sqrt(2/|e|) lhat_m ds, ds = |e|/2 dtau
            sc = np.sqrt(2.0 / length) * length / 2.0
            out.append([sc * (B @ (w * fx)), sc * (B @ (w * fy))])
    return np.array(out)


def constant_force_modes(fx_el, fy_el, nx, ny, k, lx=1.0, ly=1.0):
    """Modal coefficients of an element-wise constant force: only mode (0,0),
    equal to f * sqrt(|K|)."""
    nel = nx * ny
    f = np.zeros((nel, 2, k + 1, k + 1))
    s = np.sqrt((lx / nx) * (ly / ny))
    f[:, 0, 0, 0] = np.asarray(fx_el) * s
    f[:, 1, 0, 0] = np.asarray(fy_el) * s
    return f


# ----------------------------------------------------------------------------
# inclusion geometry
# ----------------------------------------------------------------------------
def _rect_disk_dist(nx, ny, lx, ly, cx, cy):
    hx, hy = lx / nx, ly / ny
    x0 = np.arange(nx) * hx
    y0 = np.arange(ny) * hy
    dx = np.maximum(np.maximum(x0 - cx, 0.0), cx - (x0 + hx))
    dy = np.maximum(np.maximum(y0 - cy, 0.0), cy - (y0 + hy))
    near = np.sqrt(dy[:, None] ** 2 + dx[None, :] ** 2)
    fx = np.maximum(np.abs(x0 - cx), np.abs(x0 + hx - cx))
    fy = np.maximum(np.abs(y0 - cy), np.abs(y0 + hy - cy))
    far = np.sqrt(fy[:, None] ** 2 + fx[None, :] ** 2)
    return near.ravel(), far.ravel()


def inclusion_fields(nx, ny, disks, background=1.0, lx=1.0, ly=1.0):
    """Element viscosity and 'fully inside some disk' mask.

    disks: list of (cx, cy, r, eta_i).  An element intersects a disk when its
    closed rectangle comes strictly closer than r to the centre; it is fully
    inside when its farthest corner is strictly closer than r.  eta_K is the
    maximum over the disks it intersects, and over the background when it is
    not fully covered by one disk (element-wise maximum viscosity)."""
    nel = nx * ny
    eta = np.full(nel, -np.inf)
    covered = np.zeros(nel, dtype=bool)
    for cx, cy, r, ei in disks:
        near, far = _rect_disk_dist(nx, ny, lx, ly, cx, cy)
        hit = near < r
        eta[hit] = np.maximum(eta[hit], ei)
        covered |= far < r
    eta = np.where(covered, eta, np.maximum(eta, background))
    return eta, covered


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def manufactured_stokes(n=8, k=2):
    """Dirichlet problem with an exactly representable solution:
    u = curl(x^2 y^2) = (2 x^2 y, -2 x y^2), p = x y - 1/4, eta = 1, so
    f = -div(2 eps(u)) + grad p = (-3y, 5x) and g = u on the boundary."""
    ue = lambda x, y: (2 * x * x * y, -2 * x * y * y)
    pe = lambda x, y: x * y - 0.25
    fe = lambda x, y: (-3.0 * y, 5.0 * x)
    f = project_modal(fe, n, n, k)
    g = project_boundary(ue, n, n, k)
    prob = Problem(n, n, k, np.ones(n * n), f, g,
                   (DIRICHLET, DIRICHLET, DIRICHLET, DIRICHLET),
                   name=f"manufactured-{n}x{n}-k{k}")
    prob.meta["u_exact"] = project_modal(ue, n, n, k).reshape(-1)
    prob.meta["p_exact"] = project_scalar(pe, n, n, k).reshape(-1)
    return prob


def single_inclusion(n=64, k=4, eta_in=1e4, r=0.25):
    """Centred disk of radius r with viscosity eta_in in background 1; body
    force (0, -1) on elements fully inside the disk; Navier on all sides."""
    eta, inside = inclusion_fields(n, n, [(0.5, 0.5, r, eta_in)])
    f = constant_force_modes(np.zeros(n * n), -inside.astype(float), n, n, k)
    return Problem(n, n, k, eta, f, None, name=f"inclusion-{n}x{n}-k{k}",
                   meta={"eta_in": eta_in, "r": r})


def random_inclusions(n=256, k=4, seed=0, ndisk=16, rmin=0.03, rmax=0.1,
                      log_eta=(-3.0, 3.0)):
    """ndisk seeded disks (centres uniform in the unit square, radius uniform,
    log10 viscosity uniform) on background 1; force (0, -1) inside any disk
    minus its mean; Navier on all sides."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.0, 1.0, (ndisk, 2))
    r = rng.uniform(rmin, rmax, ndisk)
    le = rng.uniform(log_eta[0], log_eta[1], ndisk)
    disks = [(c[i, 0], c[i, 1], r[i], 10.0 ** le[i]) for i in range(ndisk)]
    eta, inside = inclusion_fields(n, n, disks)
    fy = -inside.astype(float)
    fy = fy - fy.mean()
    f = constant_force_modes(np.zeros(n * n), fy, n, n, k)
    return Problem(n, n, k, eta, f, None, name=f"random-incl-{n}x{n}-k{k}-s{seed}",
                   meta={"disks": disks, "seed": seed})


def gaussian_random_field(n, seed, corr=0.1, std=1.5, nfeat=1024):
    """Mean-zero squared-exponential GRF (std, correlation length corr)
    sampled at element centres with nfeat random Fourier features."""
    rng = np.random.default_rng(seed)
    w = rng.normal(0.0, 1.0 / corr, (nfeat, 2))
    b = rng.uniform(0.0, 2 * np.pi, nfeat)
    a = rng.normal(0.0, 1.0, nfeat)
    xc = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(xc, xc, indexing="xy")
    ph = np.einsum("f,xy->fxy", w[:, 0], X) + np.einsum("f,xy->fxy", w[:, 1], Y)
    field_ = np.sqrt(2.0 / nfeat) * np.einsum("f,fxy->xy", a, np.cos(ph + b[:, None, None]))
    return std * field_.ravel()


def smooth_force(n, k, seed, nmodes=8):
    """Sum of nmodes seeded low Fourier modes, projected onto Q_k^2."""
    rng = np.random.default_rng(seed + 7919)
    kx = rng.integers(1, 4, (nmodes, 2))
    ky = rng.integers(1, 4, (nmodes, 2))
    amp = rng.normal(0.0, 1.0, (nmodes, 2))
    ph = rng.uniform(0.0, 2 * np.pi, (nmodes, 2))

    def fn(x, y):
        fx = sum(amp[i, 0] * np.sin(np.pi * kx[i, 0] * x + ph[i, 0])
                 * np.cos(np.pi * ky[i, 0] * y) for i in range(nmodes))
        fy = sum(amp[i, 1] * np.cos(np.pi * kx[i, 1] * x)
                 * np.sin(np.pi * ky[i, 1] * y + ph[i, 1]) for i in range(nmodes))
        return fx, fy

    return project_modal(fn, n, n, k, nq=k + 4)


def grf_problem(seed, n=None, k=None):
    """One request of the batched workload: n from {16,32,64,128}, k from
    {2,3,4,5}, log10 viscosity a GRF (correlation 0.1, std 1.5), smooth
    random force; Navier on all sides."""
    rng = np.random.default_rng(10_000 + seed)
    n = n or int(rng.choice([16, 32, 64, 128]))
    k = k or int(rng.choice([2, 3, 4, 5]))
    eta = 10.0 ** gaussian_random_field(n, seed)
    f = smooth_force(n, k, seed)
    return Problem(n, n, k, eta, f, None, name=f"grf-{n}x{n}-k{k}-s{seed}",
                   meta={"seed": seed})


def serving_trace(nreq=2000, rate=200.0, seed=0, nmin=32, nmax=256, kmin=2,
                  kmax=6):
    """Poisson arrivals (exponential gaps) of Stokes requests with n a multiple
    of 16 in [nmin, nmax], k in [kmin, kmax], 1-16 disks of radius
    U[0.03, 0.15] with contrast 10^U[2, 6]."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, nreq)
    t = np.cumsum(gaps)
    ns = rng.integers(nmin // 16, nmax // 16 + 1, nreq) * 16
    ks = rng.integers(kmin, kmax + 1, nreq)
    reqs = []
    for i in range(nreq):
        reqs.append({"t": float(t[i]), "n": int(ns[i]), "k": int(ks[i]),
                     "seed": 100_000 + i})
    return reqs


def serving_problem(req):
    rng = np.random.default_rng(req["seed"])
    n, k = req["n"], req["k"]
    nd = int(rng.integers(1, 17))
    c = rng.uniform(0.0, 1.0, (nd, 2))
    r = rng.uniform(0.03, 0.15, nd)
    contrast = 10.0 ** rng.uniform(2.0, 6.0)
    disks = [(c[i, 0], c[i, 1], r[i], contrast) for i in range(nd)]
    eta, inside = inclusion_fields(n, n, disks)
    fy = -inside.astype(float)
    fy = fy - fy.mean()
    f = constant_force_modes(np.zeros(n * n), fy, n, n, k)
    return Problem(n, n, k, eta, f, None, name=f"serve-{n}x{n}-k{k}",
                   meta=dict(req))


def random_problem(n, k, seed, contrast=1e4, bc=(NAVIER,) * 4):
    """Small random problem for parity tests: log-uniform element viscosity
    over the given contrast and a random modal force."""
    rng = np.random.default_rng(seed)
    eta = 10.0 ** rng.uniform(0.0, np.log10(contrast), n * n)
    f = rng.normal(0.0, 1.0, (n * n, 2, k + 1, k + 1))
    return Problem(n, n, k, eta, f, None, bc=tuple(bc), name=f"random-{n}-k{k}-s{seed}")


def c2_variant(seed, n=64, k=4, eta_in=1e4):
    """Seeded variants of the single-inclusion workload for batches of
    distinct problems: seed 0 is the centred disk of radius 0.25; other
    seeds move the centre uniformly within 0.1 of (0.5, 0.5) and draw the
    radius from U[0.2, 0.3].  Viscosity eta_in inside, 1 outside (element
    maximum), force (0, -1) on elements fully inside; Navier sides."""
    if seed == 0:
        cx, cy, r = 0.5, 0.5, 0.25
    else:
        rng = np.random.default_rng(20_000 + seed)
        cx, cy = rng.uniform(0.4, 0.6, 2)
        r = float(rng.uniform(0.2, 0.3))
    eta, inside = inclusion_fields(n, n, [(cx, cy, r, eta_in)])
    f = constant_force_modes(np.zeros(n * n), -inside.astype(float), n, n, k)
    return Problem(n, n, k, eta, f, None, name=f"inclusion-{n}x{n}-k{k}-s{seed}",
                   meta={"eta_in": eta_in, "r": r, "centre": (float(cx), float(cy)), "seed": seed})


# centres and radii of the six sedimenting inclusions (Section 8.3)
SINKERS = [(0.84, 0.39, 0.089), (0.79, 0.91, 0.059), (0.33, 0.76, 0.063),
           (0.55, 0.47, 0.081), (0.14, 0.60, 0.05), (0.24, 0.13, 0.09)]


def six_sinkers(n, k, eta2=1e6, rho2=1.2, eta1=1.0, rho1=1.0, g=10.0):
    """The six sedimenting inclusions of Section 8.3: viscosity eta2 and
    density rho2 inside, eta1 and rho1 outside, force (0, -g rho); the
    element takes the maximum viscosity and the minimum density over its
    closed area (rho2 only on elements fully inside an inclusion, as
    rho2 > rho1); Neumann on the top side, Navier on the others."""
    eta, inside = inclusion_fields(n, n, [(cx, cy, r, eta2) for cx, cy, r in SINKERS], background=eta1)
    rho = np.where(inside, rho2, rho1)
    f = constant_force_modes(np.zeros(n * n), -g * rho, n, n, k)
    return Problem(n, n, k, eta, f, None, bc=(NAVIER, NAVIER, NAVIER, NEUMANN),
                   name=f"sinkers-{n}x{n}-k{k}-eta{eta2:g}", meta={"eta2": eta2, "rho2": rho2, "g": g})


def smooth_force_elements(n, seed, nmodes=8):
    """Element-wise constant force: the seeded low Fourier modes of
    smooth_force sampled at the element centres (cheap at any mesh size);
    a force of this library's own, not a benchmark's."""
    rng = np.random.default_rng(seed + 7919)
    kx = rng.integers(1, 4, (nmodes, 2))
    ky = rng.integers(1, 4, (nmodes, 2))
    amp = rng.normal(0.0, 1.0, (nmodes, 2))
    ph = rng.uniform(0.0, 2 * np.pi, (nmodes, 2))
    c = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(c, c)  # [iy][ix]
    fx = np.zeros_like(X)
    fy = np.zeros_like(X)
    for i in range(nmodes):
        fx += amp[i, 0] * np.sin(np.pi * kx[i, 0] * X + ph[i, 0]) * np.cos(np.pi * ky[i, 0] * Y)
        fy += amp[i, 1] * np.cos(np.pi * kx[i, 1] * X) * np.sin(np.pi * ky[i, 1] * Y + ph[i, 1])
    return fx.reshape(-1), fy.reshape(-1)


def _below_half(n):
    """Fraction of each element interval [i/n, (i+1)/n] below 1/2."""
    return np.clip(n / 2.0 - np.arange(n), 0.0, 1.0)


def solcx_like(n, k, deta, seed=0):
    """The viscosity structure of the SolCx runs (Sections 7 and 8.1): one
    jump along x = 0.5, viscosity deta for x < 0.5 and 1 for x > 0.5
    (contrast eta_1 : eta_2 = deta, eta_2 = 1), Navier on all sides; with an
    even n the jump lies on element edges, with an odd n the elements of
    the middle column take the L2 projection onto constants, their mean
    (Section 8.1).  The force is this library's seeded smooth field
    (smooth_force_elements): the benchmark's own forcing and analytic
    solution are not used."""
    fl = _below_half(n)
    FL, _ = np.meshgrid(fl, fl)
    eta = (float(deta) * FL + (1.0 - FL)).reshape(-1)
    fx, fy = smooth_force_elements(n, seed)
    f = constant_force_modes(fx, fy, n, n, k)
    return Problem(n, n, k, eta, f, None, name=f"solcx-like-{n}x{n}-k{k}-deta{deta:g}", meta={"deta": deta})


def checkerboard(n, k, deta, seed=0):
    """The 2 x 2 checkerboard of Section 8.2: the SolCx jump along x = 0.5
    and a second one along y = 0.5; viscosity deta on the quadrants
    x < 0.5, y < 0.5 and x > 0.5, y > 0.5, and 1 on the other two (element
    means where an odd n puts an element across a jump); Navier on all
    sides; the force as in solcx_like."""
    fl = _below_half(n)
    FX, FY = np.meshgrid(fl, fl)
    hi = FX * FY + (1.0 - FX) * (1.0 - FY)  # area fraction of the deta quadrants (odd n: L2 mean)
    eta = (float(deta) * hi + (1.0 - hi)).reshape(-1)
    fx, fy = smooth_force_elements(n, seed)
    f = constant_force_modes(fx, fy, n, n, k)
    return Problem(n, n, k, eta, f, None, name=f"checkerboard-{n}x{n}-k{k}-deta{deta:g}", meta={"deta": deta})

