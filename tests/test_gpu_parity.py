"""Parity of the HIP library (through the C ABI) with the FP64 oracle.

Tolerances are derived from the arithmetic: a matrix-vector product in FP64
is compared componentwise against gamma |A| |u| (the standard rounding bound,
gamma well above n_row * eps with n_row <= 500); solves are compared against
the oracle's direct solution at a residual tolerance tight enough for the
stated bound.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import assemble as asm
from oracle.direct import solve_stokes, solve_viscous
from oracle.mesh import DIRICHLET, NAVIER, NEUMANN, Mesh
from oracle.multigrid import (BlockJacobi, Hierarchy, arnoldi_lambda_max,
                              p_cd, p_prolongation)
from oracle.rng import splitmix64, uniform_pm1
from paper_1607_03777_amd import inputs as gen

from gpu_helpers import (abs_bound, assert_close_componentwise, dev, host,
                          stencil_to_matrix)

pytestmark = pytest.mark.gpu

# tile shapes of the apply kernel per k+1: (TX, TY); meshes below span
# several tiles plus a ragged tail in each direction
RAGGED = {1: (35, 10), 2: (19, 11), 3: (19, 9), 4: (13, 9), 5: (9, 6), 6: (7, 6)}
BCS = [(NAVIER,) * 4, (NAVIER, NEUMANN, DIRICHLET, NAVIER), (DIRICHLET, NAVIER, NEUMANN, DIRICHLET)]


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def sdg(torch):
    from paper_1607_03777_amd import sdg as s
    s.lib()
    return s


@pytest.fixture(scope="module")
def ctx(sdg):
    c = sdg.sdg_create(0, 0)
    yield c
    sdg.sdg_destroy(c)


def make_problem(sdg, ctx, nx, ny, k, eta, bc=(NAVIER,) * 4, **opts):
    print(f"[case] problem nx={nx} ny={ny} k={k} bc={bc} opts={opts}", flush=True)
    return sdg.Problem(ctx, nx, ny, k, eta, bc=bc, **opts)


def rand_eta(n, seed, decades):
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(0, decades, n)


# ----------------------------------------------------------------------------
def test_splitmix64_bit_exact(sdg, ctx, torch):
    for seed in (0, 12345, (7 << 32) + 3):
        out = torch.empty(1000, dtype=torch.float64, device="cuda")
        sdg.sdg_uniform_pm1(ctx, seed, 1000, out, sdg.current_stream())
        torch.cuda.synchronize()
        ref = uniform_pm1(seed, 1000)
        assert np.array_equal(host(out), ref)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("bci", [0, 1, 2])
def test_apply_parity(sdg, ctx, torch, k, bci):
    nx, ny = RAGGED[k]
    bc = BCS[bci]
    eta = rand_eta(nx * ny, 100 * k + bci, 8)
    m = Mesh(nx, ny, k, bc=bc)
    A = asm.assemble_A(m, eta).tocsr()
    rng = np.random.default_rng(k)
    u = rng.normal(size=m.nu)
    P = make_problem(sdg, ctx, nx, ny, k, eta, bc)
    b = rng.normal(size=m.nu)
    # every tile shape of the kernels (the mesh leaves ragged tiles for each)
    for var in range(sdg.sdg_tile_variants(k)):
        print(f"[case] tile variant {var} {sdg.sdg_tile_shape(k, var)}", flush=True)
        for kern in (sdg.TILE_APPLY, sdg.TILE_RESIDUAL):
            for prec in (sdg.FP64, sdg.FP32):
                sdg.sdg_set_tile(P.h, kern, prec, var)
        y = P.zeros(m.nu)
        sdg.sdg_apply_viscous(P.h, dev(u), y)
        torch.cuda.synchronize()
        assert_close_componentwise(host(y), A @ u, abs_bound(A, u), 1e-13 * 64)
        # fused residual
        r = P.zeros(m.nu)
        sdg.sdg_residual_viscous(P.h, dev(b), dev(u), r)
        torch.cuda.synchronize()
        assert_close_componentwise(host(r), b - A @ u, abs_bound(A, u) + np.abs(b), 1e-13 * 64)
        # FP32 apply (same kernel in single precision)
        y32 = P.zeros(m.nu, torch.float32)
        sdg.sdg_apply_viscous_f32(P.h, dev(u.astype(np.float32)), y32)
        torch.cuda.synchronize()
        u32 = u.astype(np.float32).astype(np.float64)
        assert_close_componentwise(host(y32).astype(np.float64), A @ u32, abs_bound(A, u32), 6e-7 * 64)
    P.close()


@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_div_grad_parity(sdg, ctx, torch, k):
    nx, ny = RAGGED[k]
    for bc in BCS:
        m = Mesh(nx, ny, k, bc=bc)
        B = asm.assemble_B(m).tocsr()
        rng = np.random.default_rng(7 + k)
        u = rng.normal(size=m.nu)
        p = rng.normal(size=m.np_)
        P = make_problem(sdg, ctx, nx, ny, k, np.ones(m.nel), bc)
        q = P.zeros(m.np_)
        v = P.zeros(m.nu)
        sdg.sdg_apply_div(P.h, dev(u), q)
        sdg.sdg_apply_grad(P.h, dev(p), v)
        torch.cuda.synchronize()
        assert_close_componentwise(host(q), B.T @ u, abs(B.T) @ np.abs(u), 1e-12)
        assert_close_componentwise(host(v), B @ p, abs(B) @ np.abs(p), 1e-12)
        P.close()


@pytest.mark.parametrize("k", [1, 3, 5])
@pytest.mark.parametrize("dedup", [0, 1])
def test_blocks_and_blockjacobi(sdg, ctx, torch, k, dedup):
    nx, ny = 6, 5
    bc = (NAVIER, NEUMANN, DIRICHLET, NAVIER)
    # a two-phase field so that dedup actually shares blocks
    eta = np.where(np.arange(nx * ny) % 3 == 0, 1e4, 1.0)
    m = Mesh(nx, ny, k, bc=bc)
    Ad = asm.assemble_A(m, eta)
    BJ = BlockJacobi(Ad, m.nbu)
    P = make_problem(sdg, ctx, nx, ny, k, eta, bc, dedup=dedup)
    blocks = P.zeros(m.nel * m.nbu * m.nbu)
    sdg.sdg_get_blocks(P.h, blocks)
    torch.cuda.synchronize()
    G = host(blocks).reshape(m.nel, m.nbu, m.nbu)
    scale = np.abs(BJ.blocks).max(axis=(1, 2))
    assert np.max(np.abs(G - BJ.blocks).max(axis=(1, 2)) / scale) <= 1e-13
    rng = np.random.default_rng(3)
    r = rng.normal(size=m.nu)
    z = P.zeros(m.nu)
    sdg.sdg_apply_blockjacobi(P.h, dev(r), z)
    torch.cuda.synchronize()
    zr = BJ(r)
    # inverse applied: error bounded by cond(block) * eps; blocks here have
    # cond <= ~1e7, so compare at 1e-8 relative per element
    Z, ZR = host(z).reshape(m.nel, -1), zr.reshape(m.nel, -1)
    assert np.max(np.linalg.norm(Z - ZR, axis=1) / np.linalg.norm(ZR, axis=1)) <= 1e-8
    P.close()


@pytest.mark.parametrize("k", [2, 3, 4, 6])
@pytest.mark.parametrize("prec,field", [("fp64", "shared"), ("fp32", "shared"), ("bf16", "shared"),
                                        ("fp64", "distinct"), ("fp32", "distinct"), ("bf16", "distinct")])
def test_blockjacobi_grouped(sdg, ctx, torch, k, prec, field):
    """Grouped apply: one block shared by more elements than a workgroup
    takes (several work items and a ragged last one), shared across the
    problems of a batch; or (distinct) a viscosity that differs on every
    element, so that no two elements share a block and the low-precision
    smoother streams its factors through LDS.  FP64: the inverse applied to
    rounding accuracy.  FP32/BF16: z = s X~^T (X~ r~) with X = L^{-1} and r
    rounded to the storage type; checked against the FP64 inverse within
    the bound that rounding X and r by a unit u implies,
    |X~^T X~ - X^T X| <= (2u + u^2) |X|^T |X|, plus FP32 accumulation."""
    n, nbatch = 12, 2
    m = Mesh(n, n, k)
    if field == "shared":
        eta1 = np.ones(m.nel)
        eta1[::7] = 30.0  # a few elements with other blocks
        etas = np.stack([eta1, 2.5 * eta1])
    else:
        # contrast about 4: blocks well conditioned, so BF16 factors stay
        etas = 10.0 ** np.random.default_rng(5).uniform(-0.3, 0.3, size=(nbatch, m.nel))
    prec_s = {"fp64": sdg.FP64, "fp32": sdg.FP32, "bf16": sdg.BF16}[prec]
    P = make_problem(sdg, ctx, n, n, k, etas, prec_smoother=prec_s,
                     prec_apply=sdg.FP64 if prec == "fp64" else sdg.FP32)
    if prec == "bf16":
        assert sdg.sdg_problem_smoother_precision(P.h) == sdg.BF16
    rng = np.random.default_rng(11)
    r = rng.normal(size=(nbatch, m.nu))
    z = P.zeros(nbatch * m.nu)
    sdg.sdg_apply_blockjacobi(P.h, dev(r.ravel()), z)
    torch.cuda.synchronize()
    Z = host(z).reshape(nbatch, m.nel, m.nbu)
    for pb in range(nbatch):
        BJ = BlockJacobi(asm.assemble_A(m, etas[pb]), m.nbu)
        R = r[pb].reshape(m.nel, m.nbu)
        ZR = np.einsum("eab,eb->ea", BJ.inv, R)
        if prec == "fp64":
            err = np.linalg.norm(Z[pb] - ZR, axis=1) / np.linalg.norm(ZR, axis=1)
            assert err.max() <= 1e-10, err.max()
            continue
        u = 2.0 ** -24 if prec == "fp32" else 2.0 ** -8
        X = np.linalg.inv(np.linalg.cholesky(BJ.blocks))
        XA = np.abs(X)
        bound = np.einsum("eca,ecb,eb->ea", XA, XA, np.abs(R))
        bound *= (2 * u + u * u) + 2 * 2.0 ** -24 + 2 * m.nbu * 2.0 ** -24
        err = np.abs(Z[pb] - ZR)
        worst = np.max(err / bound)
        assert worst <= 1.0, worst
    P.close()


@pytest.mark.parametrize("k", [1, 2, 4])
def test_p_transfer_parity(sdg, ctx, torch, k):
    nx, ny = 9, 6
    m = Mesh(nx, ny, k)
    Pf = (p_prolongation(m) @ p_cd(m)).tocsr()
    P = make_problem(sdg, ctx, nx, ny, k, np.ones(m.nel))
    rng = np.random.default_rng(11)
    r = rng.normal(size=m.nu)
    nn2 = 2 * (nx + 1) * (ny + 1)
    rc = P.zeros(nn2)
    sdg.sdg_p_restrict(P.h, dev(r), rc)
    ec = rng.normal(size=nn2)
    u0 = rng.normal(size=m.nu)
    u = dev(u0)
    sdg.sdg_p_prolong_add(P.h, dev(ec), u)
    torch.cuda.synchronize()
    assert np.allclose(host(rc), Pf.T @ r, rtol=1e-13, atol=1e-13 * np.abs(r).max())
    assert np.allclose(host(u), u0 + Pf @ ec, rtol=1e-13, atol=1e-13 * np.abs(ec).max())
    P.close()


@pytest.mark.parametrize("k,bc", [(2, (NAVIER,) * 4), (3, (NAVIER, NEUMANN, DIRICHLET, NAVIER))])
def test_coarse_operators_parity(sdg, ctx, torch, k, bc):
    nx, ny = 32, 16
    eta = rand_eta(nx * ny, 5, 4)
    m = Mesh(nx, ny, k, bc=bc)
    H = Hierarchy(m, eta, coarsest_n=4)
    P = make_problem(sdg, ctx, nx, ny, k, eta, bc, coarsest_n=4)
    nlev = sdg.sdg_problem_levels(P.h)
    assert nlev - 1 == len(H.levels)
    for li, lev in enumerate(H.levels):
        nn = (lev.nx + 1) * (lev.ny + 1)
        st = P.zeros(36 * nn)
        gx, gy = sdg.sdg_get_coarse_stencil(P.h, li, st)
        torch.cuda.synchronize()
        assert (gx, gy) == (lev.nx, lev.ny)
        G = stencil_to_matrix(host(st), gx, gy)
        R = lev.A.toarray()
        assert np.abs(G - R).max() <= 1e-12 * np.abs(R).max(), li
    P.close()


def test_eig_estimates_parity(sdg, ctx, torch):
    nx = ny = 16
    k = 2
    eta = rand_eta(nx * ny, 9, 3)
    m = Mesh(nx, ny, k)
    H = Hierarchy(m, eta, coarsest_n=4, seed=77)
    P = make_problem(sdg, ctx, nx, ny, k, eta, coarsest_n=4, seed=77)
    gb = sdg.sdg_get_bounds(P.h)
    for li, (lo, hi) in enumerate(H.bounds):
        assert gb[li, 1] == pytest.approx(hi, rel=1e-9), li
        assert gb[li, 0] == pytest.approx(lo, rel=1e-9), li
    P.close()


# The batched Arnoldi of every smoothed level (classical Gram-Schmidt twice,
# coefficients, Hessenberg columns and the stopping test on the device)
# against the oracle's Arnoldi (modified Gram-Schmidt; the same Hessenberg
# matrix in exact arithmetic) problem by problem.  A 1 x 1 mesh at k = 1 has
# 8 velocity unknowns, fewer than the 10 steps: its Krylov space runs out and
# both stop at the same step.
@pytest.mark.parametrize("nx,k,bc", [(8, 2, (NAVIER, NEUMANN, DIRICHLET, NAVIER)), (1, 1, (DIRICHLET,) * 4)])
def test_eig_estimate_hessenberg_batched(sdg, ctx, torch, nx, k, bc):
    nb, seed, steps = 3, 91, 10
    etas = [rand_eta(nx * nx, 40 + i, 3) for i in range(nb)]
    m = Mesh(nx, nx, k, bc=bc)
    P = make_problem(sdg, ctx, nx, nx, k, np.stack(etas), bc, coarsest_n=2, seed=seed)
    nlev = sdg.sdg_problem_levels(P.h)
    for level in range(nlev):
        if level > 0 and level == nlev - 1:
            break  # the coarsest level has no smoother
        print(f"[case] level {level}", flush=True)
        lam, Hg = sdg.sdg_eig_estimate(P.h, level, steps)
        for pb in range(nb):
            Ho = Hierarchy(m, etas[pb], coarsest_n=2, seed=seed)
            if level == 0:
                lo, Hr = arnoldi_lambda_max(Ho.Acsr, Ho.M, seed, 0, steps)
            else:
                lev = Ho.levels[level - 1]
                lo, Hr = arnoldi_lambda_max(lev.A, lev.J, seed, level, steps)
            mm = Hr.shape[1]
            if nx == 1:
                assert mm < steps, mm  # the Krylov space ran out
            scale = np.abs(Hr).max()
            assert np.abs(Hg[pb, :mm + 1, :mm] - Hr).max() <= 1e-9 * scale, (level, pb)
            assert np.all(Hg[pb, :, mm:] == 0.0), (level, pb)  # no column after the stop
            assert lam[pb] == pytest.approx(lo, rel=1e-9), (level, pb)
    P.close()


# k = 4, 5, 6 cover the pipelined FP64 smoother's Chebyshev steps (the
# update operands read after the product)
@pytest.mark.parametrize("k", [2, 4, 5, 6])
def test_vcycle_parity(sdg, ctx, torch, k):
    nx = ny = 16
    P0 = gen.single_inclusion(nx, k, eta_in=1e4)
    m = Mesh(nx, ny, k)
    H = Hierarchy(m, P0.eta, coarsest_n=4)
    P = make_problem(sdg, ctx, nx, ny, k, P0.eta, coarsest_n=4)
    b = np.zeros((len(H.bounds) + 1, 2))
    b[: len(H.bounds)] = H.bounds
    sdg.sdg_set_bounds(P.h, b)
    rng = np.random.default_rng(2)
    r = rng.normal(size=m.nu)
    x = P.zeros(m.nu)
    sdg.sdg_vcycle(P.h, dev(r), x)
    torch.cuda.synchronize()
    xr = H.vcycle(r)
    # the coarsest solve differs in rounding (explicit inverse vs Cholesky
    # solves): allow cond(A_coarsest) * eps amplification
    kc = np.linalg.cond(H.levels[-1].A.toarray())
    tol = max(1e-11, 50.0 * kc * 2.2e-16)
    assert np.linalg.norm(host(x) - xr) <= tol * np.linalg.norm(xr), (tol, kc)
    P.close()


@pytest.mark.parametrize("n,k,contrast,bc,tol", [
    (16, 2, 1e4, (NAVIER,) * 4, 1e-9),
    (12, 3, 1e4, (NAVIER, NEUMANN, NAVIER, NAVIER), 1e-9),
    (8, 5, 1e2, (DIRICHLET,) * 4, 1e-9),
    (5, 4, 1e3, (NAVIER,) * 4, 1e-9),
    # random element viscosity over six decades: the direct solution itself
    # carries cond(A) * eps ~ 1e-8 relative error, so the bar is 1e-7 here
    (12, 3, 1e6, (NAVIER,) * 4, 1e-7),
])
def test_viscous_solve_parity(sdg, ctx, torch, n, k, contrast, bc, tol):
    P0 = gen.random_problem(n, k, 4, contrast=contrast, bc=bc)
    m = Mesh(n, n, k, bc=bc)
    ud = solve_viscous(m, P0.eta, P0.f)
    P = make_problem(sdg, ctx, n, n, k, P0.eta, bc, rtol=1e-13, max_it=3000, coarsest_n=4)
    u, st = P.solve_viscous(dev(P0.f.reshape(-1)))
    assert st["status"] == 0, st
    assert np.linalg.norm(host(u) - ud) <= tol * np.linalg.norm(ud), st
    P.close()


def test_stokes_manufactured(sdg, ctx, torch):
    """Exact polynomial Stokes solution with Dirichlet data (velocity Q_2,
    pressure Q_1): the discrete solution is the exact one.  The pressure
    amplifies the residual by about 2e5 here (measured: a residual of 5e-13
    leaves 8e-8 in p, 9e-15 leaves 2e-9), so the solve asks the extended
    refinement for rtol 1e-14; the FP64 output is then the exact
    coefficients to 1e-10 (velocity) and 5e-9 (pressure)."""
    P0 = gen.manufactured_stokes(8, 2)
    P = make_problem(sdg, ctx, 8, 8, 2, P0.eta, P0.bc, rtol=1e-14, inner_rtol=1e-6,
                     coarsest_n=4, max_it=400, refine=1)
    u, p, st = P.solve_stokes(dev(P0.f.reshape(-1)), dev(P0.g.reshape(-1)))
    assert st["status"] == 0, st
    ue, pe = P0.meta["u_exact"], P0.meta["p_exact"]
    eu = np.linalg.norm(host(u) - ue) / np.linalg.norm(ue)
    ep = np.linalg.norm(host(p) - pe) / np.linalg.norm(pe)
    print(f"[manufactured] velocity {eu:.2e} pressure {ep:.2e} {st}", flush=True)
    assert eu <= 1e-10 and ep <= 5e-9, st
    P.close()


# Against the refined (long-double) oracle solution: the FP64 LU's own
# pressure carries about 1e-7 relative error on these cases, so it cannot
# serve as the reference for a tight pressure bound.  rtol 1e-11 on the
# extended residual; velocity 1e-9, pressure 1e-8.
@pytest.mark.parametrize("n,k,ein,bc", [(8, 2, 1e2, (NAVIER,) * 4),
                                       (6, 3, 1e3, (NAVIER, NAVIER, NAVIER, NEUMANN))])
def test_stokes_solve_parity(sdg, ctx, torch, n, k, ein, bc):
    from oracle import refine as rf
    P0 = gen.single_inclusion(n, k, eta_in=ein)
    m = Mesh(n, n, k, bc=bc)
    ud, pd = rf.solve_stokes_ext(m, P0.eta, P0.f, method="lu")
    ud, pd = ud.astype(np.float64), pd.astype(np.float64)
    P = make_problem(sdg, ctx, n, n, k, P0.eta, bc, rtol=1e-11, inner_rtol=1e-6, coarsest_n=4,
                     max_it=600, refine=1)
    u, p, st = P.solve_stokes(dev(P0.f.reshape(-1)))
    assert st["status"] == 0, st
    eu = np.linalg.norm(host(u) - ud) / np.linalg.norm(ud)
    ep = np.linalg.norm(host(p) - pd) / np.linalg.norm(pd)
    print(f"[stokes parity] velocity {eu:.2e} pressure {ep:.2e} {st}", flush=True)
    assert eu <= 1e-9 and ep <= 1e-8, st
    P.close()


# The FP64 path without refinement: it may stop at the FP64 floor, and the
# library reports SDG_FLOOR only within a small factor of the floor
# estimate eps |K||x| / |b| (checked here with the same estimate).
def test_stokes_fp64_floor_is_the_floor(sdg, ctx, torch):
    P0 = gen.single_inclusion(16, 4, eta_in=1e4)
    P = make_problem(sdg, ctx, 16, 16, 4, P0.eta, rtol=1e-13, inner_rtol=1e-3, coarsest_n=4, max_it=600)
    u, p, st = P.solve_stokes(dev(P0.f.reshape(-1)))
    assert st["status"] == sdg.FLOOR, st
    x = torch.cat([u, p])
    y = torch.zeros_like(x)
    sdg.sdg_abs_apply(P.h, 1, x, y)
    torch.cuda.synchronize()
    floor = 2.0 ** -53 * float(y.norm()) / float(np.linalg.norm(P0.f))
    print(f"[fp64 floor] residual {st['rel_residual']:.2e} floor estimate {floor:.2e}", flush=True)
    assert st["rel_residual"] <= 4 * floor
    P.close()


def test_error_paths(sdg, ctx, torch):
    import ctypes
    L = sdg.lib()
    eta = dev(np.ones(16))
    for mesh, e, code in [
        (sdg.make_mesh(4, 4, 7), eta, sdg.ERR_INVALID),            # k out of range
        (sdg.make_mesh(0, 4, 2), eta, sdg.ERR_INVALID),            # empty mesh
        (sdg.make_mesh(4, 4, 2, bc=(NEUMANN,) * 4), eta, sdg.ERR_UNSUPPORTED),
        (sdg.make_mesh(4, 4, 2), dev(-np.ones(16)), sdg.ERR_INVALID),
        (sdg.make_mesh(4, 4, 2), dev(np.full(16, np.nan)), sdg.ERR_INVALID),
    ]:
        out = ctypes.c_void_p()
        rc = L.sdg_problem_create(ctx, ctypes.byref(mesh), ctypes.byref(sdg.make_options()),
                                  sdg.ptr(e), None, ctypes.byref(out))
        assert rc == code, (rc, sdg.lib().sdg_last_error())
    # memory budget too small
    small = sdg.sdg_create(0, 1024)
    out = ctypes.c_void_p()
    rc = L.sdg_problem_create(small, ctypes.byref(sdg.make_mesh(4, 4, 2)),
                              ctypes.byref(sdg.make_options()), sdg.ptr(eta), None, ctypes.byref(out))
    assert rc == sdg.ERR_NOMEM
    sdg.sdg_destroy(small)
    # iteration limit reached -> soft outcome with the last iterate
    P0 = gen.random_problem(8, 2, 1, contrast=1e3)
    P = make_problem(sdg, ctx, 8, 8, 2, P0.eta, max_it=1, rtol=1e-12)
    u, st = P.solve_viscous(dev(P0.f.reshape(-1)))
    assert st["status"] == sdg.NOT_CONVERGED and st["outer_its"] == 1
    P.close()


def test_single_element_meshes(sdg, ctx, torch):
    """Degenerate grids: one element per direction (all faces on the
    boundary) and a 1 x n strip."""
    for nx, ny, k in [(1, 1, 3), (1, 5, 2), (7, 1, 4)]:
        bc = (NAVIER, DIRICHLET, NAVIER, DIRICHLET)
        m = Mesh(nx, ny, k, bc=bc)
        eta = rand_eta(nx * ny, 1, 3)
        A = asm.assemble_A(m, eta).tocsr()
        u = np.random.default_rng(0).normal(size=m.nu)
        P = make_problem(sdg, ctx, nx, ny, k, eta, bc)
        y = P.zeros(m.nu)
        sdg.sdg_apply_viscous(P.h, dev(u), y)
        torch.cuda.synchronize()
        assert_close_componentwise(host(y), A @ u, abs_bound(A, u), 1e-13 * 64)
        P.close()


# ----------------------------------------------------------------------------
# batched problems (several problems on one mesh in one problem object)
# ----------------------------------------------------------------------------
def test_batch_apply_bit_identical(sdg, ctx, torch):
    """Problem pb of a batch runs the same arithmetic as a solo problem."""
    nx, ny, k = 13, 9, 4
    etas = [rand_eta(nx * ny, 50 + i, 6) for i in range(3)]
    Pb = make_problem(sdg, ctx, nx, ny, k, np.stack(etas))
    nu1 = nx * ny * 2 * (k + 1) ** 2
    rng = np.random.default_rng(8)
    u = rng.normal(size=3 * nu1)
    y = Pb.zeros(3 * nu1)
    sdg.sdg_apply_viscous(Pb.h, dev(u), y)
    torch.cuda.synchronize()
    yb = host(y)
    for i in range(3):
        P1 = make_problem(sdg, ctx, nx, ny, k, etas[i])
        y1 = P1.zeros(nu1)
        sdg.sdg_apply_viscous(P1.h, dev(u[i * nu1:(i + 1) * nu1]), y1)
        torch.cuda.synchronize()
        assert np.array_equal(host(y1), yb[i * nu1:(i + 1) * nu1])
        P1.close()
    Pb.close()


def test_batch_viscous_matches_solo_and_oracle(sdg, ctx, torch):
    n, k = 16, 3
    probs = [gen.random_problem(n, k, 20 + i, contrast=10.0 ** (i + 1)) for i in range(3)]
    eta = np.stack([p.eta for p in probs])
    f = np.concatenate([p.f.reshape(-1) for p in probs])
    Pb = make_problem(sdg, ctx, n, n, k, eta, rtol=1e-12, max_it=2000, coarsest_n=4)
    u, stats = Pb.solve_viscous(dev(f))
    assert all(s["status"] == 0 for s in stats), stats
    ub = host(u).reshape(3, -1)
    m = Mesh(n, n, k)
    for i, p in enumerate(probs):
        ud = solve_viscous(m, p.eta, p.f)
        assert np.linalg.norm(ub[i] - ud) <= 1e-9 * np.linalg.norm(ud), (i, stats[i])
        P1 = make_problem(sdg, ctx, n, n, k, p.eta, rtol=1e-12, max_it=2000, coarsest_n=4)
        u1, st1 = P1.solve_viscous(dev(p.f.reshape(-1)))
        assert st1["outer_its"] == stats[i]["outer_its"], (st1, stats[i])
        assert np.linalg.norm(host(u1) - ub[i]) <= 1e-10 * np.linalg.norm(ud)
        P1.close()
    Pb.close()


def test_batch_stokes_matches_oracle(sdg, ctx, torch):
    from oracle import refine as rf
    n, k = 8, 2
    probs = [gen.single_inclusion(n, k, eta_in=e) for e in (1e1, 1e3)]
    eta = np.stack([p.eta for p in probs])
    f = np.concatenate([p.f.reshape(-1) for p in probs])
    Pb = make_problem(sdg, ctx, n, n, k, eta, rtol=1e-11, inner_rtol=1e-6, coarsest_n=4, max_it=600,
                      refine=1)
    u, p, stats = Pb.solve_stokes(dev(f))
    assert all(s["status"] == 0 for s in stats), stats
    ub, pb_ = host(u).reshape(2, -1), host(p).reshape(2, -1)
    m = Mesh(n, n, k)
    for i, pr in enumerate(probs):
        ud, pd = rf.solve_stokes_ext(m, pr.eta, pr.f, method="lu")
        ud, pd = ud.astype(np.float64), pd.astype(np.float64)
        assert np.linalg.norm(ub[i] - ud) <= 1e-9 * np.linalg.norm(ud), stats[i]
        assert np.linalg.norm(pb_[i] - pd) <= 1e-8 * np.linalg.norm(pd), stats[i]
    Pb.close()


# The second case's FP64 residual floor (eps |A||u|/|F| ~ 2e-8) lies above
# its rtol: the extended refinement reaches it anyway.
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n,k,ein,rtol", [(16, 3, 1e2, 1e-9), (16, 4, 1e4, 1e-9)])
def test_mixed_precision_viscous(sdg, ctx, torch, prec, n, k, ein, rtol):
    """FP32 fine-level cycle with FP32 or BF16 block inverses inside FP64
    FGMRES with extended iterative refinement: reaches rtol on the pair and
    the refined oracle solution to 1e-9."""
    from oracle import refine as rf
    P0 = gen.single_inclusion(n, k, eta_in=ein)
    m = Mesh(n, n, k)
    ud = rf.solve_viscous_ext(m, P0.eta, P0.f).astype(np.float64)
    ps = sdg.FP32 if prec == "fp32" else sdg.BF16
    P = make_problem(sdg, ctx, n, n, k, P0.eta, rtol=rtol, max_it=400, coarsest_n=4,
                     prec_apply=sdg.FP32, prec_smoother=ps, viscous_krylov=1, restart=60, refine=1)
    u, st = P.solve_viscous(dev(P0.f.reshape(-1)))
    print(f"[mixed] {prec} n={n} k={k} eta={ein}: {st}", flush=True)
    assert st["status"] == 0, st
    assert st["rel_residual"] < rtol
    assert np.linalg.norm(host(u) - ud) <= 1e-9 * np.linalg.norm(ud), st
    P.close()


# ----------------------------------------------------------------------------
# V-cycles at 64 x 64 with the default coarsest_n = 8: the CG-Q1 levels of
# 65^2 and 33^2 nodes run the per-level kernels (Chebyshev / point-Jacobi
# sweeps, stencil residual, bilinear restriction and prolongation,
# Section 6.1.2); only the levels of at most 17^2 nodes and the dense
# coarsest solve run in the one-workgroup tail.
# ----------------------------------------------------------------------------
def _vcycle_case(sdg, torch, ctx, n, k, probs, coarsest_n=8, **opts):
    """One batched cycle on random vectors with the oracle's Chebyshev
    bounds; returns per problem (relative difference to the oracle's cycle,
    cond of the coarsest operator)."""
    m = Mesh(n, n, k)
    Hs = [Hierarchy(m, p.eta, coarsest_n=coarsest_n) for p in probs]
    nbatch = len(probs)
    P = make_problem(sdg, ctx, n, n, k, np.stack([p.eta for p in probs]), coarsest_n=coarsest_n, **opts)
    nlev = sdg.sdg_problem_levels(P.h)
    assert nlev - 1 == len(Hs[0].levels)
    b = np.zeros((nbatch, nlev, 2))
    for pb, H in enumerate(Hs):
        b[pb, : len(H.bounds)] = H.bounds
    sdg.sdg_set_bounds(P.h, b)
    rng = np.random.default_rng(5 + k)
    r = rng.normal(size=(nbatch, m.nu))
    x = P.zeros(nbatch * m.nu)
    sdg.sdg_vcycle(P.h, dev(r.ravel()), x)
    torch.cuda.synchronize()
    X = host(x).reshape(nbatch, m.nu)
    out = []
    for pb, H in enumerate(Hs):
        xr = H.vcycle(r[pb])
        kc = np.linalg.cond(H.levels[-1].A.toarray())
        out.append((np.linalg.norm(X[pb] - xr) / np.linalg.norm(xr), kc))
    P.close()
    return out, [(lev.nx, lev.ny) for lev in Hs[0].levels]


@pytest.mark.parametrize("k,nbatch", [(2, 3), (4, 1)])
def test_vcycle_parity_hlevels(sdg, ctx, torch, k, nbatch):
    """FP64 cycle: equal to the oracle's cycle up to the rounding of the
    dense coarsest solve (explicit inverse against Cholesky solves), i.e.
    within a multiple of cond(A_coarsest) * eps."""
    n = 64
    probs = [gen.random_inclusions(n, k, seed=s) for s in range(nbatch)]
    errs, levels = _vcycle_case(sdg, torch, ctx, n, k, probs)
    assert levels == [(64, 64), (32, 32), (16, 16), (8, 8)]  # 65^2, 33^2 nodes outside the tail
    for pb, (err, kc) in enumerate(errs):
        tol = max(1e-11, 50.0 * kc * 2.2e-16)
        print(f"[vcycle64] k={k} pb={pb} rel err {err:.3e} tol {tol:.1e}", flush=True)
        assert err <= tol, (pb, err, tol)


# FP32 fine-level cycle (operator apply, block smoother with FP32 factors,
# Q1 residual) around the FP64 coarse hierarchy.  The smoother applies
# s X~^T X~ r with X = L^{-1} rounded to FP32: its relative error is bounded
# by about 2 u32 kappa(M_K) (rounding X by u32 perturbs X^T X by
# 2 u32 |X|^T |X|, and |X|^T |X| ~ ||M_K^{-1}||), the FP32 operator apply by
# about n_b u32 relative to |A||u|.  Over the 2 + 2 Chebyshev steps and the
# Q1 residual (coefficients of order one) the cycle's relative deviation
# from the FP64 cycle therefore stays below 8 u32 max(kappa_max, n_b),
# kappa_max the largest condition number of the element blocks.
@pytest.mark.parametrize("n,k,coarsest", [(16, 4, 4), (64, 2, 8), (16, 5, 4), (16, 6, 4)])
def test_vcycle_parity_fp32_cycle(sdg, ctx, torch, n, k, coarsest):
    probs = [gen.single_inclusion(n, k, eta_in=1e4)]
    errs, _ = _vcycle_case(sdg, torch, ctx, n, k, probs, coarsest_n=coarsest, prec_apply=sdg.FP32,
                           prec_smoother=sdg.FP32)
    m = Mesh(n, n, k)
    BJ = BlockJacobi(asm.assemble_A(m, probs[0].eta), m.nbu)
    kappa = float(np.max(np.linalg.cond(BJ.blocks)))
    tol = 8 * 2.0 ** -24 * max(kappa, m.nbu)
    for err, _ in errs:
        print(f"[vcycle fp32] n={n} k={k} rel err {err:.3e} tol {tol:.1e} (kappa_max {kappa:.2e})", flush=True)
        assert err <= tol, (err, tol)


# k = 5 with seed 5 has an element block of condition 6e7 (a viscosity jump
# of about 1e6 between neighbours); its BF16 factor alone puts the largest
# eigenvalue of the smoothed block at 34 (tests/test_precision_cpu.py).
@pytest.mark.parametrize("k,expect", [(4, "bf16"), (5, "fp32")])
def test_bf16_factors_fall_back_to_fp32(sdg, ctx, torch, k, expect):
    """BF16 factors are kept where the smoothed operator's spectrum stays
    near that of exact inverses and replaced by FP32 factors where it does
    not; either way the solve reaches rtol and the refined oracle solution."""
    from oracle import refine as rf
    n = 32
    pr = gen.random_inclusions(n, k, seed=k)
    m = Mesh(n, n, k)
    P = make_problem(sdg, ctx, n, n, k, pr.eta, rtol=1e-9, max_it=600, prec_apply=sdg.FP32,
                     prec_smoother=sdg.BF16, viscous_krylov=1, restart=30, refine=1)
    got = {0: "fp64", 1: "fp32", 2: "bf16"}[sdg.sdg_problem_smoother_precision(P.h)]
    lam = sdg.sdg_get_bounds(P.h)[0][1] / 1.1
    print(f"[bf16] k={k}: factors {got}, lambda_max {lam:.2f}", flush=True)
    assert got == expect and lam <= 4.0
    u, st = P.solve_viscous(dev(pr.f.reshape(-1)))
    assert st["status"] == 0 and st["rel_residual"] < 1e-9, st
    ud = rf.solve_viscous_ext(m, pr.eta, pr.f).astype(np.float64)
    assert np.linalg.norm(host(u) - ud) <= 1e-8 * np.linalg.norm(ud)
    P.close()
