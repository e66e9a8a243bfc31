"""The Q_0 coarse space of Section 6.1.1 through the C ABI: the probed
Galerkin operator A_0 = (P_k^0)^T A P_k^0 and its h-hierarchy on the grid of
element centres against the oracle, one V-cycle against the oracle's
cycle, and solves (A_hp(Q_0) on odd meshes, A_p(Q_0) on an even one)
against the refined oracle solution."""
import numpy as np
import pytest

from oracle import refine as rf
from oracle.mesh import DIRICHLET, NAVIER, NEUMANN, Mesh
from oracle.multigrid import Hierarchy
from paper_1607_03777_amd import inputs as gen

from gpu_helpers import dev, host, stencil_to_matrix

pytestmark = pytest.mark.gpu
Q0 = 1


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


def rand_eta(n, seed, decades):
    return 10.0 ** np.random.default_rng(seed).uniform(0, decades, n)


@pytest.mark.parametrize("nx,ny,k,bc", [(17, 9, 2, (NAVIER,) * 4), (9, 17, 3, (NAVIER, NEUMANN, DIRICHLET, NAVIER)),
                                        (8, 6, 1, (DIRICHLET, NAVIER, NAVIER, NEUMANN))])
def test_q0_coarse_operators_match_oracle(sdg, ctx, torch, nx, ny, k, bc):
    """A_0 by probing (18 operator applies) and its Galerkin h-levels equal
    the oracle's P_0^T A P_0 and P_h^T A_H P_h to rounding."""
    eta = rand_eta(nx * ny, 5, 4)
    m = Mesh(nx, ny, k, bc=bc)
    H = Hierarchy(m, eta, coarsest_n=4, coarse_space="q0")
    print(f"[case] q0 stencil {nx}x{ny} k={k} bc={bc}", flush=True)
    P = sdg.Problem(ctx, nx, ny, k, eta, bc=bc, coarsest_n=4, coarse_space=Q0)
    assert sdg.sdg_problem_levels(P.h) - 1 == len(H.levels)
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


@pytest.mark.parametrize("n,k,nbatch,coarsest", [(17, 2, 2, 4), (33, 4, 1, 8)])
def test_q0_vcycle_matches_oracle(sdg, ctx, torch, n, k, nbatch, coarsest):
    """One batched cycle with the oracle's Chebyshev bounds.  At 33 x 33
    the 33^2-node level runs the per-level h kernels, the smaller ones the
    coarse tail."""
    m = Mesh(n, n, k)
    probs = [gen.random_inclusions(n, k, seed=s) for s in range(nbatch)]
    Hs = [Hierarchy(m, p.eta, coarsest_n=coarsest, coarse_space="q0") for p in probs]
    print(f"[case] q0 vcycle n={n} k={k} nbatch={nbatch}", flush=True)
    P = sdg.Problem(ctx, n, n, k, np.stack([p.eta for p in probs]), coarsest_n=coarsest, coarse_space=Q0)
    nlev = sdg.sdg_problem_levels(P.h)
    assert nlev - 1 == len(Hs[0].levels)
    b = np.zeros((nbatch, nlev, 2))
    for pb, H in enumerate(Hs):
        b[pb, : len(H.bounds)] = H.bounds
    sdg.sdg_set_bounds(P.h, b)
    r = np.random.default_rng(5 + k).normal(size=(nbatch, m.nu))
    x = P.zeros(nbatch * m.nu)
    sdg.sdg_vcycle(P.h, dev(r.ravel()), x)
    torch.cuda.synchronize()
    X = host(x).reshape(nbatch, m.nu)
    for pb, H in enumerate(Hs):
        xr = H.vcycle(r[pb])
        kc = np.linalg.cond(H.levels[-1].A.toarray())
        err = np.linalg.norm(X[pb] - xr) / np.linalg.norm(xr)
        tol = max(1e-11, 50.0 * kc * 2.2e-16)
        print(f"[q0 vcycle] n={n} k={k} pb={pb} rel err {err:.3e} tol {tol:.1e}", flush=True)
        assert err <= tol
    P.close()


@pytest.mark.parametrize("n,k,kind", [(17, 3, "viscous"), (15, 2, "stokes"), (16, 2, "stokes")])
def test_q0_solves_match_oracle(sdg, ctx, torch, n, k, kind):
    """A_hp(Q_0) (odd n) and A_p(Q_0) (even n: the coarse problem solved
    directly) as the viscous preconditioner: the solution equals the refined
    oracle solution."""
    pr = gen.random_problem(n, k, 60 + n, contrast=1e3)
    m = Mesh(n, n, k)
    print(f"[case] q0 {kind} n={n} k={k}", flush=True)
    # the Stokes velocity error runs about 2400 times the residual on these
    # random-viscosity problems (measured: residual 9.8e-13, velocity error
    # 2.3e-9), so the Stokes cases go to 1e-14 for the 1e-9 bar
    rtol = 1e-12 if kind == "viscous" else 1e-14
    P = sdg.Problem(ctx, n, n, k, pr.eta, rtol=rtol, inner_rtol=1e-3, max_it=3000, refine=1, coarse_space=Q0)
    u, ul = P.zeros(P.nu), P.zeros(P.nu)
    if kind == "viscous":
        rc, st = sdg.sdg_solve_viscous_ext_dev(P.h, dev(pr.f.reshape(-1)), None, u, ul)
        uref = rf.solve_viscous_ext(m, pr.eta, pr.f).astype(np.float64)
        ep = 0.0
    else:
        p, pl = P.zeros(P.np), P.zeros(P.np)
        rc, st = sdg.sdg_solve_stokes_ext_dev(P.h, dev(pr.f.reshape(-1)), None, u, ul, p, pl)
        uref, pref = rf.solve_stokes_ext(m, pr.eta, pr.f, method="lu")
        uref, pref = uref.astype(np.float64), pref.astype(np.float64)
        ep = np.linalg.norm(host(p) - pref) / np.linalg.norm(pref)
    assert st["status"] == 0, st
    eu = np.linalg.norm(host(u) - uref) / np.linalg.norm(uref)
    print(f"[q0 {kind}] n={n} k={k}: {st} velocity {eu:.2e} pressure {ep:.2e}", flush=True)
    assert eu <= 1e-9 and ep <= 1e-7
    P.close()
