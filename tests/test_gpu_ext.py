"""Extended-precision residual and refinement (the library's opts.refine),
through the C ABI, against the long-double oracle.

The residual kernel is checked where FP64 evaluation cannot pass: b is
the long-double product K x rounded to FP64 plus a small perturbation, so
the exact residual is a tiny fraction of |K||x| and an FP64 evaluation
(error about 2^-53 |K||x|) would miss it by orders of magnitude.  Solves
are checked by the long-double residual of the returned FP64 pair and by
the distance to refined long-double reference solutions.
"""
import numpy as np
import pytest

from oracle import assemble as asm
from oracle import refine as rf
from oracle.mesh import DIRICHLET, NAVIER, NEUMANN, Mesh
from paper_1607_03777_amd import inputs as gen

from gpu_helpers import dev, host

pytestmark = pytest.mark.gpu
LD = np.longdouble
BCS = [(NAVIER,) * 4, (NAVIER, NEUMANN, DIRICHLET, NAVIER), (DIRICHLET, NAVIER, NEUMANN, DIRICHLET)]
RAGGED = {1: (9, 7), 2: (8, 5), 3: (6, 5), 4: (5, 4), 5: (4, 3), 6: (3, 3)}


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


def split(x_ld):
    hi = x_ld.astype(np.float64)
    lo = (x_ld - hi.astype(LD)).astype(np.float64)
    return hi, lo


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("bci", [0, 1, 2])
def test_ext_residual_parity(sdg, ctx, torch, k, bci):
    nx, ny = RAGGED[k]
    bc = BCS[bci]
    m = Mesh(nx, ny, k, bc=bc)
    rng = np.random.default_rng(10 * k + bci)
    eta = 10.0 ** rng.uniform(-4, 4, m.nel)
    K, _ = rf.stokes_system(m, eta, np.zeros((m.nel, 2, k + 1, k + 1)))
    nu = m.nu
    x = rng.normal(size=K.shape[0]).astype(LD) * (1 + LD(2) ** -40 * rng.normal(size=K.shape[0]).astype(LD))
    xh, xl = split(x)
    x = xh.astype(LD) + xl.astype(LD)
    Kx = K @ x
    Kabs = abs(K.astype(np.float64)) @ np.abs(xh)
    # b: K x to FP64 plus 1e-12 |K||x|: the exact residual is tiny
    b = Kx.astype(np.float64) + 1e-12 * Kabs * rng.normal(size=K.shape[0])
    rex = b.astype(LD) - Kx
    print(f"[case] ext residual k={k} bc={bc}", flush=True)
    P = sdg.Problem(ctx, nx, ny, k, eta, bc=bc)
    for stokes in (0, 1):
        n = K.shape[0] if stokes else nu
        r = P.zeros(n)
        sdg.sdg_residual_ext(P.h, stokes, dev(b[:n]), dev(xh[:n]), dev(xl[:n]), r)
        torch.cuda.synchronize()
        if stokes:
            ref = rex
            scale = Kabs
        else:
            A = K[:nu, :nu]
            ref = b[:nu].astype(LD) - A @ x[:nu]
            scale = abs(A.astype(np.float64)) @ np.abs(xh[:nu])
        err = np.abs(host(r) - ref.astype(np.float64))
        # FP64 rounding of the result plus the long-double evaluation floor
        bound = 2.0 ** -52 * np.abs(ref.astype(np.float64)) + 2.0 ** -58 * (scale + np.abs(b[:n]))
        worst = float(np.max(err / (bound + 1e-300)))
        print(f"[ext] k={k} bc={bci} stokes={stokes} worst {worst:.2f} "
              f"(residual/|K||x| ~ {float(np.median(np.abs(ref.astype(np.float64)) / (scale + 1e-300))):.1e})",
              flush=True)
        assert worst <= 1.0
        # |K||x| (the floor scale behind SDG_FLOOR)
        y = P.zeros(n)
        sdg.sdg_abs_apply(P.h, stokes, dev(xh[:n]), y)
        torch.cuda.synchronize()
        # the kernel sums |scalar| |unit entry| |x| term by term, so it bounds
        # the entrywise |K||x| from above; the terms of one entry (volume,
        # consistency, penalty) differ in size, so the bound stays close
        ratio = host(y) / np.maximum(scale, 1e-300)
        print(f"[ext] |K||x| ratio min {ratio.min():.3f} p99 {np.percentile(ratio, 99):.3f}", flush=True)
        assert ratio.min() >= 1 - 1e-12 and np.percentile(ratio, 99) <= 8
    P.close()


def _pair_host(a, b):
    return host(a), host(b)


@pytest.mark.parametrize("krylov", [0, 1])
def test_ext_viscous_solve_below_fp64_floor(sdg, ctx, torch, krylov):
    """32 x 32, Q_4, inclusion of viscosity 1e4: the FP64 floor of the
    true residual is about 1e-8 here (eps |A||u| / |F| ~ 8e-8); with
    refinement the pair reaches rtol = 1e-10 in the long-double residual
    (whose own evaluation floor, 2^-64 |A||u| / |F|, is about 1e-11 at this
    size), and the velocity is the refined oracle solution to 1e-9 (CG
    corrections, or FGMRES restarts)."""
    n, k = 32, 4
    prob = gen.single_inclusion(n, k, eta_in=1e4)
    m = Mesh(n, n, k)
    P = sdg.Problem(ctx, n, n, k, prob.eta, rtol=1e-10, max_it=2000, refine=1, viscous_krylov=krylov,
                    restart=60)
    u, ul = P.zeros(P.nu), P.zeros(P.nu)
    rc, st = sdg.sdg_solve_viscous_ext_dev(P.h, dev(prob.f.reshape(-1)), None, u, ul)
    print(f"[ext viscous] krylov={krylov} {st}", flush=True)
    assert st["status"] == 0, st
    uh, ulo = _pair_host(u, ul)
    res = rf.viscous_residual(m, prob.eta, prob.f, uh, ulo)
    print(f"[ext viscous] oracle long-double residual {res:.3e}", flush=True)
    # both evaluations (library and oracle) carry about 2^-63 |A||u| / |F|
    ld_floor = 2.0 ** -63 * float(np.linalg.norm(abs(asm.assemble_A(m, prob.eta)) @ np.abs(uh))
                                  / np.linalg.norm(prob.f))
    print(f"[ext viscous] long-double evaluation floor {ld_floor:.2e}", flush=True)
    assert res <= 1e-10 + 2 * ld_floor, res
    assert abs(res - st["rel_residual"]) <= 0.1 * res + 2 * ld_floor
    uref = rf.solve_viscous_ext(m, prob.eta, prob.f)
    err = float(np.linalg.norm((uh.astype(LD) + ulo.astype(LD) - uref).astype(np.float64))
                / np.linalg.norm(uref.astype(np.float64)))
    print(f"[ext viscous] |u - u_ref| / |u_ref| = {err:.3e}", flush=True)
    assert err <= 1e-9
    P.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ext_stokes_solve(sdg, ctx, torch, prec):
    """Stokes with FGMRES restarts as refinement steps, FP64 or FP32
    fine-level cycle: long-double residual of the pair below rtol = 1e-10,
    velocity to 1e-9 and pressure to 1e-8 of the refined reference (the
    error is a few times the residual at this contrast: rtol 1e-10 is what
    the velocity bar of 1e-9 needs)."""
    n, k = 16, 4
    prob = gen.single_inclusion(n, k, eta_in=1e4)
    m = Mesh(n, n, k)
    pa = sdg.FP32 if prec == "fp32" else sdg.FP64
    P = sdg.Problem(ctx, n, n, k, prob.eta, rtol=1e-10, inner_rtol=1e-3, max_it=600, refine=1, coarsest_n=4,
                    prec_apply=pa, prec_smoother=pa)
    u, ul, p, pl = P.zeros(P.nu), P.zeros(P.nu), P.zeros(P.np), P.zeros(P.np)
    rc, st = sdg.sdg_solve_stokes_ext_dev(P.h, dev(prob.f.reshape(-1)), None, u, ul, p, pl)
    print(f"[ext stokes {prec}] {st}", flush=True)
    assert st["status"] == 0, st
    uh, ulo = _pair_host(u, ul)
    ph, plo = _pair_host(p, pl)
    res = rf.stokes_residual(m, prob.eta, prob.f, uh, ph, ulo, plo)
    print(f"[ext stokes {prec}] oracle long-double residual {res:.3e}", flush=True)
    assert res <= 1.2e-10, res
    uref, pref = rf.solve_stokes_ext(m, prob.eta, prob.f, method="lu")
    eu = float(np.linalg.norm((uh.astype(LD) + ulo.astype(LD) - uref).astype(np.float64))
               / np.linalg.norm(uref.astype(np.float64)))
    ep = float(np.linalg.norm((ph.astype(LD) + plo.astype(LD) - pref).astype(np.float64))
               / np.linalg.norm(pref.astype(np.float64)))
    print(f"[ext stokes {prec}] velocity {eu:.3e} pressure {ep:.3e}", flush=True)
    assert eu <= 1e-9 and ep <= 1e-8
    P.close()


def test_ext_batched_grf_fp32_cycle_cg(sdg, ctx, torch):
    """The options of the batched random-field workload: CG with the FP32
    fine-level cycle and extended refinement, rtol 1e-8, three requests of
    one shape in one batch (n = 32, k = 3, log10 viscosity a Gaussian random
    field): each reaches 1e-8 in the long-double residual and the refined
    oracle velocity to 1e-9."""
    n, k = 32, 3
    probs = [gen.grf_problem(s, n=n, k=k) for s in range(3)]
    m = Mesh(n, n, k)
    P = sdg.Problem(ctx, n, n, k, np.stack([p.eta for p in probs]), rtol=1e-8, max_it=3000, refine=1,
                    prec_apply=sdg.FP32, prec_smoother=sdg.FP32)
    f = np.concatenate([p.f.reshape(-1) for p in probs])
    u, ul = P.zeros(P.nu), P.zeros(P.nu)
    rc, stats = sdg.sdg_solve_viscous_ext_dev(P.h, dev(f), None, u, ul)
    U, UL = host(u).reshape(3, -1), host(ul).reshape(3, -1)
    for i, pr in enumerate(probs):
        print(f"[ext grf] {i} {stats[i]}", flush=True)
        assert stats[i]["status"] == 0, stats[i]
        res = rf.viscous_residual(m, pr.eta, pr.f, U[i], UL[i])
        uref = rf.solve_viscous_ext(m, pr.eta, pr.f)
        err = float(np.linalg.norm((U[i].astype(LD) + UL[i].astype(LD) - uref).astype(np.float64))
                    / np.linalg.norm(uref.astype(np.float64)))
        print(f"[ext grf] {i} residual {res:.3e} velocity error {err:.3e}", flush=True)
        assert res <= 1e-8 and err <= 1e-9
    P.close()
