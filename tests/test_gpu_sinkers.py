"""The six sedimenting inclusions of Section 8.3 with GCR for the Stokes
(outer) and viscous (inner) solves, and a Neumann top side, through the C
ABI against the refined long-double oracle solution.  Iteration counts are
compared with Table 4 only qualitatively (parity unpinned: the paper's
counts depend on its h-level choices and rounding).  As in the paper's
six-inclusion runs (one h-level less than for SolCx) the coarsest h-level is
16 x 16 elements: coarser levels do not resolve the small high-contrast
inclusions (the oracle's CG with coarsest level 8 x 8 needs 77 iterations to
1e-3 at 64 x 64, k = 1, against 13 with 16 x 16)."""
import json
import os

import numpy as np
import pytest

from oracle import refine as rf
from oracle.mesh import Mesh
from paper_1607_03777_amd import inputs as gen

from gpu_helpers import dev, host

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


# The force g rho = 10 acts everywhere and is balanced almost entirely by
# the hydrostatic pressure; the velocity comes from the density anomaly 0.2
# of the inclusions alone, so |b| is large against what drives u and the
# relative velocity error runs about 300 times the relative residual
# (measured: residual 8e-11, velocity error 2e-8).  rtol 1e-12 meets the
# 1e-9 velocity bar.
@pytest.mark.parametrize("eta2", [1e3, 1e6])
def test_sinkers_gcr_stokes_matches_oracle(sdg, ctx, torch, eta2):
    n, k = 32, 2
    pr = gen.six_sinkers(n, k, eta2=eta2)
    m = Mesh(n, n, k, bc=pr.bc)
    print(f"[case] sinkers n={n} k={k} eta2={eta2:g}", flush=True)
    P = sdg.Problem(ctx, n, n, k, pr.eta, bc=pr.bc, rtol=1e-12, inner_rtol=1e-3, max_it=800, refine=1,
                    outer_krylov=1, viscous_krylov=2, coarsest_n=16)
    u, ul, p, pl = P.zeros(P.nu), P.zeros(P.nu), P.zeros(P.np), P.zeros(P.np)
    rc, st = sdg.sdg_solve_stokes_ext_dev(P.h, dev(pr.f.reshape(-1)), None, u, ul, p, pl)
    print(f"[sinkers] {st}", flush=True)
    assert st["status"] == 0, st
    res = rf.stokes_residual(m, pr.eta, pr.f, host(u), host(p), host(ul), host(pl))
    uref, pref = rf.solve_stokes_ext(m, pr.eta, pr.f, method="lu")
    uref, pref = uref.astype(np.float64), pref.astype(np.float64)
    eu = np.linalg.norm(host(u) - uref) / np.linalg.norm(uref)
    ep = np.linalg.norm(host(p) - pref) / np.linalg.norm(pref)
    # the library's and the oracle's evaluations each carry about
    # 2^-63 |K||x| / |b| (5e-13 here at eta2 = 1e6)
    K, b = rf.stokes_system(m, pr.eta, pr.f)
    x = np.concatenate([host(u), host(p)])
    ld_floor = 2.0 ** -63 * float(np.linalg.norm(abs(K.astype(np.float64)) @ np.abs(x))
                                  / np.linalg.norm(b.astype(np.float64)))
    print(f"[sinkers] residual {res:.2e} (floor {ld_floor:.1e}) velocity {eu:.2e} pressure {ep:.2e}", flush=True)
    assert res <= 1e-12 + 2 * ld_floor and eu <= 1e-9 and ep <= 1e-9
    P.close()


def test_sinkers_gcr_viscous_matches_oracle(sdg, ctx, torch):
    n, k = 32, 3
    pr = gen.six_sinkers(n, k, eta2=1e6)
    m = Mesh(n, n, k, bc=pr.bc)
    P = sdg.Problem(ctx, n, n, k, pr.eta, bc=pr.bc, rtol=1e-10, max_it=800, refine=1, viscous_krylov=2,
                    coarsest_n=16)
    u, ul = P.zeros(P.nu), P.zeros(P.nu)
    rc, st = sdg.sdg_solve_viscous_ext_dev(P.h, dev(pr.f.reshape(-1)), None, u, ul)
    print(f"[sinkers viscous] {st}", flush=True)
    assert st["status"] == 0, st
    uref = rf.solve_viscous_ext(m, pr.eta, pr.f).astype(np.float64)
    err = np.linalg.norm(host(u) - uref) / np.linalg.norm(uref)
    assert err <= 1e-9, err
    P.close()


def test_sinkers_iteration_counts_qualitative(sdg, ctx, torch):
    """Paper's setting (outer rtol 1e-6, inner 1e-3, GCR both loops) on
    64 x 64: outer iterations of the same order as Table 4 and nearly
    independent of the viscosity jump (the paper's observation)."""
    ref = json.load(open(os.path.join(GOLDEN, "six_sinkers.json")))
    n = 64
    outer = {}
    for k in (1, 2, 3):
        for eta2 in (1e3, 1e6):
            pr = gen.six_sinkers(n, k, eta2=eta2)
            P = sdg.Problem(ctx, n, n, k, pr.eta, bc=pr.bc, rtol=1e-6, inner_rtol=1e-3, max_it=400,
                            outer_krylov=1, viscous_krylov=2, coarsest_n=16)
            u, p, st = P.solve_stokes(dev(pr.f.reshape(-1)))
            outer[(k, eta2)] = st["outer_its"]
            print(f"[sinkers 64] k={k} eta2={eta2:g}: outer {st['outer_its']} inner avg "
                  f"{st['inner_its_total'] / max(st['outer_its'], 1):.1f} max {st['inner_its_max']} "
                  f"(Table 4, 1e6: {ref['table4_outer_its_64x64_eta1e6']['k%d' % k]} outer, inner avg/max "
                  f"{ref['table4_inner_avg_max_64x64_eta1e6']['k%d' % k]})", flush=True)
            assert st["status"] == 0, st
            P.close()
    for k in (1, 2, 3):
        t4 = ref["table4_outer_its_64x64_eta1e6"]["k%d" % k]
        assert outer[(k, 1e6)] <= 2 * t4
        assert max(outer[(k, 1e3)], outer[(k, 1e6)]) <= 2 * min(outer[(k, 1e3)], outer[(k, 1e6)])
