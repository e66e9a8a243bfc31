"""GPU tests of the request server: requests of different shapes, kinds and
orders submitted together are admitted by memory, batched by shape and
overlapped; each result equals the same solve run alone (one-shot call)
within the stated tolerance, and the oracle's direct solution within the
solver tolerance."""
import numpy as np
import pytest

from oracle.direct import solve_stokes, solve_viscous
from oracle.mesh import Mesh
from paper_1607_03777_amd import inputs as gen

pytestmark = pytest.mark.gpu

RTOL = 1e-10
MIX_TOL = 1e-8  # |u_mix - u_alone| / |u_alone|: both solves stop at rtol 1e-10


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


def requests():
    reqs = []
    for s in range(3):  # one shape three times: one launch group
        reqs.append((gen.random_problem(8, 2, 10 + s, contrast=1e3), 0))
    for s in range(2):
        reqs.append((gen.random_problem(16, 3, 20 + s, contrast=1e2), 1))
    reqs.append((gen.single_inclusion(12, 2, eta_in=1e3), 1))
    reqs.append((gen.manufactured_stokes(8, 2), 1))
    reqs.append((gen.random_problem(8, 4, 30, contrast=1e2), 0))
    return reqs


def test_server_mix_matches_alone_and_oracle(sdg, torch):
    ctx = sdg.sdg_create(0, 0)
    srv = sdg.sdg_server_create(ctx, slots=3, max_batch=4)
    try:
        opts = sdg.make_options(rtol=RTOL, inner_rtol=1e-6, coarsest_n=4, max_it=400)
        reqs = requests()
        handles = []
        for prob, kind in reqs:
            mesh = sdg.make_mesh(prob.nx, prob.ny, prob.k, prob.bc)
            print(f"[case] submit {prob.name} kind={kind}", flush=True)
            handles.append(sdg.sdg_submit(srv, mesh, opts, kind, prob.eta, prob.f.reshape(-1),
                                          None if prob.g is None else prob.g.reshape(-1)))
        results = []
        for (prob, kind), h in zip(reqs, handles):
            rc, u, p, st, info = sdg.sdg_wait(h, prob.nu, prob.np_ if kind else 0)
            sdg.sdg_req_free(h)
            assert rc in (0, sdg.FLOOR), (prob.name, rc, st)
            assert info["start_ms"] >= info["submit_ms"] and info["end_ms"] >= info["start_ms"]
            results.append((u, p, info))
        stats = sdg.sdg_server_stats(srv)
        assert stats["completed"] == len(reqs)
        assert stats["peak_bytes"] <= stats["budget"]
        assert max(r[2]["batch"] for r in results) >= 2  # same-shape requests shared a launch
        for (prob, kind), (u, p, info) in zip(reqs, results):
            mesh = sdg.make_mesh(prob.nx, prob.ny, prob.k, prob.bc)
            ua = np.empty(prob.nu)
            g = None if prob.g is None else np.ascontiguousarray(prob.g.reshape(-1))
            f = np.ascontiguousarray(prob.f.reshape(-1))
            if kind:
                pa = np.empty(prob.np_)
                sdg.sdg_solve_stokes(ctx, mesh, opts, prob.eta, f, g, ua, pa)
                assert np.linalg.norm(p - pa) <= MIX_TOL * 10 * np.linalg.norm(pa), prob.name
            else:
                sdg.sdg_solve_viscous(ctx, mesh, opts, prob.eta, f, g, ua)
            assert np.linalg.norm(u - ua) <= MIX_TOL * np.linalg.norm(ua), prob.name
            m = Mesh(prob.nx, prob.ny, prob.k, bc=prob.bc)
            if kind:
                ud, _ = solve_stokes(m, prob.eta, prob.f, prob.g)
            else:
                ud = solve_viscous(m, prob.eta, prob.f, prob.g)
            assert np.linalg.norm(u - ud) <= 1e-7 * np.linalg.norm(ud), prob.name
    finally:
        sdg.sdg_server_destroy(srv)
        sdg.sdg_destroy(ctx)


def test_server_rejects_request_over_budget(sdg, torch):
    ctx = sdg.sdg_create(0, 0)
    srv = sdg.sdg_server_create(ctx, slots=1, max_batch=1, mem_budget=1 << 20)
    try:
        prob = gen.random_problem(32, 4, 1)
        mesh = sdg.make_mesh(32, 32, 4)
        with pytest.raises(sdg.SDGError) as e:
            sdg.sdg_submit(srv, mesh, sdg.make_options(), 0, prob.eta, prob.f.reshape(-1))
        assert e.value.code == sdg.ERR_NOMEM
    finally:
        sdg.sdg_server_destroy(srv)
        sdg.sdg_destroy(ctx)


# Combined launches (combine = 1) passed this test at this size, but runs of
# the request server with 8 slots and many requests (512 random-field
# viscous requests; 24 Poisson-arrival Stokes requests) ended in a host
# segmentation fault whose cause is not known; the option is off by default
# and its test stays skipped until the cause is found.
@pytest.mark.parametrize("combine", [
    0, pytest.param(1, marks=pytest.mark.skip(reason="combined launches: host crash at scale, cause not found"))])
def test_server_staggered_mixed_precision_matches_alone_and_oracle(sdg, torch, combine):
    """Requests of different shapes and kinds arriving one after another
    (staggered by a few milliseconds, while earlier ones run) with the
    mixed-precision options the serving workload uses (FP32 fine-level
    cycle, extended refinement): requests overlap in time (with combine,
    the later ones join the running combined launches, some launch covering
    several slots), and every result equals the same solve alone and the
    refined oracle solution."""
    import time
    from oracle import refine as rf
    ctx = sdg.sdg_create(0, 0)
    srv = sdg.sdg_server_create(ctx, slots=4, max_batch=2, combine=combine)
    try:
        # the pressure amplifies the residual by about 2e4 on the random
        # problems (measured: rtol 1e-10 leaves 2e-6 in p), so rtol is 1e-13
        opts = sdg.make_options(rtol=1e-13, inner_rtol=1e-3, coarsest_n=4, max_it=1200, refine=1,
                                prec_apply=sdg.FP32, prec_smoother=sdg.FP32)
        reqs = [(gen.random_problem(16, 2, 50, contrast=1e3), 1), (gen.single_inclusion(12, 3, eta_in=1e3), 1),
                (gen.random_problem(8, 4, 51, contrast=1e2), 0), (gen.random_problem(16, 2, 52, contrast=1e3), 1),
                (gen.random_problem(12, 3, 53, contrast=1e2), 0), (gen.single_inclusion(16, 2, eta_in=1e4), 1)]
        handles = []
        for prob, kind in reqs:
            mesh = sdg.make_mesh(prob.nx, prob.ny, prob.k, prob.bc)
            print(f"[case] staggered submit {prob.name} kind={kind}", flush=True)
            handles.append(sdg.sdg_submit(srv, mesh, opts, kind, prob.eta, prob.f.reshape(-1)))
            time.sleep(0.004)
        results = []
        for (prob, kind), h in zip(reqs, handles):
            rc, u, p, st, info = sdg.sdg_wait(h, prob.nu, prob.np_ if kind else 0)
            sdg.sdg_req_free(h)
            assert rc == 0 and st["rel_residual"] < 1e-13, (prob.name, rc, st)
            results.append((u, p, info))
        ls = sdg.sdg_server_launch_stats(srv)
        print(f"[staggered] launch stats {ls}", flush=True)
        if combine:
            assert ls["combined"] >= 1 and ls["max_width"] >= 2
        else:
            assert ls["launches"] == 0
        iv = [(r[2]["start_ms"], r[2]["end_ms"]) for r in results]
        overlap = max(min(a[1], b[1]) - max(a[0], b[0]) for i, a in enumerate(iv) for b in iv[i + 1:])
        assert overlap > 0  # at least two requests ran at the same time
        for (prob, kind), (u, p, info) in zip(reqs, results):
            mesh = sdg.make_mesh(prob.nx, prob.ny, prob.k, prob.bc)
            ua = np.empty(prob.nu)
            f = np.ascontiguousarray(prob.f.reshape(-1))
            m = Mesh(prob.nx, prob.ny, prob.k, bc=prob.bc)
            if kind:
                pa = np.empty(prob.np_)
                sdg.sdg_solve_stokes(ctx, mesh, opts, prob.eta, f, None, ua, pa)
                ud, pd = rf.solve_stokes_ext(m, prob.eta, prob.f, method="lu")
                ud, pd = ud.astype(np.float64), pd.astype(np.float64)
                assert np.linalg.norm(p - pa) <= 1e-8 * np.linalg.norm(pa), prob.name
                assert np.linalg.norm(p - pd) <= 1e-8 * np.linalg.norm(pd), prob.name
            else:
                sdg.sdg_solve_viscous(ctx, mesh, opts, prob.eta, f, None, ua)
                ud = rf.solve_viscous_ext(m, prob.eta, prob.f).astype(np.float64)
            eu_a = np.linalg.norm(u - ua) / np.linalg.norm(ua)
            eu_o = np.linalg.norm(u - ud) / np.linalg.norm(ud)
            print(f"[staggered] {prob.name}: vs alone {eu_a:.2e} vs oracle {eu_o:.2e}", flush=True)
            assert eu_a <= 1e-9 and eu_o <= 1e-9, prob.name
    finally:
        sdg.sdg_server_destroy(srv)
        sdg.sdg_destroy(ctx)
