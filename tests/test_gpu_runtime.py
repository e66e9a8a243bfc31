"""GPU tests of the runtime around the solver: kernel tracing (per-launch
HIP events and algorithmic bytes)."""
import numpy as np
import pytest

from paper_1607_03777_amd import inputs as gen

pytestmark = pytest.mark.gpu


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


def test_trace_counts_launches_and_bytes(sdg, torch):
    ctx = sdg.sdg_create(0, 0)
    try:
        n, k, nbatch = 16, 3, 2
        P0 = gen.single_inclusion(n, k, eta_in=1e2)
        print(f"[case] trace n={n} k={k} nbatch={nbatch}", flush=True)
        prob = sdg.Problem(ctx, n, n, k, np.stack([P0.eta, P0.eta]))
        u = torch.randn(prob.nu, dtype=torch.float64, device="cuda")
        y = prob.zeros(prob.nu)
        sdg.sdg_trace_enable(ctx, 1)
        for _ in range(3):
            sdg.sdg_apply_viscous(prob.h, u, y)
        sdg.sdg_apply_blockjacobi(prob.h, u, y)
        sdg.sdg_trace_enable(ctx, 0)
        sdg.sdg_apply_viscous(prob.h, u, y)  # not traced
        nel, nb = n * n * nbatch, 2 * (k + 1) ** 2
        la, ms_a, by_a = sdg.sdg_trace_read(ctx, sdg.TRACE_SIP_APPLY)
        assert la == 3 and ms_a > 0
        assert by_a == 3 * nel * (2 * nb * 8 + 8)
        ls, ms_s, by_s = sdg.sdg_trace_read(ctx, sdg.TRACE_SMOOTHER)
        assert ls == 1 and ms_s > 0 and by_s == nel * (2 * nb * 8 + 12)
        # a solve traces every class of the cycle
        sdg.sdg_trace_enable(ctx, 1)
        f = torch.as_tensor(np.concatenate([P0.f.reshape(-1)] * 2), device="cuda")
        u2, st = prob.solve_viscous(f)
        sdg.sdg_trace_enable(ctx, 0)
        for cls in (sdg.TRACE_SIP_APPLY, sdg.TRACE_SIP_RESIDUAL, sdg.TRACE_SMOOTHER,
                    sdg.TRACE_COARSE_TAIL):
            nl, ms, _ = sdg.sdg_trace_read(ctx, cls)
            assert nl > 0 and ms > 0, cls
        prob.close()
    finally:
        sdg.sdg_destroy(ctx)


def test_autotune_picks_valid_shapes_and_keeps_results(sdg, torch):
    ctx = sdg.sdg_create(0, 0)
    try:
        n, k = 24, 4
        P0 = gen.single_inclusion(n, k, eta_in=1e3)
        print(f"[case] autotune n={n} k={k}", flush=True)
        prob = sdg.Problem(ctx, n, n, k, P0.eta, prec_apply=sdg.FP32, prec_smoother=sdg.FP32, rtol=1e-10)
        f = torch.as_tensor(P0.f.reshape(-1), device="cuda")
        u0, st0 = prob.solve_viscous(f)
        var, us = sdg.sdg_autotune(prob.h, 5)
        nv = sdg.sdg_tile_variants(k)
        assert set(var) == {(sdg.TILE_APPLY, sdg.FP64), (sdg.TILE_APPLY, sdg.FP32),
                            (sdg.TILE_RESIDUAL, sdg.FP64), (sdg.TILE_RESIDUAL, sdg.FP32)}
        assert all(0 <= v < nv for v in var.values()) and all(t > 0 for t in us.values())
        u1, st1 = prob.solve_viscous(f)
        assert st1["status"] == st0["status"] == 0
        # tile shapes change the rounding order of the fused operations only
        assert float((u1 - u0).norm() / u0.norm()) <= 1e-8
        # a later problem of the same shape starts from the tuned shapes
        prob2 = sdg.Problem(ctx, n, n, k, P0.eta, prec_apply=sdg.FP32, prec_smoother=sdg.FP32, rtol=1e-10)
        for (kern, pr), v in var.items():
            assert sdg.sdg_get_tile(prob2.h, kern, pr) == v
        u2, _ = prob2.solve_viscous(f)
        assert float((u2 - u1).norm() / u1.norm()) <= 1e-8
        prob2.close()
        prob.close()
    finally:
        sdg.sdg_destroy(ctx)


def test_cg_with_tile_kernel_apply_matches_wavefront(sdg, torch):
    """The CG takes p.q from the wavefront operator kernel's per-tile partial
    sums, or, when the apply runs on a tile-kernel shape, from a separate
    first reduction stage; in both cases the update kernels finish the sums.
    A batch of two problems solved each way converges to the same solution."""
    ctx = sdg.sdg_create(0, 0)
    try:
        n, k = 24, 4
        P0 = gen.single_inclusion(n, k, eta_in=1e3)
        P1 = gen.random_problem(n, k, 7, contrast=1e2)
        etas = np.stack([P0.eta, P1.eta])
        f = torch.as_tensor(np.concatenate([P0.f.reshape(-1), P1.f.reshape(-1)]), device="cuda")
        print(f"[case] cg apply forms n={n} k={k} batch 2", flush=True)
        wave = sdg.Problem(ctx, n, n, k, etas, rtol=1e-10)
        tile = sdg.Problem(ctx, n, n, k, etas, rtol=1e-10)
        assert sdg.sdg_get_tile(wave.h, sdg.TILE_APPLY, sdg.FP64) == 0
        sdg.sdg_set_tile(tile.h, sdg.TILE_APPLY, sdg.FP64, 1)
        uw, stw = wave.solve_viscous(f)
        ut, stt = tile.solve_viscous(f)
        for a, b in zip(stw, stt):
            assert a["status"] == 0 and b["status"] == 0, (a, b)
            # the two forms differ only in rounding order (CG iterations)
            assert abs(a["outer_its"] - b["outer_its"]) <= 2, (a, b)
        assert float((ut - uw).norm() / uw.norm()) <= 1e-8
        tile.close()
        wave.close()
    finally:
        sdg.sdg_destroy(ctx)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replay_matches_eager(sdg, torch, prec):
    """CG iterations replayed from captured HIP graphs give bit-identical
    solutions to eager launches, on every solve of a sequence (the graphs are
    captured once and replayed across solves, with eager work and host
    synchronisations between the replays)."""
    ctx = sdg.sdg_create(0, 0)
    try:
        n, k = 16, 3
        P0 = gen.single_inclusion(n, k, eta_in=1e3)
        P1 = gen.random_problem(n, k, 5, contrast=1e2)
        etas = np.stack([P0.eta, P1.eta])
        f = torch.as_tensor(np.concatenate([P0.f.reshape(-1), P1.f.reshape(-1)]), device="cuda")
        p32 = sdg.FP32 if prec == "fp32" else sdg.FP64
        print(f"[case] graphs n={n} k={k} prec={prec}", flush=True)
        eager = sdg.Problem(ctx, n, n, k, etas, graphs=0, prec_apply=p32, prec_smoother=p32, rtol=1e-10)
        graph = sdg.Problem(ctx, n, n, k, etas, graphs=1, prec_apply=p32, prec_smoother=p32, rtol=1e-10)
        for rep in range(3):
            ue, ste = eager.solve_viscous(f)
            ug, stg = graph.solve_viscous(f)
            torch.cuda.synchronize()
            assert torch.equal(ue, ug), rep
            assert [s["outer_its"] for s in ste] == [s["outer_its"] for s in stg]
            ue, pe, _ = eager.solve_stokes(f)
            ug, pg, _ = graph.solve_stokes(f)
            torch.cuda.synchronize()
            assert torch.equal(ue, ug) and torch.equal(pe, pg), rep
        eager.close()
        graph.close()
    finally:
        sdg.sdg_destroy(ctx)
