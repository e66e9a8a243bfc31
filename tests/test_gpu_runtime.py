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
