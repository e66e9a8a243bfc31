"""Batching form: sdg_solve_viscous_batch over requests of different meshes
and orders (one batched problem per shape, CG iterations of all shapes in
lockstep, each iteration one replay of a combined graph), through the C ABI:
every result equals the same request solved alone and the refined oracle
solution."""
import numpy as np
import pytest

from oracle import refine as rf
from oracle.mesh import Mesh
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


SHAPES = [(16, 2, 0), (16, 2, 1), (32, 3, 2), (8, 5, 3), (16, 4, 4), (32, 3, 5)]


@pytest.mark.parametrize("prec,refine", [("fp32", 1), ("fp64", 1), ("fp64", 0)])
def test_heterogeneous_batch_matches_alone_and_oracle(sdg, torch, prec, refine):
    ctx = sdg.sdg_create(0, 0)
    try:
        pa = sdg.FP32 if prec == "fp32" else sdg.FP64
        # without refinement CG stops on its recursive residual, and the true
        # residual is then limited by the FP64 floor (a few 1e-9 here)
        rtol = 1e-10 if refine else 1e-8
        opts = sdg.make_options(rtol=rtol, max_it=3000, refine=refine, prec_apply=pa, prec_smoother=pa)
        probs = [gen.grf_problem(seed, n=n, k=k) for n, k, seed in SHAPES]
        meshes = [sdg.make_mesh(p.nx, p.ny, p.k) for p in probs]
        print(f"[case] batch {prec} refine={refine}: {[(p.nx, p.k) for p in probs]}", flush=True)
        rc, us, los, stats = sdg.sdg_solve_viscous_batch(ctx, meshes, opts, [p.eta for p in probs],
                                                         [p.f for p in probs], with_lo=True)
        for p, u, lo, st in zip(probs, us, los, stats):
            print(f"[batch] {p.name}: {st}", flush=True)
            assert st["status"] == 0, st
            if refine:
                assert st["rel_residual"] < rtol, st
            ua = np.empty(p.nu)
            rca, sta = sdg.sdg_solve_viscous(ctx, sdg.make_mesh(p.nx, p.ny, p.k), opts, p.eta,
                                             np.ascontiguousarray(p.f.reshape(-1)), None, ua)
            assert sta["status"] == 0, sta
            m = Mesh(p.nx, p.ny, p.k)
            uref = rf.solve_viscous_ext(m, p.eta, p.f).astype(np.float64)
            e_alone = np.linalg.norm(u - ua) / np.linalg.norm(ua)
            e_ref = np.linalg.norm(u - uref) / np.linalg.norm(uref)
            print(f"[batch] {p.name}: |u - u_alone| {e_alone:.2e}  |u - u_oracle| {e_ref:.2e}", flush=True)
            # both stop at rtol; at these contrasts the error is a few times the residual
            assert e_alone <= 20 * rtol
            assert e_ref <= (1e-9 if refine else 1e-7)
            if refine:
                assert rf.viscous_residual(m, p.eta, p.f, u, lo) < rtol * 1.5
            else:
                assert not np.any(lo)
    finally:
        sdg.sdg_destroy(ctx)


def test_heterogeneous_batch_setup_error_reported(sdg, torch):
    """The shape groups are set up on several host threads: a group whose
    setup fails (every side traction-free: problem creation rejects the
    rigid motions) fails the call with its own code and the message set on
    the thread that set it up, and the context then serves a valid batch."""
    from oracle.mesh import NEUMANN
    ctx = sdg.sdg_create(0, 0)
    try:
        opts = sdg.make_options(rtol=1e-8, max_it=3000, refine=1)
        probs = [gen.grf_problem(seed, n=n, k=k) for n, k, seed in SHAPES[:4]]
        meshes = [sdg.make_mesh(p.nx, p.ny, p.k) for p in probs]
        meshes[2] = sdg.make_mesh(probs[2].nx, probs[2].ny, probs[2].k, bc=(NEUMANN,) * 4)
        print("[case] batch with one traction-free group", flush=True)
        with pytest.raises(sdg.SDGError) as e:
            sdg.sdg_solve_viscous_batch(ctx, meshes, opts, [p.eta for p in probs], [p.f for p in probs])
        assert e.value.code == sdg.ERR_UNSUPPORTED
        assert "singular (rigid motions)" in str(e.value)
        good = [sdg.make_mesh(p.nx, p.ny, p.k) for p in probs]
        rc, us, _, stats = sdg.sdg_solve_viscous_batch(ctx, good, opts, [p.eta for p in probs],
                                                       [p.f for p in probs])
        assert all(st["status"] == 0 for st in stats), stats
    finally:
        sdg.sdg_destroy(ctx)
