"""The allocation-free entry point sdg_get_blocks_noalloc (element list in
the library's file-scope device array) against sdg_get_blocks, through the
C ABI: identical blocks on two calls in a row, the second with a smaller
problem, so that a stale list from the first call would show."""
import numpy as np
import pytest

from paper_1607_03777_amd import inputs as gen

from gpu_helpers import host

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


def test_get_blocks_noalloc_matches_allocating_form(sdg, torch):
    ctx = sdg.sdg_create(0, 0)
    try:
        for n, k, nbatch in ((12, 3, 3), (5, 2, 1)):  # second call smaller
            probs = [gen.random_problem(n, k, 40 + i, contrast=1e4) for i in range(nbatch)]
            print(f"[case] noalloc blocks n={n} k={k} nbatch={nbatch}", flush=True)
            P = sdg.Problem(ctx, n, n, k, np.stack([p.eta for p in probs]))
            nb = 2 * (k + 1) ** 2
            size = nbatch * n * n * nb * nb
            ref = P.zeros(size)
            got = torch.full((size,), np.nan, dtype=torch.float64, device="cuda")
            sdg.sdg_get_blocks(P.h, ref)
            sdg.sdg_get_blocks_noalloc(P.h, got)
            torch.cuda.synchronize()
            assert np.array_equal(host(got), host(ref))
            P.close()
        # beyond the limit: a clear error, nothing launched
        P = sdg.Problem(ctx, 512, 512, 1, np.ones((5, 512 * 512)))  # 5 x 262144 elements
        with pytest.raises(sdg.SDGError) as e:
            sdg.sdg_get_blocks_noalloc(P.h, torch.empty(1, dtype=torch.float64, device="cuda"))
        assert e.value.code == sdg.ERR_INVALID and "limit" in str(e.value)
        P.close()
    finally:
        sdg.sdg_destroy(ctx)
