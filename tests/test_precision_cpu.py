"""Host checks of the precision readings behind the low-precision smoother
(no GPU): the BF16 rounding of the inverse Cholesky factor X = L^{-1}
(round to nearest even of the FP32 value) keeps the smoothed element block
X~^T X~ B near the identity for moderately conditioned blocks, and moves its
largest eigenvalue far above the exact inverse's 1 for a block of condition
near the reciprocal of the BF16 unit, which is what the setup's fallback to
FP32 factors guards against."""
import numpy as np

import oracle.assemble as asm
from oracle.mesh import Mesh
from oracle.multigrid import BlockJacobi
from paper_1607_03777_amd import inputs as gen


def _bf16(x):
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _worst(n, k, seed):
    pr = gen.random_inclusions(n, k, seed=seed)
    m = Mesh(n, n, k)
    blocks = BlockJacobi(asm.assemble_A(m, pr.eta), m.nbu).blocks
    cond = np.linalg.cond(blocks)
    e = int(np.argmax(cond))
    X = np.linalg.inv(np.linalg.cholesky(blocks[e]))
    lam = np.linalg.eigvals(_bf16(X).T @ _bf16(X) @ blocks[e]).real.max()
    lam32 = np.linalg.eigvals(X.astype(np.float32).astype(np.float64).T
                              @ X.astype(np.float32).astype(np.float64) @ blocks[e]).real.max()
    return cond[e], lam, lam32


def test_bf16_factor_of_a_near_singular_block_overshoots():
    cond, lam, lam32 = _worst(32, 5, 5)
    assert cond > 1e7
    assert lam > 10.0          # BF16: an order of magnitude above the exact 1
    assert abs(lam32 - 1.0) < 0.05  # FP32 (unit 6e-8) still holds


def test_bf16_factor_of_moderate_blocks_holds():
    cond, lam, _ = _worst(32, 4, 4)
    assert cond < 1e6 and lam < 2.0
