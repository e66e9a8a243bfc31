"""Shared helpers of the GPU parity tests: device problems and oracle
references built from the same seeded inputs."""
import numpy as np

from oracle import assemble as asm
from oracle.mesh import Mesh


def torch_mod():
    import torch
    return torch


def dev(a, dtype=None):
    torch = torch_mod()
    t = torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    if dtype is not None:
        t = t.to(dtype)
    return t.contiguous()


def host(t):
    return t.detach().cpu().numpy()


def oracle_mesh(nx, ny, k, bc):
    return Mesh(nx, ny, k, bc=tuple(bc))


def abs_bound(A, u):
    """|A| |u| componentwise: the scale of rounding error in A u."""
    Aa = abs(A)
    return Aa @ np.abs(u)


def assert_close_componentwise(y, yref, bound, rel):
    """|y - yref| <= rel * (bound + 1e-2 * max(bound)) componentwise: the
    rounding bound, widened by a normwise floor for entries whose exact value
    is zero (where the quadrature-assembled reference carries roundoff)."""
    err = np.abs(y - yref)
    floor = 1e-2 * np.max(bound) if bound.size else 0.0
    worst = np.max(err / (bound + floor + 1e-300))
    assert worst <= rel, f"componentwise error {worst:.3e} > {rel:.1e} (max abs err {err.max():.3e})"


def stencil_to_matrix(st, nx, ny):
    """9-point 2x2-block stencil [36][nn] -> dense matrix on 2*nn unknowns."""
    nn = (nx + 1) * (ny + 1)
    st = st.reshape(36, nn)
    A = np.zeros((2 * nn, 2 * nn))
    for jy in range(ny + 1):
        for jx in range(nx + 1):
            node = jy * (nx + 1) + jx
            for sy in (-1, 0, 1):
                for sx in (-1, 0, 1):
                    gx, gy = jx + sx, jy + sy
                    if not (0 <= gx <= nx and 0 <= gy <= ny):
                        continue
                    s = (sy + 1) * 3 + (sx + 1)
                    nb = gy * (nx + 1) + gx
                    for d in range(2):
                        for c in range(2):
                            A[2 * node + d, 2 * nb + c] += st[s * 4 + d * 2 + c, node]
    return A
