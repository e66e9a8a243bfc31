"""1D Legendre polynomials on [-1, 1] (oracle; test infrastructure only).

The velocity and pressure spaces use tensor products of Legendre polynomials
(Section 5: pairwise orthogonal Legendre basis; the pressure basis is
orthonormal).  Here every 1D factor is scaled to be L2(-1,1)-orthonormal:
lhat_i = sqrt((2i+1)/2) L_i.  Values come from Bonnet's three-term recurrence
and derivatives from L'_{n+1} = L'_{n-1} + (2n+1) L_n, evaluated pointwise,
so nothing here relies on a closed-form trace or derivative table.
"""
import numpy as np


def legendre_values(nmax, x):
    """L_0..L_nmax at points x; shape (nmax+1, len(x))."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((nmax + 1,) + x.shape)
    out[0] = 1.0
    if nmax >= 1:
        out[1] = x
    for n in range(1, nmax):
        out[n + 1] = ((2 * n + 1) * x * out[n] - n * out[n - 1]) / (n + 1)
    return out


def legendre_derivs(nmax, x):
    """L'_0..L'_nmax at points x; shape (nmax+1, len(x))."""
    x = np.asarray(x, dtype=np.float64)
    vals = legendre_values(nmax, x)
    out = np.zeros_like(vals)
    if nmax >= 1:
        out[1] = 1.0
    for n in range(1, nmax):
        out[n + 1] = out[n - 1] + (2 * n + 1) * vals[n]
    return out


def onb_scale(nmax):
    """sqrt((2i+1)/2), the factor making L_i orthonormal on [-1, 1]."""
    i = np.arange(nmax + 1, dtype=np.float64)
    return np.sqrt((2.0 * i + 1.0) / 2.0)


def onb_values(nmax, x):
    return onb_scale(nmax)[:, None] * legendre_values(nmax, x)


def onb_derivs(nmax, x):
    return onb_scale(nmax)[:, None] * legendre_derivs(nmax, x)


def gauss(npts):
    """Gauss-Legendre points and weights on [-1, 1] (numpy's routine)."""
    return np.polynomial.legendre.leggauss(npts)
