"""1D Legendre polynomials on [-1, 1] (oracle; test infrastructure only).

The velocity and pressure spaces use tensor products of Legendre polynomials
(Section 5: pairwise orthogonal Legendre basis; the pressure basis is
orthonormal).  Here every 1D factor is scaled to be L2(-1,1)-orthonormal:
lhat_i = sqrt((2i+1)/2) L_i.  Values come from Bonnet's three-term recurrence
and derivatives from L'_{n+1} = L'_{n-1} + (2n+1) L_n, evaluated pointwise,
so nothing here relies on a closed-form trace or derivative table.

Every routine works in the floating type of its input points (float64, or
numpy.longdouble for the extended-precision residual of the refinement
check, Section 8.3.1); `gauss` takes the type as an argument.
"""
import numpy as np


def _ftype(x):
    dt = np.asarray(x).dtype
    return dt if dt == np.longdouble else np.dtype(np.float64)


def legendre_values(nmax, x):
    """L_0..L_nmax at points x; shape (nmax+1, len(x))."""
    x = np.asarray(x, dtype=_ftype(x))
    out = np.zeros((nmax + 1,) + x.shape, dtype=x.dtype)
    out[0] = 1.0
    if nmax >= 1:
        out[1] = x
    for n in range(1, nmax):
        out[n + 1] = ((2 * n + 1) * x * out[n] - n * out[n - 1]) / (n + 1)
    return out


def legendre_derivs(nmax, x):
    """L'_0..L'_nmax at points x; shape (nmax+1, len(x))."""
    x = np.asarray(x, dtype=_ftype(x))
    vals = legendre_values(nmax, x)
    out = np.zeros_like(vals)
    if nmax >= 1:
        out[1] = 1.0
    for n in range(1, nmax):
        out[n + 1] = out[n - 1] + (2 * n + 1) * vals[n]
    return out


def onb_scale(nmax, dtype=np.float64):
    """sqrt((2i+1)/2), the factor making L_i orthonormal on [-1, 1]."""
    i = np.arange(nmax + 1, dtype=dtype)
    return np.sqrt((2 * i + 1) / 2)


def onb_values(nmax, x):
    return onb_scale(nmax, _ftype(x))[:, None] * legendre_values(nmax, x)


def onb_derivs(nmax, x):
    return onb_scale(nmax, _ftype(x))[:, None] * legendre_derivs(nmax, x)


def gauss(npts, dtype=np.float64):
    """Gauss-Legendre points and weights on [-1, 1].

    float64: numpy's routine.  longdouble: numpy's points refined by Newton
    steps on L_n in long double, weights 2 / ((1 - x^2) L_n'(x)^2) (the
    standard formula), so both carry the type's full precision."""
    g, w = np.polynomial.legendre.leggauss(npts)
    if np.dtype(dtype) != np.longdouble:
        return g, w
    x = g.astype(np.longdouble)
    for _ in range(3):
        x = x - legendre_values(npts, x)[npts] / legendre_derivs(npts, x)[npts]
    d = legendre_derivs(npts, x)[npts]
    return x, 2 / ((1 - x * x) * d * d)
