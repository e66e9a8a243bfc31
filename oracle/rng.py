"""SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), used counter-style (oracle; test infrastructure).

The i-th output (i = 0, 1, ...) for seed s is mix(s + (i+1) * GOLDEN) with
the published finaliser
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9
    z ^= z >> 27; z *= 0x94D049BB133111EB
    z ^= z >> 31
all modulo 2^64.  A double in [-1, 1) is 2 * (z >> 11) * 2^-53 - 1.

The eigenvalue estimate of the Chebyshev smoother (Section 6: ten GMRES
iterations with a random right-hand side) draws its start vector from this
generator, stream seed + level * 2^32, so that the GPU library (which
implements the same published generator independently) starts from the
identical vector.
"""
import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK = (1 << 64) - 1


def splitmix64(seed, count):
    """First `count` outputs as uint64 (vectorised with numpy wrap-around)."""
    with np.errstate(over="ignore"):
        i = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed & MASK) + i * np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_scalar(seed, i):
    """Pure-Python reference of one output (for cross-checking)."""
    z = (seed + (i + 1) * GOLDEN) & MASK
    z = ((z ^ (z >> 30)) * M1) & MASK
    z = ((z ^ (z >> 27)) * M2) & MASK
    return z ^ (z >> 31)


def uniform_pm1(seed, count):
    z = splitmix64(seed, count)
    return (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 * 2.0 - 1.0


def level_stream(seed, level):
    return (seed + (level << 32)) & MASK
