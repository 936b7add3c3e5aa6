"""Seeded synthetic inputs shared by the GPU path and the oracle.

This module draws random numbers and nothing else: it holds none of the
lattice Boltzmann arithmetic.  The generator is SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014), used
as a counter-based generator: draw k of stream `seed` is
mix(seed + (k + 1) * 0x9E3779B97F4A7C15).
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Draws offset .. offset+count-1 of the SplitMix64 stream `seed` (uint64)."""
    with np.errstate(over="ignore"):
        k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of each draw."""
    return (splitmix64(seed, count, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def theta_noise(n: int, seed: int, amp: float = 1e-6) -> np.ndarray:
    """Initial temperature perturbation: amp * (2U - 1) per node, U uniform in
    [0, 1), node index x + n*(y + n*z).  Returned flat (n^3,) float64."""
    return amp * (2.0 * uniform01(seed, n ** 3) - 1.0)


def random_fields(n: int, seed: int, u_amp: float = 0.03, theta_amp: float = 0.5) -> np.ndarray:
    """Velocity and temperature fields for initialisation tests: u, v, w
    uniform in [-u_amp, u_amp) and theta in [-theta_amp, theta_amp) per node,
    FP32, shaped (4, n, n, n) indexed [field, z, y, x]."""
    u = 2.0 * uniform01(seed, 4 * n ** 3).reshape(4, n, n, n) - 1.0
    amp = np.array([u_amp, u_amp, u_amp, theta_amp])[:, None, None, None]
    return (amp * u).astype(np.float32)


def batch_cases(seed: int, count: int, sizes=(32, 48, 64, 80, 96),
                log10_ra=(3.0, 6.0), wall_types=(1, 2, 3)):
    """A batch of cavities: edge length uniform over `sizes`, Ra log-uniform in
    10**log10_ra, wall type uniform over `wall_types`; three draws per cavity."""
    u = uniform01(seed, 3 * count).reshape(count, 3)
    cases = []
    for k in range(count):
        n = sizes[min(int(u[k, 0] * len(sizes)), len(sizes) - 1)]
        ra = 10.0 ** (log10_ra[0] + (log10_ra[1] - log10_ra[0]) * u[k, 1])
        wt = wall_types[min(int(u[k, 2] * len(wall_types)), len(wall_types) - 1)]
        cases.append({"n": int(n), "ra": float(ra), "wall_type": int(wt),
                      "seed": int(splitmix64(seed ^ 0x5EED, 1, k)[0] & 0x7FFFFFFFFFFFFFFF)})
    return cases
