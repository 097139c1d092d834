"""Seeded draws: the batched-solve workload and seeded random arrays.

All random numbers come from numpy's PCG64 with an explicit seed and a fixed
draw order, so every consumer regenerates the same values.
"""

from __future__ import annotations

import numpy as np


def seeded_array(seed: int, shape, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Uniform float64 array in [lo, hi) from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=shape)


def batch_draws(n_solves: int = 64, seed: int = 1807):
    """Draws of the batched workload: per solve, in this order, the
    circumferential cell count N_theta ~ U{16..96}, the order p ~ U{1..4},
    the Mach number ~ U[0.1, 0.4] and the angle of attack ~ U[-5, 5] degrees;
    the radial count is N_theta // 2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n_solves):
        nt = int(rng.integers(16, 97))
        p = int(rng.integers(1, 5))
        ma = float(rng.uniform(0.1, 0.4))
        al = float(rng.uniform(-5.0, 5.0))
        out.append({"n_theta": nt, "n_r": nt // 2, "p": p, "mach": ma,
                    "alpha_deg": al})
    return out


def bump_centers(dim: int, n: int, seed: int = 1807) -> np.ndarray:
    """n seeded unit vectors (bump centres on the body): angles ~ U[0, 2 pi)
    in 2D; directions uniform on the sphere in 3D (normalised Gaussians)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if dim == 2:
        th = rng.uniform(0.0, 2.0 * np.pi, size=n)
        return np.stack([np.cos(th), np.sin(th)], axis=1)
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)
