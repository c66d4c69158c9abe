"""Seeded random inputs (numpy PCG64 via default_rng)."""
from __future__ import annotations

import numpy as np


def complex_normal(shape, seed: int) -> np.ndarray:
    """i.i.d. N(0,1) real and imaginary parts."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _tangent_frame(d):
    """Deterministic orthonormal (e1, e2) perpendicular to unit d."""
    a = np.array([1.0, 0.0, 0.0]) if abs(d[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = a - d * np.dot(a, d)
    e1 /= np.sqrt(np.dot(e1, e1))
    e2 = np.cross(d, e1)
    return e1, e2


def plane_wave_batch(n: int, seed: int):
    """n plane waves: directions uniform on S^2, polarisations uniform in the
    tangent plane.  Returns (d [n,3], p [n,3]), unit vectors with d.p = 0."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.sqrt(np.sum(d * d, axis=1))[:, None]
    psi = rng.uniform(0.0, 2.0 * np.pi, n)
    p = np.empty_like(d)
    for r in range(n):
        e1, e2 = _tangent_frame(d[r])
        p[r] = np.cos(psi[r]) * e1 + np.sin(psi[r]) * e2
    return d, p


def ellipsoid_batch(n: int, seed0: int, axis_range=(0.5, 3.0), eps_range=(1.5, 4.0)):
    """n ellipsoid specs (a, b, c, eps_r), body i drawn from seed seed0 + i."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed0 + i)
        a, b, c = rng.uniform(axis_range[0], axis_range[1], 3)
        eps = rng.uniform(eps_range[0], eps_range[1])
        out.append((float(a), float(b), float(c), float(eps)))
    return out
