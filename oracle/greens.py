"""Helmholtz Green's function (oracle; test infrastructure only).

G_k(x, y) = exp(i k |x - y|) / (4 pi |x - y|)        Sec. II, after eq. potential_t
grad_x G_k(x, y) = G_k(x, y) (i k - 1/r) (x - y)/r    (differentiating G in x)
Pins: symmetry G(x,y) = G(y,x), grad_x G = -grad_y G, and the radiating
Helmholtz equation checked by finite differences (tests/test_oracle_core.py).
"""
from __future__ import annotations

import numpy as np


def G(k: float, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    d = x - y
    r = np.sqrt(np.sum(d * d, axis=-1))
    return np.exp(1j * k * r) / (4.0 * np.pi * r)


def gradG(k: float, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    d = x - y
    r = np.sqrt(np.sum(d * d, axis=-1))
    g = np.exp(1j * k * r) / (4.0 * np.pi * r)
    return (g * (1j * k - 1.0 / r) / r)[..., None] * d
