"""Chebyshev tools (oracle; test infrastructure only).

- open grid u_k = cos((k + 1/2) pi / n)            Sec. III-A, eq. cheby_nodes
- Fejer weights                                     Sec. III-C, eq. fejer_weighs
- expansion f ~ sum_i w_i T_i with
  w_i = (2/n) c_i sum_j f(x_j) T_i(x_j), c_0 = 1/2  Sec. III-F (1D interpolation);
  the paper's garbled placement of c inside the sum is read as the standard
  discrete Chebyshev transform (c multiplies the output index).
- derivatives via the Chebyshev recurrence          Sec. III intro
Pins: closed forms in tests/test_oracle_cheb.py.
"""
from __future__ import annotations

import numpy as np


def nodes(n: int) -> np.ndarray:
    k = np.arange(n, dtype=np.float64)
    return np.cos((k + 0.5) * np.pi / n)


def fejer_weights(n: int) -> np.ndarray:
    """w_k = (2/n)[1 - 2 sum_{m=1}^{floor(n/2)} cos(m pi (2k+1)/n)/(4m^2-1)]."""
    k = np.arange(n, dtype=np.float64)
    s = np.zeros(n)
    for m in range(1, n // 2 + 1):
        s += np.cos(m * np.pi * (2 * k + 1) / n) / (4.0 * m * m - 1.0)
    return (2.0 / n) * (1.0 - 2.0 * s)


def T(nmax: int, x) -> np.ndarray:
    """T_0..T_{nmax-1} at x (any shape) by the three-term recurrence; last axis = degree."""
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(x.shape + (nmax,))
    out[..., 0] = 1.0
    if nmax > 1:
        out[..., 1] = x
    for k in range(2, nmax):
        out[..., k] = 2.0 * x * out[..., k - 1] - out[..., k - 2]
    return out


def dT(nmax: int, x) -> np.ndarray:
    """T'_0..T'_{nmax-1} at x: T'_k = k U_{k-1}, U by its recurrence."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape + (nmax,))
    if nmax > 1:
        U = np.empty(x.shape + (nmax,))
        U[..., 0] = 1.0
        if nmax > 1:
            U[..., 1] = 2.0 * x
        for k in range(2, nmax):
            U[..., k] = 2.0 * x * U[..., k - 1] - U[..., k - 2]
        for k in range(1, nmax):
            out[..., k] = k * U[..., k - 1]
    return out


def transform_matrix(n: int) -> np.ndarray:
    """M[i, j] = (2/n) c_i T_i(x_j): node values -> Chebyshev coefficients."""
    x = nodes(n)
    Tm = T(n, x)                    # [j, i]
    c = np.ones(n)
    c[0] = 0.5
    return (2.0 / n) * c[:, None] * Tm.T


def coefficients(f: np.ndarray, axis: int = 0) -> np.ndarray:
    """Chebyshev coefficients of node values along one axis."""
    n = f.shape[axis]
    M = transform_matrix(n)
    return np.moveaxis(np.tensordot(M, np.moveaxis(f, axis, 0), axes=(1, 0)), 0, axis)


def derivative_coefficients(c: np.ndarray, axis: int = 0) -> np.ndarray:
    """Coefficients of f' from those of f = sum_k c_k T_k.

    Uses d_{m-1} = d_{m+1} + 2 m c_m (m >= 2) and d_0 = c_1 + d_2 / 2, which
    follow from integrating T_k term by term.
    """
    c = np.moveaxis(np.asarray(c), axis, 0)
    n = c.shape[0]
    d = np.zeros((n + 1,) + c.shape[1:], dtype=c.dtype)
    for m in range(n - 1, 1, -1):
        d[m - 1] = d[m + 1] + 2.0 * m * c[m]
    if n > 1:
        d[0] = c[1] + 0.5 * d[2]
    return np.moveaxis(d[:n], 0, axis)


def evaluate(c: np.ndarray, x, axis: int = 0) -> np.ndarray:
    """sum_k c_k T_k(x) along `axis` of c, for a 1D array of points x."""
    n = c.shape[axis]
    Tx = T(n, np.asarray(x))        # [m, k]
    return np.moveaxis(np.tensordot(Tx, np.moveaxis(c, axis, 0), axes=(1, 0)), 0, axis)


def differentiate(f: np.ndarray, axis: int = 0) -> np.ndarray:
    """Values of f' at the open Chebyshev nodes from values of f there."""
    n = f.shape[axis]
    c = coefficients(f, axis)
    d = derivative_coefficients(c, axis)
    return evaluate(d, nodes(n), axis)
