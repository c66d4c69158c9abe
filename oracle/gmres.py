"""Plain GMRES (oracle; test infrastructure only).

Solves A y = b (Sec. III-A, eq. lin_system) with x0 = 0, Arnoldi by
classical Gram-Schmidt applied twice, Givens rotations, stopping when the
Arnoldi residual estimate satisfies |r| / |b| <= tol (the paper's tolerance
is 1e-4, Sec. IV); no restart up to maxit (reading A18).
Pin: converges to numpy.linalg.solve on small dense systems
(tests/test_oracle_nmuller.py).
"""
from __future__ import annotations

import numpy as np


def gmres(apply, b, tol=1e-4, maxit=500):
    """Returns (x, iterations, residual history)."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    beta = np.linalg.norm(b)
    n = b.size
    if beta == 0.0:
        return np.zeros_like(b), 0, [0.0]
    V = np.zeros((maxit + 1, n), dtype=np.complex128)
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    cs = np.zeros(maxit, dtype=np.complex128)
    sn = np.zeros(maxit, dtype=np.complex128)
    g = np.zeros(maxit + 1, dtype=np.complex128)
    g[0] = beta
    V[0] = b / beta
    hist = [1.0]
    k = 0
    for k in range(maxit):
        w = np.asarray(apply(V[k]), dtype=np.complex128).ravel()
        h = V[:k + 1].conj() @ w
        w = w - V[:k + 1].T @ h
        h2 = V[:k + 1].conj() @ w
        w = w - V[:k + 1].T @ h2
        h = h + h2
        hn = np.linalg.norm(w)
        H[:k + 1, k] = h
        H[k + 1, k] = hn
        for i in range(k):
            t = cs[i].conj() * H[i, k] + sn[i].conj() * H[i + 1, k]
            H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
            H[i, k] = t
        den = np.sqrt(abs(H[k, k]) ** 2 + abs(H[k + 1, k]) ** 2)
        cs[k] = H[k, k] / den
        sn[k] = H[k + 1, k] / den
        H[k, k] = den
        H[k + 1, k] = 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k].conj() * g[k]
        hist.append(abs(g[k + 1]) / beta)
        if hn > 0:
            V[k + 1] = w / hn
        if hist[-1] <= tol or hn == 0:
            break
    m = k + 1
    y = np.linalg.solve(np.triu(H[:m, :m]), g[:m])
    return V[:m].T @ y, m, hist
