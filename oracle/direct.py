"""O1: the plain O(N^2) regular sums (oracle; test infrastructure only).

For wavenumbers kappa_q (q = 0, 1), densities phi_k (k = 0..7), weights w:

  S_q[phi_k](x_l) = sum_{m != l} w_m phi_k(x_m) G_q(x_l, x_m)             k = 0..7
  D_q[phi_k](x_l) = sum_{m != l} w_m phi_k(x_m) n_l . grad_x G_q(x_l, x_m) k = 0..5

This is the paper's eq. ifgf_sum (self term excluded, Sec. III-E) for the
array of eight densities and two kernels of eq. ifgf_sum_em (Sec. III-I),
plus the normal derivative of eq. dl_scalar (Sec. III intro).  The divergence
densities (k = 6, 7) need S only (Sec. III intro).

Output layout: out[q, c, l] with c = 0..7 the S sums, c = 8..13 the D sums.
Pins: brute force is the definition; checked against the sphere eigenvalue
closed forms once the singular correction is added (tests/test_oracle_nmuller.py).
"""
from __future__ import annotations

import numpy as np

NS = 8   # densities with S
ND = 6   # densities with D


def regular_sums(x, normals, weights, phi, kappas, targets=None, block=None):
    """Direct regular sums.

    x [N,3], normals [N,3], weights [N], phi [8,N] complex (unweighted),
    kappas (k0, k1).  targets: optional index array of target points (the
    self term excluded is the target's own index).  Returns [2,14,T].
    Targets are taken `block` at a time (default: about 2^24 target-source
    pairs per block, which bounds the temporaries to a few GB).
    """
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    if block is None:
        block = max(1, min(256, (1 << 24) // max(N, 1)))
    a = np.asarray(phi) * np.asarray(weights)[None, :]
    tgt = np.arange(N) if targets is None else np.asarray(targets)
    out = np.zeros((2, NS + ND, tgt.size), dtype=np.complex128)
    for b0 in range(0, tgt.size, block):
        t = tgt[b0:b0 + block]
        d = x[t, None, :] - x[None, :, :]                    # [bt, N, 3]
        r = np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2])
        self_mask = np.zeros_like(r, dtype=bool)
        self_mask[np.arange(t.size), t] = True
        r = np.where(self_mask, 1.0, r)
        nd = np.sum(normals[t, None, :] * d, axis=-1)        # n_l . (x_l - x_m)
        for q, k in enumerate(kappas):
            g = np.exp(1j * k * r) / (4.0 * np.pi * r)
            g = np.where(self_mask, 0.0, g)
            out[q, :NS, b0:b0 + t.size] = (g @ a.T).T
            gd = g * (1j * k - 1.0 / r) / r * nd
            out[q, NS:, b0:b0 + t.size] = (gd @ a[:ND].T).T
    return out


def sums_at(x, weights, phi, kappas, X, dirs, block=256):
    """Direct sums at points X [M, 3] that are not sources (no term excluded):
    out[q, c, t] = sum_m w_m phi_c(x_m) G_q(X_t, x_m) (c < 8) and
    out[q, 8 + c, t] = sum_m w_m phi_c(x_m) dirs_t . grad_X G_q(X_t, x_m) (c < 6)."""
    x = np.asarray(x, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    a = np.asarray(phi) * np.asarray(weights)[None, :]
    out = np.zeros((2, NS + ND, X.shape[0]), dtype=np.complex128)
    for b0 in range(0, X.shape[0], block):
        d = X[b0:b0 + block, None, :] - x[None, :, :]
        r = np.sqrt(np.sum(d * d, axis=2))
        nd = np.sum(dirs[b0:b0 + block, None, :] * d, axis=2)
        for q, k in enumerate(kappas):
            g = np.exp(1j * k * r) / (4.0 * np.pi * r)
            out[q, :NS, b0:b0 + block] = (g @ a.T).T
            gd = g * (1j * k - 1.0 / r) / r * nd
            out[q, NS:, b0:b0 + block] = (gd @ a[:ND].T).T
    return out
