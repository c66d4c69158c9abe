"""N-Mueller operator on the Chebyshev-Nystrom discretisation (oracle; test
infrastructure only).

Sec. II of the paper (eq. potential_r, potential_k, potential_t, n_muller,
k_delta, r_delta, t_delta) with the scalar operators S and D = dS/dn of
Sec. III (eq. sl_scalar, dl_scalar) applied to eight densities (Cartesian m,
j and their surface divergences), derivatives by Chebyshev differentiation.

Units: lengths in vacuum wavelengths, omega = 2 pi, k_s = omega sqrt(eps_s mu_s).
Kernel order everywhere: q = 0 interior (k_i), q = 1 exterior (k_e).

Unknowns y[4, N] = (m.t1, m.t2, j.t1, j.t2) with t1 = d_u eta/|d_u eta|,
t2 = n x t1 (reading A14).  For a tangent density a with A_c = S_q[a_c]:
  grad A_c = grad_Gamma A_c + n D_q[a_c]     (principal value of the normal derivative)
  K_q[a] = n x curl A,  R_q[a] = n x A,  T_q[a] = n x grad_Gamma S_q[div a]
  row 1 = (mu_e + mu_i)/2 m + mu_e K_e[m] - mu_i K_i[m] - (R^D + T^D)[j]
  row 2 = (R^D + T^D)[m] + (eps_e + eps_i)/2 j + eps_e K_e[j] - eps_i K_i[j]
  R^D = (-i/omega)(k_e^2 R_e - k_i^2 R_i),  T^D = (-i/omega)(T_e - T_i)
and A y = (row1.t1, row1.t2, row2.t1, row2.t2).  The identity terms carry the
jumps n x curl S[a]|_(+/-) = K[a] +/- a/2 of the principal-value K.
Pins: sphere eigenvalues of the corrected S and D (test_oracle_singular.py),
the homogeneous-medium identity, and the Mie series (test_oracle_nmuller.py).
"""
from __future__ import annotations

import math

import numpy as np

from . import direct, singular
from .surface import PatchSurface


def cross(a, b):
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], axis=-1)


class NMuller:
    def __init__(self, surf: PatchSurface, eps_e, eps_i, mu_e=1.0, mu_i=1.0,
                 omega=2 * math.pi, sing: singular.Params | None = None, corrections=None,
                 patches=None):
        """patches: evaluate A y only on the rows of these patches (None = all).
        corrections: precomputed correction matrices ({} for geometry-only use)."""
        self.s = surf
        nq = surf.nc * surf.nc
        self.rows = (np.arange(surf.N) if patches is None else
                     np.concatenate([np.arange(p * nq, (p + 1) * nq) for p in patches]))
        self.eps_e, self.eps_i, self.mu_e, self.mu_i = eps_e, eps_i, mu_e, mu_i
        self.omega = omega
        self.ke = omega * math.sqrt(eps_e * mu_e)
        self.ki = omega * math.sqrt(eps_i * mu_i)
        self.kappas = (self.ki, self.ke)
        self.C = (corrections if corrections is not None else
                  singular.corrections(surf, self.kappas, sing,
                                       targets=None if patches is None else self.rows))

    # a1: unknowns -> eight densities ------------------------------------
    def densities(self, y):
        s = self.s
        m = y[0][:, None] * s.t1 + y[1][:, None] * s.t2
        j = y[2][:, None] * s.t1 + y[3][:, None] * s.t2
        phi = np.empty((8, s.N), dtype=np.complex128)
        phi[0:3] = m.T
        phi[3:6] = j.T
        phi[6] = s.surface_div(m)
        phi[7] = s.surface_div(j)
        return phi

    # a2..a7: corrected layer sums ----------------------------------------
    def layer_sums(self, phi, regular=None):
        """out[q, 0..7] = S_q[phi_k], out[q, 8..13] = D_q[phi_k] (k < 6), corrected."""
        s = self.s
        if regular is None:
            out = np.zeros((2, 14, s.N), dtype=np.complex128)
            out[:, :, self.rows] = direct.regular_sums(s.x, s.n, s.w, phi, self.kappas, targets=self.rows)
        else:
            out = regular.copy()
        for q in range(2):
            out[q, :8] += (self.C[("S", q)] @ phi.T).T
            out[q, 8:] += (self.C[("D", q)] @ phi[:6].T).T
        return out

    # a8: operator assembly -------------------------------------------------
    def _KRT(self, SD, q, base, div_index):
        s = self.s
        A = SD[q, base:base + 3].T                         # [N, 3] = S_q[a_c]
        Dn = SD[q, 8 + base:8 + base + 3].T                # [N, 3] = D_q[a_c]
        grad = np.empty((s.N, 3, 3), dtype=np.complex128)  # grad[:, c, i] = d_i A_c
        for c in range(3):
            grad[:, c, :] = s.surface_grad(A[:, c]) + Dn[:, c][:, None] * s.n
        curl = np.stack([grad[:, 2, 1] - grad[:, 1, 2], grad[:, 0, 2] - grad[:, 2, 0],
                         grad[:, 1, 0] - grad[:, 0, 1]], axis=1)
        K = cross(s.n, curl)
        R = cross(s.n, A)
        T = cross(s.n, s.surface_grad(SD[q, div_index]))
        return K, R, T

    def assemble(self, y, SD):
        s = self.s
        w = self.omega
        m = y[0][:, None] * s.t1 + y[1][:, None] * s.t2
        j = y[2][:, None] * s.t1 + y[3][:, None] * s.t2
        Ki_m, Ri_m, Ti_m = self._KRT(SD, 0, 0, 6)
        Ke_m, Re_m, Te_m = self._KRT(SD, 1, 0, 6)
        Ki_j, Ri_j, Ti_j = self._KRT(SD, 0, 3, 7)
        Ke_j, Re_j, Te_j = self._KRT(SD, 1, 3, 7)
        RT_j = (-1j / w) * (self.ke ** 2 * Re_j - self.ki ** 2 * Ri_j + Te_j - Ti_j)
        RT_m = (-1j / w) * (self.ke ** 2 * Re_m - self.ki ** 2 * Ri_m + Te_m - Ti_m)
        row1 = 0.5 * (self.mu_e + self.mu_i) * m + self.mu_e * Ke_m - self.mu_i * Ki_m - RT_j
        row2 = RT_m + 0.5 * (self.eps_e + self.eps_i) * j + self.eps_e * Ke_j - self.eps_i * Ki_j
        return np.stack([np.sum(row1 * s.t1, axis=1), np.sum(row1 * s.t2, axis=1),
                         np.sum(row2 * s.t1, axis=1), np.sum(row2 * s.t2, axis=1)])

    def apply(self, y, regular=None):
        """A y for y [4, N] (the forward map of eq. lin_system), on self.rows."""
        phi = self.densities(y)
        return self.assemble(y, self.layer_sums(phi, regular))[:, self.rows]

    # right-hand side of eq. n_muller --------------------------------------
    def incident_plane_wave(self, d, p, x=None):
        """E = p exp(i k_e d.x), H = (k_e / (omega mu_e)) (d x p) exp(i k_e d.x)."""
        x = self.s.x if x is None else x
        d = np.asarray(d, dtype=np.float64)
        p = np.asarray(p, dtype=np.complex128)
        ph = np.exp(1j * self.ke * (x @ d))
        E = ph[:, None] * p[None, :]
        H = (self.ke / (self.omega * self.mu_e)) * ph[:, None] * np.cross(d, p)[None, :]
        return E, H

    def rhs(self, E, H):
        s = self.s
        a = cross(s.n, E) / self.omega
        b = cross(s.n, H) / self.omega
        return np.stack([np.sum(a * s.t1, axis=1), np.sum(a * s.t2, axis=1),
                         np.sum(b * s.t1, axis=1), np.sum(b * s.t2, axis=1)])


def interior_field(nm: NMuller, y, X):
    """Total interior field (E, H) at points X [M, 3] strictly inside Gamma.

    From the representation that reproduces eq. n_muller through the jump
    relations (the interior Stratton-Chu representation with the surface
    densities m and j):
      E_i = -omega mu_i curl S_i[m] - i (k_i^2 S_i[j] + grad S_i[div j])
      H_i = -omega eps_i curl S_i[j] + i (k_i^2 S_i[m] + grad S_i[div m])
    with S_i evaluated by the regular (Fejer) quadrature, valid away from Gamma.
    """
    s = nm.s
    k = nm.ki
    phi = nm.densities(y)
    a = phi * s.w[None, :]
    E = np.zeros((X.shape[0], 3), dtype=np.complex128)
    H = np.zeros_like(E)
    for b0 in range(0, X.shape[0], 64):
        Xb = X[b0:b0 + 64]
        d = Xb[:, None, :] - s.x[None, :, :]
        r = np.sqrt(np.sum(d * d, axis=2))
        G = np.exp(1j * k * r) / (4 * np.pi * r)
        gG = (G * (1j * k - 1.0 / r) / r)[:, :, None] * d      # grad_x G [M, N, 3]
        Sm = G @ a[0:3].T
        Sj = G @ a[3:6].T
        curl_m = np.einsum("mnc,dn->mcd", gG, a[0:3])           # [M, c, d] = d_c G * m_d
        curl_j = np.einsum("mnc,dn->mcd", gG, a[3:6])
        cm = np.stack([curl_m[:, 1, 2] - curl_m[:, 2, 1], curl_m[:, 2, 0] - curl_m[:, 0, 2],
                       curl_m[:, 0, 1] - curl_m[:, 1, 0]], axis=1)
        cj = np.stack([curl_j[:, 1, 2] - curl_j[:, 2, 1], curl_j[:, 2, 0] - curl_j[:, 0, 2],
                       curl_j[:, 0, 1] - curl_j[:, 1, 0]], axis=1)
        gdj = np.einsum("mnc,n->mc", gG, a[7])
        gdm = np.einsum("mnc,n->mc", gG, a[6])
        E[b0:b0 + 64] = -nm.omega * nm.mu_i * cm - 1j * (k * k * Sj + gdj)
        H[b0:b0 + 64] = -nm.omega * nm.eps_i * cj + 1j * (k * k * Sm + gdm)
    return E, H
