"""Mie series for plane-wave scattering by a dielectric sphere (oracle; test
infrastructure only).

Textbook solution (vector spherical wave functions, time factor exp(-i w t)),
written for an incident field E = x-hat exp(i k z), H = (k/(w mu)) y-hat exp(i k z)
and a sphere of radius a centred at the origin with wavenumbers k (outside)
and k1 (inside), mu = mu1 = 1.  The paper compares its solver with this
series on the unit sphere (Sec. IV-B).

Pins (tests/test_oracle_nmuller.py, test_mie_series_self_consistent): the incident expansion reproduces the plane
wave, tangential E and H are continuous across r = a, and the small-sphere
(Rayleigh) limit of the interior field is the uniform 3/(eps_r + 2) E_inc.
"""
from __future__ import annotations

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def _zfun(kind, n, rho):
    j = spherical_jn(n, rho)
    dj = spherical_jn(n, rho, derivative=True)
    if kind == 1:
        return j, j + rho * dj                    # z_n, (rho z_n)'
    y = spherical_yn(n, rho)
    dy = spherical_yn(n, rho, derivative=True)
    h = j + 1j * y
    return h, h + rho * (dj + 1j * dy)


def _pi_tau(nmax, mu):
    pi = np.zeros((nmax + 1,) + mu.shape)
    tau = np.zeros_like(pi)
    pi[1] = 1.0
    for n in range(2, nmax + 1):
        pi[n] = ((2 * n - 1) / (n - 1)) * mu * pi[n - 1] - (n / (n - 1)) * pi[n - 2]
    for n in range(1, nmax + 1):
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi, tau


def _vsh(kind, n, rho, th, ph, pi_n, tau_n):
    """M_o1n, M_e1n, N_e1n, N_o1n in spherical components (r, theta, phi)."""
    z, dz = _zfun(kind, n, rho)
    c, s = np.cos(ph), np.sin(ph)
    st = np.sin(th)
    zero = np.zeros_like(rho, dtype=complex)
    M_o = np.stack([zero, c * pi_n * z, -s * tau_n * z])
    M_e = np.stack([zero, -s * pi_n * z, -c * tau_n * z])
    N_e = np.stack([c * n * (n + 1) * st * pi_n * z / rho, c * tau_n * dz / rho, -s * pi_n * dz / rho])
    N_o = np.stack([s * n * (n + 1) * st * pi_n * z / rho, s * tau_n * dz / rho, c * pi_n * dz / rho])
    return M_o, M_e, N_e, N_o


def _to_cart(V, th, ph):
    r, t, p = V
    st, ct, sp, cp = np.sin(th), np.cos(th), np.sin(ph), np.cos(ph)
    return np.stack([r * st * cp + t * ct * cp - p * sp,
                     r * st * sp + t * ct * sp + p * cp,
                     r * ct - t * st], axis=-1)


class MieSphere:
    def __init__(self, a, k, k1, omega, nmax=None):
        self.a, self.k, self.k1, self.omega = a, k, k1, omega
        x = k * a
        m = k1 / k
        self.nmax = nmax or int(x + 4 * x ** (1 / 3) + 12)
        n = np.arange(1, self.nmax + 1)
        jx, djx = _zfun(1, n, x)
        hx, dhx = _zfun(3, n, x)
        jmx, djmx = _zfun(1, n, m * x)
        # Bohren & Huffman (4.52)-(4.53) with mu = mu1
        self.a_n = (m * m * jmx * djx - jx * djmx) / (m * m * jmx * dhx - hx * djmx)
        self.b_n = (jmx * djx - jx * djmx) / (jmx * dhx - hx * djmx)
        self.c_n = (jx * dhx - hx * djx) / (jmx * dhx - hx * djmx)
        self.d_n = (m * jx * dhx - m * hx * djx) / (m * m * jmx * dhx - hx * djmx)
        self.E_n = (1j ** n) * (2 * n + 1) / (n * (n + 1))

    def fields(self, X, region):
        """(E, H) at points X [M, 3]; region in {'inc', 'sca', 'int'}."""
        r = np.sqrt(np.sum(X * X, axis=1))
        th = np.arccos(np.clip(X[:, 2] / r, -1, 1))
        ph = np.arctan2(X[:, 1], X[:, 0])
        pi, tau = _pi_tau(self.nmax, np.cos(th))
        kk = self.k1 if region == "int" else self.k
        rho = kk * r
        E = np.zeros((3, X.shape[0]), dtype=complex)
        H = np.zeros_like(E)
        kind = 3 if region == "sca" else 1
        for i, n in enumerate(range(1, self.nmax + 1)):
            Mo, Me, Ne, No = _vsh(kind, n, rho, th, ph, pi[n], tau[n])
            En = self.E_n[i]
            if region == "inc":
                E += En * (Mo - 1j * Ne)
                H += (-kk / self.omega) * En * (Me + 1j * No)
            elif region == "int":
                E += En * (self.c_n[i] * Mo - 1j * self.d_n[i] * Ne)
                H += (-kk / self.omega) * En * (self.d_n[i] * Me + 1j * self.c_n[i] * No)
            else:
                E += En * (1j * self.a_n[i] * Ne - self.b_n[i] * Mo)
                H += (kk / self.omega) * En * (1j * self.b_n[i] * No + self.a_n[i] * Me)
        return _to_cart(E, th, ph), _to_cart(H, th, ph)
