"""Incident fields (oracle; test infrastructure only).

Electric dipole at a complex source point, the end-face excitation of the
paper's waveguide example (Sec. IV): moment p at x_s = x_0 + i b d.  From the
Hertz potential Pi = p G, G = exp(i k r) / (4 pi r), r = sqrt(R.R) with
R = x - x_s on the principal branch:
  E = (k^2 Pi + grad div Pi) / eps,   H = -i omega curl Pi,
i.e. E = (k^2 G p + (p . grad) grad G) / eps and H = -i omega grad G x p, with
grad G = G (i k - 1/r) R / r and
(p . grad) grad G = G (i k - 1/r) p / r + G (-k^2 - 3 i k / r + 3 / r^2) (R.p) R / r^2.
Pins (tests/test_oracle_excitation.py): Maxwell's equations by central
differences, div E = 0, the far field of the real dipole, and the forward
beam of the complex source.
"""
from __future__ import annotations

import numpy as np


def dipole_fields(X, k, eps, omega, p, x0, beam):
    """E, H [M, 3] complex at points X [M, 3]."""
    X = np.asarray(X, dtype=np.float64)
    p = np.asarray(p, dtype=np.complex128)
    R = X - np.asarray(x0, float)[None, :] - 1j * np.asarray(beam, float)[None, :]
    r = np.sqrt(np.sum(R * R, axis=1))                 # principal branch: Re r >= 0
    G = np.exp(1j * k * r) / (4 * np.pi * r)
    dG = G * (1j * k - 1.0 / r) / r                    # grad G = dG R
    ddG = G * (-k * k - 3j * k / r + 3.0 / r ** 2) / r ** 2
    Rp = R @ p
    E = (k * k * G[:, None] * p[None, :] + dG[:, None] * p[None, :] + (ddG * Rp)[:, None] * R) / eps
    H = -1j * omega * dG[:, None] * np.cross(R, p[None, :])
    return E, H
