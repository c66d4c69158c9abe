"""Pins for the oracle's incident dipole field (end-face excitation of the
paper's waveguide example, Sec. IV): Maxwell's equations by central
differences, the far field of the real dipole, and the forward beam of the
complex source point.  A dropped term or a wrong sign in E or H breaks
Maxwell's equations; a wrong branch of r breaks the beam direction."""
import math

import numpy as np
import pytest

from oracle import excitation

OMEGA = 2 * math.pi
EPS = 2.1
K = OMEGA * math.sqrt(EPS)       # mu = 1


def _curl_div(f, X, h=1e-3):
    """Fourth-order central differences of a vector field f(X) -> [M, 3]."""
    J = np.zeros((X.shape[0], 3, 3), dtype=np.complex128)     # J[:, i, j] = d_j f_i
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        J[:, :, j] = (-f(X + 2 * e) + 8 * f(X + e) - 8 * f(X - e) + f(X - 2 * e)) / (12 * h)
    curl = np.stack([J[:, 2, 1] - J[:, 1, 2], J[:, 0, 2] - J[:, 2, 0], J[:, 1, 0] - J[:, 0, 1]], axis=1)
    return curl, J[:, 0, 0] + J[:, 1, 1] + J[:, 2, 2]


@pytest.mark.parametrize("b", [0.0, 0.728])
def test_maxwell_equations_by_finite_differences(b):
    rng = np.random.default_rng(1)
    p = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    x0 = np.array([-1.0, 0.2, 0.1])
    d = np.array([1.0, 0.0, 0.0])
    X = x0 + rng.uniform(1.0, 3.0, (40, 1)) * rng.standard_normal((40, 3)) / math.sqrt(3)
    X = X[np.abs((X - x0) @ d) > 0.3]               # away from the branch-cut disk
    E, H = excitation.dipole_fields(X, K, EPS, OMEGA, p, x0, b * d)
    cE, dE = _curl_div(lambda Y: excitation.dipole_fields(Y, K, EPS, OMEGA, p, x0, b * d)[0], X)
    cH, _ = _curl_div(lambda Y: excitation.dipole_fields(Y, K, EPS, OMEGA, p, x0, b * d)[1], X)
    assert np.linalg.norm(cE - 1j * OMEGA * H) < 1e-6 * np.linalg.norm(cE)
    assert np.linalg.norm(cH + 1j * OMEGA * EPS * E) < 1e-6 * np.linalg.norm(cH)
    assert np.max(np.abs(dE)) < 1e-6 * np.max(np.abs(cE))


def test_far_field_of_the_real_dipole():
    # E -> (k^2 / eps) G (p - r (r.p)), |H| = sqrt(eps / mu) |E| (plane-wave impedance)
    p = np.array([0.3, -1.0, 0.5 + 0.2j])
    rng = np.random.default_rng(2)
    u = rng.standard_normal((20, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    R = 3000.0
    E, H = excitation.dipole_fields(R * u, K, EPS, OMEGA, p, np.zeros(3), np.zeros(3))
    G = np.exp(1j * K * R) / (4 * np.pi * R)
    want = (K * K / EPS) * G * (p[None, :] - u * (u @ p)[:, None])
    assert np.linalg.norm(E - want) < 1e-3 * np.linalg.norm(want)
    assert abs(np.linalg.norm(H) - math.sqrt(EPS) * np.linalg.norm(E)) < 1e-3 * np.linalg.norm(H)


def test_complex_source_launches_a_forward_beam():
    # on the axis d, r = (L - i b) forward and (L + i b) backward: the transverse
    # field ratio is exp(2 k b) up to 1 / (k L) corrections
    b = K * 0.4 ** 2 / 2
    d = np.array([1.0, 0.0, 0.0])
    x0 = np.zeros(3)
    L = 60.0
    X = np.array([x0 + L * d, x0 - L * d])
    E, _ = excitation.dipole_fields(X, K, EPS, OMEGA, np.array([0, 1.0, 0]), x0, b * d)
    ratio = np.linalg.norm(E[0]) / np.linalg.norm(E[1])
    assert abs(math.log(ratio) - 2 * K * b) < 0.02
    # across the beam the field follows the paraxial Gaussian profile
    # exp(-rho^2 / w(z)^2), w(z) = w0 sqrt(1 + (z / b)^2), b the Rayleigh range
    w0, z = 0.4, 2.0
    wz = w0 * math.sqrt(1 + (z / b) ** 2)
    Y = np.array([[z, 0.0, 0.0], [z, 0.4, 0.0], [z, 0.8, 0.0]])
    Ey, _ = excitation.dipole_fields(Y, K, EPS, OMEGA, np.array([0, 0, 1.0]), x0, b * d)
    a = np.linalg.norm(Ey, axis=1)
    for i, rho in ((1, 0.4), (2, 0.8)):
        assert abs(a[i] / a[0] - math.exp(-rho ** 2 / wz ** 2)) < 0.05
