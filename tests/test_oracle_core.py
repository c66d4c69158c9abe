"""Pins for the Green's function and the O1 direct sums."""
import numpy as np

import synth
from oracle import direct, greens


def test_green_symmetry_and_gradient():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((50, 3))
    y = rng.standard_normal((50, 3))
    k = 7.3
    assert np.allclose(greens.G(k, x, y), greens.G(k, y, x), rtol=1e-15, atol=0)
    assert np.allclose(greens.gradG(k, x, y), -greens.gradG(k, y, x), rtol=1e-14, atol=1e-14)
    # gradient against central differences
    h = 1e-6
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        fd = (greens.G(k, x + e, y) - greens.G(k, x - e, y)) / (2 * h)
        assert np.allclose(fd, greens.gradG(k, x, y)[:, c], rtol=1e-6, atol=1e-8)


def test_green_solves_helmholtz():
    # Laplacian G + k^2 G = 0 away from the source (7-point stencil)
    k = 5.0
    x = np.array([[0.7, -0.2, 0.4]])
    y = np.zeros((1, 3))
    h = 1e-3
    lap = -6 * greens.G(k, x, y)
    for c in range(3):
        e = np.zeros(3)
        e[c] = h
        lap = lap + greens.G(k, x + e, y) + greens.G(k, x - e, y)
    lap /= h * h
    assert abs(lap[0] + k * k * greens.G(k, x, y)[0]) < 1e-4 * abs(k * k * greens.G(k, x, y)[0])


def test_direct_sums_match_pairwise_loop():
    # pure-Python double loop on a tiny input is the definition written out
    s = synth.cube_sphere(1, 2)
    n = s.n
    rng = np.random.default_rng(1)
    w = rng.uniform(0.5, 1.5, n)
    phi = synth.complex_normal((8, n), 2)
    ks = (3.0, 4.5)
    out = direct.regular_sums(s.x, s.normal, w, phi, ks, block=5)
    for l in range(n):
        for q, k in enumerate(ks):
            S = np.zeros(8, complex)
            D = np.zeros(6, complex)
            for m in range(n):
                if m == l:
                    continue
                d = s.x[l] - s.x[m]
                r = np.sqrt(d @ d)
                g = np.exp(1j * k * r) / (4 * np.pi * r)
                S += w[m] * phi[:, m] * g
                D += w[m] * phi[:6, m] * g * (1j * k - 1 / r) * (s.normal[l] @ d) / r
            assert np.allclose(out[q, :8, l], S, rtol=1e-13, atol=1e-15)
            assert np.allclose(out[q, 8:, l], D, rtol=1e-13, atol=1e-15)


def test_direct_target_subset():
    s = synth.cube_sphere(1, 3)
    w = np.ones(s.n)
    phi = synth.complex_normal((8, s.n), 3)
    full = direct.regular_sums(s.x, s.normal, w, phi, (2.0, 3.0))
    idx = np.array([0, 5, 17, 40])
    sub = direct.regular_sums(s.x, s.normal, w, phi, (2.0, 3.0), targets=idx)
    assert np.allclose(sub, full[:, :, idx], rtol=1e-14, atol=1e-15)
