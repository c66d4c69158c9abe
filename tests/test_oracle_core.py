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


def test_rounded_box_area_and_volume_closed_forms():
    """The rounded-box generator (the waveguide stand-in) against Steiner's
    formulas for the Minkowski sum of a box (edges A, B, C) and a ball of
    radius r: area 2(AB+BC+CA) + 2 pi r (A+B+C) + 4 pi r^2; volume
    ABC + 2 r (AB+BC+CA) + pi r^2 (A+B+C) + 4/3 pi r^3 (divergence theorem:
    the integral of x.n is 3 V); the integral of n vanishes."""
    import synth
    from oracle.surface import PatchSurface
    r = 0.1
    s = synth.rounded_box((2.0, 0.5, 0.25), r, 0.3, 10)
    surf = PatchSurface(s.P, s.nc, s.x, s.du, s.dv)
    A, B, C = 2 * (2.0 - r), 2 * (0.5 - r), 2 * (0.25 - r)
    area = 2 * (A * B + B * C + C * A) + 2 * np.pi * r * (A + B + C) + 4 * np.pi * r * r
    vol = A * B * C + 2 * r * (A * B + B * C + C * A) + np.pi * r * r * (A + B + C) + 4.0 / 3.0 * np.pi * r ** 3
    assert abs(surf.w.sum() - area) < 1e-9 * area
    flux = np.sum(surf.w * np.sum(s.x * s.normal, axis=1))
    assert abs(flux - 3 * vol) < 2e-9 * 3 * vol
    assert np.max(np.abs((surf.w[:, None] * s.normal).sum(0))) < 1e-9 * area
    # outward normals agree with the patch orientation
    assert np.all(np.sum(surf.n * s.normal, axis=1) > 0.999)


def test_sums_at_off_node_points_match_regular_sums():
    # the sums at a point that is not a source equal the regular sums of the
    # source set extended by that point, at that point (its own term excluded)
    import math
    import numpy as np
    import synth
    from oracle import direct
    s = synth.cube_sphere(1, 5, 1.0)
    rng = np.random.default_rng(7)
    w = rng.uniform(0.5, 1.5, s.n)
    phi = synth.complex_normal((8, s.n), 8)
    X = np.array([[0.2, -0.3, 0.4], [1.3, 0.1, -0.2]])
    dirs = np.array([[0.0, 0.6, 0.8], [1.0, 0.0, 0.0]])
    ks = (2.5 * math.pi, 1.5 * math.pi)
    got = direct.sums_at(s.x, w, phi, ks, X, dirs)
    for t in range(2):
        x = np.vstack([s.x, X[t:t + 1]])
        nrm = np.vstack([s.normal, dirs[t:t + 1]])
        ww = np.r_[w, 1.0]
        ph = np.hstack([phi, rng.standard_normal((8, 1))])
        want = direct.regular_sums(x, nrm, ww, ph, ks, targets=[s.n])
        assert np.allclose(got[:, :, t], want[:, :, 0], rtol=1e-13, atol=0)
