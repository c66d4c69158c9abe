"""Pins for the singular quadrature (Sec. III-D) and local corrections (Sec. III-H)."""
import math

import numpy as np
import pytest
from scipy.special import spherical_jn, spherical_yn

import synth
from oracle import direct, singular, surface


def test_kress_map_endpoints_and_flatness():
    d = 4
    assert abs(singular.kress_w(0.0, d)) < 1e-15
    assert abs(singular.kress_w(math.pi, d) - math.pi) < 1e-14
    assert abs(singular.kress_w(2 * math.pi, d) - 2 * math.pi) < 1e-14
    # derivatives up to order d-1 vanish at the end points: w(t) = O(t^d)
    for t in (1e-2, 5e-3):
        assert singular.kress_w(t, d) / t ** d < 50
        assert abs(singular.kress_dw(t, d)) / t ** (d - 1) < 200
    # analytic derivative vs central differences in the interior
    for t in (0.7, 2.0, 4.1):
        h = 1e-6
        fd = (singular.kress_w(t + h, d) - singular.kress_w(t - h, d)) / (2 * h)
        assert abs(fd - singular.kress_dw(t, d)) < 1e-7


@pytest.mark.parametrize("alpha", [-1.0, -0.3, 0.0, 0.55, 1.0])
def test_xi_endpoints_and_derivative(alpha):
    d = 4
    t = np.array([-1.0, 1.0])
    u, _ = singular.xi(np.array([alpha]), t, d)
    assert np.allclose(u[0], [-1.0, 1.0], atol=1e-14)
    if abs(alpha) < 1:
        u0, _ = singular.xi(np.array([alpha]), np.array([0.0]), d)
        assert abs(u0[0, 0] - alpha) < 1e-15
    tt = np.linspace(-0.95, 0.95, 9)
    tt = tt[np.abs(tt) > 1e-3]
    h = 1e-6
    up, _ = singular.xi(np.array([alpha]), tt + h, d)
    um, _ = singular.xi(np.array([alpha]), tt - h, d)
    _, mu = singular.xi(np.array([alpha]), tt, d)
    assert np.allclose((up - um) / (2 * h), mu, atol=1e-6)
    # the map is monotone and onto [-1, 1]
    tg = np.linspace(-1, 1, 401)
    ug, _ = singular.xi(np.array([alpha]), tg, d)
    assert np.all(np.diff(ug[0]) >= -1e-15)


def test_mapped_quadrature_integrates_polynomials():
    # int_{-1}^{1} of a smooth function through the clustering map
    d = 4
    nb = 48
    from oracle import cheb
    t, w = cheb.nodes(nb), cheb.fejer_weights(nb)
    for alpha in (-1.0, -0.2, 0.6, 1.0):
        u, mu = singular.xi(np.array([alpha]), t, d)
        val = np.sum(np.exp(u[0]) * mu[0] * w)
        assert abs(val - (math.e - 1 / math.e)) < 1e-5


def test_closest_point_on_own_and_neighbour_patches():
    s = synth.cube_sphere(2, 8, 1.0)
    surf = surface.PatchSurface(s.P, s.nc, s.x, s.du, s.dv)
    A = singular.patch_coefficients(surf)
    prm = singular.Params()
    # own patch: exact node parameters, distance 0
    tg = np.array([0, 77, 130])
    pa = tg // 64
    u, v, dist = singular.closest_points(surf, A, tg, pa, prm)
    from oracle import cheb
    t = cheb.nodes(8)
    assert np.array_equal(u, t[(tg % 64) // 8]) and np.array_equal(v, t[tg % 8])
    assert np.all(dist == 0)
    # a point pushed off the sphere along the normal above a patch point: the
    # closest point is (numerically) that point, at the offset distance
    rng = np.random.default_rng(4)
    for p in (3, 11, 20):
        uu, vv = rng.uniform(-0.8, 0.8, 2)
        X = singular.eval_patch(A[p:p + 1], np.array([[uu]]), np.array([[vv]]))[0, 0, 0]
        n = X / np.linalg.norm(X)
        surf2 = surface.PatchSurface(s.P, s.nc, s.x, s.du, s.dv)
        surf2.x = np.vstack([surf.x, X + 0.05 * n])
        u2, v2, d2 = singular.closest_points(surf2, A, np.array([surf.N]), np.array([p]), prm)
        assert abs(u2[0] - uu) < 1e-5 and abs(v2[0] - vv) < 1e-5
        assert abs(d2[0] - 0.05) < 1e-7


def _h1(n, z, der=False):
    return spherical_jn(n, z, derivative=der) + 1j * spherical_yn(n, z, derivative=der)


@pytest.mark.parametrize("n_harm", [1, 2, 3])
def test_sphere_eigenvalues_with_corrections(n_harm):
    # S[Y_n] = i k a^2 j_n(ka) h_n(ka) Y_n, D_pv[Y_n] = (i k^2 a^2 / 2)(j_n h_n' + j_n' h_n) Y_n
    s = synth.cube_sphere(2, 8, 1.0)
    surf = surface.PatchSurface(s.P, s.nc, s.x, s.du, s.dv)
    ks = (3 * math.pi, 2 * math.pi)
    rng = np.random.default_rng(n_harm)
    tg = np.sort(rng.choice(surf.N, 120, replace=False))
    C = singular.corrections(surf, ks, targets=tg)
    x = s.x
    Y = {1: x[:, 2], 2: 3 * x[:, 2] ** 2 - 1, 3: x[:, 0] * x[:, 1] * x[:, 2]}[n_harm]
    phi = np.zeros((8, surf.N), complex)
    phi[0] = Y
    reg = direct.regular_sums(x, surf.n, surf.w, phi, ks, targets=tg)
    for q, k in enumerate(ks):
        S = reg[q, 0] + (C[("S", q)] @ Y)[tg]
        D = reg[q, 8] + (C[("D", q)] @ Y)[tg]
        lamS = 1j * k * spherical_jn(n_harm, k) * _h1(n_harm, k)
        lamD = 0.5j * k * k * (spherical_jn(n_harm, k) * _h1(n_harm, k, True)
                               + spherical_jn(n_harm, k, derivative=True) * _h1(n_harm, k))
        eS = np.linalg.norm(S - lamS * Y[tg]) / np.linalg.norm(lamS * Y[tg])
        eD = np.linalg.norm(D - lamD * Y[tg]) / np.linalg.norm(lamD * Y[tg])
        # Nc = 8 on 24 patches, N_beta = 48: ~1e-4 for S, ~1e-5 for D
        assert eS < 3e-4, eS
        assert eD < 1e-4, eD
        # without the correction the error is O(1): the correction is doing the work
        eS0 = np.linalg.norm(reg[q, 0] - lamS * Y[tg]) / np.linalg.norm(lamS * Y[tg])
        assert eS0 > 100 * eS
