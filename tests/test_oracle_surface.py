"""Pins for the oracle's surface calculus (Sec. III-A node grid, Chebyshev
differentiation per patch): tangential gradient and surface divergence
against closed forms, and the surface divergence theorem.

A mistake in the metric inverse (swapped or missing terms), a missing
Jacobian in the divergence, or a sign error fails one of these."""
import numpy as np
import pytest

import synth
from oracle import surface


@pytest.fixture(scope="module")
def sphere():
    s = synth.cube_sphere(2, 12, 1.0)
    return surface.PatchSurface(s.P, s.nc, s.x, s.du, s.dv)


@pytest.fixture(scope="module")
def ellipsoid():
    s = synth.ellipsoid(1.3, 0.8, 1.1, 2, 12)
    return surface.PatchSurface(s.P, s.nc, s.x, s.du, s.dv)


def test_normals_are_outward_radial_on_the_unit_sphere(sphere):
    assert np.max(np.abs(sphere.n - sphere.x)) < 1e-12


def test_gradient_of_a_coordinate(sphere):
    # on the unit sphere grad_Gamma x_3 = e_3 - n n_3
    g = sphere.surface_grad(sphere.x[:, 2].copy())
    want = np.array([0.0, 0.0, 1.0])[None, :] - sphere.n * sphere.n[:, 2:3]
    assert np.max(np.abs(g - want)) < 1e-7


def test_gradient_is_tangent_and_complex_linear(sphere):
    rng = np.random.default_rng(3)
    k = rng.standard_normal(3)
    f = np.exp(1j * (sphere.x @ k))
    g = sphere.surface_grad(f)
    assert np.max(np.abs(np.sum(g * sphere.n, axis=1))) < 1e-12 * np.max(np.abs(g))
    # the tangential part of the ambient gradient i k f
    amb = 1j * k[None, :] * f[:, None]
    want = amb - sphere.n * np.sum(amb * sphere.n, axis=1)[:, None]
    assert np.max(np.abs(g - want)) < 1e-6 * np.max(np.abs(want))


@pytest.mark.parametrize("deg,f", [
    (1, lambda x: x[:, 2]),
    (2, lambda x: x[:, 0] * x[:, 1]),
    (3, lambda x: x[:, 2] * (5 * x[:, 2] ** 2 - 3)),
])
def test_laplace_beltrami_of_spherical_harmonics(sphere, deg, f):
    # div_Gamma grad_Gamma Y_n = -n (n + 1) Y_n on the unit sphere; two
    # spectral differentiations at Nc = 12 leave ~1e-6 relative to n (n + 1) |Y|
    y = f(sphere.x).astype(float)
    lap = sphere.surface_div(sphere.surface_grad(y))
    assert np.max(np.abs(lap + deg * (deg + 1) * y)) < 1e-5 * deg * (deg + 1) * np.max(np.abs(y))


def test_divergence_of_a_rotation_field(sphere):
    # a = c x n is tangent and divergence free on the sphere
    c = np.array([0.3, -1.2, 0.7])
    a = np.cross(c[None, :], sphere.n)
    assert np.max(np.abs(sphere.surface_div(a))) < 1e-6


def test_divergence_of_a_projected_constant(sphere):
    # a = c - n (n.c) on the unit sphere: div_Gamma a = -2 n.c
    c = np.array([0.4, 0.9, -0.5])
    a = c[None, :] - sphere.n * (sphere.n @ c)[:, None]
    assert np.max(np.abs(sphere.surface_div(a) + 2 * (sphere.n @ c))) < 1e-6


def test_divergence_theorem_on_an_ellipsoid(ellipsoid):
    # closed surface: int div_Gamma a = 0 and int f div_Gamma a = -int grad_Gamma f . a
    s = ellipsoid
    rng = np.random.default_rng(4)
    k = rng.standard_normal(3)
    c = np.array([0.2, 1.0, -0.6])
    a = (c[None, :] - s.n * (s.n @ c)[:, None]) * np.exp(1j * (s.x @ k))[:, None]
    div = s.surface_div(a)
    scale = np.sum(s.w * np.abs(div))
    assert abs(np.sum(s.w * div)) < 1e-7 * scale
    f = np.cos(s.x @ np.array([1.0, -0.5, 0.3]))
    lhs = np.sum(s.w * f * div)
    rhs = -np.sum(s.w * np.sum(s.surface_grad(f) * a, axis=1))
    assert abs(lhs - rhs) < 1e-7 * scale


def test_weights_integrate_the_ellipsoid(ellipsoid):
    # int n = 0 and int x.n = 3 volume (divergence theorem in R^3)
    s = ellipsoid
    vol = 4.0 / 3.0 * np.pi * 1.3 * 0.8 * 1.1
    assert np.max(np.abs(np.sum(s.w[:, None] * s.n, axis=0))) < 1e-10
    assert abs(np.sum(s.w * np.sum(s.x * s.n, axis=1)) - 3 * vol) < 1e-8 * vol
