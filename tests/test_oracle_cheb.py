"""Pins for the oracle's Chebyshev tools against closed forms."""
import numpy as np
import pytest

from oracle import cheb


@pytest.mark.parametrize("n", [2, 3, 5, 8, 10, 12, 16])
def test_fejer_integrates_chebyshev_exactly(n):
    # Fejer's rule on n open Chebyshev nodes is exact for polynomials of degree < n:
    # int_{-1}^{1} T_k = 2/(1-k^2) for even k, 0 for odd k.
    w = cheb.fejer_weights(n)
    x = cheb.nodes(n)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(n):
        exact = 2.0 / (1.0 - k * k) if k % 2 == 0 else 0.0
        assert abs(np.sum(w * np.cos(k * np.arccos(x))) - exact) < 1e-14


def test_fejer_matches_gauss_on_smooth_integrand():
    # int_{-1}^1 exp(x) dx = e - 1/e; Fejer converges spectrally.
    n = 16
    val = np.sum(cheb.fejer_weights(n) * np.exp(cheb.nodes(n)))
    assert abs(val - (np.e - 1.0 / np.e)) < 1e-14


@pytest.mark.parametrize("n", [3, 5, 8])
def test_interpolation_reproduces_polynomials(n):
    rng = np.random.default_rng(n)
    coef = rng.standard_normal(n)                     # monomial coefficients, degree n-1
    f = lambda t: np.polyval(coef, t)
    c = cheb.coefficients(f(cheb.nodes(n)))
    t = np.linspace(-1, 1, 37)
    assert np.max(np.abs(cheb.evaluate(c, t) - f(t))) < 1e-12


@pytest.mark.parametrize("n", [3, 5, 8, 12])
def test_differentiation_exact_for_polynomials(n):
    rng = np.random.default_rng(10 + n)
    coef = rng.standard_normal(n)
    f = lambda t: np.polyval(coef, t)
    df = lambda t: np.polyval(np.polyder(coef), t)
    x = cheb.nodes(n)
    assert np.max(np.abs(cheb.differentiate(f(x)) - df(x))) < 1e-11


def test_T_and_dT_closed_forms():
    t = np.linspace(-0.99, 0.99, 11)
    Tm = cheb.T(6, t)
    dTm = cheb.dT(6, t)
    th = np.arccos(t)
    for k in range(6):
        assert np.allclose(Tm[:, k], np.cos(k * th), atol=1e-14)
        # T_k'(t) = k sin(k th) / sin(th)
        assert np.allclose(dTm[:, k], k * np.sin(k * th) / np.sin(th), atol=1e-12)
