"""Pins for the oracle's Gauss-Legendre quadrature (a1 setup step)."""
import numpy as np
import pytest

from oracle.quadrature import gauss_legendre

NS = [2, 4, 8, 16, 32, 64, 128, 256]


@pytest.mark.parametrize("n", NS)
def test_polynomial_exactness(n):
    # An n-point Gauss rule integrates every polynomial of degree <= 2n-1 exactly.
    mu, w = gauss_legendre(n)
    for k in range(0, 2 * n):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        got = float(np.sum(w * mu ** k))
        assert abs(got - exact) <= 2e-14 * max(1.0, n / 16), (n, k, got, exact)


@pytest.mark.parametrize("n", NS)
def test_symmetry_order_and_weights(n):
    mu, w = gauss_legendre(n)
    assert np.all(np.diff(mu) > 0)
    np.testing.assert_allclose(mu[::-1], -mu, atol=1e-15)
    np.testing.assert_allclose(w[::-1], w, rtol=1e-13)
    assert np.all(w > 0)
    assert abs(np.sum(w) - 2.0) < 1e-13
    assert abs(np.sum(w * mu * mu) - 2.0 / 3.0) < 1e-13
    assert np.all(mu[: n // 2] < 0) and np.all(mu[n // 2:] > 0)


@pytest.mark.parametrize("n", NS)
def test_matches_library_rule(n):
    ref_x, ref_w = np.polynomial.legendre.leggauss(n)
    mu, w = gauss_legendre(n)
    np.testing.assert_allclose(mu, ref_x, atol=3e-15)
    # the library's weights carry ~1e-11 relative error at N = 256; ours ~1e-13
    np.testing.assert_allclose(w, ref_w, rtol=1e-10, atol=1e-15)
