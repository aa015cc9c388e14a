"""Pins of the oracle's 1D building blocks against closed forms."""
import numpy as np

from oracle.refelem import gauss_rule, gll_nodes, lagrange, lagrange_deriv


def test_gll_closed_forms():
    assert np.allclose(gll_nodes(1), [0, 1])
    assert np.allclose(gll_nodes(2), [0, 0.5, 1])
    # k = 3: interior nodes at 1/2 -+ sqrt(5)/10 (roots of P_3' = (15x^2-3)/2)
    assert np.allclose(gll_nodes(3), [0, 0.5 - np.sqrt(5) / 10, 0.5 + np.sqrt(5) / 10, 1])
    # k = 4: interior nodes 1/2 and 1/2 -+ sqrt(21)/14
    assert np.allclose(gll_nodes(4), [0, 0.5 - np.sqrt(21) / 14, 0.5, 0.5 + np.sqrt(21) / 14, 1])


def test_gauss_exactness():
    for n in range(1, 8):
        x, w = gauss_rule(n)
        for p in range(2 * n):
            assert abs(np.sum(w * x ** p) - 1.0 / (p + 1)) < 1e-14
        # and not exact one degree higher
        assert abs(np.sum(w * x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12


def test_lagrange_cardinal_and_derivative():
    for k in range(1, 7):
        xi = gll_nodes(k)
        assert np.allclose(lagrange(xi, xi), np.eye(k + 1), atol=1e-13)
        x = np.linspace(0.03, 0.97, 11)
        eps = 1e-6
        fd = (lagrange(xi, x + eps) - lagrange(xi, x - eps)) / (2 * eps)
        assert np.allclose(lagrange_deriv(xi, x), fd, atol=1e-6 * (k + 1) ** 3)
        # partition of unity and reproduction of x^k
        assert np.allclose(lagrange(xi, x).sum(0), 1)
        assert np.allclose(xi ** k @ lagrange(xi, x), x ** k)
