"""P14: the oracle's adjoint gradient against complex-step and central
differences (the adjoint is derived from eqs. HDG and HDG_flux; it is not
in the paper)."""
import numpy as np
import pytest

from oracle import adjoint
from oracle.hdg import HDG


@pytest.mark.parametrize("d,n,k", [(2, 4, 2), (2, 2, 3), (3, 2, 1)])
def test_P14_complex_step(d, n, k):
    rng = np.random.default_rng(7)
    P = HDG(d, n, k, 1.0, np.ones(n ** d))
    theta = 0.5 * rng.standard_normal(n ** d)
    f = np.ones((n ** d, P.nv))
    u_obs = 0.01 * rng.standard_normal((n ** d, P.nv))
    J, grad = adjoint.gradient(P, theta, f, u_obs)
    cs = np.zeros(n ** d)
    for T in range(n ** d):
        th = theta.astype(complex)
        th[T] += 1e-30j
        u, q, lam, A = adjoint.forward(P, th, f)
        cs[T] = adjoint.misfit(P, u, u_obs).imag / 1e-30
    assert np.abs(grad - cs).max() <= 1e-12 * np.abs(cs).max()


def test_P14_central_difference_and_continuous_sign():
    rng = np.random.default_rng(8)
    n, k = 8, 2
    P = HDG(2, n, k, 1.0, np.ones(n * n))
    theta = rng.standard_normal(n * n)
    f = np.ones((n * n, P.nv))
    u0, _, _, _ = adjoint.forward(P, np.zeros(n * n), f)
    u_obs = u0 + 0.01 * np.sqrt(np.mean(u0 ** 2)) * rng.standard_normal(u0.shape)
    J, grad = adjoint.gradient(P, theta, f, u_obs)
    for _ in range(3):
        v = rng.standard_normal(n * n)
        eps = 1e-5
        Jp = adjoint.misfit(P, adjoint.forward(P, theta + eps * v, f)[0], u_obs)
        Jm = adjoint.misfit(P, adjoint.forward(P, theta - eps * v, f)[0], u_obs)
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - grad @ v) <= 1e-6 * max(abs(fd), 1e-12)
    # with u_obs = 0 and f = 1, raising kappa everywhere lowers u (and J):
    # the continuous sensitivity -int kappa^-1 q . q* is then negative in sum
    J0, g0 = adjoint.gradient(P, theta, f, np.zeros_like(u0))
    assert g0.sum() < 0
