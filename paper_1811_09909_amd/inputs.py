"""Seeded synthetic workloads (shared by the HIP path, its tests and the oracle).

This module holds none of the method's arithmetic: only random draws, in a
fixed order from ``numpy.random.default_rng(seed)`` (PCG64), and closed-form
coefficient, source and exact-solution functions.  Where an input is a
function of position, each consumer evaluates it at its own nodes or
quadrature points.

Workloads (all on the unit box, tau = 1, zero Dirichlet data):

* ``poisson2d``    -- -lap u = f, u = sin(pi x) sin(pi y), kappa = 1.
* ``diffusion2d``  -- kappa per element log-uniform in [lo, hi] (drawn first,
                      one per element, elements lexicographic), then nodal f
                      i.i.d. N(0,1) ([N_T][(k+1)^2], element-major).
* ``diffusion3d``  -- kappa(x) = 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z),
                      u = sin(pi x) sin(pi y) sin(pi z), f = -div(kappa grad u).
* ``batched2d``    -- per problem: n from {32,64,128,256}, k from {2,..,5},
                      kappa per element log-uniform, then nrhs nodal N(0,1)
                      right-hand sides.
* ``adjoint2d``    -- f = 1, theta = log kappa per element ~ N(0,1).
* ``ipdg2d``       -- the hybridized IPDG workload: kappa per element
                      1 + 0.5 sin(2 pi x) cos(3 pi y) at the element centre
                      (the coefficient of Example III on the unit square),
                      f = -kappa_T lap u for u = x y exp(x^2 y^3) (Example I),
                      zero Dirichlet data; stabilization kappa_T (p+1)(p+2)/h_min.
* ``multinumerics2d`` -- Example VI's coefficient 1 + 0.5 sin(4 pi x) cos(3 pi y)
                      at element centres, f = 1, zero Dirichlet data; NIPG-H on
                      the elements whose centre lies within 0.3 of
                      (0.45, 0.55), RT-H on the others.
"""
import numpy as np


class Workload:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def kappa_loguniform(rng, n_el, lo, hi):
    """kappa = 10^U(log10 lo, log10 hi), one draw per element."""
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), n_el)


def poisson2d(n=8, k=2):
    pi = np.pi

    def u(X):
        return np.sin(pi * X[..., 0]) * np.sin(pi * X[..., 1])

    def grad(X):
        return np.stack([pi * np.cos(pi * X[..., 0]) * np.sin(pi * X[..., 1]),
                         pi * np.sin(pi * X[..., 0]) * np.cos(pi * X[..., 1])], axis=-1)

    def f(X):
        return 2 * pi * pi * u(X)

    return Workload(d=2, n=n, k=k, tau=1.0, kappa=np.ones(n * n), f=f, u_exact=u,
                    grad_exact=grad, kappa_fn=None, name=f"poisson2d n={n} k={k}")


def diffusion2d(n=512, k=4, lo=1e-3, hi=1e3, seed=0):
    rng = np.random.default_rng(seed)
    kappa = kappa_loguniform(rng, n * n, lo, hi)
    f = rng.standard_normal((n * n, (k + 1) ** 2))
    return Workload(d=2, n=n, k=k, tau=1.0, kappa=kappa, f=f, seed=seed,
                    name=f"diffusion2d n={n} k={k} kappa=logU[{lo:g},{hi:g}] seed={seed}")


def diffusion3d(n=32, k=3):
    pi = np.pi

    def kap(X):
        return 1 + 0.5 * np.sin(2 * pi * X[..., 0]) * np.sin(2 * pi * X[..., 1]) * np.sin(2 * pi * X[..., 2])

    def gkap(X):
        s = [np.sin(2 * pi * X[..., i]) for i in range(3)]
        c = [np.cos(2 * pi * X[..., i]) for i in range(3)]
        return 0.5 * 2 * pi * np.stack([c[0] * s[1] * s[2], s[0] * c[1] * s[2], s[0] * s[1] * c[2]], axis=-1)

    def u(X):
        return np.sin(pi * X[..., 0]) * np.sin(pi * X[..., 1]) * np.sin(pi * X[..., 2])

    def grad(X):
        s = [np.sin(pi * X[..., i]) for i in range(3)]
        c = [np.cos(pi * X[..., i]) for i in range(3)]
        return pi * np.stack([c[0] * s[1] * s[2], s[0] * c[1] * s[2], s[0] * s[1] * c[2]], axis=-1)

    def f(X):
        # -div(kappa grad u) = -grad kappa . grad u - kappa lap u, lap u = -3 pi^2 u
        return -np.sum(gkap(X) * grad(X), axis=-1) + kap(X) * 3 * pi * pi * u(X)

    return Workload(d=3, n=n, k=k, tau=1.0, kappa=kap, f=f, u_exact=u, grad_exact=grad,
                    kappa_fn=kap, name=f"diffusion3d n={n} k={k}")


def batched2d(nprob=64, nrhs=16, ns=(32, 64, 128, 256), ks=(2, 3, 4, 5), lo=1e-2, hi=1e2, seed=0):
    rng = np.random.default_rng(seed)
    probs = []
    for _ in range(nprob):
        n = int(rng.choice(ns))
        k = int(rng.choice(ks))
        kappa = kappa_loguniform(rng, n * n, lo, hi)
        f = rng.standard_normal((nrhs, n * n, (k + 1) ** 2))
        probs.append(Workload(d=2, n=n, k=k, tau=1.0, kappa=kappa, f=f))
    return probs


def adjoint2d(n=256, k=3, seed=0):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(n * n)
    f = np.ones((n * n, (k + 1) ** 2))
    return Workload(d=2, n=n, k=k, tau=1.0, theta=theta, f=f, rng=rng,
                    name=f"adjoint2d n={n} k={k} seed={seed}")


def observation_noise(rng, shape):
    """xi ~ N(0,1) per nodal value, drawn after theta."""
    return rng.standard_normal(shape)


def ipdg2d(n=512, k=4):
    c = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(c, c, indexing="xy")  # element index x + n y
    kappa = (1.0 + 0.5 * np.sin(2 * np.pi * X) * np.cos(3 * np.pi * Y)).ravel()

    def lap_u(P):
        x, y = P[..., 0], P[..., 1]
        e = np.exp(x ** 2 * y ** 3)
        return y * e * (6 * x * y ** 3 + 4 * x ** 3 * y ** 6) + x * e * (12 * x ** 2 * y ** 2 + 9 * x ** 4 * y ** 5)

    def f(P):
        """-kappa_T lap u at points P [N_T, m, 2] (element-major)."""
        return -kappa[:, None] * lap_u(P)

    return Workload(d=2, n=n, k=k, tau=(k + 1) * (k + 2) * n / np.sqrt(2.0), kappa=kappa, f=f,
                    name=f"ipdg2d NIPG-H n={n} k={k} kappa=1+0.5sin(2pi x)cos(3pi y) tau=kappa(p+1)(p+2)/h_min")


def multinumerics2d(n=512, k=1):
    c = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(c, c, indexing="xy")  # element index x + n y
    kappa = (1.0 + 0.5 * np.sin(4 * np.pi * X) * np.cos(3 * np.pi * Y)).ravel()
    use_rt = ((X - 0.45) ** 2 + (Y - 0.55) ** 2 > 0.09).ravel()
    schemes = ["rt" if r else "nipg" for r in use_rt]
    return Workload(d=2, n=n, k=k, tau=(k + 1) * (k + 2) * n / np.sqrt(2.0), kappa=kappa, schemes=schemes,
                    f=np.ones((n * n, (k + 1) ** 2)),
                    name=f"multinumerics2d RT-H + NIPG-H n={n} k={k} kappa=1+0.5sin(4pi x)cos(3pi y) f=1")
