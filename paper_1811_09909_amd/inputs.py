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
* ``unstructured2d`` -- Example II's setting (kappa = 1, f = 1, tau = 1) on
                      ``box_with_holes``, a seeded Delaunay mesh of the box
                      [0, 2] x [0, 1] with eight circular holes, and the seed
                      points of two coarsening strategies.
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


def box_with_holes(nx=32, holes=True, seed=0):
    """An unstructured triangulation of the box [0, 2] x [0, 1], by default
    with eight circular holes of radius 0.12 centred at (0.25 + 0.5 i,
    0.25 + 0.5 j), i < 4, j < 2 (a stand-in for the mesh of Example II,
    which is published only as a figure).

    Vertices: a grid of spacing h = 1 / nx over the box, the interior ones
    moved by U(-0.3 h, 0.3 h) per coordinate (drawn in vertex order, x then
    y), minus those within 0.12 + 0.6 h of a hole centre, plus
    ceil(2 pi 0.12 / h) equally spaced points on every hole's circle.
    Triangles: the Delaunay triangulation of these points, without those
    whose centroid lies inside a hole, each listed counter-clockwise, in
    order of their lowest vertex, then their highest.
    Returns (vertices [nv, 2] float64, triangles [nt, 3] int32)."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    h = 1.0 / nx
    xs = np.arange(2 * nx + 1) * h
    ys = np.arange(nx + 1) * h
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    P = np.stack([X.ravel(), Y.ravel()], axis=1)
    jit = rng.uniform(-0.3 * h, 0.3 * h, P.shape)
    inner = (P[:, 0] > 0) & (P[:, 0] < 2.0) & (P[:, 1] > 0) & (P[:, 1] < 1.0)
    P[inner] += jit[inner]
    r = 0.12
    centres = np.array([(0.25 + 0.5 * i, 0.25 + 0.5 * j) for j in range(2) for i in range(4)]) if holes \
        else np.zeros((0, 2))
    keep = np.ones(len(P), dtype=bool)
    for c in centres:
        keep &= np.hypot(P[:, 0] - c[0], P[:, 1] - c[1]) > r + 0.6 * h
    pts = [P[keep]]
    m = int(np.ceil(2 * np.pi * r / h))
    th = 2 * np.pi * np.arange(m) / m
    for c in centres:
        pts.append(np.stack([c[0] + r * np.cos(th), c[1] + r * np.sin(th)], axis=1))
    V = np.concatenate(pts)
    tri = Delaunay(V).simplices.astype(np.int64)
    cen = V[tri].mean(axis=1)
    ok = np.ones(len(tri), dtype=bool)
    for c in centres:
        ok &= np.hypot(cen[:, 0] - c[0], cen[:, 1] - c[1]) > r
    tri = tri[ok]
    a, b, c3 = V[tri[:, 0]], V[tri[:, 1]], V[tri[:, 2]]
    area2 = (b[:, 0] - a[:, 0]) * (c3[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c3[:, 0] - a[:, 0])
    flip = area2 < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    used = np.unique(tri)
    remap = -np.ones(len(V), dtype=np.int64)
    remap[used] = np.arange(len(used))
    tri = remap[tri]
    order = np.lexsort((tri.max(axis=1), tri.min(axis=1)))  # by lowest vertex, then highest
    return V[used].copy(), tri[order].astype(np.int32)


def unstructured2d(nx=32, k=2, strategy=1, holes=True, seed=0):
    """The unstructured workload (Example II's setting on a synthetic mesh):
    kappa = 1, f = 1, zero Dirichlet data, tau = 1, on ``box_with_holes``.
    Seed points of the level-1 macro-elements: strategy 1 takes eight
    (0.25 + 0.5 i, 0.25 + 0.5 j), strategy 2 four (0.25 + 0.5 i, 0.5).
    ``hlevels``: the most agglomeration levels whose finest macro-elements
    hold at least three triangles on average (seeds 4^(hlevels-1) 3 <= N_T)."""
    V, T = box_with_holes(nx, holes, seed)
    if strategy == 1:
        seeds = np.array([(0.25 + 0.5 * i, 0.25 + 0.5 * j) for j in range(2) for i in range(4)])
    else:
        seeds = np.array([(0.25 + 0.5 * i, 0.5) for i in range(4)])
    nt = len(T)
    hl = 1
    while len(seeds) * 4 ** hl * 3 <= nt:
        hl += 1
    nv = (k + 1) * (k + 2) // 2
    return Workload(d=2, k=k, tau=1.0, vertices=V, triangles=T, seeds=seeds, hlevels=hl,
                    kappa=np.ones(nt), f=np.ones((nt, nv)),
                    name=f"unstructured2d box with 8 holes nx={nx} ({nt} triangles) k={k} strategy {strategy}")


def disk_mesh(h, seed=0):
    """An unstructured triangulation of the unit disk: the points of a grid of
    spacing h inside radius 1 - 0.6 h, moved by U(-0.3 h, 0.3 h) per
    coordinate (drawn in point order, x then y), plus ceil(2 pi / h) equally
    spaced points on the circle; the Delaunay triangulation of these points
    (all inside the inscribed polygon), counter-clockwise, listed by lowest
    then highest vertex.  Returns (vertices, triangles)."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    m = int(np.ceil(1.0 / h))
    g = np.arange(-m, m + 1) * h
    X, Y = np.meshgrid(g, g, indexing="xy")
    P = np.stack([X.ravel(), Y.ravel()], axis=1)
    P = P[np.hypot(P[:, 0], P[:, 1]) < 1.0 - 0.6 * h]
    P = P + rng.uniform(-0.3 * h, 0.3 * h, P.shape)
    nb = int(np.ceil(2 * np.pi / h))
    th = 2 * np.pi * np.arange(nb) / nb
    V = np.concatenate([P, np.stack([np.cos(th), np.sin(th)], axis=1)])
    tri = Delaunay(V).simplices.astype(np.int64)
    a, b, c = V[tri[:, 0]], V[tri[:, 1]], V[tri[:, 2]]
    flip = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    order = np.lexsort((tri.max(axis=1), tri.min(axis=1)))
    return V, tri[order].astype(np.int32)


def example3_disk(levels=4, k=2):
    """Example III's setting on a synthetic disk mesh: kappa = 1 + 0.5
    sin(2 pi x) cos(3 pi y) at the triangle centroids, u = x y exp(x^2 y^3),
    f = -div(kappa grad u) with the smooth kappa, Dirichlet data u, tau = 1.
    The mesh of ``levels`` has about 84 4^(levels - 2) triangles (the sizes of
    the paper's hierarchy), and 21 seed points on a grid of spacing 0.4 give
    about 84 macro-elements on level 2 and four times more per level below."""
    ntri = 84 * 4 ** (levels - 2)
    V, T = disk_mesh(np.sqrt(2 * np.pi / ntri))
    cen = V[T].mean(axis=1)
    kappa = 1.0 + 0.5 * np.sin(2 * np.pi * cen[:, 0]) * np.cos(3 * np.pi * cen[:, 1])
    g = np.arange(-2, 3) * 0.4
    S = np.stack(np.meshgrid(g, g, indexing="xy"), axis=-1).reshape(-1, 2)
    seeds = S[np.hypot(S[:, 0], S[:, 1]) < 0.95]

    def u(P):
        x, y = P[..., 0], P[..., 1]
        return x * y * np.exp(x ** 2 * y ** 3)

    def grad(P):
        x, y = P[..., 0], P[..., 1]
        e = np.exp(x ** 2 * y ** 3)
        return np.stack([y * e * (1 + 2 * x ** 2 * y ** 3), x * e * (1 + 3 * x ** 2 * y ** 3)], axis=-1)

    def f(P):
        x, y = P[..., 0], P[..., 1]
        e = np.exp(x ** 2 * y ** 3)
        lap = y * e * (6 * x * y ** 3 + 4 * x ** 3 * y ** 6) + x * e * (12 * x ** 2 * y ** 2 + 9 * x ** 4 * y ** 5)
        kap = 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.cos(3 * np.pi * y)
        kx = np.pi * np.cos(2 * np.pi * x) * np.cos(3 * np.pi * y)
        ky = -1.5 * np.pi * np.sin(2 * np.pi * x) * np.sin(3 * np.pi * y)
        gu = grad(P)
        return -(kap * lap + kx * gu[..., 0] + ky * gu[..., 1])

    hl = 1
    while len(seeds) * 4 ** hl * 3 <= len(T):
        hl += 1
    return Workload(d=2, k=k, tau=1.0, vertices=V, triangles=T, seeds=seeds, hlevels=hl, kappa=kappa, f=f,
                    u_exact=u, grad_exact=grad,
                    name=f"example3 disk mesh level {levels} ({len(T)} triangles) k={k} "
                         f"kappa=1+0.5sin(2pi x)cos(3pi y) u=xy exp(x^2y^3) tau=1")
