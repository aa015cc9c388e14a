"""Pins of the oracle's hybridized Raviart-Thomas method and multinumerics
(Sec. 2, eqs. mixed_local1 and mixed_local2 with the conservation of the
normal flux; Sec. 4.6).

R1  element maps symmetric positive semidefinite, constants in their kernel.
R2  polynomial reproduction: u in Q^k with f = -kappa lap u gives exact
    traces, scalar and flux at the nodes (q = -kappa grad u in RT_k).
R3  static condensation = the uncondensed (q, u, lambda) system.
R4  convergence: u and q of order k+1 in L2.
M1  multinumerics couples consistently: linear u is reproduced across
    RT-H / NIPG-H interfaces (constant kappa), and u = 1 + 2x under kappa
    layered along x with the elements mixed at random.
M2  multinumerics: condensed = uncondensed with random kappa, f, Dirichlet
    data and element mix.
M3  multigrid on the mixed trace system (Sec. 3 unchanged): the Galerkin
    chain with the nonsymmetric restriction, and h-independent counts of MG
    and GMRES on the Example VI coefficient with a disk of NIPG-H elements
    inside RT-H (the paper's unstructured mesh and element pattern are not
    available: its counts are "parity unpinned").
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import mg
from oracle.rth import RTH, Multinumerics

from .test_oracle_ipdg import _poly, _tau


@pytest.mark.parametrize("k", [1, 2, 3])
def test_R1_symmetric_semidefinite_constants(k):
    n = 2
    kap = np.array([0.3, 7.0, 1.0, 2.0])
    P = RTH(n, k, kap)
    for T in range(n * n):
        Ae = P.element_dtn(T)
        assert np.abs(Ae - Ae.T).max() <= 1e-13 * np.abs(Ae).max()
        assert np.linalg.eigvalsh(0.5 * (Ae + Ae.T)).min() >= -1e-12 * np.abs(Ae).max()
        assert np.abs(Ae @ np.ones(P.nl)).max() <= 1e-13 * np.abs(Ae).max()
        u, q = P.recover_element(T, np.ones(P.nl))
        assert np.abs(u - 1).max() <= 1e-13 and np.abs(q).max() <= 1e-11


@pytest.mark.parametrize("k", [1, 2, 3])
def test_R2_polynomial_reproduction(k):
    n, kap = 3, 2.5
    rng = np.random.default_rng(20 + k)
    coef = rng.standard_normal((k + 1) ** 2)
    u, grad, f = _poly(2, k, coef, kap)
    P = RTH(n, k, kap * np.ones(n * n))
    Xn = P.volume_nodes().reshape(-1, 2)
    fn = f(Xn).reshape(n * n, -1)
    A, g, lb = P.assemble(fn, u)
    lam = spla.spsolve(A.tocsc(), g)
    uh, qh = P.reconstruct(lam, fn, lb)
    scale = np.abs(u(Xn)).max()
    assert np.abs(lam - u(P.interior_trace_nodes())).max() <= 1e-11 * scale
    assert np.abs(uh.ravel() - u(Xn)).max() <= 1e-11 * scale
    qe = -kap * grad(Xn).reshape(n * n, P.nv, 2).transpose(0, 2, 1)
    assert np.abs(qh - qe).max() <= 1e-10 * np.abs(qe).max()


@pytest.mark.parametrize("k", [1, 2])
def test_R3_condensed_equals_uncondensed(k):
    n = 4
    rng = np.random.default_rng(8)
    kap = 10.0 ** rng.uniform(-1, 1, n * n)
    P = RTH(n, k, kap)
    f = rng.standard_normal((n * n, P.nv))

    def gD(X):
        return np.cos(X.sum(axis=1))
    A, g, lb = P.assemble(f, gD)
    lam = spla.spsolve(A.tocsc(), g)
    u, q = P.reconstruct(lam, f, lb)
    lm, um, qm = P.monolithic_solve(f, gD)
    assert np.abs(lam - lm).max() <= 1e-11 * np.abs(lm).max()
    assert np.abs(u - um).max() <= 1e-11 * np.abs(um).max()
    assert np.abs(q - qm).max() <= 1e-10 * np.abs(qm).max()


@pytest.mark.parametrize("k", [1, 2])
def test_R4_convergence_rates(k):
    pi = np.pi

    def u(X):
        return np.sin(pi * X[:, 0]) * np.sin(pi * X[:, 1])

    def grad(X):
        return np.stack([pi * np.cos(pi * X[:, 0]) * np.sin(pi * X[:, 1]),
                         pi * np.sin(pi * X[:, 0]) * np.cos(pi * X[:, 1])], axis=1)
    eu, eq = [], []
    for n in (4, 8, 16):
        P = RTH(n, k, np.ones(n * n))
        fn = (2 * pi ** 2 * u(P.volume_nodes().reshape(-1, 2))).reshape(n * n, -1)
        A, g, lb = P.assemble(fn, u)
        lam = spla.spsolve(A.tocsc(), g)
        uh, qh = P.reconstruct(lam, fn, lb)
        a, b = P.errors(uh, qh, u, grad)
        eu.append(a)
        eq.append(b)
    assert np.log2(eu[1] / eu[2]) >= k + 1 - 0.1
    assert np.log2(eq[1] / eq[2]) >= k + 1 - 0.1


def _mix(n, seed=0):
    return np.random.default_rng(seed).random(n * n) < 0.5


def test_M1_multinumerics_reproduction():
    n, k = 4, 1
    use = _mix(n)
    assert use.any() and not use.all()
    P = Multinumerics(n, k, _tau(2, n, k), np.full(n * n, 1.7), use)

    def lin(X):
        return 0.3 + X[:, 0] - 2.0 * X[:, 1]
    A, g, lb = P.assemble(None, lin)
    lam = spla.spsolve(A.tocsc(), g)
    uh, qh = P.reconstruct(lam, None, lb)
    Xn = P.volume_nodes().reshape(-1, 2)
    assert np.abs(uh.ravel() - lin(Xn)).max() <= 1e-12
    assert np.abs(qh[:, 0] + 1.7).max() <= 1e-12 and np.abs(qh[:, 1] - 3.4).max() <= 1e-12
    kap = np.repeat(10.0 ** np.linspace(-1, 1, n), n)
    P2 = Multinumerics(n, k, _tau(2, n, k), kap, _mix(n, 1))

    def u2(X):
        return 1.0 + 2.0 * X[:, 0]
    A, g, lb = P2.assemble(None, u2)
    lam = spla.spsolve(A.tocsc(), g)
    uh, qh = P2.reconstruct(lam, None, lb)
    assert np.abs(uh.ravel() - u2(Xn)).max() <= 1e-11
    assert np.abs(qh[:, 0, :] + 2.0 * kap[:, None]).max() <= 1e-10


@pytest.mark.parametrize("k", [1, 2])
def test_M2_multinumerics_condensed_equals_uncondensed(k):
    n = 4
    rng = np.random.default_rng(9)
    kap = 10.0 ** rng.uniform(-1, 1, n * n)
    P = Multinumerics(n, k, _tau(2, n, k), kap, _mix(n, 2))
    f = rng.standard_normal((n * n, P.nv))

    def gD(X):
        return np.sin(2 * X[:, 0]) + X[:, 1]
    A, g, lb = P.assemble(f, gD)
    lam = spla.spsolve(A.tocsc(), g)
    u, q = P.reconstruct(lam, f, lb)
    lm, um, qm = P.monolithic_solve(f, gD)
    assert np.abs(lam - lm).max() <= 1e-11 * np.abs(lm).max()
    assert np.abs(u - um).max() <= 1e-11 * np.abs(um).max()
    assert np.abs(q - qm).max() <= 1e-10 * np.abs(qm).max()


def example6(n, k=1):
    """Example VI coefficient 1 + 0.5 sin(4 pi x) cos(3 pi y) at the element
    centres, NIPG-H inside the disk of radius 0.3 about (0.45, 0.55), RT-H
    outside; tau = kappa (p+1)(p+2)/h_min on the NIPG-H elements."""
    c = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(c, c, indexing="xy")
    kap = (1.0 + 0.5 * np.sin(4 * np.pi * X) * np.cos(3 * np.pi * Y)).ravel()
    use_rt = ((X - 0.45) ** 2 + (Y - 0.55) ** 2 > 0.09).ravel()
    return Multinumerics(n, k, _tau(2, n, k), kap, use_rt)


def test_M3_multigrid_on_multinumerics():
    P = example6(8)
    A, g, _ = P.assemble(np.ones((64, P.nv)))
    H = mg.Hierarchy(A, 2, 8, 1)
    for i in range(len(H.levels) - 1):
        L, Lc = H.levels[i], H.levels[i + 1]
        G = (L.Q @ L.A @ L.I).toarray()
        assert np.abs(G - Lc.A.toarray()).max() <= 1e-12 * np.abs(Lc.A).max()
    counts = []
    for L in (3, 4, 5):
        n = 2 ** L
        P = example6(n)
        A, g, _ = P.assemble(np.ones((n * n, P.nv)))
        H = mg.Hierarchy(A, 2, n, 1, sweeps=3, growth=2)
        r1 = mg.mg_solve(H, A, g, tol=1e-9)
        r2 = mg.gmres_solve(H, A, g, tol=1e-9, side="left")
        assert r1.converged and r2.converged
        counts.append((r1.iters, r2.iters))
    assert max(c[0] for c in counts) <= 18 and abs(counts[2][0] - counts[1][0]) <= 2, counts
    assert max(c[1] for c in counts) <= 8, counts
