"""Pins of the oracle's unstructured-mesh path (Sec. 2 on P^k triangles;
Sec. 3.1.2 seed-point agglomeration and the P^1 parameterization of
macro-edges; Sec. 3 multigrid on the agglomerated levels).

U1  the triangle rule integrates x^a y^b exactly (a! b! / (a + b + 2)!).
U2  element maps symmetric positive semidefinite, constants in their kernel.
U3  polynomial reproduction: u in P^k with f = -kappa lap u gives exact
    traces and nodal u on an unstructured mesh (any wrong normal, edge
    orientation, quadrature or basis breaks it).
U4  static condensation = the uncondensed (q, u, lambda) system.
U5  convergence: u and q of order k + 1 in L2 under refinement.
U6  agglomeration: level 1 is the nearest-seed partition (brute force),
    every level splits each macro-element of the previous one into at most
    four parts of sizes that differ by at most one, and the levels nest.
U7  macro-edges: every boundary face of the finer level lies in exactly one
    chain, chains are connected from start to end vertex, J has unit row
    sums and maps the coarse arc-length coordinate (0 at the start, L at the
    end) onto the arc length of every finer face end.
U8  the Galerkin chain A_{k-1} = Q A I holds and every level is SPD.
U9  GMRES and MG counts stay bounded as the mesh is refined (Example II's
    mesh is available only as a figure, so its table counts are "parity
    unpinned": the synthetic box with eight holes stands in).
U10 Example III on a synthetic disk mesh (tests/golden/ex3_hdg_smooth_iterations.txt,
    Table HDG_smooth_k_tau1): hierarchy sizes near the paper's, GMRES
    within 3 and MG within twice the table (parity unpinned: other mesh),
    u converging to the exact solution.
U11 SIPG-H, IIPG-H, NIPG-H on P^k triangles reproduce u in P^k (traces, u,
    q = -kappa grad u); SIPG-H maps symmetric, the others not.
U12 NIPG-H multigrid on the box with holes: Galerkin chain with Q != I^T,
    bounded MG / GMRES counts.
"""
from math import factorial

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import mg
from oracle import unstructured as U
from paper_1811_09909_amd import inputs


def _mesh(nx=8, holes=True):
    w = inputs.unstructured2d(nx, 1, holes=holes)
    return U.TriMesh(w.vertices, w.triangles), w


@pytest.mark.parametrize("q", [2, 3, 5])
def test_U1_triangle_quadrature(q):
    X, W = U.tri_quadrature(q)
    for a in range(2 * q):
        for b in range(2 * q - 1 - a):
            exact = factorial(a) * factorial(b) / factorial(a + b + 2)
            assert abs(np.sum(W * X[:, 0] ** a * X[:, 1] ** b) - exact) <= 1e-15 * max(1.0, exact) + 1e-17


@pytest.mark.parametrize("k", [1, 2, 3])
def test_U2_element_maps_spsd(k):
    m, _ = _mesh()
    P = U.TriHDG(m, k, 1.0, np.random.default_rng(k).uniform(0.1, 10.0, m.nel))
    for t in range(0, m.nel, 37):
        Ae = P.element_dtn(t)
        sc = np.abs(Ae).max()
        assert np.abs(Ae - Ae.T).max() <= 1e-13 * sc
        assert np.linalg.eigvalsh(0.5 * (Ae + Ae.T)).min() >= -1e-12 * sc
        assert np.abs(Ae @ np.ones(P.nl)).max() <= 1e-13 * sc


def _poly(k, coef):
    ex = U.tri_monomials(k)

    def u(X):
        return sum(c * X[:, 0] ** a * X[:, 1] ** b for c, (a, b) in zip(coef, ex))

    def lap(X):
        s = np.zeros(len(X))
        for c, (a, b) in zip(coef, ex):
            if a >= 2:
                s = s + c * a * (a - 1) * X[:, 0] ** (a - 2) * X[:, 1] ** b
            if b >= 2:
                s = s + c * b * (b - 1) * X[:, 0] ** a * X[:, 1] ** (b - 2)
        return s
    return u, lap


@pytest.mark.parametrize("k", [1, 2, 3])
def test_U3_polynomial_reproduction(k):
    m, _ = _mesh()
    kap = 2.5
    u, lap = _poly(k, np.random.default_rng(30 + k).standard_normal((k + 1) * (k + 2) // 2))
    P = U.TriHDG(m, k, 1.0, np.full(m.nel, kap))
    Xn = P.volume_nodes().reshape(-1, 2)
    fn = (-kap * lap(Xn)).reshape(m.nel, -1)
    A, g, lb = P.assemble(fn, u)
    lam = spla.spsolve(A.tocsc(), g)
    sc = np.abs(u(Xn)).max()
    assert np.abs(lam - u(P.interior_trace_nodes())).max() <= 1e-10 * sc
    uh, _ = P.reconstruct(lam, fn, lb)
    assert np.abs(uh.ravel() - u(Xn)).max() <= 1e-10 * sc


@pytest.mark.parametrize("k", [1, 2])
def test_U4_condensed_equals_uncondensed(k):
    m, _ = _mesh()
    rng = np.random.default_rng(4)
    P = U.TriHDG(m, k, 1.0, 10.0 ** rng.uniform(-1, 1, m.nel))
    f = rng.standard_normal((m.nel, P.nv))

    def gD(X):
        return np.cos(X.sum(axis=1))
    A, g, lb = P.assemble(f, gD)
    lam = spla.spsolve(A.tocsc(), g)
    u, q = P.reconstruct(lam, f, lb)
    lm, um, qm = P.monolithic_solve(f, gD)
    assert np.abs(lam - lm).max() <= 1e-11 * np.abs(lm).max()
    assert np.abs(u - um).max() <= 1e-11 * np.abs(um).max()
    assert np.abs(q - qm).max() <= 1e-10 * np.abs(qm).max()


def _square(nx, jit=0.3, seed=0):
    """Delaunay triangulation of a jittered (nx+1)^2 grid on the unit square."""
    from scipy.spatial import Delaunay
    xs = np.linspace(0.0, 1.0, nx + 1)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    V = np.stack([X.ravel(), Y.ravel()], axis=1)
    inner = (V[:, 0] > 0) & (V[:, 0] < 1) & (V[:, 1] > 0) & (V[:, 1] < 1)
    V[inner] += np.random.default_rng(seed).uniform(-jit / nx, jit / nx, V[inner].shape)
    T = Delaunay(V).simplices
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    neg = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]) < 0
    T[neg] = T[neg][:, [0, 2, 1]]
    return V, T


@pytest.mark.parametrize("k", [1, 2])
def test_U5_convergence_rates(k):
    pi = np.pi

    def u(X):
        return np.sin(pi * X[:, 0]) * np.sin(pi * X[:, 1])

    def grad(X):
        return np.stack([pi * np.cos(pi * X[:, 0]) * np.sin(pi * X[:, 1]),
                         pi * np.sin(pi * X[:, 0]) * np.cos(pi * X[:, 1])], axis=1)
    eu, eq = [], []
    for nx in (4, 8, 16):
        m = U.TriMesh(*_square(nx))
        P = U.TriHDG(m, k, 1.0, np.ones(m.nel))
        fn = (2 * pi ** 2 * u(P.volume_nodes().reshape(-1, 2))).reshape(m.nel, -1)
        A, g, lb = P.assemble(fn, u)
        lam = spla.spsolve(A.tocsc(), g)
        uh, qh = P.reconstruct(lam, fn, lb)
        a, b = P.errors(uh, qh, u, grad)
        eu.append(a)
        eq.append(b)
    assert np.log2(eu[1] / eu[2]) >= k + 1 - 0.1, eu
    assert np.log2(eq[1] / eq[2]) >= k + 1 - 0.1, eq


def test_U6_agglomeration():
    m, w = _mesh(16)
    parts = U.agglomerate(m, w.seeds, 4)
    cen = m.centroids()
    d2 = ((cen[:, None, :] - w.seeds[None, :, :]) ** 2).sum(axis=2)
    near = np.array([min(range(len(w.seeds)), key=lambda s: (d2[t, s], s)) for t in range(m.nel)])
    # level 1: the seeds in order, those that win no triangle dropped
    used = sorted(set(near))
    assert np.array_equal(parts[0], np.array([used.index(s) for s in near]))
    for lev in range(1, len(parts)):
        fine, coarse = parts[lev], parts[lev - 1]
        assert fine.min() == 0 and len(np.unique(fine)) == fine.max() + 1
        for c in range(coarse.max() + 1):
            kids = np.unique(fine[coarse == c])
            assert 1 <= len(kids) <= 4
            sizes = [np.sum(fine == q) for q in kids]
            assert max(sizes) - min(sizes) <= 1
            # nesting: the children's triangles are exactly the parent's
            assert np.array_equal(np.sort(np.nonzero(np.isin(fine, kids))[0]), np.nonzero(coarse == c)[0])


def test_U7_macro_edges_arc_length():
    m, w = _mesh(16)
    parts = U.agglomerate(m, w.seeds, 4)
    fine = U.triangle_faces(m)
    cell_of = np.arange(m.nel)
    V = m.V
    for p in reversed(parts):
        coarse_of = np.zeros(cell_of.max() + 1, dtype=np.int64)
        coarse_of[cell_of] = p
        I_f, B_f, J, cf = U.macro_faces(fine, coarse_of)
        assert len(I_f) + len(B_f) == fine.nface and len(np.intersect1d(I_f, B_f)) == 0
        J = J.toarray()
        assert np.abs(J.sum(axis=1) - 1).max() <= 1e-15
        # every B face feeds exactly one macro-edge
        owner = [set(np.nonzero(J[2 * b] + J[2 * b + 1])[0] // 2) for b in range(len(B_f))]
        assert all(len(o) == 1 for o in owner)
        # chains of triangle edges: connected from start to end, lengths add up
        for E in range(cf.nface):
            v = cf.ends[E, 0]
            tot = 0.0
            for e, fwd in cf.chains[E]:
                lo, hi = m.faces[e]
                a, b = (lo, hi) if fwd else (hi, lo)
                assert a == v
                v = b
                tot += np.hypot(*(V[hi] - V[lo]))
            assert v == cf.ends[E, 1]
            assert abs(tot - cf.length[E]) <= 1e-12 * tot
        # J maps the coarse coordinate (0 at the start, L at the end) to the
        # arc length from the macro-edge's start of every fine face end
        s_coarse = np.zeros(2 * cf.nface)
        s_coarse[1::2] = cf.length
        s_fine = J @ s_coarse
        for E in range(cf.nface):
            pos = {int(cf.ends[E, 0]): 0.0}
            s = 0.0
            for e, fwd in cf.chains[E]:
                lo, hi = m.faces[e]
                a, b = (lo, hi) if fwd else (hi, lo)
                s += np.hypot(*(V[hi] - V[lo]))
                pos.setdefault(int(b), s)
            for bi, f in enumerate(B_f):
                if 2 * E in np.nonzero(J[2 * bi])[0] or 2 * E + 1 in np.nonzero(J[2 * bi])[0]:
                    for i in range(2):
                        v = int(fine.ends[f, i])
                        assert abs(s_fine[2 * bi + i] - pos[v]) <= 1e-12 * cf.length[E]
        fine, cell_of = cf, p


@pytest.mark.parametrize("k", [1, 3])
def test_U8_galerkin_chain_spd(k):
    m, w = _mesh(16)
    P = U.TriHDG(m, k, 1.0, 10.0 ** np.random.default_rng(8).uniform(-1, 1, m.nel))
    A, g, _ = P.assemble()
    H = U.UHierarchy(A, m, k, U.agglomerate(m, w.seeds, w.hlevels))
    assert len(H.levels) == w.hlevels + (2 if k > 1 else 1)
    for i in range(len(H.levels) - 1):
        L, Lc = H.levels[i], H.levels[i + 1]
        G = (L.Q @ L.A @ L.I).toarray()
        assert np.abs(G - Lc.A.toarray()).max() <= 1e-12 * np.abs(Lc.A).max()
        Ad = Lc.A.toarray()
        assert np.abs(Ad - Ad.T).max() <= 1e-12 * np.abs(Ad).max()
        assert np.linalg.eigvalsh(Ad).min() > 0


def test_U9_bounded_counts():
    counts = []
    for nx in (16, 32):
        for k in (1, 3):
            w = inputs.unstructured2d(nx, k)
            m = U.TriMesh(w.vertices, w.triangles)
            P = U.TriHDG(m, k, w.tau, w.kappa)
            A, g, _ = P.assemble(w.f)
            H = U.UHierarchy(A, m, k, U.agglomerate(m, w.seeds, w.hlevels))
            r1 = mg.mg_solve(H, A, g, tol=1e-9)
            r2 = mg.gmres_solve(H, A, g, tol=1e-9)
            assert r1.converged and r2.converged
            counts.append((nx, k, r1.iters, r2.iters))
    assert max(c[3] for c in counts) <= 18, counts
    assert max(c[2] for c in counts) <= 50, counts


def _golden_ex3():
    import os
    rows = {}
    path = os.path.join(os.path.dirname(__file__), "golden", "ex3_hdg_smooth_iterations.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        tok = line.split()
        rows[(tok[0], int(tok[1]))] = [int(x) for x in tok[2:]]
    return rows


def test_U10_example3_disk():
    """Example III on a synthetic disk mesh (Table HDG_smooth_k_tau1; the
    paper's meshes of the circle are not available, so its counts are
    "parity unpinned"): with 21 seed points the hierarchy has about the
    paper's element counts per level, the GMRES counts stay within 3 of the
    table for p = 1, 2 at L = 2 .. 4, MG within twice the table, and the
    recovered u approaches x y exp(x^2 y^3)."""
    tab = _golden_ex3()
    errs = []
    for L in (2, 3, 4):
        for k in (1, 2):
            w = inputs.example3_disk(L, k)
            m = U.TriMesh(w.vertices, w.triangles)
            assert abs(m.nel - 84 * 4 ** (L - 2)) <= 0.25 * 84 * 4 ** (L - 2)
            P = U.TriHDG(m, k, w.tau, w.kappa)
            Xn = P.volume_nodes().reshape(-1, 2)
            fn = w.f(Xn).reshape(m.nel, -1)
            A, g, lb = P.assemble(fn, w.u_exact)
            H = U.UHierarchy(A, m, k, U.agglomerate(m, w.seeds, w.hlevels))
            r1 = mg.mg_solve(H, A, g, tol=1e-9)
            r2 = mg.gmres_solve(H, A, g, tol=1e-9, side="left")
            assert r1.converged and r2.converged
            assert abs(r2.iters - tab[("gmres", k)][L - 2]) <= 3, (L, k, r2.iters)
            assert r1.iters <= 2 * tab[("mg", k)][L - 2], (L, k, r1.iters)
            uh, _ = P.reconstruct(r1.lam, fn, lb)
            errs.append((k, np.abs(uh.ravel() - w.u_exact(Xn)).max()))
    for k in (1, 2):
        e = [v for kk, v in errs if kk == k]
        assert e[0] > e[1] > e[2]


def _hmin(w):
    V, T = w.vertices, w.triangles
    e = np.concatenate([T[:, [0, 1]], T[:, [1, 2]], T[:, [2, 0]]])
    return np.hypot(*(V[e[:, 0]] - V[e[:, 1]]).T).min()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_U11_ipdg_triangles_reproduction(k):
    """SIPG-H, IIPG-H and NIPG-H on P^k triangles (eq. IPG_H): u in P^k with
    f = -kappa lap u and its Dirichlet data gives exact traces, u and q =
    -kappa grad u at the nodes (tau = (p+1)(p+2)/h_min); SIPG-H element maps
    are symmetric, IIPG-H and NIPG-H ones are not."""
    m, w = _mesh()
    kap = 2.5
    coef = np.random.default_rng(50 + k).standard_normal((k + 1) * (k + 2) // 2)
    u, lap = _poly(k, coef)
    ex = U.tri_monomials(k)

    def grad(X):
        gx, gy = np.zeros(len(X)), np.zeros(len(X))
        for c, (a, b) in zip(coef, ex):
            if a >= 1:
                gx = gx + c * a * X[:, 0] ** (a - 1) * X[:, 1] ** b
            if b >= 1:
                gy = gy + c * b * X[:, 0] ** a * X[:, 1] ** (b - 1)
        return np.stack([gx, gy], axis=1)
    for scheme in ("sipg", "iipg", "nipg"):
        P = U.TriIPDG(m, k, (k + 1) * (k + 2) / _hmin(w), np.full(m.nel, kap), scheme)
        Xn = P.volume_nodes().reshape(-1, 2)
        fn = (-kap * lap(Xn)).reshape(m.nel, -1)
        A, g, lb = P.assemble(fn, u)
        lam = spla.spsolve(A.tocsc(), g)
        uh, qh = P.reconstruct(lam, fn, lb)
        sc = np.abs(u(Xn)).max()
        qe = -kap * grad(Xn).reshape(m.nel, -1, 2).transpose(0, 2, 1)
        assert np.abs(lam - u(P.interior_trace_nodes())).max() <= 1e-10 * sc
        assert np.abs(uh.ravel() - u(Xn)).max() <= 1e-10 * sc
        assert np.abs(qh - qe).max() <= 1e-8 * np.abs(qe).max()
        Ae = P.element_dtn(0)
        asym = np.abs(Ae - Ae.T).max() / np.abs(Ae).max()
        assert (asym <= 1e-13) if scheme == "sipg" else (asym >= 1e-3)


def test_U12_nipg_multigrid_triangles():
    """NIPG-H on the box with holes: the Galerkin chain with the nonsymmetric
    restriction Q != I^T, and MG / GMRES converging with counts bounded
    under refinement (Example II's Table NIPG: "parity unpinned", other
    mesh)."""
    counts = []
    for nx in (16, 32):
        w = inputs.unstructured2d(nx, 1)
        m = U.TriMesh(w.vertices, w.triangles)
        P = U.TriIPDG(m, 1, 6.0 / _hmin(w), w.kappa, "nipg")
        A, g, _ = P.assemble(w.f)
        H = U.UHierarchy(A, m, 1, U.agglomerate(m, w.seeds, w.hlevels))
        L0 = H.levels[0]
        assert abs(L0.Q - L0.I.T).max() > 1e-3
        for i in range(len(H.levels) - 1):
            L, Lc = H.levels[i], H.levels[i + 1]
            G = (L.Q @ L.A @ L.I).toarray()
            assert np.abs(G - Lc.A.toarray()).max() <= 1e-11 * np.abs(Lc.A).max()
        r1 = mg.mg_solve(H, A, g, tol=1e-9)
        r2 = mg.gmres_solve(H, A, g, tol=1e-9)
        assert r1.converged and r2.converged
        counts.append((r1.iters, r2.iters))
    assert max(c[1] for c in counts) <= 20 and max(c[0] for c in counts) <= 60, counts
