"""HDG on unstructured triangle meshes and the agglomeration multigrid of
Sec. 3.1.2 (oracle; test infrastructure only).

* ``TriMesh``  -- vertices and counter-clockwise triangles; the edges, the
  interior ones numbered by their sorted vertex pair (the trace unknowns),
  the boundary ones apart (Dirichlet data).  Every edge carries P^k traces
  nodal at the GLL points of its own parameter t in [0, 1], which runs from
  its lower-numbered vertex to the other one.
* ``TriHDG``   -- the HDG local problem (eqs. HDG, HDG_flux) on P^k
  triangles, static condensation into the trace system (eq.
  trace_linear_system), local recovery and the uncondensed system.  The
  volume basis is nodal at the equispaced lattice of the reference
  triangle; integrals use the collapsed (Duffy) product of Gauss rules.
* ``TriIPDG``  -- the hybridized interior penalty family (eq. IPG_H:
  SIPG-H, IIPG-H, NIPG-H) on the same triangles and traces.
* ``agglomerate`` -- the seed-point agglomeration of Sec. 3.1.2: the
  level-1 macro-elements gather the triangles nearest to each seed point,
  and every level's macro-elements are split into four to form the next.
* ``macro_faces`` -- the interface grid of a coarser partition (every
  macro-edge is a connected chain of the finer level's faces shared by the
  same two macro-elements) and the P^1 coarse space on it, parameterized by
  arc length along the chain (the remark of Sec. 3: macro-edges of
  agglomerated meshes are not straight), with the injection J of that space
  into the finer level's P^1 traces.
* ``UHierarchy`` -- the multigrid of Sec. 3 on these levels: p-coarsening
  to P^1 on the triangles, then h-coarsening through the partitions; the
  Galerkin operators, transfers, smoothers and the V-cycle of
  ``oracle.mg``.

Numbering shared by every level (so that level operators compare entry by
entry): cells are triangles, then macro-elements in the order of
``agglomerate``; faces of the triangle levels are the interior edges in
order of their sorted vertex pair; macro-edges of a coarser level are
ordered by (lower macro-element, higher macro-element, smallest finer face
in the chain).  Face f holds DOFs f m .. f m + m - 1 (m = k + 1 on the
finest level, 2 on P^1 levels); a macro-edge's two DOFs sit at its start
and its end vertex.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import mg
from .refelem import gauss_rule, gll_nodes, lagrange


# ---------------------------------------------------------------------------
# reference triangle (vertices (0,0), (1,0), (0,1))
def tri_lattice(k):
    """The (k+1)(k+2)/2 equispaced nodes (i/k, j/k), i + j <= k, j slowest."""
    return np.array([(i / k, j / k) for j in range(k + 1) for i in range(k + 1 - j)])


def tri_monomials(k):
    """Exponents (a, b) of x^a y^b, a + b <= k."""
    return np.array([(a, t - a) for t in range(k + 1) for a in range(t, -1, -1)])


def tri_quadrature(q):
    """Collapsed Gauss rule on the reference triangle: x = s (1 - r),
    y = r, weight w_s w_r (1 - r); exact for x^a y^b with a < 2q and
    a + b + 1 < 2q."""
    g, w = gauss_rule(q)
    X, W = [], []
    for j in range(q):
        for i in range(q):
            X.append((g[i] * (1 - g[j]), g[j]))
            W.append(w[i] * w[j] * (1 - g[j]))
    return np.array(X), np.array(W)


class RefTriangle:
    """Nodal P^k basis on the reference triangle through the monomial
    Vandermonde matrix: phi_i = sum_m C[m, i] x^a_m y^b_m with
    phi_i(node_j) = delta_ij."""

    def __init__(self, k):
        self.k = k
        self.nodes = tri_lattice(k)
        self.exps = tri_monomials(k)
        self.nv = len(self.nodes)
        self.C = np.linalg.inv(self.mono(self.nodes))

    def mono(self, X):
        X = np.atleast_2d(X)
        return X[:, 0:1] ** self.exps[None, :, 0] * X[:, 1:2] ** self.exps[None, :, 1]

    def mono_grad(self, X):
        X = np.atleast_2d(X)
        a, b = self.exps[:, 0], self.exps[:, 1]
        with np.errstate(divide="ignore", invalid="ignore"):
            dx = np.where(a > 0, a * X[:, 0:1] ** np.maximum(a - 1, 0) * X[:, 1:2] ** b, 0.0)
            dy = np.where(b > 0, b * X[:, 0:1] ** a * X[:, 1:2] ** np.maximum(b - 1, 0), 0.0)
        return dx, dy

    def values(self, X):
        """phi_i(X_q) as [nq, nv]."""
        return self.mono(X) @ self.C

    def grads(self, X):
        """(d phi / dx, d phi / dy) at X_q on the reference triangle, each [nq, nv]."""
        dx, dy = self.mono_grad(X)
        return dx @ self.C, dy @ self.C


# ---------------------------------------------------------------------------
class TriMesh:
    """Triangles (counter-clockwise vertex triples) and their edges.

    Slot s of triangle T is its edge from vertex T[s] to T[(s+1) % 3]."""

    def __init__(self, V, T):
        self.V = np.asarray(V, dtype=float)
        self.T = np.asarray(T, dtype=np.int64)
        self.nel = len(self.T)
        a, b, c = self.V[self.T[:, 0]], self.V[self.T[:, 1]], self.V[self.T[:, 2]]
        area2 = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
        if np.any(area2 <= 0):
            raise ValueError("triangles must be counter-clockwise and non-degenerate")
        keys = {}
        for t in range(self.nel):
            for s in range(3):
                u, v = int(self.T[t, s]), int(self.T[t, (s + 1) % 3])
                keys.setdefault((min(u, v), max(u, v)), []).append((t, s))
        inter = sorted(k for k, w in keys.items() if len(w) == 2)
        bnd = sorted(k for k, w in keys.items() if len(w) == 1)
        if any(len(w) > 2 for w in keys.values()):
            raise ValueError("an edge is shared by more than two triangles")
        self.faces = np.array(inter, dtype=np.int64).reshape(-1, 2)   # (lo, hi) vertex of each interior edge
        self.bfaces = np.array(bnd, dtype=np.int64).reshape(-1, 2)
        self.nface, self.nbface = len(inter), len(bnd)
        self.face_cells = np.zeros((self.nface, 2, 2), dtype=np.int64)  # [f][side] = (triangle, slot)
        self.slot_face = np.zeros((self.nel, 3), dtype=np.int64)         # interior face id, or -1 - boundary id
        for f, key in enumerate(inter):
            w = sorted(keys[key])
            self.face_cells[f] = w
            for (t, s) in w:
                self.slot_face[t, s] = f
        for b, key in enumerate(bnd):
            (t, s), = keys[key]
            self.slot_face[t, s] = -1 - b
        self.d = 2

    def centroids(self):
        """((x0 + x1) + x2) / 3 per triangle, coordinate by coordinate."""
        P = self.V[self.T]
        return ((P[:, 0] + P[:, 1]) + P[:, 2]) / 3.0

    def edge_length(self, lo, hi):
        d = self.V[hi] - self.V[lo]
        return float(np.hypot(d[0], d[1]))


class TriHDG:
    """HDG with P^k volume and trace spaces on a ``TriMesh`` (Sec. 2), kappa
    one value per triangle, scalar tau.  Local unknowns [q_x, q_y, u]."""

    def __init__(self, mesh, k, tau, kappa):
        self.mesh, self.k, self.tau = mesh, k, float(tau)
        self.d = 2
        self.kappa = np.asarray(kappa, dtype=float)
        if self.kappa.shape != (mesh.nel,):
            raise ValueError("kappa: one value per triangle")
        self.ref = RefTriangle(k)
        self.nv = self.ref.nv
        self.ne = k + 1
        self.nf = 3
        self.nl = 3 * self.ne
        self.nlam = mesh.nface * self.ne
        self.nbdof = mesh.nbface * self.ne
        self.xi = gll_nodes(k)
        self.qX, self.qW = tri_quadrature(k + 2)
        self.eg, self.ew = gauss_rule(k + 2)
        self.Mu = lagrange(self.xi, self.eg).T            # [nfq, ne]
        gmap = -np.ones((mesh.nel, self.nl), dtype=np.int64)
        bmap = -np.ones((mesh.nel, self.nl), dtype=np.int64)
        for t in range(mesh.nel):
            for s in range(3):
                f = mesh.slot_face[t, s]
                rng = np.arange(self.ne)
                if f >= 0:
                    gmap[t, s * self.ne:(s + 1) * self.ne] = f * self.ne + rng
                else:
                    bmap[t, s * self.ne:(s + 1) * self.ne] = (-1 - f) * self.ne + rng
        self.gmap, self.bmap = gmap, bmap

    # -- element matrices ---------------------------------------------------
    def geometry(self, t):
        P = self.mesh.V[self.mesh.T[t]]
        Jm = np.stack([P[1] - P[0], P[2] - P[0]], axis=1)
        return P, Jm, np.linalg.det(Jm), np.linalg.inv(Jm)

    def element_blocks(self, t):
        """Mass M, (q, grad)-blocks, face blocks of triangle t (physical)."""
        ref, nv, ne, nl = self.ref, self.nv, self.ne, self.nl
        P, Jm, det, Ji = self.geometry(t)
        Phi = ref.values(self.qX)
        gx, gy = ref.grads(self.qX)
        dPhi = [Ji[0, c] * gx + Ji[1, c] * gy for c in range(2)]   # d/dx_c = sum_r (J^-1)_{rc} d/dxi_r
        W = self.qW * det
        M = (Phi.T * W) @ Phi
        Bdiv = np.zeros((2 * nv, nv))
        C = np.zeros((nv, 2 * nv))
        for c in range(2):
            Bdiv[c * nv:(c + 1) * nv] = -(dPhi[c].T * W) @ Phi
            C[:, c * nv:(c + 1) * nv] = -(dPhi[c].T * W) @ Phi
        F = np.zeros((2 * nv, nl))
        E = np.zeros((nv, nv))
        G = np.zeros((nv, nl))
        H = np.zeros((nl, nl))
        T = self.mesh.T[t]
        for s in range(3):
            va, vb = int(T[s]), int(T[(s + 1) % 3])
            lo, hi = min(va, vb), max(va, vb)
            A, B = self.mesh.V[lo], self.mesh.V[hi]
            ln = float(np.hypot(*(B - A)))
            dvec = self.mesh.V[vb] - self.mesh.V[va]
            nrm = np.array([dvec[1], -dvec[0]]) / ln
            X = A[None, :] + self.eg[:, None] * (B - A)[None, :]
            Xi = (X - P[0]) @ Ji.T
            Pf = ref.values(Xi)
            wf = self.ew * ln
            cols = slice(s * ne, (s + 1) * ne)
            Ef = (Pf.T * wf) @ Pf
            E += Ef
            G[:, cols] = (Pf.T * wf) @ self.Mu
            H[cols, cols] = (self.Mu.T * wf) @ self.Mu
            for c in range(2):
                F[c * nv:(c + 1) * nv, cols] = nrm[c] * (Pf.T * wf) @ self.Mu
                C[:, c * nv:(c + 1) * nv] += nrm[c] * Ef
        return M, Bdiv, C, F, E, G, H

    def local_matrix(self, t):
        """L_T = [[M / kappa_T (per component), Bdiv], [C, tau E]]."""
        M, Bdiv, C, F, E, G, H = self.element_blocks(t)
        nv = self.nv
        L = np.zeros((3 * nv, 3 * nv))
        for c in range(2):
            L[c * nv:(c + 1) * nv, c * nv:(c + 1) * nv] = M / self.kappa[t]
        L[:2 * nv, 2 * nv:] = Bdiv
        L[2 * nv:, :2 * nv] = C
        L[2 * nv:, 2 * nv:] = self.tau * E
        R = np.vstack([-F, self.tau * G])
        S = np.vstack([F, self.tau * G])
        return L, R, S, H, M

    def element_dtn(self, t, f_t=None):
        """A^e = tau H - S^T L^-1 R and b^e = S^T L^-1 [0; M f_T]."""
        L, R, S, H, M = self.local_matrix(t)
        Ae = self.tau * H - S.T @ np.linalg.solve(L, R)
        if f_t is None:
            return Ae
        rhs = np.zeros(L.shape[0])
        rhs[2 * self.nv:] = M @ f_t
        return Ae, S.T @ np.linalg.solve(L, rhs)

    def all_element_dtn(self):
        return np.stack([self.element_dtn(t) for t in range(self.mesh.nel)])

    # -- node coordinates ---------------------------------------------------
    def volume_nodes(self):
        """Physical coordinates of every triangle's nodes, [N_T, nv, 2]."""
        P = self.mesh.V[self.mesh.T]
        ref = self.ref.nodes
        return P[:, None, 0, :] + ref[None, :, 0:1] * (P[:, None, 1, :] - P[:, None, 0, :]) \
            + ref[None, :, 1:2] * (P[:, None, 2, :] - P[:, None, 0, :])

    def _edge_nodes(self, pairs):
        V = self.mesh.V
        A, B = V[pairs[:, 0]], V[pairs[:, 1]]
        return (A[:, None, :] + self.xi[None, :, None] * (B - A)[:, None, :]).reshape(-1, 2)

    def interior_trace_nodes(self):
        return self._edge_nodes(self.mesh.faces)

    def boundary_nodes(self):
        return self._edge_nodes(self.mesh.bfaces)

    # -- trace system -------------------------------------------------------
    def assemble(self, f_nodal=None, gD=None):
        """(A, g, lam_bnd) of eq. trace_linear_system, Dirichlet data gD."""
        nel, nl = self.mesh.nel, self.nl
        f_nodal = np.zeros((nel, self.nv)) if f_nodal is None else np.asarray(f_nodal, dtype=float)
        lam_b = np.zeros(self.nbdof) if gD is None else np.asarray(gD(self.boundary_nodes()), dtype=float)
        rows, cols, vals = [], [], []
        g = np.zeros(self.nlam)
        self.Ae = np.zeros((nel, nl, nl))
        for t in range(nel):
            Ae, be = self.element_dtn(t, f_nodal[t])
            self.Ae[t] = Ae
            gi, bi = self.gmap[t], self.bmap[t]
            ii = np.nonzero(gi >= 0)[0]
            jb = np.nonzero(bi >= 0)[0]
            rr, cc = np.meshgrid(gi[ii], gi[ii], indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(Ae[np.ix_(ii, ii)].ravel())
            np.add.at(g, gi[ii], be[ii])
            if len(jb):
                np.add.at(g, gi[ii], -Ae[np.ix_(ii, jb)] @ lam_b[bi[jb]])
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.nlam, self.nlam)).tocsr()
        A.sum_duplicates()
        return A, g, lam_b

    def reconstruct(self, lam, f_nodal=None, lam_b=None):
        """u [N_T, nv] and q [N_T, 2, nv] (nodal) from the traces (Sec. 2)."""
        nel, nv = self.mesh.nel, self.nv
        f_nodal = np.zeros((nel, nv)) if f_nodal is None else np.asarray(f_nodal, dtype=float)
        lam_b = np.zeros(self.nbdof) if lam_b is None else lam_b
        u = np.zeros((nel, nv))
        q = np.zeros((nel, 2, nv))
        for t in range(nel):
            LT = np.where(self.gmap[t] >= 0, lam[np.maximum(self.gmap[t], 0)], lam_b[np.maximum(self.bmap[t], 0)])
            L, R, S, H, M = self.local_matrix(t)
            rhs = R @ LT
            rhs[2 * nv:] += M @ f_nodal[t]
            w = np.linalg.solve(L, rhs)
            u[t], q[t] = w[2 * nv:], w[:2 * nv].reshape(2, nv)
        return u, q

    def monolithic_solve(self, f_nodal=None, gD=None):
        """Every triangle's local equations and the conservation rows of
        every interior edge solved at once (sparse direct): (lambda, u, q)."""
        nel, nv, nl = self.mesh.nel, self.nv, self.nl
        f_nodal = np.zeros((nel, nv)) if f_nodal is None else np.asarray(f_nodal, dtype=float)
        lam_b = np.zeros(self.nbdof) if gD is None else np.asarray(gD(self.boundary_nodes()), dtype=float)
        nw = 3 * nv
        Nt = nel * nw + self.nlam
        rows, cols, vals = [], [], []
        rhs = np.zeros(Nt)

        def put(r, c, blk):
            rr, cc = np.meshgrid(r, c, indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(np.asarray(blk).ravel())

        for t in range(nel):
            L, R, S, H, M = self.local_matrix(t)
            wr = t * nw + np.arange(nw)
            gi, bi = self.gmap[t], self.bmap[t]
            ii = np.nonzero(gi >= 0)[0]
            jb = np.nonzero(bi >= 0)[0]
            put(wr, wr, L)
            put(wr, nel * nw + gi[ii], -R[:, ii])
            rhs[wr[2 * nv:]] += M @ f_nodal[t]
            rhs[wr] += R[:, jb] @ lam_b[bi[jb]]
            lr = nel * nw + gi[ii]
            put(lr, wr, S.T[ii, :])
            put(lr, nel * nw + gi[ii], -self.tau * H[np.ix_(ii, ii)])
            rhs[lr] += self.tau * H[np.ix_(ii, jb)] @ lam_b[bi[jb]]
        K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(Nt, Nt)).tocsc()
        sol = spla.spsolve(K, rhs)
        w = sol[:nel * nw].reshape(nel, nw)
        return sol[nel * nw:], w[:, 2 * nv:], w[:, :2 * nv].reshape(nel, 2, nv)

    def errors(self, u, q, u_exact, grad_exact, kappa=1.0):
        """L2 errors of u and q = -kappa grad u (kappa constant)."""
        eu = eq = 0.0
        Phi = self.ref.values(self.qX)
        for t in range(self.mesh.nel):
            P, Jm, det, Ji = self.geometry(t)
            X = P[0] + self.qX @ Jm.T
            W = self.qW * det
            eu += np.sum(W * (Phi @ u[t] - u_exact(X)) ** 2)
            qe = -kappa * grad_exact(X)
            for c in range(2):
                eq += np.sum(W * (Phi @ q[t, c] - qe[:, c]) ** 2)
        return np.sqrt(eu), np.sqrt(eq)


class TriIPDG(TriHDG):
    """The hybridized interior penalty family (eq. IPG_H; SIPG-H, IIPG-H,
    NIPG-H with s_f = 1, 0, -1) on P^k triangles, kappa per triangle, scalar
    tau.  Rows for the test function, per triangle:

        L = kappa (K - s_f N - N^T) + tau E,   K_ij = (grad phi_j, grad phi_i),
                                               N_ij = <phi_j, grad phi_i . n>,
        R = tau G - s_f kappa D,               D_il = <mu_l, grad phi_i . n>,
        C = tau G^T - kappa D^T,

    A^e = tau H - C L^-1 R, b^e = C L^-1 M f; recovery u = L^-1 (R Lambda +
    M f) and q = -kappa grad u at the nodes."""

    SCHEMES = {"sipg": 1.0, "iipg": 0.0, "nipg": -1.0}

    def __init__(self, mesh, k, tau, kappa, scheme="nipg"):
        super().__init__(mesh, k, tau, kappa)
        if scheme not in self.SCHEMES:
            raise ValueError(f"unknown scheme {scheme}")
        self.scheme, self.sf = scheme, self.SCHEMES[scheme]

    def ipdg_blocks(self, t):
        """(L, R, C, H, M) of triangle t."""
        ref, nv, ne, nl = self.ref, self.nv, self.ne, self.nl
        P, Jm, det, Ji = self.geometry(t)
        Phi = ref.values(self.qX)
        gx, gy = ref.grads(self.qX)
        dPhi = [Ji[0, c] * gx + Ji[1, c] * gy for c in range(2)]
        W = self.qW * det
        M = (Phi.T * W) @ Phi
        K = sum((dPhi[c].T * W) @ dPhi[c] for c in range(2))
        N = np.zeros((nv, nv))
        D = np.zeros((nv, nl))
        E = np.zeros((nv, nv))
        G = np.zeros((nv, nl))
        H = np.zeros((nl, nl))
        T = self.mesh.T[t]
        for s in range(3):
            va, vb = int(T[s]), int(T[(s + 1) % 3])
            lo, hi = min(va, vb), max(va, vb)
            A, B = self.mesh.V[lo], self.mesh.V[hi]
            ln = float(np.hypot(*(B - A)))
            dvec = self.mesh.V[vb] - self.mesh.V[va]
            nrm = np.array([dvec[1], -dvec[0]]) / ln
            X = A[None, :] + self.eg[:, None] * (B - A)[None, :]
            Xi = (X - P[0]) @ Ji.T
            Pf = ref.values(Xi)
            fx, fy = ref.grads(Xi)
            dn = sum(nrm[c] * (Ji[0, c] * fx + Ji[1, c] * fy) for c in range(2))   # grad phi_i . n
            wf = self.ew * ln
            cols = slice(s * ne, (s + 1) * ne)
            N += (dn.T * wf) @ Pf
            D[:, cols] = (dn.T * wf) @ self.Mu
            E += (Pf.T * wf) @ Pf
            G[:, cols] = (Pf.T * wf) @ self.Mu
            H[cols, cols] = (self.Mu.T * wf) @ self.Mu
        kap, tau, sf = self.kappa[t], self.tau, self.sf
        L = kap * (K - sf * N - N.T) + tau * E
        R = tau * G - sf * kap * D
        C = tau * G.T - kap * D.T
        return L, R, C, H, M

    def element_dtn(self, t, f_t=None):
        L, R, C, H, M = self.ipdg_blocks(t)
        Ae = self.tau * H - C @ np.linalg.solve(L, R)
        if f_t is None:
            return Ae
        return Ae, C @ np.linalg.solve(L, M @ f_t)

    def reconstruct(self, lam, f_nodal=None, lam_b=None):
        """u (nodal) and q = -kappa grad u at the nodes, [N_T, 2, nv]."""
        nel, nv = self.mesh.nel, self.nv
        f_nodal = np.zeros((nel, nv)) if f_nodal is None else np.asarray(f_nodal, dtype=float)
        lam_b = np.zeros(self.nbdof) if lam_b is None else lam_b
        gx, gy = self.ref.grads(self.ref.nodes)
        u = np.zeros((nel, nv))
        q = np.zeros((nel, 2, nv))
        for t in range(nel):
            LT = np.where(self.gmap[t] >= 0, lam[np.maximum(self.gmap[t], 0)], lam_b[np.maximum(self.bmap[t], 0)])
            L, R, C, H, M = self.ipdg_blocks(t)
            u[t] = np.linalg.solve(L, R @ LT + M @ f_nodal[t])
            _, _, _, Ji = self.geometry(t)
            for c in range(2):
                q[t, c] = -self.kappa[t] * (Ji[0, c] * gx + Ji[1, c] * gy) @ u[t]
        return u, q


# ---------------------------------------------------------------------------
# seed-point agglomeration (Sec. 3.1.2)
def _split2(ids, cen):
    """Halve a set of triangles at the median of their centroids along the
    axis of larger centroid extent (x on ties): the floor(n/2) lowest
    (coordinate, id) first."""
    if len(ids) == 0:
        return []
    c = cen[ids]
    ext = c.max(axis=0) - c.min(axis=0)
    ax = 0 if ext[0] >= ext[1] else 1
    order = np.lexsort((ids, c[:, ax]))
    s = ids[order]
    h = len(s) // 2
    return [np.sort(s[:h]), np.sort(s[h:])]


def agglomerate(mesh, seeds, hlevels):
    """Partitions T_1 .. T_hlevels of the triangles: level 1 assigns every
    triangle to its nearest seed point (centroid distance, lowest seed on
    ties; seeds that win no triangle are dropped), level l + 1 splits every
    macro-element of level l into four (two halvings, ``_split2``; empty
    parts dropped), macro-elements numbered in order of their parent, then
    of their part.  Returns [part_1, ..., part_hlevels] (triangle -> macro
    id) and the macro counts."""
    cen = mesh.centroids()
    seeds = np.asarray(seeds, dtype=float)
    d2 = (cen[:, None, 0] - seeds[None, :, 0]) ** 2 + (cen[:, None, 1] - seeds[None, :, 1]) ** 2
    near = np.argmin(d2, axis=1)
    groups = [np.nonzero(near == s)[0] for s in range(len(seeds))]
    groups = [g for g in groups if len(g)]
    parts = []
    for lev in range(hlevels):
        if lev > 0:
            nxt = []
            for g in groups:
                for half in _split2(g, cen):
                    for q in _split2(half, cen):
                        if len(q):
                            nxt.append(q)
            groups = nxt
        p = -np.ones(mesh.nel, dtype=np.int64)
        for i, g in enumerate(groups):
            p[g] = i
        parts.append(p)
    return parts


class FaceLevel:
    """The faces of one level: per face its two cells, its chain of
    triangle edges (edge index into ``TriMesh.faces``, forward flag), its
    start and end vertex and its length."""

    def __init__(self, cells, chains, ends, lengths):
        self.cells = np.asarray(cells, dtype=np.int64).reshape(-1, 2)
        self.chains, self.ends = chains, np.asarray(ends, dtype=np.int64).reshape(-1, 2)
        self.length = np.asarray(lengths, dtype=float)
        self.nface = len(self.cells)
        self.d = 2


def triangle_faces(mesh):
    """Faces of the triangle levels: the interior edges (start = lower vertex)."""
    cells = mesh.face_cells[:, :, 0]
    chains = [[(f, True)] for f in range(mesh.nface)]
    lengths = [mesh.edge_length(lo, hi) for lo, hi in mesh.faces]
    return FaceLevel(cells, chains, mesh.faces, lengths)


def macro_faces(fine, coarse_of):
    """The interface grid of the coarser partition (cell c of the finer
    level lies in coarse cell coarse_of[c]).

    Faces of the finer level whose two cells share a coarse cell are
    interior (E_I); the others (E_B) are grouped by their pair of coarse
    cells, and each group into chains joined at vertices that exactly two
    of its faces share.  A chain with two distinct end vertices starts at
    the lower one; a closed chain (or one that returns to its branch
    vertex) starts at that vertex (the lowest one of a cycle), leaving
    through the one of its two faces there with the lower id.  Positions
    along a chain are arc lengths, summed face by face from the start.

    Returns (interior face ids, boundary face ids, J [2 n_B, 2 n_coarse]
    (row 2 b + i: DOF i of boundary face b; column 2 E + j: DOF j of
    macro-edge E), coarse FaceLevel)."""
    cc = coarse_of[fine.cells]
    interior = np.nonzero(cc[:, 0] == cc[:, 1])[0]
    bnd = np.nonzero(cc[:, 0] != cc[:, 1])[0]
    groups = {}
    for f in bnd:
        key = (min(cc[f]), max(cc[f]))
        groups.setdefault(key, []).append(int(f))
    edges = []      # (key, min face, ordered [(face, forward)], start, end)
    for key in sorted(groups):
        fl = sorted(groups[key])
        inc = {}
        for f in fl:
            for v in fine.ends[f]:
                inc.setdefault(int(v), []).append(f)
        deg = {v: len(fs) for v, fs in inc.items()}
        seen = set()
        for f0 in fl:
            if f0 in seen:
                continue
            # collect the component through degree-2 vertices
            comp, stack = {f0}, [f0]
            while stack:
                f = stack.pop()
                for v in fine.ends[f]:
                    v = int(v)
                    if deg[v] == 2:
                        for g in inc[v]:
                            if g not in comp:
                                comp.add(g)
                                stack.append(g)
            seen |= comp
            # end vertices: ends of the component's faces at vertices of degree != 2
            ends = []
            for f in sorted(comp):
                for v in fine.ends[f]:
                    if deg[int(v)] != 2:
                        ends.append(int(v))
            if len(ends) == 2 and ends[0] != ends[1]:
                start = min(ends)
            elif len(ends) == 2:
                start = ends[0]
            elif len(ends) == 0:
                start = min(int(v) for f in comp for v in fine.ends[f])
            else:
                raise ValueError("macro-edge chain with a branch inside")
            first = min(g for g in inc[start] if g in comp)
            order, v, f = [], start, first
            used = set()
            while True:
                a, b = int(fine.ends[f][0]), int(fine.ends[f][1])
                fwd = a == v
                order.append((f, fwd))
                used.add(f)
                v = b if fwd else a
                if deg[v] != 2:
                    break
                nxt = [g for g in inc[v] if g not in used]
                if not nxt:
                    break
                f = nxt[0]
            if len(used) != len(comp):
                raise ValueError("macro-edge chain is not a simple path")
            edges.append((key, min(comp), order, start, v))
    edges.sort(key=lambda e: (e[0][0], e[0][1], e[1]))
    Bpos = -np.ones(fine.nface, dtype=np.int64)
    Bpos[bnd] = np.arange(len(bnd))
    rows, cols, vals = [], [], []
    cells, chains, ends, lengths = [], [], [], []
    for E, (key, _, order, start, end) in enumerate(edges):
        L = 0.0
        pos = []
        for f, fwd in order:
            s0 = L
            L = L + fine.length[f]
            pos.append((s0, L) if fwd else (L, s0))
        for (f, fwd), (p0, p1) in zip(order, pos):
            for i, p in enumerate((p0, p1)):
                t = p / L
                for j, wgt in enumerate((1.0 - t, t)):
                    if wgt != 0.0:
                        rows.append(2 * Bpos[f] + i)
                        cols.append(2 * E + j)
                        vals.append(wgt)
        chain = []
        for f, fwd in order:
            sub = fine.chains[f]
            chain.extend(sub if fwd else [(e, not w) for e, w in reversed(sub)])
        cells.append(key)
        chains.append(chain)
        ends.append((start, end))
        lengths.append(L)
    J = sp.coo_matrix((vals, (rows, cols)), shape=(2 * len(bnd), 2 * len(edges))).tocsr()
    return interior, bnd, J, FaceLevel(cells, chains, ends, lengths)


def dofs_of(faces, m):
    faces = np.asarray(faces, dtype=np.int64)
    return (faces[:, None] * m + np.arange(m)[None, :]).ravel()


class UHierarchy(mg.Hierarchy):
    """Levels ordered from finest (index 0) to coarsest: P^k on the
    triangles, P^1 on the triangles (when k > 1), then one level per
    partition T_hlevels, ..., T_1 of ``agglomerate``."""

    def __init__(self, A, mesh, k, parts, sweeps=2, growth=1, omega=1.0, local_corr=mg.LC_PRE,
                 smoother="block_jacobi"):
        if smoother not in mg.SMOOTHERS:
            raise ValueError(f"unknown smoother {smoother}")
        self.coarse, self.omega, self.local_corr = "p1", omega, local_corr
        self.smoother = smoother
        faces = triangle_faces(mesh)
        lev = mg.Level(A, faces, k + 1)
        self.levels = [lev]
        self.face_levels = [faces]
        if k > 1:
            J = mg.p_injection(faces, k)
            lev.kind, lev.I, lev.Q = "p", J, J.T.tocsr()
            lev = mg.Level((J.T @ lev.A @ J).tocsr(), faces, 2)
            self.levels.append(lev)
            self.face_levels.append(faces)
        cell_of = np.arange(mesh.nel)          # finest cells: the triangles
        fine = faces
        for p in reversed(parts):
            coarse_of = np.zeros(cell_of.max() + 1, dtype=np.int64)
            coarse_of[cell_of] = p
            I_f, B_f, J, cf = macro_faces(fine, coarse_of)
            lev = self._h_step(lev, dofs_of(I_f, 2), dofs_of(B_f, 2), J, 2, cf)
            self.levels.append(lev)
            self.face_levels.append(cf)
            fine, cell_of = cf, p
        self._finish(sweeps, growth, smoother)
