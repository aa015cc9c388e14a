"""HDG discretization and static condensation (oracle; test infrastructure only).

Model problem (Sec. 2, eqs. primal_elliptic and mixed_elliptic), written
with the scalar unknown ``u`` and the flux ``q = -kappa grad u`` (the paper
names them the other way round).  On every element T the HDG local
problem (eq. HDG) with numerical flux (eq. HDG_flux)

    (kappa^-1 q, v)_T - (u, div v)_T + <lambda, v.n>_dT        = 0
    -(q, grad w)_T + <qhat.n, w>_dT                           = (f, w)_T
    qhat.n = q.n + tau (u - lambda)

is solved for (q, u) given the trace lambda; the conservation condition
(eq. conservation) over interior faces then gives the trace system
A lambda = g (eq. trace_linear_system), and (q, u) is recovered element
by element (Sec. 2, last paragraph).

Discretization contract (readings of points the paper leaves open):
  * quads/hexes of the unit box, n per direction, h = 1/n;
  * Q^k on elements, nodal at tensor GLL points (x fastest);
  * Q^k on faces (P^k in 2D), nodal at GLL points ordered by increasing
    global coordinate, first tangential direction fastest;
  * element-local face slots x-, x+, y-, y+, (z-, z+);
  * tensor Gauss rules with k+2 points per direction on elements and
    faces; k+4 points for error norms;
  * source given by its nodal values (load M f); Dirichlet data imposed
    strongly through the boundary traces (Sec. 4.1, Example I).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .refelem import gll_nodes, gauss_rule, lagrange, lagrange_deriv


def lex(shape):
    """All multi-indices of ``shape`` as rows, first index fastest."""
    grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    return np.stack([g.ravel(order="F") for g in grids], axis=1)


class Mesh:
    """Structured mesh of [0,1]^d with n^d equal elements and its skeleton.

    Elements: index sum_c e_c n^c.  Interior faces of normal direction c
    sit at positions p = 1..n-1 along c; within a direction they are
    numbered lexicographically on the grid with extent n-1 along c and n
    elsewhere (x fastest), and the directions follow one another.
    Boundary faces: block (c, side) holds the n^(d-1) faces at x_c = side,
    numbered over the tangential coordinates, first fastest.
    """

    def __init__(self, d, n):
        if d not in (2, 3) or n < 1:
            raise ValueError("need d in {2,3}, n >= 1")
        self.d, self.n, self.h = d, n, 1.0 / n
        self.nel = n ** d
        self.elem_coords = lex((n,) * d)
        self.nface_dir = [(n - 1) * n ** (d - 1) for _ in range(d)]
        self.face_off = np.concatenate([[0], np.cumsum(self.nface_dir)]).astype(int)
        self.nface = int(self.face_off[-1])
        self.nbface = 2 * d * n ** (d - 1)

    def tangential(self, c):
        return [t for t in range(self.d) if t != c]

    def interior_face_id(self, c, coords):
        """coords: face grid coordinates, coords[c] = p in 1..n-1."""
        n, idx, stride = self.n, 0, 1
        for dim in range(self.d):
            if dim == c:
                idx += (coords[dim] - 1) * stride
                stride *= n - 1
            else:
                idx += coords[dim] * stride
                stride *= n
        return int(self.face_off[c] + idx)

    def interior_face_coords(self, fid):
        c = int(np.searchsorted(self.face_off, fid, side="right") - 1)
        r = fid - self.face_off[c]
        coords = []
        for dim in range(self.d):
            ext = self.n - 1 if dim == c else self.n
            coords.append(r % ext + (1 if dim == c else 0))
            r //= ext
        return c, coords

    def boundary_face_id(self, c, side, coords):
        n, idx, stride = self.n, 0, 1
        for t in self.tangential(c):
            idx += coords[t] * stride
            stride *= n
        return int((2 * c + side) * n ** (self.d - 1) + idx)

    def slot_face(self, T, s):
        """Face in local slot s = 2c+side of element T: ('i'|'b', id, coords)."""
        c, side = divmod(s, 2)
        coords = list(self.elem_coords[T])
        p = coords[c] + side
        coords[c] = p
        if p == 0 or p == self.n:
            return "b", self.boundary_face_id(c, 1 if p == self.n else 0, coords), coords
        return "i", self.interior_face_id(c, coords), coords


class HDG:
    """Element matrices, condensed trace system and local recovery.

    ``kappa`` is either one value per element (shape [N_T]) or values at
    the volume Gauss points (shape [N_T, (k+2)^d], points lexicographic
    with x fastest).  Complex kappa is accepted (complex-step checks).
    ``tau_kappa``: the stabilization of element T is tau * kappa_T (the
    paper's tau = kappa / h_min of Example IV, Sec. 4.4); needs one kappa
    per element.
    """

    def __init__(self, d, n, k, tau, kappa, tau_kappa=False):
        self.mesh = Mesh(d, n)
        self.d, self.n, self.k, self.tau = d, n, k, tau
        self.tau_kappa = tau_kappa
        h = self.mesh.h
        self.nv = (k + 1) ** d
        self.ne = (k + 1) ** (d - 1)
        self.nf = 2 * d
        self.nl = self.nf * self.ne
        self.nlam = self.mesh.nface * self.ne

        xi = gll_nodes(k)
        gq, gw = gauss_rule(k + 2)
        self.xi = xi
        l1 = lagrange(xi, gq)
        dl1 = lagrange_deriv(xi, gq)
        Iidx = lex((k + 1,) * d)
        Qidx = lex((k + 2,) * d)
        self.nq = len(Qidx)
        # volume basis and gradients at the Gauss points, Gauss weights
        Phi = np.ones((self.nq, self.nv))
        for dim in range(d):
            Phi *= l1[Iidx[:, dim]][:, Qidx[:, dim]].T
        dPhi = []
        for c in range(d):
            D = np.ones((self.nq, self.nv))
            for dim in range(d):
                tab = dl1 if dim == c else l1
                D *= tab[Iidx[:, dim]][:, Qidx[:, dim]].T
            dPhi.append(D / h)
        W = np.prod(gw[Qidx], axis=1) * h ** d
        self.Phi, self.dPhi, self.W = Phi, dPhi, W
        self.qpoints_ref = gq[Qidx]

        # face quadrature: for slot s, tangential Gauss points, weights
        fIdx = lex((k + 1,) * (d - 1))
        fQ = lex((k + 2,) * (d - 1))
        Wf = np.prod(gw[fQ], axis=1) * h ** (d - 1) if d > 1 else np.ones(1)
        Mu = np.ones((len(fQ), self.ne))
        for j in range(d - 1):
            Mu *= l1[fIdx[:, j]][:, fQ[:, j]].T
        Phif = []
        for s in range(self.nf):
            c, side = divmod(s, 2)
            end = lagrange(xi, [float(side)])[:, 0]
            P = np.ones((len(fQ), self.nv)) * end[Iidx[:, c]][None, :]
            for j, t in enumerate([t for t in range(d) if t != c]):
                P *= l1[Iidx[:, t]][:, fQ[:, j]].T
            Phif.append(P)
        self.Wf, self.Mu, self.Phif = Wf, Mu, Phif

        nv, ne, nl = self.nv, self.ne, self.nl
        # (q, div v) and <lambda, v.n> blocks of the first local equation
        Bdiv = np.zeros((d * nv, nv))
        F = np.zeros((d * nv, nl))
        for c in range(d):
            Bdiv[c * nv:(c + 1) * nv] = -(dPhi[c].T * W) @ Phi
        for s in range(self.nf):
            c, side = divmod(s, 2)
            nrm = 1.0 if side == 1 else -1.0
            F[c * nv:(c + 1) * nv, s * ne:(s + 1) * ne] = nrm * (Phif[s].T * Wf) @ Mu
        # -(q, grad w) + <q.n, w>, tau <u, w>, <lambda, w> and face mass
        C = np.zeros((nv, d * nv))
        for c in range(d):
            blk = -(dPhi[c].T * W) @ Phi
            for side in (0, 1):
                s = 2 * c + side
                nrm = 1.0 if side == 1 else -1.0
                blk = blk + nrm * (Phif[s].T * Wf) @ Phif[s]
            C[:, c * nv:(c + 1) * nv] = blk
        E = np.zeros((nv, nv))
        G = np.zeros((nv, nl))
        H = np.zeros((nl, nl))
        for s in range(self.nf):
            E += (Phif[s].T * Wf) @ Phif[s]
            G[:, s * ne:(s + 1) * ne] = (Phif[s].T * Wf) @ Mu
            H[s * ne:(s + 1) * ne, s * ne:(s + 1) * ne] = (Mu.T * Wf) @ Mu
        self.Bdiv, self.F, self.C, self.E, self.G, self.H = Bdiv, F, C, E, G, H
        self.M = (Phi.T * W) @ Phi
        self.R = np.vstack([-F, tau * G])
        self.S = np.vstack([F, tau * G])

        self.set_kappa(kappa)
        self._build_maps()

    # ------------------------------------------------------------------
    def set_kappa(self, kappa):
        kappa = np.asarray(kappa)
        if self.tau_kappa and kappa.ndim != 1:
            raise ValueError("tau proportional to kappa needs one kappa per element")
        self.kappa_el = kappa if kappa.ndim == 1 else None
        if kappa.ndim == 1:
            kappa = np.repeat(kappa[:, None], self.nq, axis=1)
        if kappa.shape != (self.mesh.nel, self.nq):
            raise ValueError("kappa has the wrong shape")
        self.kappa_qp = kappa
        self.dtype = np.result_type(kappa.dtype, np.float64)

    def tau_of(self, T):
        """The stabilization of element T: tau, or tau * kappa_T."""
        return self.tau * self.kappa_el[T] if self.tau_kappa else self.tau

    def R_of(self, T):
        """R_T = [-F; tau_T G] (right-hand side of the local problem)."""
        return self.R if not self.tau_kappa else np.vstack([-self.F, self.tau_of(T) * self.G])

    def S_of(self, T):
        """S_T = [F; tau_T G] (the flux terms of the conservation rows)."""
        return self.S if not self.tau_kappa else np.vstack([self.F, self.tau_of(T) * self.G])

    def local_matrix(self, T):
        """L_T = [[A_T, Bdiv], [C, tau E]] for element T (first local eq. on
        top, second below; unknowns ordered [q_x, q_y, (q_z), u])."""
        d, nv = self.d, self.nv
        Mk = (self.Phi.T * (self.W / self.kappa_qp[T])) @ self.Phi
        L = np.zeros(((d + 1) * nv, (d + 1) * nv), dtype=self.dtype)
        for c in range(d):
            L[c * nv:(c + 1) * nv, c * nv:(c + 1) * nv] = Mk
        L[:d * nv, d * nv:] = self.Bdiv
        L[d * nv:, :d * nv] = self.C
        L[d * nv:, d * nv:] = self.tau_of(T) * self.E
        return L

    def element_dtn(self, T, b=None):
        """Element DtN matrix and load: A^e = tau H - S^T L^-1 R and
        b^e = S^T L^-1 [0; b] (static condensation, Sec. 2)."""
        L = self.local_matrix(T)
        S = self.S_of(T)
        Ae = self.tau_of(T) * self.H - S.T @ np.linalg.solve(L, self.R_of(T))
        if b is None:
            return Ae
        rhs = np.zeros(L.shape[0], dtype=np.result_type(self.dtype, b.dtype))
        rhs[self.d * self.nv:] = b
        return Ae, S.T @ np.linalg.solve(L, rhs)

    def all_element_dtn(self):
        """A^e for every element, shape [N_T, n_f n_e, n_f n_e]."""
        out = np.zeros((self.mesh.nel, self.nl, self.nl), dtype=self.dtype)
        for T in range(self.mesh.nel):
            out[T] = self.element_dtn(T)
        return out

    # ------------------------------------------------------------------
    def _build_maps(self):
        m, ne = self.mesh, self.ne
        gmap = -np.ones((m.nel, self.nl), dtype=np.int64)
        bmap = -np.ones((m.nel, self.nl), dtype=np.int64)
        for T in range(m.nel):
            for s in range(self.nf):
                kind, fid, _ = m.slot_face(T, s)
                rng = np.arange(ne)
                if kind == "i":
                    gmap[T, s * ne:(s + 1) * ne] = fid * ne + rng
                else:
                    bmap[T, s * ne:(s + 1) * ne] = fid * ne + rng
        self.gmap, self.bmap = gmap, bmap
        self.nbdof = m.nbface * ne

    def volume_nodes(self):
        """Coordinates of the volume GLL nodes, shape [N_T, N_v, d]."""
        m, d = self.mesh, self.d
        Iidx = lex((self.k + 1,) * d)
        ref = self.xi[Iidx]
        return (m.elem_coords[:, None, :] + ref[None, :, :]) * m.h

    def volume_qpoints(self):
        """Coordinates of the volume Gauss points, shape [N_T, (k+2)^d, d]."""
        m = self.mesh
        return (m.elem_coords[:, None, :] + self.qpoints_ref[None]) * m.h

    def boundary_nodes(self):
        """Coordinates of the boundary-face GLL nodes, [N_bdof, d]."""
        m, d, ne = self.mesh, self.d, self.ne
        fIdx = lex((self.k + 1,) * (d - 1))
        X = np.zeros((self.nbdof, d))
        for c in range(d):
            tang = m.tangential(c)
            for side in (0, 1):
                for tc in lex((m.n,) * (d - 1)):
                    coords = [0] * d
                    for j, t in enumerate(tang):
                        coords[t] = tc[j]
                    bid = m.boundary_face_id(c, side, coords)
                    for a, ai in enumerate(fIdx):
                        x = np.zeros(d)
                        x[c] = side
                        for j, t in enumerate(tang):
                            x[t] = (tc[j] + self.xi[ai[j]]) * m.h
                        X[bid * ne + a] = x
        return X

    def interior_trace_nodes(self):
        """Coordinates of the interior trace GLL nodes, [N_lambda, d]."""
        m, d, ne = self.mesh, self.d, self.ne
        fIdx = lex((self.k + 1,) * (d - 1))
        X = np.zeros((self.nlam, d))
        for fid in range(m.nface):
            c, coords = m.interior_face_coords(fid)
            tang = m.tangential(c)
            for a, ai in enumerate(fIdx):
                x = np.zeros(d)
                x[c] = coords[c] * m.h
                for j, t in enumerate(tang):
                    x[t] = (coords[t] + self.xi[ai[j]]) * m.h
                X[fid * ne + a] = x
        return X

    # ------------------------------------------------------------------
    def assemble(self, f_nodal=None, gD=None):
        """Trace system of eq. trace_linear_system.

        Returns (A, g, lam_bnd): A = sum_T P_T^T A^e P_T over interior
        trace DOFs (CSR); g = sum_T P_T^T b^e - A_{I,bnd} lam_bnd, where
        lam_bnd are the Dirichlet boundary traces (nodal interpolant of
        gD; zero if gD is None) and b_T = M f_T.
        """
        m, nl = self.mesh, self.nl
        nel = m.nel
        f_nodal = np.zeros((nel, self.nv)) if f_nodal is None else np.asarray(f_nodal)
        lam_b = np.zeros(self.nbdof) if gD is None else np.asarray(gD(self.boundary_nodes()), dtype=float)
        dt = np.result_type(self.dtype, f_nodal.dtype)
        rows, cols, vals = [], [], []
        g = np.zeros(self.nlam, dtype=dt)
        self.Ae = np.zeros((nel, nl, nl), dtype=dt)
        for T in range(nel):
            b = self.M @ f_nodal[T]
            Ae, be = self.element_dtn(T, b)
            self.Ae[T] = Ae
            gi = self.gmap[T]
            bi = self.bmap[T]
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

    def local_traces(self, lam, lam_b):
        """Lambda_T for all elements, [N_T, n_f n_e] (boundary values included)."""
        out = np.zeros((self.mesh.nel, self.nl), dtype=np.result_type(lam.dtype, lam_b.dtype))
        mi = self.gmap >= 0
        out[mi] = lam[self.gmap[mi]]
        mb = self.bmap >= 0
        out[mb] = lam_b[self.bmap[mb]]
        return out

    def reconstruct(self, lam, f_nodal=None, lam_b=None):
        """Local recovery w_T = L_T^-1 (R_T Lambda_T + [0; b_T]) (Sec. 2).

        Returns u [N_T, N_v] and q [N_T, d, N_v].
        """
        nel, d, nv = self.mesh.nel, self.d, self.nv
        f_nodal = np.zeros((nel, nv)) if f_nodal is None else np.asarray(f_nodal)
        lam_b = np.zeros(self.nbdof) if lam_b is None else lam_b
        LT = self.local_traces(np.asarray(lam), lam_b)
        dt = np.result_type(self.dtype, LT.dtype, f_nodal.dtype)
        u = np.zeros((nel, nv), dtype=dt)
        q = np.zeros((nel, d, nv), dtype=dt)
        for T in range(nel):
            u[T], q[T] = self.recover_element(T, LT[T], f_nodal[T])
        return u, q

    def recover_element(self, T, lam_T, f_T=None):
        """w_T = L_T^-1 (R_T Lambda_T + [0; M f_T]) for one element (Sec. 2):
        (u_T [N_v], q_T [d, N_v]) from its local traces Lambda_T [n_f n_e]."""
        d, nv = self.d, self.nv
        lam_T = np.asarray(lam_T)
        rhs = (self.R_of(T) @ lam_T).astype(np.result_type(self.dtype, lam_T.dtype))
        if f_T is not None:
            rhs = rhs.astype(np.result_type(rhs.dtype, np.asarray(f_T).dtype))
            rhs[d * nv:] += self.M @ f_T
        w = np.linalg.solve(self.local_matrix(T), rhs)
        return w[d * nv:], w[:d * nv].reshape(d, nv)

    # -- rows of the assembled system, one face at a time ------------------
    # (for sampled checks on meshes too large to assemble)
    def face_elements(self, fid):
        """The two elements that share interior face fid, each with the local
        slot the face occupies in it: [(T_below, 2c+1), (T_above, 2c)]."""
        c, coords = self.mesh.interior_face_coords(fid)
        out = []
        for side in (0, 1):
            e = list(coords)
            e[c] = coords[c] - 1 + side
            T = int(sum(e[a] * self.n ** a for a in range(self.d)))
            out.append((T, 2 * c + 1 - side))
        return out

    def _dtn_cached(self, T, cache):
        if cache is None:
            return self.element_dtn(T)
        if T not in cache:
            cache[T] = self.element_dtn(T)
        return cache[T]

    def apply_rows(self, fids, x, cache=None):
        """(A x) restricted to interior faces fids, [len(fids), n_e]:
        sum over the two elements T of face F of A^e_T[slot rows, :] x_T
        (x_T gathered with zero boundary traces), eq. trace_linear_system."""
        ne = self.ne
        x = np.asarray(x)
        out = np.zeros((len(fids), ne), dtype=np.result_type(self.dtype, x.dtype))
        for i, F in enumerate(fids):
            for T, s in self.face_elements(F):
                Ae = self._dtn_cached(T, cache)
                gi = self.gmap[T]
                xT = np.where(gi >= 0, x[np.maximum(gi, 0)], 0.0)
                out[i] += Ae[s * ne:(s + 1) * ne] @ xT
        return out

    def load_rows(self, fids, f_nodal):
        """g restricted to interior faces fids (zero Dirichlet data):
        sum over the two elements of face F of b^e_T[slot rows], b_T = M f_T."""
        ne = self.ne
        out = np.zeros((len(fids), ne))
        for i, F in enumerate(fids):
            for T, s in self.face_elements(F):
                _, be = self.element_dtn(T, self.M @ np.asarray(f_nodal[T]))
                out[i] += be[s * ne:(s + 1) * ne]
        return out

    def diag_block(self, fid, cache=None):
        """Assembled diagonal block of face fid: A^e_{T-}[s,s] + A^e_{T+}[s,s]."""
        ne = self.ne
        D = np.zeros((ne, ne), dtype=self.dtype)
        for T, s in self.face_elements(fid):
            Ae = self._dtn_cached(T, cache)
            D += Ae[s * ne:(s + 1) * ne, s * ne:(s + 1) * ne]
        return D

    def monolithic_solve(self, f_nodal=None, gD=None):
        """Solve the uncondensed HDG system (eqs. HDG, HDG_flux and
        conservation) for (q, u, lambda) at once with a sparse direct solver."""
        m, d, nv, nl = self.mesh, self.d, self.nv, self.nl
        nel = m.nel
        nw = (d + 1) * nv
        f_nodal = np.zeros((nel, nv)) if f_nodal is None else np.asarray(f_nodal)
        lam_b = np.zeros(self.nbdof) if gD is None else np.asarray(gD(self.boundary_nodes()), dtype=float)
        N = nel * nw + self.nlam
        rows, cols, vals = [], [], []
        rhs = np.zeros(N)

        def put(r, c, blk):
            rr, cc = np.meshgrid(r, c, indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(np.asarray(blk).ravel())

        for T in range(nel):
            L = self.local_matrix(T)
            wr = T * nw + np.arange(nw)
            gi, bi = self.gmap[T], self.bmap[T]
            ii = np.nonzero(gi >= 0)[0]
            jb = np.nonzero(bi >= 0)[0]
            # local equations: L w - R Lambda = [0; b]
            put(wr, wr, L)
            R, S, tT = self.R_of(T), self.S_of(T), self.tau_of(T)
            put(wr, nel * nw + gi[ii], -R[:, ii])
            rhs[wr[d * nv:]] += self.M @ f_nodal[T]
            rhs[wr] += R[:, jb] @ lam_b[bi[jb]]
            # conservation rows: sum_T (S^T w - tau H Lambda) = 0
            lr = nel * nw + gi[ii]
            put(lr, wr, S.T[ii, :])
            put(lr, nel * nw + gi[ii], -tT * self.H[np.ix_(ii, ii)])
            rhs[lr] += tT * self.H[np.ix_(ii, jb)] @ lam_b[bi[jb]]
        K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(N, N)).tocsc()
        sol = spla.spsolve(K, rhs)
        w = sol[:nel * nw].reshape(nel, nw)
        lam = sol[nel * nw:]
        q = w[:, :d * nv].reshape(nel, d, nv)
        u = w[:, d * nv:]
        return lam, u, q

    def errors(self, u, q, u_exact, grad_exact, kappa_fn=None):
        """L2 errors of u and q = -kappa grad u with a (k+4)-point Gauss rule."""
        d, k, m = self.d, self.k, self.mesh
        gq, gw = gauss_rule(k + 4)
        Iidx = lex((k + 1,) * d)
        Qidx = lex((k + 4,) * d)
        l1 = lagrange(self.xi, gq)
        P = np.ones((len(Qidx), self.nv))
        for dim in range(d):
            P *= l1[Iidx[:, dim]][:, Qidx[:, dim]].T
        W = np.prod(gw[Qidx], axis=1) * m.h ** d
        X = (m.elem_coords[:, None, :] + gq[Qidx][None]) * m.h
        Xf = X.reshape(-1, d)
        ue = u_exact(Xf).reshape(m.nel, -1)
        ge = grad_exact(Xf).reshape(m.nel, -1, d)
        kap = np.ones(Xf.shape[0]) if kappa_fn is None else kappa_fn(Xf)
        qe = -kap.reshape(m.nel, -1, 1) * ge
        uh = u @ P.T
        eu = np.sqrt(np.sum(W[None] * (uh - ue) ** 2))
        eq = 0.0
        for c in range(d):
            qh = q[:, c, :] @ P.T
            eq += np.sum(W[None] * (qh - qe[:, :, c]) ** 2)
        return eu, np.sqrt(eq)
