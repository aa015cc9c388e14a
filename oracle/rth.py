"""Hybridized Raviart-Thomas mixed method and multinumerics (oracle; test
infrastructure only).

RT-H (Sec. 2, eqs. mixed_local1 and mixed_local2 with the conservation
condition on the normal flux): on every element T, for all v in RT_k(T)
and w in Q^k(T),

    (kappa^-1 q, v)_T - (u, div v)_T + <lambda, v.n>_dT = 0
    (div q, w)_T                                         = (f, w)_T

and sum_T <q.n, mu>_dT = 0 on every interior face.  On the square
elements used here RT_k = Q_{k+1,k} x Q_{k,k+1} (the x component of
degree k+1 in x and k in y, the y component the other way round), the
scalar lives in Q^k and the traces in P^k, so the trace space is the one
of HDG and of the IPDG family (inf-sup stable spaces, no stabilization).

With the velocity coefficients Q and the scalar U the local system reads

    [ Mq  -B ] [Q]   [-F Lambda]      Mq_ij = (kappa^-1 v_j, v_i),
    [ B^T  0 ] [U] = [  M f    ],     B_ij  = (w_j, div v_i),
                                      F_il  = <mu_l, v_i . n>,

the conservation rows are F^T Q, and eliminating (Q, U) gives the element
map of the trace system (eq. trace_linear_system)

    A^e = -S^T L^-1 R,  b^e = S^T L^-1 [0; M f],  R = [-F; 0], S = [F; 0],

a symmetric positive semidefinite map (the HDG form with tau = 0).

Multinumerics (Sec. 4.6): every element carries its own method; the
trace system is assembled from the element maps of each, and the
multigrid of Sec. 3 runs on it unchanged.

Velocity basis: nodal, tensor GLL points of degree k+1 along the
component's own direction and k across it (x fastest); velocity
coefficients ordered [x component, y component].  2D only.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .hdg import HDG, lex
from .ipdg import IPDG
from .refelem import gll_nodes, gauss_rule, lagrange, lagrange_deriv


class RTH(HDG):
    """Element matrices, condensed trace system and recovery of RT_k-H on
    the square elements of ``oracle.hdg`` (d = 2)."""

    def __init__(self, n, k, kappa):
        super().__init__(2, n, k, 0.0, kappa)
        d, h = 2, self.mesh.h
        xi_hi, xi_lo = gll_nodes(k + 1), gll_nodes(k)
        gq, gw = gauss_rule(k + 2)
        Qidx = lex((k + 2,) * d)
        fQ = lex((k + 2,) * (d - 1))
        self.nqc = (k + 2) * (k + 1)        # coefficients per velocity component
        self.nqv = d * self.nqc
        # per component c: index tuples (a_0, a_1), with degree k+1 along c
        self.comp_idx = []
        for c in range(d):
            shape = tuple(k + 2 if t == c else k + 1 for t in range(d))
            self.comp_idx.append(lex(shape))
        self.node_sets = [[xi_hi if t == c else xi_lo for t in range(d)] for c in range(d)]

        def comp_values(c, pts_per_dir, deriv_dir=None):
            """[npts, nqc] values (or the derivative along deriv_dir) of the
            basis of component c at a tensor set of points (x fastest)."""
            idx = self.comp_idx[c]
            tabs = []
            for t in range(d):
                nodes = self.node_sets[c][t]
                tab = lagrange_deriv(nodes, pts_per_dir[t]) / h if deriv_dir == t else lagrange(nodes, pts_per_dir[t])
                tabs.append(tab)
            P = lex(tuple(len(p) for p in pts_per_dir))
            V = np.ones((len(P), len(idx)))
            for t in range(d):
                V *= tabs[t][idx[:, t]][:, P[:, t]].T
            return V

        W = self.W
        # velocity mass without kappa (per component, at the volume Gauss points)
        self.Vq = [comp_values(c, [gq] * d) for c in range(d)]
        self.Dq = [comp_values(c, [gq] * d, deriv_dir=c) for c in range(d)]
        B = np.zeros((self.nqv, self.nv))
        for c in range(d):
            B[c * self.nqc:(c + 1) * self.nqc] = (self.Dq[c].T * W) @ self.Phi
        self.Bd = B
        # normal traces on each face slot: F_il = <mu_l, v_i . n>
        ne = self.ne
        F = np.zeros((self.nqv, self.nl))
        for s in range(self.nf):
            c, side = divmod(s, 2)
            nrm = 1.0 if side == 1 else -1.0
            pts = [gq if t != c else np.array([float(side)]) for t in range(d)]
            Vf = comp_values(c, pts)                    # [nfq, nqc], face points lexicographic
            F[c * self.nqc:(c + 1) * self.nqc, s * ne:(s + 1) * ne] = nrm * (Vf.T * self.Wf) @ self.Mu
        self.Fr = F
        self.Rr = np.vstack([-F, np.zeros((self.nv, self.nl))])
        self.Sr = np.vstack([F, np.zeros((self.nv, self.nl))])
        # velocity basis at the scalar's nodes, for the flux output
        xi = self.xi
        self.Vnode = [comp_values(c, [xi] * d) for c in range(d)]

    def local_matrix(self, T):
        """L_T = [[Mq, -B], [B^T, 0]] of element T."""
        nqc, nqv, nv = self.nqc, self.nqv, self.nv
        wk = self.W / self.kappa_qp[T]
        L = np.zeros((nqv + nv, nqv + nv))
        for c in range(2):
            L[c * nqc:(c + 1) * nqc, c * nqc:(c + 1) * nqc] = (self.Vq[c].T * wk) @ self.Vq[c]
        L[:nqv, nqv:] = -self.Bd
        L[nqv:, :nqv] = self.Bd.T
        return L

    def element_dtn(self, T, b=None):
        """A^e = -S^T L^-1 R and b^e = S^T L^-1 [0; b]."""
        L = self.local_matrix(T)
        Ae = -self.Sr.T @ np.linalg.solve(L, self.Rr)
        if b is None:
            return Ae
        rhs = np.zeros(L.shape[0])
        rhs[self.nqv:] = b
        return Ae, self.Sr.T @ np.linalg.solve(L, rhs)

    def recover_element(self, T, lam_T, f_T=None):
        """(Q, U) = L^-1 (R Lambda + [0; M f]); returns u = U and the flux
        at the scalar's nodes, q_c(x_a) = sum_i Q_i v_{c,i}(x_a)."""
        rhs = self.Rr @ np.asarray(lam_T, dtype=float)
        if f_T is not None:
            rhs[self.nqv:] += self.M @ np.asarray(f_T)
        w = np.linalg.solve(self.local_matrix(T), rhs)
        Q = w[:self.nqv]
        q = np.stack([self.Vnode[c] @ Q[c * self.nqc:(c + 1) * self.nqc] for c in range(2)])
        return w[self.nqv:], q

    def local_system(self, T):
        """(L, R, conservation rows, tau_T H, first load row, flux map) of the
        uncondensed system; the flux map takes local unknowns to nodal flux."""
        nqc = self.nqc
        Fmap = np.zeros((2 * self.nv, self.nqv + self.nv))
        for c in range(2):
            Fmap[c * self.nv:(c + 1) * self.nv, c * nqc:(c + 1) * nqc] = self.Vnode[c]
        return self.local_matrix(T), self.Rr, self.Sr.T, 0.0 * self.H, self.nqv, Fmap

    def monolithic_solve(self, f_nodal=None, gD=None):
        return uncondensed_solve(self, f_nodal, gD)


def _ipdg_local_system(P, T):
    L, R, C = P.blocks(T)
    Fmap = np.vstack([-float(P.kappa_el[T]) * Dc for Dc in P.Dnode])
    return L, R, C, P.tau_of(T) * P.H, 0, Fmap


class Multinumerics(HDG):
    """RT_k-H on the elements with ``use_rt[T]`` true and an IPDG scheme on
    the others, one trace system (Sec. 4.6).  kappa per element; the IPDG
    elements are stabilized with tau (times kappa_T if ``tau_kappa``)."""

    def __init__(self, n, k, tau, kappa, use_rt, scheme="nipg", tau_kappa=True):
        kappa = np.asarray(kappa, dtype=float)
        super().__init__(2, n, k, tau, kappa, tau_kappa)
        self.use_rt = np.asarray(use_rt, dtype=bool)
        if self.use_rt.shape != (n * n,):
            raise ValueError("use_rt: one flag per element")
        self.rt = RTH(n, k, kappa)
        self.dg = IPDG(2, n, k, tau, kappa, scheme, tau_kappa=tau_kappa)

    def _m(self, T):
        return self.rt if self.use_rt[T] else self.dg

    def element_dtn(self, T, b=None):
        return self._m(T).element_dtn(T, b)

    def recover_element(self, T, lam_T, f_T=None):
        return self._m(T).recover_element(T, lam_T, f_T)

    def local_system(self, T):
        return self.rt.local_system(T) if self.use_rt[T] else _ipdg_local_system(self.dg, T)

    def monolithic_solve(self, f_nodal=None, gD=None):
        return uncondensed_solve(self, f_nodal, gD)


def uncondensed_solve(P, f_nodal=None, gD=None):
    """Solve every element's local equations and the conservation rows of
    every interior face for (local unknowns, lambda) at once with a sparse
    direct solver, for any mix of element methods (each provides
    ``local_system(T)``).  Returns (lambda, u, q), q the flux at the nodes."""
    m, nv = P.mesh, P.nv
    nel = m.nel
    f_nodal = np.zeros((nel, nv)) if f_nodal is None else np.asarray(f_nodal)
    lam_b = np.zeros(P.nbdof) if gD is None else np.asarray(gD(P.boundary_nodes()), dtype=float)
    systems = [P.local_system(T) for T in range(nel)]
    sizes = np.array([s[0].shape[0] for s in systems])
    off = np.concatenate([[0], np.cumsum(sizes)])
    nw = int(off[-1])
    Nt = nw + P.nlam
    rows, cols, vals = [], [], []
    rhs = np.zeros(Nt)

    def put(r, c, blk):
        rr, cc = np.meshgrid(r, c, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(np.asarray(blk).ravel())

    for T, (L, R, Cons, tH, r0, _) in enumerate(systems):
        wr = off[T] + np.arange(sizes[T])
        gi, bi = P.gmap[T], P.bmap[T]
        ii = np.nonzero(gi >= 0)[0]
        jb = np.nonzero(bi >= 0)[0]
        put(wr, wr, L)
        put(wr, nw + gi[ii], -R[:, ii])
        rhs[wr[r0:]] += P.M @ f_nodal[T]
        rhs[wr] += R[:, jb] @ lam_b[bi[jb]]
        lr = nw + gi[ii]
        put(lr, wr, Cons[ii, :])
        put(lr, nw + gi[ii], -tH[np.ix_(ii, ii)])
        rhs[lr] += tH[np.ix_(ii, jb)] @ lam_b[bi[jb]]
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(Nt, Nt)).tocsc()
    sol = spla.spsolve(K, rhs)
    lam = sol[nw:]
    u = np.zeros((nel, nv))
    q = np.zeros((nel, 2, nv))
    for T, (L, R, Cons, tH, r0, Fmap) in enumerate(systems):
        w = sol[off[T]:off[T + 1]]
        u[T] = w[r0:r0 + nv] if r0 > 0 else w[:nv]
        q[T] = (Fmap @ w).reshape(2, nv)
    return lam, u, q
