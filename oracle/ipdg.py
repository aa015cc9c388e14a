"""Hybridized interior penalty DG schemes (oracle; test infrastructure only).

The primal hybridized IPDG family of Sec. 2 (eqs. IPDG_flux_form,
IPDG_flux, SIPG_H and IPG_H): on every element T, for all w in Q^k(T),

    (kappa grad u, grad w)_T - s_f <u - lambda, kappa grad w . n>_dT
        - <kappa grad u . n, w>_dT + <tau (u - lambda), w>_dT = (f, w)_T

with the numerical flux qhat.n = -kappa grad u . n + tau (u - lambda)
(eq. IPDG_flux), made single valued by the conservation condition
sum_T <qhat.n, mu>_dT = 0 on every interior face (eq. conservation).
s_f = 1 is SIPG-H, s_f = 0 IIPG-H, s_f = -1 NIPG-H.

Written with rows for the test function w = phi_i and columns for the
trial function, per element (kappa constant on the element):

    L_T = kappa (K - s_f N - N^T) + tau E,   K_ij = (grad phi_j, grad phi_i)_T,
                                             N_ij = <phi_j, grad phi_i . n>_dT,
    R_T = tau G - s_f kappa D,               D_il = <mu_l, grad phi_i . n>_dT,
    C_T = tau G^T - kappa D^T,               (conservation rows)

with E, G, H the boundary mass matrices of the HDG element.  The local
problem reads L_T u = R_T Lambda_T + M f_T, the conservation rows
C_T u - tau H Lambda_T, and eliminating u gives the element map of the
trace system (eq. trace_linear_system)

    A^e = tau H - C_T L_T^-1 R_T,    b^e = C_T L_T^-1 M f_T.

For s_f = 1, C_T = R_T^T and L_T is symmetric, so A^e is symmetric; for
s_f = 0, -1 it is not, and the trace system is solved by GMRES (Sec. 4).
The flux is recovered as q = -kappa grad u_h; with Q^k elements every
component of grad u_h lies in Q^k, so its nodal values represent it exactly.

Discretization contract: the HDG element of ``oracle.hdg`` (meshes, node
sets, face numbering, quadrature, strong Dirichlet data); kappa is one value
per element (the face terms take the element's own value); with
``tau_kappa`` the stabilization of element T is tau * kappa_T (the paper's
tau = kappa (p+1)(p+2)/h_min of Examples III and IV).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .hdg import HDG, lex
from .refelem import gll_nodes, gauss_rule, lagrange, lagrange_deriv

SCHEMES = {"sipg": 1.0, "iipg": 0.0, "nipg": -1.0}


class IPDG(HDG):
    """Element matrices, condensed trace system and recovery of SIPG-H,
    IIPG-H and NIPG-H (eq. IPG_H with s_f = 1, 0, -1)."""

    def __init__(self, d, n, k, tau, kappa, scheme="nipg", tau_kappa=False):
        if scheme not in SCHEMES:
            raise ValueError(f"unknown scheme {scheme}")
        kappa = np.asarray(kappa)
        if kappa.shape != (n ** d,):
            raise ValueError("IPDG takes one kappa per element")
        self.scheme, self.sf = scheme, SCHEMES[scheme]
        super().__init__(d, n, k, tau, kappa, tau_kappa)
        h = self.mesh.h
        nv, ne, nl = self.nv, self.ne, self.nl
        xi = self.xi
        gq, _ = gauss_rule(k + 2)
        l1 = lagrange(xi, gq)
        Iidx = lex((k + 1,) * d)
        fQ = lex((k + 2,) * (d - 1))
        # K: stiffness matrix
        self.K = sum((self.dPhi[c].T * self.W) @ self.dPhi[c] for c in range(d))
        # outward normal derivative of every volume basis function at the
        # Gauss points of each face slot s = 2c + side: n_c d_c phi_i
        Dnf = []
        for s in range(self.nf):
            c, side = divmod(s, 2)
            nrm = 1.0 if side == 1 else -1.0
            dend = lagrange_deriv(xi, [float(side)])[:, 0] / h
            P = np.ones((len(fQ), nv)) * dend[Iidx[:, c]][None, :]
            for j, t in enumerate([t for t in range(d) if t != c]):
                P *= l1[Iidx[:, t]][:, fQ[:, j]].T
            Dnf.append(nrm * P)
        self.Dnf = Dnf
        self.N = sum((Dnf[s].T * self.Wf) @ self.Phif[s] for s in range(self.nf))
        D = np.zeros((nv, nl))
        for s in range(self.nf):
            D[:, s * ne:(s + 1) * ne] = (Dnf[s].T * self.Wf) @ self.Mu
        self.Dn = D
        # derivative of the basis at its own nodes, one matrix per direction
        dnode = lagrange_deriv(xi, xi)   # dnode[j, a] = l_j'(xi_a)
        lnode = lagrange(xi, xi)         # identity up to rounding
        self.Dnode = []
        for c in range(d):
            Dc = np.ones((nv, nv))
            for dim in range(d):
                tab = dnode if dim == c else lnode
                Dc *= tab[Iidx[:, dim]][:, Iidx[:, dim]].T
            self.Dnode.append(Dc / h)

    # ------------------------------------------------------------------
    def blocks(self, T):
        """(L_T, R_T, C_T) of element T."""
        kap, tau, sf = float(self.kappa_el[T]), self.tau_of(T), self.sf
        L = kap * (self.K - sf * self.N - self.N.T) + tau * self.E
        R = tau * self.G - sf * kap * self.Dn
        C = tau * self.G.T - kap * self.Dn.T
        return L, R, C

    def local_matrix(self, T):
        return self.blocks(T)[0]

    def element_dtn(self, T, b=None):
        """A^e = tau H - C L^-1 R and b^e = C L^-1 b (static condensation)."""
        L, R, C = self.blocks(T)
        Ae = self.tau_of(T) * self.H - C @ np.linalg.solve(L, R)
        if b is None:
            return Ae
        return Ae, C @ np.linalg.solve(L, np.asarray(b, dtype=float))

    def recover_element(self, T, lam_T, f_T=None):
        """u_T = L_T^-1 (R_T Lambda_T + M f_T), q_T = -kappa_T grad u_T at the
        nodes: (u_T [N_v], q_T [d, N_v])."""
        L, R, _ = self.blocks(T)
        rhs = R @ np.asarray(lam_T, dtype=float)
        if f_T is not None:
            rhs = rhs + self.M @ np.asarray(f_T)
        u = np.linalg.solve(L, rhs)
        q = -float(self.kappa_el[T]) * np.stack([Dc @ u for Dc in self.Dnode])
        return u, q

    def reconstruct(self, lam, f_nodal=None, lam_b=None):
        nel, d, nv = self.mesh.nel, self.d, self.nv
        f_nodal = np.zeros((nel, nv)) if f_nodal is None else np.asarray(f_nodal)
        lam_b = np.zeros(self.nbdof) if lam_b is None else lam_b
        LT = self.local_traces(np.asarray(lam), lam_b)
        u = np.zeros((nel, nv))
        q = np.zeros((nel, d, nv))
        for T in range(nel):
            u[T], q[T] = self.recover_element(T, LT[T], f_nodal[T])
        return u, q

    def monolithic_solve(self, f_nodal=None, gD=None):
        """Solve the uncondensed system (eq. IPG_H on every element, eq.
        conservation on every interior face) for (u, lambda) at once with a
        sparse direct solver.  Returns (lambda, u, q = -kappa grad u)."""
        m, nv = self.mesh, self.nv
        nel = m.nel
        f_nodal = np.zeros((nel, nv)) if f_nodal is None else np.asarray(f_nodal)
        lam_b = np.zeros(self.nbdof) if gD is None else np.asarray(gD(self.boundary_nodes()), dtype=float)
        Nt = nel * nv + self.nlam
        rows, cols, vals = [], [], []
        rhs = np.zeros(Nt)

        def put(r, c, blk):
            rr, cc = np.meshgrid(r, c, indexing="ij")
            rows.append(rr.ravel())
            cols.append(cc.ravel())
            vals.append(np.asarray(blk).ravel())

        for T in range(nel):
            L, R, C = self.blocks(T)
            ur = T * nv + np.arange(nv)
            gi, bi = self.gmap[T], self.bmap[T]
            ii = np.nonzero(gi >= 0)[0]
            jb = np.nonzero(bi >= 0)[0]
            put(ur, ur, L)
            put(ur, nel * nv + gi[ii], -R[:, ii])
            rhs[ur] += self.M @ f_nodal[T] + R[:, jb] @ lam_b[bi[jb]]
            lr = nel * nv + gi[ii]
            put(lr, ur, C[ii, :])
            put(lr, nel * nv + gi[ii], -self.tau_of(T) * self.H[np.ix_(ii, ii)])
            rhs[lr] += self.tau_of(T) * self.H[np.ix_(ii, jb)] @ lam_b[bi[jb]]
        Kg = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                           shape=(Nt, Nt)).tocsc()
        sol = spla.spsolve(Kg, rhs)
        u = sol[:nel * nv].reshape(nel, nv)
        lam = sol[nel * nv:]
        q = np.stack([-self.kappa_el[:, None] * (u @ Dc.T) for Dc in self.Dnode], axis=1)
        return lam, u, q

