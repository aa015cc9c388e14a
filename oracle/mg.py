"""Unified geometric multigrid for the trace system (oracle; test infrastructure only).

Everything here works on the global sparse trace operators, exactly as the
paper writes them:

* p-coarsening (Sec. 3.1.1): level N keeps P^k traces, level N-1 the same
  faces with P^1 (Q^1 in 3D) traces; J_N interpolates P^1 into P^k;
  I_N = J_N, Q_{N-1} = J_N^T, A_{N-1} = J_N^T A_N J_N (eqs. n_g1_Ik,
  n_g1_Qk, ANm1).
* h-coarsening by agglomeration (Sec. 3.1.2): 2^d macro-elements of level
  k form one macro-element of level k-1.  Faces inside a coarse
  macro-element form E_{k,I}, faces on coarse macro-element boundaries
  form E_{k,B} (eq. trace_partition); the coarse space is P^1 (Q^1) on
  each coarse macro-face and J_k interpolates it onto E_{k,B}.
* prolongation I_k = [-A_II^-1 A_IB J_k ; J_k] (eq. n_1_Ik), restriction
  Q_{k-1} = [-J_k^T A_BI A_II^-1 , J_k^T] (eq. n_1_Qk), Galerkin coarse
  operator A_{k-1} = Q_{k-1} A_k I_k = J_k^T (A_BB - A_BI A_II^-1 A_IB) J_k
  (eqs. coarse, Akm1).  J_k^* is taken as the matrix transpose with
  residuals in assembled (weak) form.
* smoothing (Sec. 4.1), m_k sweeps (Sec. 3.3): face-block Jacobi, one block
  per face of the level, damping omega (1 by default); or one of the
  paper's point smoothers: damped point Jacobi (omega = 2/3), Chebyshev-
  accelerated point Jacobi (the largest eigenvalue of D^-1 A estimated by
  power iteration, the smallest taken as a thirtieth of it), and LU-SGS
  (one forward and one backward point Gauss-Seidel sweep per step, in the
  trace numbering); and the multicolour variant of LU-SGS the GPU runs
  (faces in colours no two of which share an element, point Gauss-Seidel
  within a face).
* local correction T_k: e_I += A_II^-1 (r - A e)_I (eq. localCorrection).
* V-cycle: Algorithm 1, with B_1 = A_1^-1 by a dense direct solve.
* outer iterations: fixed point lambda += B_N (g - A lambda) (Sec. 3.6),
  preconditioned CG, and GMRES (right or left preconditioned).

The hierarchy stops at 2^d macro-elements by default: one macro-element
has no interior faces under Dirichlet conditions, so its level would be
empty.  ``coarsest_n`` stops the h-coarsening earlier, at the first macro
grid with at most that many macro-elements per direction; the paper treats
the number of levels N as a free parameter (Sec. 3.1.2, Sec. 4.5) and always
solves the coarsest level directly (Algorithm 1, B_1 = A_1^-1).

``coarse='exact'`` keeps every trace unknown of E_{k,B} on the coarse level
(J_k = identity, no p-coarsening): the coarse operators become exact Schur
complements and the V-cycle with zero smoothing is a direct solver (nested
dissection, Sec. 3.5).  It exists to pin the recursion.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from .hdg import Mesh, lex
from .refelem import gll_nodes

LC_NONE, LC_PRE, LC_POST, LC_BOTH = 0, 1, 2, 3
SMOOTHERS = ("block_jacobi", "jacobi", "chebyshev", "lusgs", "lusgs_mc")
CHEB_POWER_ITS = 20      # power iterations of the largest-eigenvalue estimate
CHEB_SAFETY = 1.1        # the estimate is raised by this factor
CHEB_RATIO = 30.0        # smallest eigenvalue taken as largest / CHEB_RATIO


def block_inverse(A):
    """Inverse of a sparse matrix that is block diagonal up to a permutation:
    the blocks are the connected components of its graph, each inverted
    densely."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    if n == 0:
        return sp.csr_matrix((0, 0))
    ncomp, lab = connected_components(A, directed=False)
    order = np.argsort(lab, kind="stable")
    bounds = np.concatenate([[0], np.cumsum(np.bincount(lab, minlength=ncomp))])
    rows, cols, vals = [], [], []
    for b in range(ncomp):
        idx = order[bounds[b]:bounds[b + 1]]
        inv = np.linalg.inv(A[idx][:, idx].toarray())
        rr, cc = np.meshgrid(idx, idx, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(inv.ravel())
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def face_dofs(mesh, m):
    """DOF ids of every interior face of ``mesh`` with m DOFs per face."""
    return np.arange(mesh.nface * m).reshape(mesh.nface, m)


def p_injection(mesh, k):
    """J_N: P^1 (Q^1) vertex values on each face -> P^k GLL nodal values."""
    d = mesh.d
    xi = gll_nodes(k)
    ne, nc = (k + 1) ** (d - 1), 2 ** (d - 1)
    aidx = lex((k + 1,) * (d - 1))
    vidx = lex((2,) * (d - 1))
    blk = np.ones((ne, nc))
    for a in range(ne):
        for v in range(nc):
            for j in range(d - 1):
                t = xi[aidx[a, j]]
                blk[a, v] *= t if vidx[v, j] == 1 else 1.0 - t
    return sp.kron(sp.identity(mesh.nface), sp.csr_matrix(blk)).tocsr()


def h_partition(mesh, m, coarse):
    """Split the faces of ``mesh`` (m DOFs each) into E_I (odd position
    along the normal) and E_B (even position) and build J_k from the coarse
    space on the coarse mesh (n/2 per direction) onto E_B.

    Returns (I_dofs, B_dofs, J_B, m_coarse, coarse_mesh)."""
    d, n = mesh.d, mesh.n
    cm = Mesh(d, n // 2)
    I_dofs, B_dofs = [], []
    for fid in range(mesh.nface):
        c, coords = mesh.interior_face_coords(fid)
        (I_dofs if coords[c] % 2 == 1 else B_dofs).append(fid * m + np.arange(m))
    I_dofs = np.concatenate(I_dofs) if I_dofs else np.zeros(0, dtype=int)
    B_dofs = np.concatenate(B_dofs) if B_dofs else np.zeros(0, dtype=int)
    Bpos = -np.ones(mesh.nface * m, dtype=np.int64)
    Bpos[B_dofs] = np.arange(len(B_dofs))
    nsub = 2 ** (d - 1)
    sidx = lex((2,) * (d - 1))
    if coarse == "p1":
        if m != 2 ** (d - 1):
            raise ValueError("P1 h-coarsening needs P1 traces on the fine level")
        mc = nsub
    else:
        mc = nsub * m
    rows, cols, vals = [], [], []
    for F in range(cm.nface):
        c, cc = cm.interior_face_coords(F)
        tang = cm.tangential(c)
        for si, s in enumerate(sidx):
            fc = list(cc)
            fc[c] = 2 * cc[c]
            for j, t in enumerate(tang):
                fc[t] = 2 * cc[t] + s[j]
            f = mesh.interior_face_id(c, fc)
            if coarse == "p1":
                for v in range(m):
                    vv = sidx[v]
                    for V in range(mc):
                        VV = sidx[V]
                        w = 1.0
                        for j in range(d - 1):
                            t = 0.5 * (s[j] + vv[j])
                            w *= t if VV[j] == 1 else 1.0 - t
                        if w != 0.0:
                            rows.append(Bpos[f * m + v])
                            cols.append(F * mc + V)
                            vals.append(w)
            else:
                for a in range(m):
                    rows.append(Bpos[f * m + a])
                    cols.append(F * mc + si * m + a)
                    vals.append(1.0)
    J = sp.coo_matrix((vals, (rows, cols)), shape=(len(B_dofs), cm.nface * mc)).tocsr()
    return I_dofs, B_dofs, J, mc, cm


class Level:
    def __init__(self, A, mesh, m):
        self.A = sp.csr_matrix(A)
        self.mesh = mesh
        self.m = m
        self.faces = face_dofs(mesh, m)
        self.kind = None
        self.Dinv = None

    def face_block_inverses(self):
        """Inverses of the assembled diagonal blocks D_e, one per face (Sec. 4.1)."""
        if self.faces.size:
            r = np.repeat(self.faces[:, :, None], self.m, axis=2)
            c = np.repeat(self.faces[:, None, :], self.m, axis=1)
            D = np.asarray(self.A[r.ravel(), c.ravel()]).reshape(r.shape)
            self.Dinv = np.linalg.inv(D)
        return self


def block_jacobi(L, res, m, omega=1.0):
    """m face-block Jacobi sweeps on L.A delta = res from delta = 0."""
    delta = np.zeros_like(res)
    for _ in range(m):
        t = res - L.A @ delta
        delta = delta.copy()
        delta[L.faces] += omega * np.einsum("fab,fb->fa", L.Dinv, t[L.faces])
    return delta


def point_jacobi(L, res, m, omega):
    """m damped point-Jacobi sweeps: delta += omega D^-1 (res - A delta)."""
    dinv = 1.0 / L.A.diagonal()
    delta = np.zeros_like(res)
    for _ in range(m):
        delta = delta + omega * dinv * (res - L.A @ delta)
    return delta


def lambda_max_estimate(A):
    """Largest eigenvalue of D^-1 A by power iteration from the all-ones
    vector: CHEB_POWER_ITS normalised steps v <- D^-1 A v / ||D^-1 A v||,
    then ||D^-1 A v|| for the last unit v, raised by CHEB_SAFETY (Sec. 4.1
    asks for an estimate to about 1e-2)."""
    N = A.shape[0]
    if N == 0:
        return 1.0
    d = A.diagonal()
    v = np.ones(N)
    for _ in range(CHEB_POWER_ITS):
        w = (A @ v) / d
        v = w / np.linalg.norm(w)
    return CHEB_SAFETY * float(np.linalg.norm((A @ v) / d))


def chebyshev(L, res, m, lmax):
    """m steps of Chebyshev-accelerated point Jacobi on [lmax / CHEB_RATIO,
    lmax] from delta = 0, by the three-term recurrence of the shifted and
    scaled Chebyshev polynomials."""
    dinv = 1.0 / L.A.diagonal()
    lmin = lmax / CHEB_RATIO
    theta, dlt = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    sigma = theta / dlt
    rho = 1.0 / sigma
    d = dinv * res / theta
    delta = d.copy()
    for _ in range(1, m):
        rho_new = 1.0 / (2.0 * sigma - rho)
        r = res - L.A @ delta
        d = rho_new * rho * d + (2.0 * rho_new / dlt) * (dinv * r)
        delta = delta + d
        rho = rho_new
    return delta if m > 0 else np.zeros_like(res)


def lusgs(L, res, m):
    """m LU-SGS steps from delta = 0: a forward then a backward point
    Gauss-Seidel sweep over the unknowns in the trace numbering."""
    A = sp.csr_matrix(L.A)
    N = A.shape[0]
    delta = np.zeros_like(res)
    indptr, indices, data = A.indptr, A.indices, A.data
    diag = A.diagonal()
    for _ in range(m):
        for order in (range(N), range(N - 1, -1, -1)):
            for i in order:
                lo, hi = indptr[i], indptr[i + 1]
                s = res[i] - data[lo:hi] @ delta[indices[lo:hi]]
                delta[i] += s / diag[i]
    return delta


def face_colors(mesh):
    """Colour of each interior face: 2 c + (grid position along its normal
    c, 1 .. n-1) mod 2.  Faces of one colour share no element."""
    col = np.zeros(mesh.nface, dtype=np.int64)
    for F in range(mesh.nface):
        c, coords = mesh.interior_face_coords(F)
        col[F] = 2 * c + (coords[c] % 2)
    return col


def lusgs_mc(L, res, m):
    """Multicolour LU-SGS: per step, the face colours in increasing order,
    then decreasing; within a colour every face at once, within a face its
    unknowns in increasing (forward) or decreasing (backward) order, each a
    point Gauss-Seidel update with the current values."""
    A = sp.csr_matrix(L.A)
    diag = A.diagonal()
    col = face_colors(L.mesh)
    ncol = 2 * L.mesh.d
    delta = np.zeros_like(res)
    m_e = L.m
    for _ in range(m):
        for colors, dofs in ((range(ncol), range(m_e)), (range(ncol - 1, -1, -1), range(m_e - 1, -1, -1))):
            for c in colors:
                faces = np.nonzero(col == c)[0]
                for a in dofs:
                    rows = L.faces[faces, a]
                    s = res[rows] - A[rows] @ delta
                    delta[rows] += s / diag[rows]
    return delta


class Hierarchy:
    """Levels ordered from finest (index 0) to coarsest."""

    def __init__(self, A, d, n, k, coarse="p1", sweeps=2, growth=1, omega=1.0,
                 local_corr=LC_PRE, coarsest_n=2, smoother="block_jacobi"):
        if smoother not in SMOOTHERS:
            raise ValueError(f"unknown smoother {smoother}")
        self.coarse, self.omega, self.local_corr = coarse, omega, local_corr
        self.smoother = smoother
        mesh = Mesh(d, n)
        lev = Level(A, mesh, (k + 1) ** (d - 1))
        self.levels = [lev]
        if n < 2 or (n & (n - 1)) != 0:
            raise ValueError("h-coarsening needs n = 2^m")
        if k > 1 and coarse == "p1":
            J = p_injection(mesh, k)
            lev.kind = "p"
            lev.I = J
            lev.Q = J.T.tocsr()
            Ac = (J.T @ lev.A @ J).tocsr()
            lev = Level(Ac, mesh, 2 ** (d - 1))
            self.levels.append(lev)
        while lev.mesh.n > max(2, coarsest_n):
            I_d, B_d, JB, mc, cm = h_partition(lev.mesh, lev.m, coarse)
            lev = self._h_step(lev, I_d, B_d, JB, mc, cm)
            self.levels.append(lev)
        self._finish(sweeps, growth, smoother)

    def _h_step(self, lev, I_d, B_d, JB, mc, cm):
        """One h-coarsening (eq. trace_partition): E_I DOFs I_d, E_B DOFs
        B_d, J_k = JB; fills lev's transfers and returns the coarse level."""
        A = lev.A
        AII = A[I_d][:, I_d]
        AIB = A[I_d][:, B_d]
        ABI = A[B_d][:, I_d]
        ABB = A[B_d][:, B_d]
        AIIinv = block_inverse(AII)
        X = (AIIinv @ AIB).tocsr()
        Ac = (JB.T @ (ABB - ABI @ X) @ JB).tocsr()
        N = A.shape[0]
        # prolongation and restriction in the level's own DOF order
        PI = sp.vstack([-(X @ JB), JB]).tocsr()
        perm = np.concatenate([I_d, B_d])
        Pmat = sp.csr_matrix((np.ones(N), (perm, np.arange(N))), shape=(N, N))
        lev.I = (Pmat @ PI).tocsr()
        Qblk = sp.hstack([-(JB.T @ ABI @ AIIinv), JB.T]).tocsr()
        lev.Q = (Qblk @ Pmat.T).tocsr()
        lev.kind = "h"
        lev.I_dofs, lev.B_dofs, lev.JB = I_d, B_d, JB
        lev.AIIinv = AIIinv
        lev.AII = AII
        return Level(Ac, cm, mc)

    def _finish(self, sweeps, growth, smoother):
        """Coarsest factorization, sweeps per level, smoother data."""
        self.coarse_lu = sla.lu_factor(self.levels[-1].A.toarray()) if self.levels[-1].A.shape[0] else None
        for i, L in enumerate(self.levels):
            L.sweeps = sweeps * (2 ** i if growth == 2 else 1)
            L.face_block_inverses()
            if smoother == "chebyshev":
                L.lmax = lambda_max_estimate(L.A)

    # ---- smoothing, local correction, cycle --------------------------------
    def block_jacobi(self, i, res, m):
        """m face-block Jacobi sweeps on A_i delta = res from delta = 0."""
        return block_jacobi(self.levels[i], res, m, self.omega)

    def smooth(self, i, res, m):
        """Smooth(i, res, m): m steps of the hierarchy's smoother on
        A_i delta = res from delta = 0 (Sec. 4.1)."""
        L = self.levels[i]
        if self.smoother == "block_jacobi":
            return block_jacobi(L, res, m, self.omega)
        if self.smoother == "jacobi":
            return point_jacobi(L, res, m, self.omega)
        if self.smoother == "chebyshev":
            return chebyshev(L, res, m, L.lmax)
        if self.smoother == "lusgs":
            return lusgs(L, res, m)
        return lusgs_mc(L, res, m)

    def local_correction(self, i, rho):
        """T_i rho = [A_II^-1 rho_I ; 0] (eq. localCorrection)."""
        L = self.levels[i]
        out = np.zeros_like(rho)
        out[L.I_dofs] = L.AIIinv @ rho[L.I_dofs]
        return out

    def vcycle(self, r, i=0):
        """B_i r by Algorithm 1."""
        L = self.levels[i]
        if i == len(self.levels) - 1:
            if r.size == 0:
                return r.copy()
            return sla.lu_solve(self.coarse_lu, r)
        A = L.A
        e = np.zeros_like(r)
        e = e + self.smooth(i, r - A @ e, L.sweeps)
        if L.kind == "h" and self.local_corr in (LC_PRE, LC_BOTH):
            e = e + self.local_correction(i, r - A @ e)
        e = e + L.I @ self.vcycle(L.Q @ (r - A @ e), i + 1)
        if L.kind == "h" and self.local_corr in (LC_POST, LC_BOTH):
            e = e + self.local_correction(i, r - A @ e)
        e = e + self.smooth(i, r - A @ e, L.sweeps)
        return e


class Result:
    def __init__(self, lam, iters, relres, history, converged):
        self.lam, self.iters, self.relres = lam, iters, relres
        self.history, self.converged = history, converged


def mg_solve(H, A, g, tol=1e-10, maxit=200, lam0=None):
    """Fixed point lambda^{i+1} = lambda^i + B_N (g - A lambda^i) (Sec. 3.6)."""
    lam = np.zeros_like(g) if lam0 is None else lam0.copy()
    gn = np.linalg.norm(g)
    if gn == 0:
        return Result(np.zeros_like(g), 0, 0.0, [0.0], True)
    r = g - A @ lam
    hist = [np.linalg.norm(r) / gn]
    it = 0
    while hist[-1] > tol and it < maxit and np.isfinite(hist[-1]):
        lam = lam + H.vcycle(r)
        r = g - A @ lam
        it += 1
        hist.append(np.linalg.norm(r) / gn)
    return Result(lam, it, hist[-1], hist, hist[-1] <= tol)


def pcg_solve(H, A, g, tol=1e-10, maxit=200, lam0=None):
    """Conjugate gradients preconditioned by one V-cycle per iteration.
    Stops on the recursively updated residual, then confirms with the true
    residual and restarts from the current iterate if that is not yet
    below tol."""
    lam = np.zeros_like(g) if lam0 is None else lam0.copy()
    gn = np.linalg.norm(g)
    if gn == 0:
        return Result(np.zeros_like(g), 0, 0.0, [0.0], True)
    it = 0
    hist = []
    while True:
        r = g - A @ lam
        hist.append(np.linalg.norm(r) / gn)
        if hist[-1] <= tol or it >= maxit or not np.isfinite(hist[-1]):
            break
        z = H.vcycle(r)
        p = z.copy()
        rz = r @ z
        while it < maxit:
            Ap = A @ p
            alpha = rz / (p @ Ap)
            lam = lam + alpha * p
            r = r - alpha * Ap
            it += 1
            rel = np.linalg.norm(r) / gn
            if rel <= tol or not np.isfinite(rel):
                break
            hist.append(rel)
            z = H.vcycle(r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
    return Result(lam, it, hist[-1], hist, hist[-1] <= tol)


def gmres_solve(H, A, g, tol=1e-10, maxit=200, lam0=None, side="right"):
    """GMRES without restart, modified Gram-Schmidt, Givens rotations.
    ``side='right'`` minimises the true residual ||g - A lambda||;
    ``side='left'`` (the paper's choice, Sec. 4) minimises ||B(g - A lambda)||
    and stops on the preconditioned residual normalised by ||B g||."""
    lam = np.zeros_like(g) if lam0 is None else lam0.copy()
    gn = np.linalg.norm(g)
    if gn == 0:
        return Result(np.zeros_like(g), 0, 0.0, [0.0], True)
    r = g - A @ lam
    if side == "left":
        r = H.vcycle(r)
        ref = np.linalg.norm(H.vcycle(g))
    else:
        ref = gn
    beta = np.linalg.norm(r)
    hist = [beta / ref]
    if hist[-1] <= tol:
        return Result(lam, 0, hist[-1], hist, True)
    V = [r / beta]
    Z = []
    Hh = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    s = np.zeros(maxit + 1)
    s[0] = beta
    j = 0
    while j < maxit:
        if side == "right":
            z = H.vcycle(V[j])
            Z.append(z)
            w = A @ z
        else:
            w = H.vcycle(A @ V[j])
        for i in range(j + 1):
            Hh[i, j] = w @ V[i]
            w = w - Hh[i, j] * V[i]
        hnext = np.linalg.norm(w)
        Hh[j + 1, j] = hnext
        for i in range(j):
            t = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
            Hh[i + 1, j] = -sn[i] * Hh[i, j] + cs[i] * Hh[i + 1, j]
            Hh[i, j] = t
        den = np.hypot(Hh[j, j], Hh[j + 1, j])
        cs[j], sn[j] = Hh[j, j] / den, Hh[j + 1, j] / den
        Hh[j, j] = den
        Hh[j + 1, j] = 0.0
        s[j + 1] = -sn[j] * s[j]
        s[j] = cs[j] * s[j]
        j += 1
        hist.append(abs(s[j]) / ref)
        if hist[-1] <= tol or hnext == 0.0 or not np.isfinite(hist[-1]):
            break
        V.append(w / hnext)
    y = sla.solve_triangular(Hh[:j, :j], s[:j])
    if side == "right":
        lam = lam + sum(y[i] * Z[i] for i in range(j))
    else:
        lam = lam + sum(y[i] * V[i] for i in range(j))
    return Result(lam, j, hist[-1], hist, hist[-1] <= tol)
