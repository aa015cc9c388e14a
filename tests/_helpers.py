"""Shared test utilities: assembling element-form matrices with the documented
trace numbering, and tolerance helpers.  Test code only."""
import numpy as np
import scipy.sparse as sp

from oracle.hdg import Mesh


def local_to_global(d, n, ne):
    """[n^d, 2d*ne] interior trace DOF of every element-local DOF (-1 on the boundary)."""
    m = Mesh(d, n)
    out = -np.ones((m.nel, 2 * d * ne), dtype=np.int64)
    for T in range(m.nel):
        for s in range(2 * d):
            kind, fid, _ = m.slot_face(T, s)
            if kind == "i":
                out[T, s * ne:(s + 1) * ne] = fid * ne + np.arange(ne)
    return out, m.nface * ne


def assemble(Ae, d, n, ne):
    gmap, N = local_to_global(d, n, ne)
    rows, cols, vals = [], [], []
    for T in range(Ae.shape[0]):
        ii = np.nonzero(gmap[T] >= 0)[0]
        rr, cc = np.meshgrid(gmap[T, ii], gmap[T, ii], indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(Ae[T][np.ix_(ii, ii)].ravel())
    if not rows:
        return sp.csr_matrix((N, N))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N)).tocsr()


def relerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0)


def ge_solve_longdouble(A, B):
    """Gaussian elimination with partial pivoting in extended precision."""
    A = np.array(A, dtype=np.longdouble)
    B = np.array(B, dtype=np.longdouble)
    n = A.shape[0]
    for k in range(n):
        p = k + int(np.argmax(np.abs(A[k:, k])))
        if p != k:
            A[[k, p]] = A[[p, k]]
            B[[k, p]] = B[[p, k]]
        f = A[k + 1:, k] / A[k, k]
        A[k + 1:, k:] -= f[:, None] * A[k, k:][None, :]
        B[k + 1:] -= f[:, None] * B[k][None, :]
    X = np.zeros_like(B)
    for k in range(n - 1, -1, -1):
        X[k] = (B[k] - A[k, k + 1:] @ X[k + 1:]) / A[k, k]
    return X


def rowerr(a, b, scale):
    """Largest entrywise difference |a - b| measured against a per-entry
    scale (e.g. (|A| |x|)_i for a product A x): what a normwise error hides
    on entries much smaller than the vector's norm."""
    a, b, s = np.asarray(a).ravel(), np.asarray(b).ravel(), np.asarray(scale).ravel()
    d = np.abs(a - b)
    tiny = np.finfo(float).tiny
    return float(np.max(d / np.maximum(s, tiny))) if d.size else 0.0


def load_scale(O, f, lam_b=None):
    """Per trace DOF, the sum of the magnitudes of the terms that make up g:
    sum_T |b^e_T| + |A^e_{T,I bnd}| |lambda_bnd| (the entrywise scale of g)."""
    sc = np.zeros(O.nlam)
    for T in range(O.mesh.nel):
        Ae, be = O.element_dtn(T, O.M @ np.asarray(f[T]))
        gi, bi = O.gmap[T], O.bmap[T]
        ii = np.nonzero(gi >= 0)[0]
        jb = np.nonzero(bi >= 0)[0]
        np.add.at(sc, gi[ii], np.abs(be[ii]))
        if lam_b is not None and len(jb):
            np.add.at(sc, gi[ii], np.abs(Ae[np.ix_(ii, jb)]) @ np.abs(lam_b[bi[jb]]))
    return sc


def local_cond(kap, n, tau=1.0):
    """Largest kappa / (tau h) over the elements (h = 1/n): the factor by which
    the element-local solves' rounding grows (the DtN map and the recovered
    flux are differences of terms that much larger than themselves)."""
    return float(np.max(np.asarray(kap))) * n / tau


def elem_bound(kap, n, tau=1.0, floor=1e-12):
    """FP64 parity bound for results formed from element-local solves:
    floor, or 4 eps times the largest kappa / (tau h) where that is larger."""
    return max(floor, 4 * np.finfo(float).eps * (1.0 + local_cond(kap, n, tau)))


def load_scale_weighted(O, f, kap, n, lam_b=None, tau=1.0):
    """load_scale with each element's terms weighted by 1 + kappa_T/(tau h):
    the entrywise scale of g against which both codes' rounding is bounded."""
    kmax = np.asarray(kap).reshape(O.mesh.nel, -1).max(axis=1)
    sc = np.zeros(O.nlam)
    for T in range(O.mesh.nel):
        Ae, be = O.element_dtn(T, O.M @ np.asarray(f[T]))
        c = 1.0 + kmax[T] * n / tau
        gi, bi = O.gmap[T], O.bmap[T]
        ii = np.nonzero(gi >= 0)[0]
        jb = np.nonzero(bi >= 0)[0]
        np.add.at(sc, gi[ii], c * np.abs(be[ii]))
        if lam_b is not None and len(jb):
            np.add.at(sc, gi[ii], c * (np.abs(Ae[np.ix_(ii, jb)]) @ np.abs(lam_b[bi[jb]])))
    return sc
