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
