"""1D building blocks of the nodal spaces (oracle; test infrastructure only).

The paper uses polynomial spaces of degree p on every element and face
(Sec. 2, definition of V_h, W_h, M_h).  On the tensor-product quads and
hexes used here they are read as Q^k spaces, nodal at tensor
Gauss-Lobatto-Legendre (GLL) points; integrals use tensor Gauss-Legendre
rules.  Everything lives on the unit interval [0, 1].
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gll_nodes(k):
    """The k+1 Gauss-Lobatto-Legendre points on [0, 1], increasing.

    They are the two end points together with the roots of P_k', the
    derivative of the Legendre polynomial of degree k.
    """
    if k < 1:
        raise ValueError("degree must be >= 1")
    coeffs = np.zeros(k + 1)
    coeffs[k] = 1.0
    inner = npleg.legroots(npleg.legder(coeffs)) if k > 1 else np.zeros(0)
    x = np.concatenate(([-1.0], np.sort(np.real(inner)), [1.0]))
    return 0.5 * (x + 1.0)


def gauss_rule(npts):
    """Gauss-Legendre points and weights on [0, 1] (exact to degree 2*npts-1)."""
    x, w = npleg.leggauss(npts)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange(nodes, x):
    """V[i, q] = l_i(x_q) for the Lagrange basis through ``nodes``."""
    nodes = np.asarray(nodes, dtype=float)
    x = np.atleast_1d(np.asarray(x, dtype=float))
    n = len(nodes)
    V = np.ones((n, len(x)))
    for i in range(n):
        for j in range(n):
            if j != i:
                V[i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
    return V


def lagrange_deriv(nodes, x):
    """D[i, q] = l_i'(x_q), by the product rule over the factors of l_i."""
    nodes = np.asarray(nodes, dtype=float)
    x = np.atleast_1d(np.asarray(x, dtype=float))
    n = len(nodes)
    D = np.zeros((n, len(x)))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.ones(len(x)) / (nodes[i] - nodes[m])
            for j in range(n):
                if j != i and j != m:
                    term = term * (x - nodes[j]) / (nodes[i] - nodes[j])
            D[i] += term
    return D
