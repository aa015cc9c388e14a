"""Discrete adjoint of the condensed HDG system (oracle; test infrastructure only).

Not in the paper; derived from the local problem (eqs. HDG, HDG_flux) and
the conservation condition.  With kappa_T = exp(theta_T) constant on each
element and the misfit J = 1/2 sum_T (u_T - u_obs,T)^T M_T (u_T - u_obs,T):

* the local operator satisfies L_T^T = P L_T P with P = diag(-I_q, I_u),
  and S_T = P R_T, so the adjoint trace system is the forward trace system
  with the volume load b_T replaced by j_T = dJ/du_T = M_T (u_T - u_obs,T);
* the adjoint volume fields (q*, u*) are the local recovery of that
  adjoint trace solution with load j;
* dJ/dtheta_T = -(q*_T)^T A_T q_T, where A_T is the kappa^-1 weighted
  vector mass matrix of the first local equation (d A_T / d theta_T = -A_T).

Pinned by complex-step differentiation through the whole forward path and
by central differences (tests/test_oracle_adjoint.py).
"""
import numpy as np
import scipy.sparse.linalg as spla


def misfit(P, u, u_obs):
    """J = 1/2 sum_T (u_T - u_obs,T)^T M_T (u_T - u_obs,T) (no conjugation,
    so that it continues analytically for complex-step checks)."""
    r = u - u_obs
    return 0.5 * np.sum(r * (r @ P.M.T))


def forward(P, theta, f_nodal, gD=None, solver=None):
    """u, q, lambda at kappa_T = exp(theta_T)."""
    P.set_kappa(np.exp(theta))
    A, g, lam_b = P.assemble(f_nodal, gD)
    lam = spla.spsolve(A.tocsc(), g) if solver is None else solver(A, g)
    u, q = P.reconstruct(lam, f_nodal, lam_b)
    return u, q, lam, A


def gradient(P, theta, f_nodal, u_obs, gD=None, solver=None):
    """(J, dJ/dtheta) by one forward and one adjoint solve."""
    u, q, lam, A = forward(P, theta, f_nodal, gD, solver)
    J = misfit(P, u, u_obs)
    jnod = u - u_obs                      # load j_T = M_T (u_T - u_obs,T)
    _, gadj, _ = P.assemble(jnod, None)   # same operator, load j, zero traces on the boundary
    mu = spla.spsolve(A.tocsc(), gadj) if solver is None else solver(A, gadj)
    _, qs = P.reconstruct(mu, jnod, None)
    kap = np.exp(theta)
    Mk = P.M
    grad = np.zeros(P.mesh.nel, dtype=np.result_type(qs.dtype, q.dtype))
    for c in range(P.d):
        grad -= np.einsum("ti,ij,tj->t", qs[:, c, :], Mk, q[:, c, :]) / kap
    return J, grad
