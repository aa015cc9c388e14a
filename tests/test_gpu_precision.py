"""Mixed precision as FP64 iterative refinement, solution accuracy against
the oracle's direct solve, and solver bookkeeping, through the C ABI.

* 3D, k = 3, kappa(x) of the 3D workload at n = 16 and 32: the FP32
  V-cycle inside FP64 refinement reaches a true FP64 relative residual of
  1e-10 (recomputed by the oracle at n = 16, by the GPU's FP64 apply at
  n = 32), and the same trace as the FP64 solve.
* 2D, 64 x 64, k = 4, kappa over six decades (the benchmark's
  distribution): FP64 and mixed traces, u and q against the oracle's
  sparse direct solve, at the benchmark tolerance and at the FP64 floor.
* GMRES over several right-hand sides gives each single solve bit for bit.
* The autograd adjoint stays correct when the handle was re-formed at
  another theta between the forward and the backward pass.
"""
import sys

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import mg as omg
from oracle.hdg import HDG
from paper_1811_09909_amd import inputs

from ._helpers import relerr

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _cube(torch, n):
    from paper_1811_09909_amd.hdg import Problem
    wl = inputs.diffusion3d(n, 3)
    probe = Problem(3, n, 3, torch.ones(n ** 3, dtype=torch.float64), tau=1.0, store_recovery=False)
    kq = wl.kappa_fn(probe.volume_qpoints().numpy())
    f = wl.f(probe.volume_nodes().numpy())
    probe.close()
    P = Problem(3, n, 3, torch.as_tensor(kq), tau=1.0, kappa_kind="qp", store_recovery=False)
    return wl, P, kq, f


@pytest.mark.parametrize("n", [16, 32])
def test_mixed_refinement_3d(torch_cuda, n):
    """FP32 V-cycle + FP64 refinement on the 3D workload converges to the
    FP64 tolerance; its trace matches the FP64 solve's."""
    from paper_1811_09909_amd import _lib as L
    say(f"[mixed 3d] n={n} k=3")
    wl, P, kq, f = _cube(torch_cuda, n)
    ft = torch_cuda.as_tensor(f)
    out = {}
    for nm, prec in (("fp64", L.FP64), ("mixed", L.MIXED)):
        P.build(local_corr=L.LC_BOTH, method=L.METHOD_PCG, precision=prec, max_it=3000)
        lam, info = P.solve(ft, tol=1e-10)
        g = P.rhs(ft)
        rel = float((g - P.level_apply(0, lam)).norm() / g.norm())
        say(f"  {nm}: {info['iters']} iterations, {info['outer_iters']} true residuals, reported relres "
            f"{info['relres']:.2e}, recomputed {rel:.2e}")
        assert info["relres"] <= 1e-10 and rel <= 1.05e-10
        out[nm] = (lam, info)
    # FP32 operator blocks with FP64 sums and FP64 finest-level vectors keep
    # the FP64 cycle's count
    assert out["mixed"][1]["iters"] <= 1.05 * out["fp64"][1]["iters"] + 5
    d = float((out["mixed"][0] - out["fp64"][0]).norm() / out["fp64"][0].norm())
    say(f"  |lam_mixed - lam_fp64| / |lam_fp64| = {d:.2e}")
    assert d <= 1e-9
    if n == 16:
        # the oracle's own residual of the mixed trace
        O = HDG(3, n, 3, 1.0, np.ones(n ** 3))
        O.set_kappa(kq)
        A, go, _ = O.assemble(f)
        x = out["mixed"][0].cpu().numpy()
        ro = np.linalg.norm(go - A @ x) / np.linalg.norm(go)
        say(f"  oracle residual of the mixed trace {ro:.2e}")
        assert ro <= 1.05e-10


@pytest.fixture(scope="module")
def sq64(torch_cuda):
    """64 x 64, k = 4, kappa log-uniform over six decades, nodal f ~ N(0,1):
    the benchmark's distribution on a mesh the oracle factors directly."""
    wl = inputs.diffusion2d(64, 4, 1e-3, 1e3, seed=0)
    O = HDG(2, 64, 4, 1.0, wl.kappa)
    A, g, lb = O.assemble(wl.f)
    lu = spla.splu(A.tocsc())
    lam = lu.solve(g)
    u, q = O.reconstruct(lam, wl.f, lb)
    say(f"[sq64] oracle direct solve: relres {np.linalg.norm(g - A @ lam) / np.linalg.norm(g):.2e}")
    return wl, O, A, g, lu, lam, u, q


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solution_vs_direct_solve(torch_cuda, sq64, prec):
    """Trace, u and q of the GPU solve against the oracle's direct solve,
    at the benchmark tolerance and at the FP64 floor of the residual:
    1e-10 relative (FP64) and 1e-9 (mixed), and within what the two
    residuals allow (A^-1 applied to each, with the oracle's LU)."""
    from paper_1811_09909_amd import _lib as L
    from paper_1811_09909_amd.hdg import Problem
    wl, O, A, g, lu, lam_d, u_d, q_d = sq64
    pr = L.FP64 if prec == "fp64" else L.MIXED
    P = Problem(2, 64, 4, torch_cuda.as_tensor(wl.kappa), tau=1.0, store_recovery=True)
    f = torch_cuda.as_tensor(wl.f)
    P.build(local_corr=L.LC_BOTH, method=L.METHOD_PCG, precision=pr, max_it=3000, coarse_n=16)
    lam, info = P.solve(f, tol=1e-10)
    its = info["iters"]
    target = 1e-10 if prec == "fp64" else 1e-9
    e_d = np.linalg.norm(lu.solve(g - A @ lam_d))
    for label, tol, maxit in (("tol 1e-10", 1e-10, 3000), ("floor", 1e-13, its + 300)):
        P.build(local_corr=L.LC_BOTH, method=L.METHOD_PCG, precision=pr, max_it=maxit, coarse_n=16)
        lam, info = P.solve(f, tol=tol, allow_not_converged=True)
        u, q = P.reconstruct(lam, f)
        x = lam.cpu().numpy()
        ro = np.linalg.norm(g - A @ x) / np.linalg.norm(g)
        el, eu, eq = relerr(x, lam_d), relerr(u.cpu().numpy(), u_d), relerr(q.cpu().numpy(), q_d)
        bound = 1.5 * (np.linalg.norm(lu.solve(g - A @ x)) + e_d) / np.linalg.norm(lam_d) + 1e-14
        say(f"  {prec} {label}: {info['iters']} iterations ({info['outer_iters']} true residuals), "
            f"oracle relres {ro:.2e}; errors lambda {el:.2e} (residual bound {bound:.2e}) u {eu:.2e} q {eq:.2e}")
        if tol == 1e-10:
            assert info["relres"] <= 1e-10 and ro <= 1.05e-10
        assert el <= bound
        assert el <= target and eu <= target and eq <= target


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_gmres_several_rhs_match_single_solves(torch_cuda, prec):
    """GMRES with a build for three right-hand sides solves each in its own
    rows: bit for bit the single solves (right-hand side 0 included)."""
    from paper_1811_09909_amd import _lib as L
    from paper_1811_09909_amd.hdg import Problem
    wl = inputs.diffusion2d(32, 3, 1e-2, 1e2, seed=8)
    rng = np.random.default_rng(9)
    F = np.stack([wl.f, rng.standard_normal(wl.f.shape), 1e-3 * rng.standard_normal(wl.f.shape)])
    pr = L.FP64 if prec == "fp64" else L.MIXED
    P = Problem(2, 32, 3, torch_cuda.as_tensor(wl.kappa), tau=1.0, store_recovery=False)
    P.build(local_corr=L.LC_PRE, method=L.METHOD_GMRES, precision=pr, max_it=200)
    singles = [P.solve(torch_cuda.as_tensor(F[i]), tol=1e-10) for i in range(3)]
    P.build(local_corr=L.LC_PRE, method=L.METHOD_GMRES, precision=pr, max_it=200, nrhs=3)
    lam, info = P.solve(torch_cuda.as_tensor(F), tol=1e-10, nrhs=3)
    lam = lam.reshape(3, -1)
    for i in range(3):
        diff = float((lam[i] - singles[i][0]).abs().max())
        g = P.rhs(torch_cuda.as_tensor(F[i]))
        rel = float((g - P.level_apply(0, lam[i])).norm() / g.norm())
        say(f"[gmres x3 {prec}] rhs {i}: single {singles[i][1]['iters']} iterations, true relres {rel:.2e}, "
            f"max diff vs single {diff:.1e}")
        assert diff == 0.0 and rel <= 1.05e-10


def test_adjoint_after_handle_reformed(torch_cuda):
    """Forward at theta1, forward at theta2 on the same handle, then the
    backward pass of the theta1 graph: the gradient equals that of a fresh
    forward and backward at theta1."""
    import torch
    from paper_1811_09909_amd import _lib as L
    from paper_1811_09909_amd.hdg import HDGMass, HDGSolve, Problem
    n, k = 16, 2
    rng = np.random.default_rng(12)
    P = Problem(2, n, k, torch.ones(n * n, dtype=torch.float64), tau=1.0, store_recovery=True)
    f = torch.ones(n * n, (k + 1) ** 2, dtype=torch.float64, device=P.device)
    kw = dict(method=L.METHOD_PCG, local_corr=L.LC_BOTH, precision=L.FP64, max_it=500)
    u_obs = torch.as_tensor(rng.standard_normal((n * n, (k + 1) ** 2)) * 1e-2, device=P.device)

    def J(theta):
        u = HDGSolve.apply(theta, P, f, 1e-13, kw)
        r = u - u_obs
        return 0.5 * (r * HDGMass.apply(r, P)).sum()

    t1 = torch.as_tensor(rng.standard_normal(n * n), device=P.device).requires_grad_(True)
    t2 = torch.as_tensor(rng.standard_normal(n * n), device=P.device).requires_grad_(True)
    J1 = J(t1)
    J2 = J(t2)  # re-forms the handle at theta2
    J1.backward()
    g1 = t1.grad.detach().clone()
    t1.grad = None
    J(t1).backward()
    ref = t1.grad.detach().clone()
    e = float((g1 - ref).norm() / ref.norm())
    say(f"[adjoint after reform] J1 {J1.item():.6e} J2 {J2.item():.6e}: gradient vs fresh {e:.2e}")
    assert e <= 1e-12


@pytest.mark.parametrize("d,n,k,variant", [(3, 8, 3, 0), (3, 4, 2, 0), (2, 32, 4, "fine64"), (2, 32, 4, 0)])
def test_mixed_cycle_against_oracle(torch_cuda, d, n, k, variant):
    """The cycle the mixed solve applies (in 3D, and by choice in 2D: FP64
    vectors and sums over FP32 operator blocks; in 2D by default the FP32
    cycle) against the oracle's FP64 Algorithm 1: single-precision
    agreement."""
    from paper_1811_09909_amd import _lib as L
    from paper_1811_09909_amd.hdg import Problem
    rng = np.random.default_rng(3)
    if d == 3:
        wl = inputs.diffusion3d(n, k)
        O = HDG(3, n, k, 1.0, np.ones(n ** 3))
        kap = wl.kappa_fn(O.volume_qpoints())
        O.set_kappa(kap)
        P = Problem(3, n, k, torch_cuda.as_tensor(kap), tau=1.0, kappa_kind="qp", store_recovery=False)
    else:
        kap = 10.0 ** rng.uniform(-2, 2, n * n)
        O = HDG(2, n, k, 1.0, kap)
        P = Problem(2, n, k, torch_cuda.as_tensor(kap), tau=1.0, store_recovery=False)
    A, _, _ = O.assemble()
    H = omg.Hierarchy(A, d, n, k, local_corr=omg.LC_BOTH)
    var = L.VARIANT_FP64_VECTORS if variant == "fine64" else 0
    P.build(local_corr=L.LC_BOTH, method=L.METHOD_PCG, precision=L.MIXED, variant=var)
    r = rng.standard_normal(A.shape[0])
    eo = H.vcycle(r)
    e = P.vcycle(torch_cuda.as_tensor(r), precision=L.MIXED_CYCLE).cpu().numpy()
    e64 = P.vcycle(torch_cuda.as_tensor(r)).cpu().numpy()
    say(f"[mixed cycle] d={d} n={n} k={k} variant={variant}: vs oracle {relerr(e, eo):.2e}, "
        f"FP64 cycle vs oracle {relerr(e64, eo):.2e}")
    assert relerr(e, eo) <= 1e-5
