"""Persistent coarse cycle (HDG_VARIANT_GRID_TAIL) through the C ABI.

The coarse h-levels of the 2D fused V-cycle (from 128 x 128 down) and the
dense coarsest solve run in one launch with grid-wide barriers.  Each phase
is the same work item, in the same lane layout, that the per-level kernels
run, so the cycle must equal the per-level form bit for bit: single
V-cycles in FP64 and FP32, and whole CG solves (FP64 and mixed) with their
iteration counts, over graph replays.  One case also checks the cycle
against the oracle's Algorithm 1 with the same levels.
"""
import sys

import numpy as np
import pytest

from oracle import mg as omg
from oracle.hdg import HDG
from paper_1811_09909_amd import inputs

from ._helpers import relerr

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="persistent coarse cycle switched off: single eager V-cycles matched the per-level "
                            "kernels bit for bit (and the oracle to 3.4e-14), but a graph-captured CG solve with it "
                            "failed on the device and lost the queue, cause not yet shown; hdg_mg_build refuses "
                            "HDG_VARIANT_GRID_TAIL"),
]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _problem(torch, n, k, seed=0):
    from paper_1811_09909_amd.hdg import Problem
    rng = np.random.default_rng(seed)
    kap = inputs.kappa_loguniform(rng, n * n, 1e-3, 1e3)
    return Problem(2, n, k, torch.as_tensor(kap), tau=1.0), kap, rng


@pytest.mark.parametrize("n,k,cn,lc", [(256, 2, 16, "both"), (128, 1, 8, "pre"), (256, 4, 32, "post")])
def test_grid_tail_vcycle_bitwise(torch_cuda, n, k, cn, lc):
    """One V-cycle with and without the persistent coarse cycle: identical
    results in FP64 and FP32, on two calls in a row."""
    from paper_1811_09909_amd import _lib as L
    LCM = {"both": L.LC_BOTH, "pre": L.LC_PRE, "post": L.LC_POST}[lc]
    say(f"[grid tail vcycle] n={n} k={k} coarse_n={cn} lc={lc}")
    P, kap, rng = _problem(torch_cuda, n, k)
    nlam = P.nlam
    R = [rng.standard_normal(nlam) for _ in range(2)]
    outs = {}
    for var in (0, L.VARIANT_GRID_TAIL):
        P.build(sweeps=2, local_corr=LCM, coarse_n=cn, variant=var)
        start = P.query(L.Q_GRID_TAIL)
        if var:
            assert start >= 1, "the persistent coarse cycle was not set up"
        else:
            assert start == -1
        outs[var] = [(P.vcycle(torch_cuda.as_tensor(r)).cpu().numpy(),
                      P.vcycle(torch_cuda.as_tensor(r, dtype=torch_cuda.float32), precision=L.FP32).cpu().numpy())
                     for r in R]
        say(f"  variant {var}: levels {P.level_sizes()}, persistent cycle from level {start}")
    for i in range(2):
        for j in range(2):
            a, b = outs[L.VARIANT_GRID_TAIL][i][j], outs[0][i][j]
            say(f"  call {i} {'fp64' if j == 0 else 'fp32'}: max |diff| {np.abs(a - b).max():.3e}")
            assert np.array_equal(a, b)
    P.close()


def test_grid_tail_against_oracle(torch_cuda):
    """The cycle with the persistent coarse part against the oracle's
    Algorithm 1 on the same hierarchy (64 x 64, k = 2, coarsest 8 x 8)."""
    from paper_1811_09909_amd import _lib as L
    n, k, cn = 64, 2, 8
    P, kap, rng = _problem(torch_cuda, n, k, seed=3)
    P.build(sweeps=2, local_corr=L.LC_BOTH, coarse_n=cn, variant=L.VARIANT_GRID_TAIL)
    assert P.query(L.Q_GRID_TAIL) >= 1
    O = HDG(2, n, k, 1.0, kap)
    A, _, _ = O.assemble()
    H = omg.Hierarchy(A, 2, n, k, sweeps=2, local_corr=omg.LC_BOTH, coarsest_n=cn)
    assert P.level_sizes() == [Lv.A.shape[0] for Lv in H.levels]
    r = rng.standard_normal(A.shape[0])
    eo = H.vcycle(r)
    e = P.vcycle(torch_cuda.as_tensor(r)).cpu().numpy()
    say(f"[grid tail vs oracle] n={n} k={k} levels {P.level_sizes()}: relerr {relerr(e, eo):.2e}")
    assert relerr(e, eo) <= 1e-10
    P.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_grid_tail_pcg_bitwise(torch_cuda, prec):
    """Whole CG solves (graph-captured iterations) with and without the
    persistent coarse cycle: same iteration count, same trace bit for bit."""
    from paper_1811_09909_amd import _lib as L
    n, k = 256, 3
    say(f"[grid tail pcg] n={n} k={k} {prec}")
    P, kap, rng = _problem(torch_cuda, n, k, seed=1)
    f = rng.standard_normal(P.volume_nodes().shape[0])
    res = {}
    for var in (0, L.VARIANT_GRID_TAIL):
        P.build(sweeps=2, local_corr=L.LC_BOTH, coarse_n=16, method=L.METHOD_PCG,
                precision=L.MIXED if prec == "mixed" else L.FP64, max_it=2000, variant=var)
        lam, info = P.solve(torch_cuda.as_tensor(f), tol=1e-10)
        res[var] = (lam.cpu().numpy(), info)
        say(f"  variant {var}: iters {info['iters']} relres {info['relres']:.2e}")
    a, ia = res[L.VARIANT_GRID_TAIL]
    b, ib = res[0]
    assert ia["iters"] == ib["iters"] and ia["relres"] <= 1e-10
    assert np.array_equal(a, b)
    P.close()


def test_grid_tail_refused_in_batches(torch_cuda):
    """Batched solves run problems on several streams at once, which cannot
    promise that every workgroup of a persistent launch is resident: a
    handle built with it is refused there."""
    from paper_1811_09909_amd import _lib as L
    from paper_1811_09909_amd.hdg import solve_batch
    P, kap, rng = _problem(torch_cuda, 256, 2, seed=2)
    P.build(sweeps=2, local_corr=L.LC_BOTH, coarse_n=16, method=L.METHOD_PCG, variant=L.VARIANT_GRID_TAIL)
    f = torch_cuda.as_tensor(rng.standard_normal(P.volume_nodes().shape[0]))
    with pytest.raises(L.HDGError) as ei:
        solve_batch([P], [f], tol=1e-8)
    assert ei.value.status == L.HDG_ERR_UNSUPPORTED
    P.close()
