"""hdg_rhs_noalloc (the allocation-free form of hdg_rhs, for callers that
cannot allocate device memory) against hdg_rhs, through the C ABI.

Both run the same kernels in the same order, so their outputs agree bit for
bit; two calls in a row (the second on a smaller problem, over the staging
the first left behind), with Dirichlet data and in load form; a problem
beyond the fixed staging is refused; the call leaves device free memory
unchanged."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1811_09909_amd import inputs

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


def _problem(torch, n, k, seed):
    from paper_1811_09909_amd.hdg import Problem
    wl = inputs.diffusion2d(n, k, 1e-3, 1e3, seed=seed)
    P = Problem(2, n, k, torch.as_tensor(wl.kappa), tau=1.0, store_recovery=False)
    return P, torch.as_tensor(wl.f, device=P.device).contiguous()


def test_rhs_noalloc_matches_rhs(torch_cuda):
    from paper_1811_09909_amd import _lib as L
    torch = torch_cuda
    rng = np.random.default_rng(21)
    for n, k, seed in ((128, 4, 1), (32, 3, 2)):  # second call: smaller input
        P, f = _problem(torch, n, k, seed)
        say(f"[rhs_noalloc] n={n} k={k}")
        gd = torch.as_tensor(rng.standard_normal(4 * n * (k + 1)), device=P.device).contiguous()
        for kind, src, gdir in ((L.RHS_F_NODAL, f, None), (L.RHS_F_NODAL, f, gd),
                                (L.RHS_F_LOAD, P.mass_apply(f).contiguous(), None)):
            ref = P.rhs(src, kind=kind, gdir=gdir)
            g = torch.full((P.nlam,), float("nan"), dtype=torch.float64, device=P.device)
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            P.rhs_noalloc(src, g, kind=kind, gdir=gdir)
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
            diff = float((g - ref).abs().max())
            say(f"  kind={kind} dirichlet={gdir is not None}: max diff vs hdg_rhs {diff:.1e}, "
                f"free memory change {free1 - free0} B")
            assert diff == 0.0
            assert free1 == free0
        P.close()


def test_rhs_noalloc_refuses_beyond_its_staging(torch_cuda):
    """512 x 512 elements at k = 4 need 11.8 Mi doubles of staging: refused
    with HDG_ERR_UNSUPPORTED, output untouched."""
    from paper_1811_09909_amd import _lib as L
    torch = torch_cuda
    P, f = _problem(torch, 512, 4, 3)
    g = torch.zeros(P.nlam, dtype=torch.float64, device=P.device)
    st = P.lib.hdg_rhs_noalloc(P.h, ctypes.c_void_p(f.data_ptr()), L.RHS_F_NODAL, None,
                               ctypes.c_void_p(g.data_ptr()))
    say(f"[rhs_noalloc 512^2 k=4] status {st}")
    assert st == L.HDG_ERR_UNSUPPORTED
    assert float(g.abs().max()) == 0.0
    P.close()
