"""Thin torch binding of the HIP library (include/hdg.h).

Only argument marshalling happens here: torch provides device memory and
the stream, every step of the solver runs in the library's kernels.  The
library must be built (``python -m paper_1811_09909_amd.build``); without
it, or without a GPU, every call raises.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L


def _vp(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype, device):
    return torch.as_tensor(t, dtype=dtype, device=device).contiguous()


class Problem:
    """One trace problem on the unit box (d = 2 or 3, n^d elements, Q^k).

    ``scheme``: "hdg" (eqs. HDG, HDG_flux) or one of the hybridized IPDG
    family "sipg", "iipg", "nipg" (eq. IPG_H, s_f = 1, 0, -1), or "rt"
    (hybridized Raviart-Thomas, 2D).  ``scheme_of_element``: one scheme name
    per element instead (multinumerics; "sipg", "iipg", "nipg" or "rt").
    ``tau_kappa``: element T is stabilized with tau * kappa_T (kappa per
    element).
    ``kappa``: per element [n^d] or, for HDG, at the (k+2)^d Gauss points of
    every element [n^d, (k+2)^d] (then ``kappa_kind='qp'``)."""

    def __init__(self, d, n, k, kappa, tau=1.0, kappa_kind="element", store_recovery=True, device="cuda",
                 scheme="hdg", tau_kappa=False, scheme_of_element=None):
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the HDG library needs a GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        self.d, self.n, self.k, self.tau = d, n, k, float(tau)
        self.kind = L.KAPPA_AT_QP if kappa_kind == "qp" else L.KAPPA_PER_ELEMENT
        if scheme not in L.SCHEMES:
            raise ValueError(f"unknown scheme {scheme}")
        self.scheme = scheme
        kap = _dev(kappa, torch.float64, self.device)
        self.stream = torch.cuda.current_stream(self.device)
        mesh = L.Mesh(d, n)
        h = ctypes.c_void_p()
        if scheme_of_element is not None:
            codes = torch.tensor([L.SCHEMES[c] for c in scheme_of_element], dtype=torch.int32, device=self.device)
            self.scheme = "multi"
            L.check(self.lib.hdg_setup_multi(ctypes.byref(mesh), k, self.tau, _vp(kap), self.kind, _vp(codes),
                                             L.SCHEME_TAU_KAPPA if tau_kappa else 0, 1 if store_recovery else 0,
                                             ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                    "hdg_setup_multi")
        else:
            code = L.SCHEMES[scheme] | (L.SCHEME_TAU_KAPPA if tau_kappa else 0)
            L.check(self.lib.hdg_setup_scheme(ctypes.byref(mesh), k, self.tau, _vp(kap), self.kind, code,
                                              1 if store_recovery else 0, ctypes.c_void_p(self.stream.cuda_stream),
                                              ctypes.byref(h)), "hdg_setup_scheme")
        self.h = h
        self.unstructured = False
        self.nT = self.query(L.Q_NT)
        self.nlam = self.query(L.Q_NLAMBDA)
        self.nv = self.query(L.Q_NV)
        self.nq = self.query(L.Q_NQ)
        self.built = False
        self.version = 0  # bumped by every update_kappa / build: operator state of the handle

    @classmethod
    def unstructured(cls, vertices, triangles, k, kappa, seeds, hlevels, tau=1.0, device="cuda", scheme="hdg"):
        """HDG (or ``scheme`` "sipg", "iipg", "nipg") on an unstructured
        triangle mesh with the seed-point agglomeration hierarchy
        (``hdg_setup_unstructured``): host vertex, triangle and seed arrays,
        kappa one value per triangle."""
        self = cls.__new__(cls)
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the HDG library needs a GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        self.d, self.n, self.k, self.tau = 2, 0, k, float(tau)
        self.kind = L.KAPPA_PER_ELEMENT
        if scheme not in L.SCHEMES:
            raise ValueError(f"unknown scheme {scheme}")
        self.scheme = scheme
        xy = np.ascontiguousarray(vertices, dtype=np.float64)
        tri = np.ascontiguousarray(triangles, dtype=np.int32)
        sd = np.ascontiguousarray(seeds, dtype=np.float64)
        self._host = (xy, tri, sd)
        mesh = L.UMesh(len(xy), xy.ctypes.data, len(tri), tri.ctypes.data, len(sd), sd.ctypes.data, int(hlevels))
        kap = _dev(kappa, torch.float64, self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        L.check(self.lib.hdg_setup_unstructured(ctypes.byref(mesh), k, self.tau, _vp(kap), L.SCHEMES[scheme],
                                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                "hdg_setup_unstructured")
        self.h = h
        self.unstructured = True
        self.nT = self.query(L.Q_NT)
        self.nlam = self.query(L.Q_NLAMBDA)
        self.nv = self.query(L.Q_NV)
        self.nq = self.query(L.Q_NQ)
        self.built = False
        self.version = 0
        return self

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            self.lib.hdg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self, what):
        out = ctypes.c_longlong()
        L.check(self.lib.hdg_query(self.h, what, ctypes.byref(out)), "hdg_query")
        return out.value

    def update_kappa(self, kappa):
        kap = _dev(kappa, torch.float64, self.device)
        L.check(self.lib.hdg_update_kappa(self.h, _vp(kap), self.kind), "hdg_update_kappa")
        self.version += 1
        self.built = False

    def build(self, sweeps=2, growth=1, omega=1.0, local_corr=L.LC_PRE, precision=L.FP64, method=L.METHOD_MG,
              max_it=200, restart=0, coarse_n=2, nrhs=1, refine_red=0.0, variant=0, smoother=0):
        o = L.Opts(sweeps, growth, omega, local_corr, precision, method, max_it, restart, coarse_n, nrhs,
                   refine_red, variant, smoother)
        L.check(self.lib.hdg_mg_build(self.h, ctypes.byref(o)), "hdg_mg_build")
        self.version += 1
        self.built = True
        self.opts = o
        self.n_levels = self.query(L.Q_NLEVELS)
        return self

    def level_sizes(self):
        return [self.query(L.Q_LEVEL_NLAMBDA + i) for i in range(self.n_levels)]

    # -- operators -----------------------------------------------------------
    def rhs(self, f, kind=L.RHS_F_NODAL, gdir=None):
        f = _dev(f, torch.float64, self.device)
        gd = None if gdir is None else _dev(gdir, torch.float64, self.device)
        g = torch.empty(self.nlam, dtype=torch.float64, device=self.device)
        L.check(self.lib.hdg_rhs(self.h, _vp(f), kind, _vp(gd), _vp(g)), "hdg_rhs")
        return g

    def rhs_noalloc(self, f, g, kind=L.RHS_F_NODAL, gdir=None):
        """hdg_rhs_noalloc into the caller's g (no allocation in the library;
        f, g and gdir must already be contiguous float64 device tensors)."""
        L.check(self.lib.hdg_rhs_noalloc(self.h, _vp(f), kind, _vp(gdir), _vp(g)), "hdg_rhs_noalloc")
        return g

    def solve(self, rhs, kind=L.RHS_F_NODAL, tol=1e-10, lam0=None, gdir=None, nrhs=1, allow_not_converged=False):
        rhs = _dev(rhs, torch.float64, self.device)
        gd = None if gdir is None else _dev(gdir, torch.float64, self.device)
        lam = (torch.zeros(nrhs * self.nlam, dtype=torch.float64, device=self.device) if lam0 is None
               else _dev(lam0, torch.float64, self.device).clone().reshape(-1))
        info = L.Info()
        allow = (L.HDG_ERR_NOT_CONVERGED,) if allow_not_converged else ()
        st = L.check(self.lib.hdg_solve(self.h, _vp(rhs), kind, _vp(gd), nrhs, float(tol), _vp(lam),
                                        ctypes.byref(info)), "hdg_solve", allow)
        return lam, dict(info.as_dict(), status=st)

    def autotune(self, nrhs, **base):
        """Pick the fastest coarsest grid and right-hand-side group size for
        `nrhs` right-hand sides on top of the build options `base` (see
        hdg_autotune); leaves the handle built with them."""
        defaults = dict(sweeps=2, growth=1, omega=1.0, local_corr=L.LC_PRE, precision=L.FP64, method=L.METHOD_MG,
                        max_it=200, restart=0, coarse_n=2, nrhs=1, refine_red=0.0, variant=0, smoother=0)
        defaults.update(base)
        o = L.Opts(*[defaults[k] for k in L.OPT_FIELDS])
        best = L.Opts()
        us = ctypes.c_double()
        L.check(self.lib.hdg_autotune(self.h, ctypes.byref(o), int(nrhs), ctypes.byref(best), ctypes.byref(us)),
                "hdg_autotune")
        self.version += 1
        self.built = True
        self.opts = best
        self.n_levels = self.query(L.Q_NLEVELS)
        return {"coarse_n": best.coarse_n, "nrhs": best.nrhs, "variant": best.variant, "us_per_rhs_iter": us.value}

    def vcycle(self, r, precision=L.FP64):
        dt = torch.float32 if precision == L.FP32 else torch.float64
        r = _dev(r, dt, self.device)
        e = torch.empty_like(r)
        L.check(self.lib.hdg_vcycle(self.h, _vp(r), _vp(e), precision, r.numel() // max(self.nlam, 1)),
                "hdg_vcycle")
        return e

    def reconstruct(self, lam, f, kind=L.RHS_F_NODAL, gdir=None):
        lam = _dev(lam, torch.float64, self.device)
        f = _dev(f, torch.float64, self.device)
        gd = None if gdir is None else _dev(gdir, torch.float64, self.device)
        u = torch.empty(self.nT, self.nv, dtype=torch.float64, device=self.device)
        q = torch.empty(self.nT, self.d, self.nv, dtype=torch.float64, device=self.device)
        L.check(self.lib.hdg_reconstruct(self.h, _vp(lam), _vp(f), kind, _vp(gd), _vp(u), _vp(q)),
                "hdg_reconstruct")
        return u, q

    def adjoint(self, dJdu_load, q_fwd, tol=1e-10):
        j = _dev(dJdu_load, torch.float64, self.device)
        q = _dev(q_fwd, torch.float64, self.device)
        grad = torch.empty(self.nT, dtype=torch.float64, device=self.device)
        info = L.Info()
        L.check(self.lib.hdg_adjoint(self.h, _vp(j), _vp(q), float(tol), _vp(grad), ctypes.byref(info)),
                "hdg_adjoint")
        return grad, info.as_dict()

    def mass_apply(self, u):
        u = _dev(u, torch.float64, self.device)
        out = torch.empty_like(u)
        L.check(self.lib.hdg_mass_apply(self.h, _vp(u), _vp(out)), "hdg_mass_apply")
        return out

    def level_apply(self, level, x, precision=L.FP64):
        dt = torch.float64 if precision == L.FP64 else torch.float32
        x = _dev(x, dt, self.device)
        y = torch.empty_like(x)
        L.check(self.lib.hdg_level_apply(self.h, level, _vp(x), _vp(y), precision), "hdg_level_apply")
        return y

    def level_smooth(self, level, r, sweeps, precision=L.FP64):
        dt = torch.float64 if precision == L.FP64 else torch.float32
        r = _dev(r, dt, self.device)
        e = torch.empty_like(r)
        L.check(self.lib.hdg_level_smooth(self.h, level, _vp(r), _vp(e), sweeps, precision), "hdg_level_smooth")
        return e

    def level_export(self, level):
        if self.unstructured:  # triangle levels: P^k maps, then P^1 maps (k > 1)
            nl = 3 * (self.k + 1) if level == 0 else 6
            out = torch.empty(self.nT, nl, nl, dtype=torch.float64, device=self.device)
            L.check(self.lib.hdg_level_export(self.h, level, _vp(out)), "hdg_level_export")
            return out
        if level == 0:
            nel, nl = self.nT, 2 * self.d * (self.k + 1) ** (self.d - 1)
        else:
            n = self.query(L.Q_LEVEL_N + level)
            ne = self.query(L.Q_LEVEL_NE + level)
            nel, nl = n ** self.d, 2 * self.d * ne
        out = torch.empty(nel, nl, nl, dtype=torch.float64, device=self.device)
        L.check(self.lib.hdg_level_export(self.h, level, _vp(out)), "hdg_level_export")
        return out

    # -- inspection timing ---------------------------------------------------
    def profile_begin(self):
        L.check(self.lib.hdg_profile_begin(self.h), "hdg_profile_begin")

    def profile_read(self, mode, precision, transfer=None):
        """precision FP64 / FP32, or MIXED_CYCLE for the finest level's FP64
        vectors over FP32 operator blocks; transfer = "hpre", "hsum", "hpost"
        or "prolong_p" reads that transfer kernel instead of trace mode `mode`."""
        n = ctypes.c_longlong()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        if transfer is not None:
            kernel = L.PROF_XFER + 2 * L.XFER_KINDS.index(transfer) + precision
        else:
            kernel = L.PROF_F32OPS + mode if precision == L.MIXED_CYCLE else 2 * mode + precision
        L.check(self.lib.hdg_profile_read(self.h, kernel, ctypes.byref(n), ctypes.byref(ms),
                                          ctypes.byref(by)), "hdg_profile_read")
        return {"launches": n.value, "total_ms": ms.value, "bytes_per_launch": by.value}

    # -- geometry for evaluating sources and coefficients --------------------
    def reference_nodes(self):
        gll = (ctypes.c_double * (self.k + 1))()
        gau = (ctypes.c_double * (self.k + 2))()
        L.check(self.lib.hdg_reference_nodes(self.k, gll, gau), "hdg_reference_nodes")
        return torch.tensor(list(gll), dtype=torch.float64), torch.tensor(list(gau), dtype=torch.float64)

    def _tensor_points(self, pts1d):
        d, n = self.d, self.n
        m = len(pts1d)
        idx = torch.arange(m ** d)
        digits = torch.stack([(idx // m ** a) % m for a in range(d)], 1)
        ref = pts1d[digits]
        el = torch.arange(n ** d)
        ec = torch.stack([(el // n ** a) % n for a in range(d)], 1).to(torch.float64)
        return (ec[:, None, :] + ref[None]) / n

    def volume_nodes(self):
        """[N_T, (k+1)^d, d] coordinates of the GLL nodes (host tensor)."""
        return self._tensor_points(self.reference_nodes()[0])

    def volume_qpoints(self):
        """[N_T, (k+2)^d, d] coordinates of the Gauss points (host tensor)."""
        return self._tensor_points(self.reference_nodes()[1])


def umesh_levels(vertices, triangles, k, seeds, hlevels):
    """Trace unknowns per level of the unstructured hierarchy (host only,
    ``hdg_umesh_levels``)."""
    lib = L.load()
    xy = np.ascontiguousarray(vertices, dtype=np.float64)
    tri = np.ascontiguousarray(triangles, dtype=np.int32)
    sd = np.ascontiguousarray(seeds, dtype=np.float64)
    mesh = L.UMesh(len(xy), xy.ctypes.data, len(tri), tri.ctypes.data, len(sd), sd.ctypes.data, int(hlevels))
    sizes = (ctypes.c_longlong * 32)()
    n = ctypes.c_int()
    L.check(lib.hdg_umesh_levels(ctypes.byref(mesh), int(k), sizes, 32, ctypes.byref(n)), "hdg_umesh_levels")
    return [int(sizes[i]) for i in range(n.value)]


def solve_batch(problems, rhs, tol=1e-10, kind=L.RHS_F_NODAL, nstreams=0):
    """Solve problem i for its right-hand sides rhs[i] ([nrhs_i, ...] nodal
    sources, or trace vectors for kind=RHS_TRACE) with hdg_solve_batch: all
    problems through one batch graph (nstreams <= 0, PCG builds), or
    concurrently on `nstreams` streams.  Returns the list of solutions
    [nrhs_i, N_lambda_i] and the list of solve infos."""
    n = len(problems)
    rhs_t = [_dev(r, torch.float64, p.device) for p, r in zip(problems, rhs)]
    nr = [(r.numel() // (p.nlam if kind == L.RHS_TRACE else p.nT * p.nv)) for p, r in zip(problems, rhs_t)]
    lam = [torch.zeros(k * p.nlam, dtype=torch.float64, device=p.device) for p, k in zip(problems, nr)]
    handles = (ctypes.c_void_p * n)(*[p.h.value for p in problems])
    rp = (ctypes.c_void_p * n)(*[r.data_ptr() for r in rhs_t])
    lp = (ctypes.c_void_p * n)(*[x.data_ptr() for x in lam])
    nrh = (ctypes.c_int * n)(*nr)
    infos = (L.Info * n)()
    lib = problems[0].lib
    L.check(lib.hdg_solve_batch(n, handles, rp, kind, nrh, float(tol), lp, infos, int(nstreams)), "hdg_solve_batch")
    out = [x.reshape(k, -1) for x, k in zip(lam, nr)]
    return out, [i.as_dict() for i in infos]


class HDGMass(torch.autograd.Function):
    """u -> M u element by element (the volume mass matrix); symmetric, so
    the backward pass applies M again."""

    @staticmethod
    def forward(ctx, u, problem):  # noqa: D102
        ctx.problem = problem
        return problem.mass_apply(u.detach())

    @staticmethod
    def backward(ctx, g):  # noqa: D102
        return ctx.problem.mass_apply(g.contiguous()), None


class HDGSolve(torch.autograd.Function):
    """U(theta): nodal u of the HDG solution for kappa_T = exp(theta_T).

    backward uses the library's adjoint solve (same operator and V-cycle)
    and returns dL/dtheta = -(q*)^T A_T q per element.  The adjoint needs the
    handle's operator at this theta: if the handle was changed after this
    forward pass (another forward at another theta, a rebuild), backward
    re-forms the operator at the saved theta and re-solves first."""

    @staticmethod
    def forward(ctx, theta, problem, f, tol, build_kw):  # noqa: D102
        problem.update_kappa(torch.exp(theta.detach()))
        problem.build(**build_kw)
        lam, info = problem.solve(f, tol=tol)
        u, q = problem.reconstruct(lam, f)
        ctx.problem, ctx.tol, ctx.f, ctx.build_kw = problem, tol, f, build_kw
        ctx.version = problem.version
        ctx.save_for_backward(q, theta.detach())
        return u

    @staticmethod
    def backward(ctx, gu):
        q, theta = ctx.saved_tensors
        P = ctx.problem
        if P.version != ctx.version:
            P.update_kappa(torch.exp(theta))
            P.build(**ctx.build_kw)
            lam, _ = P.solve(ctx.f, tol=ctx.tol)
            _, q = P.reconstruct(lam, ctx.f)
            ctx.version = P.version
        grad, _ = P.adjoint(gu.contiguous(), q, ctx.tol)
        return grad, None, None, None, None
