"""ctypes declarations of the C ABI in include/hdg.h (marshalling only)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# HDG_LIBRARY selects another build of the same library (a variant build)
LIB_PATH = os.environ.get("HDG_LIBRARY", os.path.join(_HERE, "_lib", "libhdg.so"))

HDG_OK, HDG_ERR_INVALID_ARG, HDG_ERR_UNSUPPORTED, HDG_ERR_STATE = 0, -1, -2, -3
HDG_ERR_NOT_CONVERGED, HDG_ERR_BREAKDOWN, HDG_ERR_DEVICE = -4, -5, -6
KAPPA_PER_ELEMENT, KAPPA_AT_QP = 0, 1
FP64, FP32, MIXED = 0, 1, 1
MIXED_CYCLE = 2  # hdg_vcycle: the mixed solve's cycle on FP64 vectors
LC_NONE, LC_PRE, LC_POST, LC_BOTH = 0, 1, 2, 3
METHOD_MG, METHOD_PCG, METHOD_GMRES = 0, 1, 2
RHS_F_NODAL, RHS_F_LOAD, RHS_TRACE = 0, 1, 2
Q_NT, Q_NLAMBDA, Q_NLEVELS, Q_NV, Q_NQ = 0, 1, 2, 3, 4
Q_LEVEL_NLAMBDA, Q_LEVEL_N, Q_LEVEL_NE, Q_DEVICE_BYTES = 100, 200, 300, 400
Q_GRID_TAIL = 401

EXPORTS = [
    "hdg_default_opts", "hdg_setup", "hdg_update_kappa", "hdg_mg_build", "hdg_vcycle", "hdg_rhs", "hdg_solve",
    "hdg_reconstruct", "hdg_adjoint", "hdg_mass_apply", "hdg_level_apply", "hdg_level_smooth",
    "hdg_level_export", "hdg_query", "hdg_reference_nodes", "hdg_destroy", "hdg_status_string",
    "hdg_profile_begin", "hdg_profile_read", "hdg_solve_batch", "hdg_autotune", "hdg_rhs_noalloc",
    "hdg_setup_scheme", "hdg_setup_multi", "hdg_setup_unstructured", "hdg_umesh_levels",
]


MAX_NRHS = 64  # HDG_MAX_NRHS


class Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int)]


class UMesh(ctypes.Structure):
    """hdg_umesh: host vertex, triangle and seed arrays, agglomeration levels."""
    _fields_ = [("nvert", ctypes.c_long), ("xy", ctypes.c_void_p), ("ntri", ctypes.c_long),
                ("tri", ctypes.c_void_p), ("nseeds", ctypes.c_int), ("seeds", ctypes.c_void_p),
                ("hlevels", ctypes.c_int)]


class Opts(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int), ("growth", ctypes.c_int), ("omega", ctypes.c_double),
                ("local_corr", ctypes.c_int), ("precision", ctypes.c_int), ("method", ctypes.c_int),
                ("max_it", ctypes.c_int), ("restart", ctypes.c_int), ("coarse_n", ctypes.c_int),
                ("nrhs", ctypes.c_int), ("refine_red", ctypes.c_double), ("variant", ctypes.c_int),
                ("smoother", ctypes.c_int)]


# hdg_mg_opts.variant bits (HDG_VARIANT_*)
VARIANT_NO_GRAPH, VARIANT_NO_FUSE, VARIANT_NO_TAIL, VARIANT_NO_PACK, VARIANT_NO_STRIP = 1, 2, 4, 8, 16
VARIANT_FP32_VECTORS, VARIANT_FP64_VECTORS = 32, 64
VARIANT_LANES1, VARIANT_LANES4 = 128, 256
VARIANT_GRID_TAIL = 512
PROF_F32OPS = 14  # hdg_profile_read: kernel = 14 + mode for FP64 vectors over FP32 operator blocks
PROF_XFER = 21    # hdg_profile_read: kernel = 21 + 2 t + precision, t = 0 hpre, 1 hsum, 2 hpost, 3 p-prolongation
XFER_KINDS = ("hpre", "hsum", "hpost", "prolong_p")
OPT_FIELDS = ("sweeps", "growth", "omega", "local_corr", "precision", "method", "max_it", "restart", "coarse_n",
              "nrhs", "refine_red", "variant", "smoother")
SMOOTHER_BLOCK_JACOBI, SMOOTHER_JACOBI, SMOOTHER_CHEBYSHEV, SMOOTHER_LUSGS = 0, 1, 2, 3
# HDG_SCHEME_*: HDG, and the hybridized IPDG family (eq. IPG_H, s_f = 1, 0, -1)
SCHEME_HDG, SCHEME_SIPG, SCHEME_IIPG, SCHEME_NIPG, SCHEME_RT = 0, 1, 2, 3, 4
SCHEMES = {"hdg": SCHEME_HDG, "sipg": SCHEME_SIPG, "iipg": SCHEME_IIPG, "nipg": SCHEME_NIPG, "rt": SCHEME_RT}
SCHEME_TAU_KAPPA = 16  # or-ed into the scheme: element T stabilized with tau * kappa_T


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("relres", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
                ("n_levels", ctypes.c_int), ("outer_iters", ctypes.c_int), ("t_setup_ms", ctypes.c_double),
                ("t_build_ms", ctypes.c_double)]

    def as_dict(self):
        return {"iters": self.iters, "relres": self.relres, "t_solve_ms": self.t_solve_ms,
                "n_levels": self.n_levels, "outer_iters": self.outer_iters, "t_setup_ms": self.t_setup_ms,
                "t_build_ms": self.t_build_ms}


_lib = None
P = ctypes.c_void_p
I = ctypes.c_int
D = ctypes.c_double


def load():
    """Open libhdg.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run python -m paper_1811_09909_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "hdg_default_opts": (None, [ctypes.POINTER(Opts)]),
        "hdg_setup": (I, [ctypes.POINTER(Mesh), I, D, P, I, I, P, ctypes.POINTER(P)]),
        "hdg_setup_scheme": (I, [ctypes.POINTER(Mesh), I, D, P, I, I, I, P, ctypes.POINTER(P)]),
        "hdg_setup_multi": (I, [ctypes.POINTER(Mesh), I, D, P, I, P, I, I, P, ctypes.POINTER(P)]),
        "hdg_setup_unstructured": (I, [ctypes.POINTER(UMesh), I, D, P, I, P, ctypes.POINTER(P)]),
        "hdg_umesh_levels": (I, [ctypes.POINTER(UMesh), I, ctypes.POINTER(ctypes.c_longlong), I,
                                 ctypes.POINTER(I)]),
        "hdg_update_kappa": (I, [P, P, I]),
        "hdg_mg_build": (I, [P, ctypes.POINTER(Opts)]),
        "hdg_vcycle": (I, [P, P, P, I, I]),
        "hdg_rhs": (I, [P, P, I, P, P]),
        "hdg_rhs_noalloc": (I, [P, P, I, P, P]),
        "hdg_solve": (I, [P, P, I, P, I, D, P, ctypes.POINTER(Info)]),
        "hdg_solve_batch": (I, [I, P, P, I, P, D, P, ctypes.POINTER(Info), I]),
        "hdg_autotune": (I, [P, ctypes.POINTER(Opts), I, ctypes.POINTER(Opts), ctypes.POINTER(D)]),
        "hdg_reconstruct": (I, [P, P, P, I, P, P, P]),
        "hdg_adjoint": (I, [P, P, P, D, P, ctypes.POINTER(Info)]),
        "hdg_mass_apply": (I, [P, P, P]),
        "hdg_level_apply": (I, [P, I, P, P, I]),
        "hdg_level_smooth": (I, [P, I, P, P, I, I]),
        "hdg_level_export": (I, [P, I, P]),
        "hdg_query": (I, [P, I, ctypes.POINTER(ctypes.c_longlong)]),
        "hdg_reference_nodes": (I, [I, ctypes.POINTER(D), ctypes.POINTER(D)]),
        "hdg_destroy": (I, [P]),
        "hdg_profile_begin": (I, [P]),
        "hdg_profile_read": (I, [P, I, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(D), ctypes.POINTER(D)]),
        "hdg_status_string": (ctypes.c_char_p, [I]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class HDGError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = load().hdg_status_string(status).decode()
        super().__init__(f"{where}: {msg} ({status})")


def check(status, where, allow=()):
    if status != HDG_OK and status not in allow:
        raise HDGError(status, where)
    return status
