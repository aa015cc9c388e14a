"""CPU checks of the C ABI: the built library loads, exports every entry point
that include/hdg.h declares, and its host-side reference data (no GPU call)
matches closed forms."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hdg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hdg_[a-z_]+)\s*\(", src)))


def _lib():
    from paper_1811_09909_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libhdg.so not built")
    return L


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["hdg_setup", "hdg_mg_build", "hdg_vcycle", "hdg_solve", "hdg_reconstruct", "hdg_adjoint",
                 "hdg_destroy"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(L.EXPORTS) == _declared()


def test_reference_nodes_host_side():
    L = _lib()
    lib = L.load()
    for k in range(1, 7):
        gll = (ctypes.c_double * (k + 1))()
        gau = (ctypes.c_double * (k + 2))()
        assert lib.hdg_reference_nodes(k, gll, gau) == 0
        g = np.array(list(gll))
        x = np.array(list(gau))
        from numpy.polynomial import legendre
        xr, _ = legendre.leggauss(k + 2)
        assert np.allclose(x, (xr + 1) / 2, atol=1e-15)
        assert g[0] == 0.0 and g[-1] == 1.0 and np.all(np.diff(g) > 0)
        if k == 2:
            assert np.allclose(g, [0, 0.5, 1], atol=1e-15)
        if k == 3:
            assert np.allclose(g[1], 0.5 - np.sqrt(5) / 10, atol=1e-15)
    assert lib.hdg_reference_nodes(0, gll, gau) == L.HDG_ERR_INVALID_ARG


def test_invalid_arguments_rejected_before_any_device_work():
    L = _lib()
    lib = L.load()
    h = ctypes.c_void_p()
    mesh = L.Mesh(4, 8)
    kap = (ctypes.c_double * 1)(1.0)
    assert lib.hdg_setup(ctypes.byref(mesh), 2, 1.0, kap, 0, 1, None, ctypes.byref(h)) == L.HDG_ERR_UNSUPPORTED
    mesh = L.Mesh(2, 8)
    assert lib.hdg_setup(ctypes.byref(mesh), 9, 1.0, kap, 0, 1, None, ctypes.byref(h)) == L.HDG_ERR_UNSUPPORTED
    assert lib.hdg_setup(ctypes.byref(mesh), 2, -1.0, kap, 0, 1, None, ctypes.byref(h)) == L.HDG_ERR_INVALID_ARG
    assert lib.hdg_setup(ctypes.byref(mesh), 2, 1.0, None, 0, 1, None, ctypes.byref(h)) == L.HDG_ERR_INVALID_ARG
    assert lib.hdg_solve(None, None, 0, None, 1, 1e-10, None, None) == L.HDG_ERR_INVALID_ARG
    assert lib.hdg_status_string(L.HDG_ERR_NOT_CONVERGED) == b"not converged"


def test_product_path_has_no_oracle_or_cpu_fallback():
    """The package never imports the oracle; a missing library raises."""
    pkg = os.path.join(ROOT, "paper_1811_09909_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert not re.search(r"^\s*(from|import)\s+oracle", src, flags=re.M), fn
    from paper_1811_09909_amd import _lib as L
    saved = L.LIB_PATH, L._lib
    try:
        L.LIB_PATH, L._lib = "/nonexistent/libhdg.so", None
        with pytest.raises(RuntimeError):
            L.load()
    finally:
        L.LIB_PATH, L._lib = saved


@pytest.mark.parametrize("nx,k,strategy", [(8, 1, 1), (16, 2, 1), (16, 3, 2), (32, 1, 2), (45, 2, 1)])
def test_unstructured_hierarchy_host_side(nx, k, strategy):
    """The library's host-side agglomeration (seed points, four-way splits,
    macro-edge chains) gives the oracle's level sizes on the box with holes."""
    _lib()
    from oracle import unstructured as U
    from paper_1811_09909_amd import inputs
    from paper_1811_09909_amd.hdg import umesh_levels
    w = inputs.unstructured2d(nx, k, strategy=strategy)
    m = U.TriMesh(w.vertices, w.triangles)
    parts = U.agglomerate(m, w.seeds, w.hlevels)
    sizes = [m.nface * (k + 1)] + ([m.nface * 2] if k > 1 else [])
    fine, cell_of = U.triangle_faces(m), np.arange(m.nel)
    for p in reversed(parts):
        co = np.zeros(cell_of.max() + 1, dtype=np.int64)
        co[cell_of] = p
        _, _, _, fine = U.macro_faces(fine, co)
        cell_of = p
        sizes.append(2 * fine.nface)
    assert umesh_levels(w.vertices, w.triangles, k, w.seeds, w.hlevels) == sizes
