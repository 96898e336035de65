"""The C-ABI library loads and exports every function include/dg_sipdg.h
declares (no device work: runs without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dg_sipdg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dg_mesh_create", "dg_mesh_destroy", "helmholtz_apply", "helmholtz_solve",
                     "poisson_solve", "helmholtz_solve_batched", "dg_server_create",
                     "dg_server_submit", "dg_server_poll", "dg_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import ctypes
    from paper_2112_04167_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("HIP library not built (run __graft_entry__.build())")
    L = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_argument_errors_without_device():
    # argument validation happens on the host before any device call
    import ctypes
    from paper_2112_04167_amd import binding
    L = binding.lib()
    h = ctypes.c_void_p()
    v = (ctypes.c_double * 3)(0.0, 0.5, 1.0)
    bc = (ctypes.c_int * 3)(0, 0, 0)
    rc = L.dg_mesh_create(2, 2, 2, 2, v, v, v, bc, None, ctypes.byref(h))   # P=2 unsupported
    assert rc == binding.DG_ERR_ARG
    assert "P" in binding.last_error()
    bad = (ctypes.c_double * 3)(0.0, 0.7, 0.5)
    rc = L.dg_mesh_create(2, 2, 2, 4, bad, v, v, bc, None, ctypes.byref(h))
    assert rc == binding.DG_ERR_ARG
    bcx = (ctypes.c_int * 3)(0, 7, 0)
    rc = L.dg_mesh_create(2, 2, 2, 4, v, v, v, bcx, None, ctypes.byref(h))
    assert rc == binding.DG_ERR_ARG
