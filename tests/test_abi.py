"""CPU checks of the C-ABI boundary: the built library loads and exports every symbol
include/gqd.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gqd.h")
LIB = os.path.join(ROOT, "paper_1902_04661_amd", "libgqd.so")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:gqd_status|void|const char\*)\s+(gqd_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["gqd_create", "gqd_destroy", "gqd_set_surfaces", "gqd_apply_H",
                     "gqd_implicit_step", "gqd_propagate", "gqd_adjoint", "gqd_diag",
                     "gqd_inner", "gqd_workspace_size", "gqd_set_workspace", "gqd_last_error"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgqd.so not built (run python -m paper_1902_04661_amd.build)")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgqd.so not built (run python -m paper_1902_04661_amd.build)")
def test_binding_lists_the_same_symbols():
    from paper_1902_04661_amd import gqd
    assert sorted(gqd.exported_symbols()) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgqd.so not built (run python -m paper_1902_04661_amd.build)")
def test_invalid_arguments_fail_without_a_gpu():
    # argument validation happens before any device work
    from paper_1902_04661_amd import gqd
    lib = gqd.load_library()
    h = ctypes.c_void_p()
    assert lib.gqd_create(ctypes.byref(h), None) == -1
    assert b"NULL" in lib.gqd_last_error()
    assert lib.gqd_set_wait_limit(None, 1) == -1
    assert b"NULL" in lib.gqd_last_error()
    n = (ctypes.c_int * 1)(300)
    qmin = (ctypes.c_double * 1)(0.0)
    qmax = (ctypes.c_double * 1)(1.0)
    mass = (ctypes.c_double * 1)(1.0)
    desc = gqd._GridDesc(1, 2, 1, n, qmin, qmax, mass)
    assert lib.gqd_create(ctypes.byref(h), ctypes.byref(desc)) == -5   # unsupported size
    n[0] = 256
    desc = gqd._GridDesc(1, 2, 0, n, qmin, qmax, mass)
    assert lib.gqd_create(ctypes.byref(h), ctypes.byref(desc)) == -1   # empty batch
    assert b"batch" in lib.gqd_last_error()
    n[0] = 300
    desc = gqd._GridDesc(3, 2, 1, n, qmin, qmax, mass)
    assert lib.gqd_create(ctypes.byref(h), ctypes.byref(desc)) == -5   # dims
    # 2D: n x n with n in {64, 128, 256, 512}, two masses
    n2 = (ctypes.c_int * 2)(128, 256)
    q0 = (ctypes.c_double * 2)(0.0, 0.0)
    q1 = (ctypes.c_double * 2)(1.0, 1.0)
    m2 = (ctypes.c_double * 2)(1.0, 1.0)
    desc = gqd._GridDesc(2, 2, 1, n2, q0, q1, m2)
    assert lib.gqd_create(ctypes.byref(h), ctypes.byref(desc)) == -5   # not square
    n2 = (ctypes.c_int * 2)(96, 96)
    desc = gqd._GridDesc(2, 2, 1, n2, q0, q1, m2)
    assert lib.gqd_create(ctypes.byref(h), ctypes.byref(desc)) == -5   # unsupported n
    n2 = (ctypes.c_int * 2)(64, 64)
    m2 = (ctypes.c_double * 2)(1.0, -1.0)
    desc = gqd._GridDesc(2, 2, 1, n2, q0, q1, m2)
    assert lib.gqd_create(ctypes.byref(h), ctypes.byref(desc)) == -1   # mass of the second axis


def header_struct_fields(name):
    """Member names, in order, of `typedef struct { ... } name;` in the header."""
    text = open(HEADER).read()
    end = re.search(r"\}\s*" + name + r";", text)
    assert end, name
    start = text.rfind("typedef struct {", 0, end.start())
    body = re.sub(r"/\*.*?\*/", "", text[start + len("typedef struct {"):end.start()], flags=re.S)
    return re.findall(r"(\w+)\s*;", body)


@pytest.mark.parametrize("cname,pyname", [("gqd_solver_opts", "_SolverOpts"), ("gqd_stats", "_Stats"),
                                          ("gqd_grid_desc", "_GridDesc")])
def test_binding_structs_mirror_the_header(cname, pyname):
    from paper_1902_04661_amd import gqd
    fields = [f[0] for f in getattr(gqd, pyname)._fields_]
    assert fields == header_struct_fields(cname)
