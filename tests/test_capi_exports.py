"""The C-ABI library loads and exports every entry point include/bo.h declares
(no GPU work: only host-side calls that validate arguments)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bo.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bo_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_2111_14991_amd as bo
    if not os.path.exists(bo.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return bo


def test_every_declared_symbol_is_exported(L):
    lib = C.CDLL(L.LIB_PATH)
    names = declared_functions()
    assert "bo_gp_fit" in names and "bo_posterior" in names and "bo_acquire" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps each of them under the same name
    assert set(names) <= set(L.exported_symbols())


def test_workspace_query_and_limits(L):
    b = L.bo_workspace_query(1536, 4, 20, L.BO_FP64)
    assert b > 1536 * 4 * 8
    assert b % 256 == 0
    b3 = L.bo_workspace_query(1 << 20, 10, 1000, L.BO_BF16X3)
    assert b3 > (1 << 20) * 10 * 8
    for bad in [(0, 4, 20, 0), (10, 0, 5, 0), (10, 17, 5, 0), (10, 4, 0, 0), (10, 4, 1025, 0), (10, 4, 5, 3)]:
        with pytest.raises(L.BOError) as e:
            L.bo_workspace_query(*bad)
        assert e.value.status == L.BO_E_INVALID_ARG


def test_session_create_rejects_bad_workspace(L):
    lib = L.lib()
    h = C.c_void_p()
    prob = L.bo_problem(100, 3, 10, L.BO_FP64, 0)
    rc = lib.bo_session_create(C.byref(h), C.byref(prob), None, None, 0, None)
    assert rc == L.BO_E_WORKSPACE
    assert "workspace" in L.last_error()
    rc = lib.bo_session_create(C.byref(h), C.byref(prob), None, 0x1000 + 8, 1 << 30, None)
    assert rc == L.BO_E_WORKSPACE
    g = L.bo_gp_params(4, 7, 1.0, 1.0, 1e-6)
    rc = lib.bo_session_create(C.byref(h), C.byref(prob), C.byref(g), 0x100000, 1 << 30, None)
    assert rc == L.BO_E_INVALID_ARG
    assert L.bo_version().startswith("bo-mi355x")
