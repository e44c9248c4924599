"""The C-ABI library loads and exports every entry point include/cq.h
declares (no GPU needed: nothing here launches work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cq.h")
LIB = os.path.join(ROOT, "paper_1905_01381_amd", "libcq.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cq_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("cq_basis_create", "cq_schwarz", "cq_jk_build", "cq_fock2e_2c", "cq_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcq.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcq.so not built")
def test_argument_errors_without_gpu_work():
    """Argument validation returns CQ_EINVAL before touching the device."""
    from paper_1905_01381_amd import cq
    L = cq.lib()
    h = ctypes.c_void_p()
    st = L.cq_basis_create(0, None, None, None, None, None, None, ctypes.byref(h))
    assert st == cq.CQ_EINVAL
    assert b"nshell" in L.cq_last_error()
    assert L.cq_jk_build(None, 1, None, None, None, None, None, None) == cq.CQ_EINVAL
    assert L.cq_boys(99, 1, None, None, None) == cq.CQ_EINVAL
    assert L.cq_basis_nbf(None) == -1
    assert L.cq_basis_nmol(None) == -1
    assert L.cq_basis_create_batch(0, None, None, None, None, None, None, None, ctypes.byref(h)) == cq.CQ_EINVAL
    ns = (ctypes.c_int * 2)(3, 0)
    assert L.cq_basis_create_batch(2, ns, None, None, None, None, None, None, ctypes.byref(h)) == cq.CQ_EINVAL
    assert b"molecule 1" in L.cq_last_error()
    assert L.cq_autotune(None, 1, 1, None) == cq.CQ_EINVAL
