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
    assert L.cq_boys(99, 1, None, None, 0, None) == cq.CQ_EINVAL
    assert L.cq_boys(3, 1, None, None, 2, None) == cq.CQ_EINVAL
    assert L.cq_sync_status(None, None) == cq.CQ_EINVAL
    assert L.cq_basis_nbf(None) == -1
    assert L.cq_basis_nmol(None) == -1
    assert L.cq_basis_create_batch(0, None, None, None, None, None, None, None, ctypes.byref(h)) == cq.CQ_EINVAL
    ns = (ctypes.c_int * 2)(3, 0)
    assert L.cq_basis_create_batch(2, ns, None, None, None, None, None, None, ctypes.byref(h)) == cq.CQ_EINVAL
    assert b"molecule 1" in L.cq_last_error()
    assert L.cq_autotune(None, 1, 1, None) == cq.CQ_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcq.so not built")
def test_size_check_guards_32bit_offsets():
    """The kernels address a molecule's [nbf][nbf][slots] blocks with 32-bit
    offsets; builds that would overflow them are refused before any work
    (checked on the host, no GPU)."""
    from paper_1905_01381_amd import cq
    assert cq.jk_size_check(600, 8, 1, 8) == cq.CQ_OK
    assert cq.jk_size_check(3000, 16, 16, 16) == cq.CQ_OK
    assert cq.jk_size_check(16383, 8, 8, 8) == cq.CQ_OK          # 2.147e9 - 8 * 32767 < 2^31
    assert cq.jk_size_check(16384, 8, 8, 8) == cq.CQ_EUNSUPPORTED  # exactly 2^31
    assert cq.jk_size_check(11586, 16, 1, 1) == cq.CQ_EUNSUPPORTED  # 16 slots above 11585 functions
    assert cq.jk_size_check(11585, 1, 16, 1) == cq.CQ_OK
    assert cq.jk_size_check(11586, 1, 1, 16) == cq.CQ_EUNSUPPORTED
    assert b"2^31" in cq.lib().cq_last_error()
    assert cq.jk_size_check(-1, 1, 1, 1) == cq.CQ_EINVAL
    # every (nbf, slots) pair agrees with the 64-bit product
    for nbf in (1, 4095, 11585, 11586, 16383, 16384, 46340, 46341):
        for w in (1, 2, 8, 9, 16):
            want = cq.CQ_OK if nbf * nbf * w < 2 ** 31 else cq.CQ_EUNSUPPORTED
            assert cq.jk_size_check(nbf, w, 1, 1) == want, (nbf, w)


def test_thresholds_flags():
    from paper_1905_01381_amd import cq
    assert cq.thresholds().flags == cq.CQ_DETERMINISTIC
    assert cq.thresholds(accumulate=True).flags == cq.CQ_DETERMINISTIC | cq.CQ_ACCUMULATE


@pytest.mark.skipif(not os.path.exists(LIB), reason="libcq.so not built")
def test_general_basis_argument_errors():
    """cq_basis_create_general refuses l = 4 (CQ_EUNSUPPORTED) and ncontr or
    pure outside their ranges (CQ_EINVAL) before touching the device."""
    import numpy as np
    from paper_1905_01381_amd import cq, inputs
    L = cq.lib()
    mol = inputs.small(1, [0, 1, 2], seed=1).mol
    dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    xyz = np.ascontiguousarray(mol.shell_xyz, dtype=np.float64)
    a = np.ascontiguousarray(mol.alpha)
    c = np.ascontiguousarray(mol.coef)
    npr = np.ascontiguousarray(mol.nprim, dtype=np.int32)
    nsm = np.array([3], np.int32)

    def create(ls, nco, pure):
        ls, nco, pure = (np.ascontiguousarray(v, dtype=np.int32) for v in (ls, nco, pure))
        h = ctypes.c_void_p()
        return L.cq_basis_create_general(1, nsm.ctypes.data_as(ip), xyz.ctypes.data_as(dp), ls.ctypes.data_as(ip),
                                         npr.ctypes.data_as(ip), nco.ctypes.data_as(ip), pure.ctypes.data_as(ip),
                                         a.ctypes.data_as(dp), c.ctypes.data_as(dp), None, ctypes.byref(h))
    assert create([0, 1, 4], [1, 1, 1], [0, 0, 1]) == cq.CQ_EUNSUPPORTED
    assert b"l=4" in L.cq_last_error()
    assert create([0, 1, 2], [1, 0, 1], [0, 0, 1]) == cq.CQ_EINVAL
    assert create([0, 1, 2], [1, 65, 1], [0, 0, 1]) == cq.CQ_EINVAL
    assert create([0, 1, 2], [1, 1, 1], [0, 0, 2]) == cq.CQ_EINVAL


def test_general_recipe_counts():
    """The spherical and general-contraction variants of the input recipe:
    3s2p1d gives 14 functions per atom with spherical d (nbf 560 for the
    40-atom two-component workload), the general variant keeps the function
    count with one shell per angular momentum."""
    import numpy as np
    from paper_1905_01381_amd import inputs
    assert inputs.c2(spherical=True).mol.nbf == 560
    m = inputs.general_molecule(2, inputs.SHELLS_3S2P1D, 0.1, 1e3, np.random.default_rng(0))
    assert list(m.shell_l) == [0, 1, 2] * 2
    assert list(m.ncontr) == [3, 2, 1] * 2 and list(m.nprim) == [8, 6, 3] * 2
    assert m.nbf == 28 and m.coef.size == 2 * (24 + 12 + 3)
    f = inputs.small(2, inputs.SHELLS_4S3P2D1F, spherical=True, general=True).mol
    assert list(f.shell_l) == [0, 1, 2, 3] * 2 and list(f.ncontr) == [4, 3, 2, 1] * 2
    assert f.nbf == 2 * (4 + 9 + 10 + 7)
    assert inputs.small(2, inputs.SHELLS_4S3P2D1F).mol.nbf == 2 * 35
