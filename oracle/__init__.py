"""CPU FP64 oracle for the integral-direct J/K build (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path.

* ``cq_oracle.c``: Boys function (series / erf), McMurchie-Davidson ERIs,
  one-electron integrals, J/K by the plain definition and by canonical
  quartets with deduplicated permutation images, sampled J/K blocks, Schwarz.
* ``twocomp.py``: the Pauli split / merge and the two-component Fock pieces.
* ``rt.py``: the EM2 real-time step with an eigendecomposition exponential.
* ``mlp.py``: the pointwise midpoint MLP (forward, backward, Adam) in FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cq_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB_PATH)
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int)
            L.ora_boys.restype = ctypes.c_double
            L.ora_boys.argtypes = [ctypes.c_int, ctypes.c_double]
            L.ora_boys_vec.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
            L.ora_basis_create.restype = ctypes.c_void_p
            L.ora_basis_create.argtypes = [ctypes.c_int, dp, ip, ip, dp, dp]
            L.ora_basis_destroy.argtypes = [ctypes.c_void_p]
            L.ora_nbf.restype = ctypes.c_int
            L.ora_nbf.argtypes = [ctypes.c_void_p]
            L.ora_shell_offsets.argtypes = [ctypes.c_void_p, ip]
            L.ora_eri_prim.restype = ctypes.c_double
            L.ora_eri_prim.argtypes = [ip, ctypes.c_double, dp] * 4
            L.ora_eri_shell.argtypes = [ctypes.c_void_p] + [ctypes.c_int] * 4 + [dp]
            L.ora_one_electron.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, dp,
                                           ctypes.c_int, dp, dp, dp]
            L.ora_jk_full.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp, dp]
            L.ora_jk_sym.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp, dp]
            L.ora_j_block.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
            L.ora_k_block.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
            L.ora_schwarz.argtypes = [ctypes.c_void_p, dp]
            L.ora_num_threads.restype = ctypes.c_int
            L.ora_set_threads.argtypes = [ctypes.c_int]
            L.ora_basis_coefs.argtypes = [ctypes.c_void_p, dp, dp]
            _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def boys(m: int, T: float) -> float:
    return lib().ora_boys(int(m), float(T))


def boys_table(mmax: int, T) -> np.ndarray:
    T = _f64(np.atleast_1d(T))
    out = np.zeros((T.size, mmax + 1))
    lib().ora_boys_vec(mmax, T.size, _dp(T), _dp(out))
    return out


def eri_prim(ea, a, A, eb, b, B, ec, c, C, ed, d, D) -> float:
    """Unnormalized primitive Cartesian ERI (x^i y^j z^k exp(-a r^2))."""
    args = []
    for e, x, X in ((ea, a, A), (eb, b, B), (ec, c, C), (ed, d, D)):
        ei = np.ascontiguousarray(e, dtype=np.int32)
        Xd = _f64(X)
        args += [ei, float(x), Xd]
    keep = args
    call = []
    for k in range(4):
        call += [_ip(keep[3 * k]), keep[3 * k + 1], _dp(keep[3 * k + 2])]
    return lib().ora_eri_prim(*call)


class Basis:
    """Oracle-side contracted basis (normalization done in C)."""

    def __init__(self, shell_xyz, shell_l, nprim, alpha, coef):
        self.xyz = _f64(shell_xyz).reshape(-1, 3)
        self.l = np.ascontiguousarray(shell_l, dtype=np.int32)
        self.nprim = np.ascontiguousarray(nprim, dtype=np.int32)
        self.alpha = _f64(alpha)
        self.coef = _f64(coef)
        self.nshell = int(self.l.size)
        self.h = lib().ora_basis_create(self.nshell, _dp(self.xyz), _ip(self.l), _ip(self.nprim),
                                        _dp(self.alpha), _dp(self.coef))
        self.nbf = lib().ora_nbf(self.h)
        off = np.zeros(self.nshell + 1, dtype=np.int32)
        lib().ora_shell_offsets(self.h, _ip(off))
        self.offsets = off

    @classmethod
    def from_molecule(cls, mol) -> "Basis":
        return cls(mol.shell_xyz, mol.shell_l, mol.nprim, mol.alpha, mol.coef)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().ora_basis_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def normalized_coefs(self) -> tuple[np.ndarray, np.ndarray]:
        """(primitive coefficients incl. x^l factor, per-function factors)."""
        c = np.zeros(self.alpha.size)
        f = np.zeros(self.nbf)
        lib().ora_basis_coefs(self.h, _dp(c), _dp(f))
        return c, f

    def nfunc(self, s: int) -> int:
        return int(self.offsets[s + 1] - self.offsets[s])

    def eri_shell(self, a, b, c, d) -> np.ndarray:
        shape = (self.nfunc(a), self.nfunc(b), self.nfunc(c), self.nfunc(d))
        out = np.zeros(shape)
        lib().ora_eri_shell(self.h, int(a), int(b), int(c), int(d), _dp(out))
        return out

    def eri_full(self) -> np.ndarray:
        """Every (mn|ls) as an nbf^4 array (tiny bases only)."""
        n = self.nbf
        g = np.zeros((n, n, n, n))
        o = self.offsets
        for a in range(self.nshell):
            for b in range(self.nshell):
                for c in range(self.nshell):
                    for d in range(self.nshell):
                        g[o[a]:o[a + 1], o[b]:o[b + 1], o[c]:o[c + 1], o[d]:o[d + 1]] = self.eri_shell(a, b, c, d)
        return g

    def one_electron(self, kind: str, direction: int = 2, origin=(0.0, 0.0, 0.0),
                     charges=None, centers=None) -> np.ndarray:
        k = {"overlap": 0, "kinetic": 1, "dipole": 2, "nuclear": 3}[kind]
        out = np.zeros((self.nbf, self.nbf))
        org = _f64(origin)
        if charges is None:
            Z = np.zeros(1); C = np.zeros(3); nc = 0
        else:
            Z = _f64(charges); C = _f64(centers).reshape(-1); nc = Z.size
        lib().ora_one_electron(self.h, k, int(direction), _dp(org), nc, _dp(Z), _dp(C), _dp(out))
        return out

    def overlap(self) -> np.ndarray:
        return self.one_electron("overlap")

    def _jk(self, fn, X, want_j=True, want_k=True):
        X = _f64(X)
        single = X.ndim == 2
        if single:
            X = X[None]
        nmat = X.shape[0]
        J = np.zeros_like(X) if want_j else None
        K = np.zeros_like(X) if want_k else None
        fn(self.h, nmat, _dp(X), _dp(J) if want_j else None, _dp(K) if want_k else None)
        if single:
            J = J[0] if want_j else None
            K = K[0] if want_k else None
        return J, K

    def jk_full(self, X, want_j=True, want_k=True):
        """J[X] and K[X] by the plain definition over every ordered quartet."""
        return self._jk(lib().ora_jk_full, X, want_j, want_k)

    def jk(self, X, want_j=True, want_k=True):
        """J[X] and K[X] via canonical quartets and their distinct images."""
        return self._jk(lib().ora_jk_sym, X, want_j, want_k)

    def j_block(self, a, b, X) -> np.ndarray:
        X = _f64(X)
        if X.ndim == 2:
            X = X[None]
        out = np.zeros((X.shape[0], self.nfunc(a), self.nfunc(b)))
        lib().ora_j_block(self.h, int(a), int(b), X.shape[0], _dp(X), _dp(out))
        return out

    def k_block(self, a, c, X) -> np.ndarray:
        X = _f64(X)
        if X.ndim == 2:
            X = X[None]
        out = np.zeros((X.shape[0], self.nfunc(a), self.nfunc(c)))
        lib().ora_k_block(self.h, int(a), int(c), X.shape[0], _dp(X), _dp(out))
        return out

    def schwarz(self) -> np.ndarray:
        Q = np.zeros((self.nshell, self.nshell))
        lib().ora_schwarz(self.h, _dp(Q))
        return Q


def set_threads(n: int) -> None:
    lib().ora_set_threads(int(n))


def num_threads() -> int:
    return lib().ora_num_threads()


def inv_sqrt(S: np.ndarray) -> np.ndarray:
    """S^{-1/2} by symmetric eigendecomposition (Loewdin)."""
    w, v = np.linalg.eigh(S)
    return (v / np.sqrt(w)) @ v.T


def density_real(S: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """P = C C^T with C = S^{-1/2} Q (S-orthonormal occupied orbitals)."""
    C = inv_sqrt(S) @ Q
    return C @ C.T


def density_2c(S: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Spin-blocked P^{2C} = C C^dagger with C = diag(S,S)^{-1/2} Q."""
    n = S.shape[0]
    X = inv_sqrt(S)
    C = np.empty_like(Q)
    C[:n] = X @ Q[:n]
    C[n:] = X @ Q[n:]
    return C @ C.conj().T
