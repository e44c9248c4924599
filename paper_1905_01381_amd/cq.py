"""Thin Python binding of libcq (include/cq.h): argument marshalling only.

Every computation runs in the HIP library.  PyTorch provides device memory
and streams; the library raises ``RuntimeError`` if it is missing or was not
built (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcq.so")

CQ_OK, CQ_EINVAL, CQ_ENOMEM, CQ_EHIP, CQ_EUNSUPPORTED, CQ_ENONFINITE, CQ_ENOTCONV = range(7)
CQ_ACCUMULATE = 1
CQ_DETERMINISTIC = 2
CQ_MAX_DENSITIES = 16
_STATUS = {0: "CQ_OK", 1: "CQ_EINVAL", 2: "CQ_ENOMEM", 3: "CQ_EHIP", 4: "CQ_EUNSUPPORTED",
           5: "CQ_ENONFINITE", 6: "CQ_ENOTCONV"}

_lib = None


class CqError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Thresholds(ctypes.Structure):
    _fields_ = [("skip", ctypes.c_double), ("fp32_below", ctypes.c_double),
                ("mode", ctypes.c_int), ("flags", ctypes.c_uint)]


def lib():
    """Load libcq.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libcq.so not found at {LIB_PATH}; run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip, i = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.c_int
        L.cq_last_error.restype = ctypes.c_char_p
        L.cq_basis_create.argtypes = [i, dp, ip, ip, dp, dp, vp, ctypes.POINTER(vp)]
        L.cq_basis_create_batch.argtypes = [i, ip, dp, ip, ip, dp, dp, vp, ctypes.POINTER(vp)]
        L.cq_basis_create_general.argtypes = [i, ip, dp, ip, ip, ip, ip, dp, dp, vp, ctypes.POINTER(vp)]
        L.cq_basis_nmol.argtypes = [vp]
        L.cq_basis_nmol.restype = i
        L.cq_basis_mol_nbf.argtypes = [vp, ip]
        L.cq_autotune.argtypes = [vp, i, i, vp]
        L.cq_autotune_read.argtypes = [vp, i, ip, ctypes.POINTER(ctypes.c_float), ip]
        L.cq_plan_set.argtypes = [vp, i, ip]
        L.cq_basis_destroy.argtypes = [vp]
        L.cq_basis_nbf.argtypes = [vp]
        L.cq_basis_nbf.restype = i
        L.cq_basis_nshell.argtypes = [vp]
        L.cq_basis_nshell.restype = i
        L.cq_schwarz.argtypes = [vp, vp, vp]
        L.cq_jk_build.argtypes = [vp, i, ctypes.POINTER(vp), ip, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                  ctypes.POINTER(Thresholds), vp]
        L.cq_jk_build_noalloc.argtypes = L.cq_jk_build.argtypes
        L.cq_fock2e_2c.argtypes = [vp, vp, vp, ctypes.POINTER(Thresholds), vp]
        L.cq_boys.argtypes = [i, i, vp, vp, i, vp]
        L.cq_sync_status.argtypes = [vp, vp]
        L.cq_jk_size_check.argtypes = [i, i, i, i]
        L.cq_eri_quartet.argtypes = [vp, i, i, i, i, dp, vp]
        L.cq_one_electron.argtypes = [vp, i, i, dp, i, dp, dp, vp, vp]
        llp = ctypes.POINTER(ctypes.c_longlong)
        L.cq_quartet_counts.argtypes = [vp, i, ip, llp, ip]
        L.cq_prim_quartet_counts.argtypes = [vp, i, ip, llp, ip]
        L.cq_profile.argtypes = [vp, i]
        L.cq_trace.argtypes = [vp, i]
        L.cq_build_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_ulonglong), vp]
        fp = ctypes.POINTER(ctypes.c_float)
        L.cq_rt_create.argtypes = [vp, vp, vp, vp, vp, ctypes.c_double, i, vp, ctypes.POINTER(vp)]
        L.cq_rt_destroy.argtypes = [vp]
        L.cq_rt_set_mode.argtypes = [vp, i]
        L.cq_rt_set_params.argtypes = [vp, ctypes.c_double, i, ctypes.c_double]
        L.cq_rt_set_restart.argtypes = [vp, i]
        L.cq_rt_set_field.argtypes = [vp, i, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.cq_rt_step.argtypes = [vp, i, dp, dp, ip]
        L.cq_rt_density.argtypes = [vp, vp, vp]
        L.cq_rt_stats.argtypes = [vp, llp]
        L.cq_rt_record.argtypes = [vp, i, i, ctypes.c_uint]
        L.cq_rt_recorded.argtypes = [vp, ip]
        L.cq_rt_train.argtypes = [vp, i, ctypes.c_float, fp]
        L.cq_rt_mlp_weights.argtypes = [vp, fp, fp]
        L.cq_rt_mlp_scales.argtypes = [vp, fp, dp]
        L.cq_expm.argtypes = [i, vp, ctypes.c_double, vp, vp]
        L.cq_zgemm.argtypes = [i, vp, vp, i, vp, vp]
        L.cq_mlp_eval.argtypes = [vp, vp, vp, i, vp, vp, vp]
        L.cq_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_float, i, vp]
        L.cq_profile_read.argtypes = [vp, i, ip, dp, llp, ip]
        for name in ("cq_basis_create", "cq_basis_create_batch", "cq_basis_create_general", "cq_basis_mol_nbf",
                     "cq_autotune", "cq_plan_set",
                     "cq_autotune_read", "cq_basis_destroy", "cq_schwarz", "cq_jk_build", "cq_fock2e_2c",
                     "cq_boys", "cq_eri_quartet", "cq_one_electron", "cq_quartet_counts", "cq_prim_quartet_counts",
                     "cq_profile", "cq_trace",
                     "cq_profile_read", "cq_build_stats", "cq_rt_create", "cq_rt_destroy", "cq_rt_set_mode",
                     "cq_rt_set_params", "cq_rt_step", "cq_rt_density", "cq_rt_stats", "cq_rt_record",
                     "cq_rt_recorded", "cq_rt_train", "cq_rt_mlp_weights", "cq_rt_mlp_scales", "cq_expm",
                     "cq_mlp_eval", "cq_mlp_adam", "cq_sync_status", "cq_jk_size_check", "cq_jk_build_noalloc", "cq_rt_set_restart", "cq_rt_set_field", "cq_zgemm"):
            getattr(L, name).restype = i
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != CQ_OK:
        raise CqError(status, lib().cq_last_error().decode())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _req_dev(t, dtype, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("expected a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")


@dataclass
class JKResult:
    J: list
    K: list


def thresholds(skip: float = 0.0, fp32_below: float = 0.0, mode: int = 0, accumulate: bool = False) -> Thresholds:
    """Build thresholds (accumulation is always deterministic: CQ_DETERMINISTIC)."""
    flags = (CQ_ACCUMULATE if accumulate else 0) | CQ_DETERMINISTIC
    return Thresholds(float(skip), float(fp32_below), int(mode), flags)


def jk_size_check(nbf: int, nx: int, nj: int, nk: int) -> int:
    """Status of cq_jk_size_check (host only): CQ_OK or CQ_EUNSUPPORTED."""
    return int(lib().cq_jk_size_check(int(nbf), int(nx), int(nj), int(nk)))


class Basis:
    """A libcq basis handle (device resident).  With ``nshell_mol`` the shell
    arrays hold several molecules one after another and the handle is a
    batch: its matrices are flat tensors of the concatenated per-molecule
    [nbf_m, nbf_m] blocks (see ``pack`` / ``unpack``)."""

    def __init__(self, shell_xyz, shell_l, nprim, alpha, coef, stream=None, nshell_mol=None, ncontr=None,
                 pure=None):
        """``ncontr`` / ``pure`` (per shell) select cq_basis_create_general:
        generally contracted shells (``coef`` then holds ncontr rows of nprim
        per shell) and spherical d shells."""
        xyz = np.ascontiguousarray(shell_xyz, dtype=np.float64).reshape(-1)
        l = np.ascontiguousarray(shell_l, dtype=np.int32)
        npr = np.ascontiguousarray(nprim, dtype=np.int32)
        a = np.ascontiguousarray(alpha, dtype=np.float64)
        c = np.ascontiguousarray(coef, dtype=np.float64)
        h = ctypes.c_void_p()
        dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        if ncontr is not None or pure is not None:
            nco = np.ascontiguousarray(np.ones(l.size) if ncontr is None else ncontr, dtype=np.int32)
            pu = np.ascontiguousarray(np.zeros(l.size) if pure is None else pure, dtype=np.int32)
            nsm = np.ascontiguousarray([l.size] if nshell_mol is None else nshell_mol, dtype=np.int32)
            if nco.size != l.size or pu.size != l.size or int(nsm.sum()) != l.size:
                raise ValueError("ncontr, pure and nshell_mol must match the shells")
            _check(lib().cq_basis_create_general(int(nsm.size), nsm.ctypes.data_as(ip), xyz.ctypes.data_as(dp),
                                                 l.ctypes.data_as(ip), npr.ctypes.data_as(ip),
                                                 nco.ctypes.data_as(ip), pu.ctypes.data_as(ip),
                                                 a.ctypes.data_as(dp), c.ctypes.data_as(dp), _stream(stream),
                                                 ctypes.byref(h)))
        elif nshell_mol is None:
            _check(lib().cq_basis_create(int(l.size), xyz.ctypes.data_as(dp), l.ctypes.data_as(ip),
                                         npr.ctypes.data_as(ip), a.ctypes.data_as(dp), c.ctypes.data_as(dp),
                                         _stream(stream), ctypes.byref(h)))
        else:
            nsm = np.ascontiguousarray(nshell_mol, dtype=np.int32)
            if int(nsm.sum()) != l.size:
                raise ValueError("nshell_mol does not add up to the number of shells")
            _check(lib().cq_basis_create_batch(int(nsm.size), nsm.ctypes.data_as(ip), xyz.ctypes.data_as(dp),
                                               l.ctypes.data_as(ip), npr.ctypes.data_as(ip),
                                               a.ctypes.data_as(dp), c.ctypes.data_as(dp), _stream(stream),
                                               ctypes.byref(h)))
        self.h = h
        self.nbf = lib().cq_basis_nbf(h)
        self.nshell = lib().cq_basis_nshell(h)
        # shells as the library holds them: general contractions expanded
        self.shell_l = np.repeat(l, np.asarray(ncontr, dtype=np.int64)) if ncontr is not None else l.copy()
        self.nmol = lib().cq_basis_nmol(h)
        nb = np.zeros(self.nmol, np.int32)
        _check(lib().cq_basis_mol_nbf(h, nb.ctypes.data_as(ip)))
        self.mol_nbf = [int(x) for x in nb]
        self.mol_off = [0]
        for n in self.mol_nbf:
            self.mol_off.append(self.mol_off[-1] + n * n)
        self.nel = self.mol_off[-1]
        self.batch = nshell_mol is not None

    @classmethod
    def from_molecule(cls, mol, stream=None) -> "Basis":
        return cls(mol.shell_xyz, mol.shell_l, mol.nprim, mol.alpha, mol.coef, stream,
                   ncontr=getattr(mol, "ncontr", None), pure=getattr(mol, "pure", None))

    @classmethod
    def from_molecules(cls, mols, stream=None) -> "Basis":
        """A batch handle over a list of molecules."""
        general = any(getattr(m, "ncontr", None) is not None or getattr(m, "pure", None) is not None for m in mols)
        kw = {}
        if general:
            kw["ncontr"] = np.concatenate([m.ncontr if getattr(m, "ncontr", None) is not None
                                           else np.ones(m.nshell, np.int32) for m in mols])
            kw["pure"] = np.concatenate([m.pure if getattr(m, "pure", None) is not None
                                         else np.zeros(m.nshell, np.int32) for m in mols])
        return cls(np.concatenate([np.asarray(m.shell_xyz).reshape(-1, 3) for m in mols]),
                   np.concatenate([m.shell_l for m in mols]), np.concatenate([m.nprim for m in mols]),
                   np.concatenate([m.alpha for m in mols]), np.concatenate([m.coef for m in mols]), stream,
                   nshell_mol=[len(m.shell_l) for m in mols], **kw)

    def pack(self, mats):
        """Concatenate per-molecule [nbf_m, nbf_m] device matrices into one flat batch tensor."""
        import torch
        return torch.cat([m.reshape(-1) for m in mats]).contiguous()

    def unpack(self, flat):
        """Views of a flat batch tensor as the per-molecule [nbf_m, nbf_m] blocks."""
        return [flat[self.mol_off[i]:self.mol_off[i + 1]].view(n, n) for i, n in enumerate(self.mol_nbf)]

    def autotune(self, nmat: int = 1, reps: int = 1, stream=None) -> list:
        """Time candidate task shapes and grid caps per class and keep the fastest."""
        _check(lib().cq_autotune(self.h, int(nmat), int(reps), _stream(stream)))
        return self.plan()

    def plan(self) -> list:
        """The launch plan per class: (la, lb, lc, ld), c-range length, grid
        cap, tasks, orientation, LDS level (-1: highest that fits), walk
        rotation, tuned ms."""
        n = ctypes.c_int()
        rec = np.zeros(10 * 32, np.int32)
        ms = np.zeros(32, np.float32)
        _check(lib().cq_autotune_read(self.h, 32, rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                      ms.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(n)))
        out = []
        for k in range(min(n.value, 32)):
            r = rec[10 * k:10 * k + 10]
            out.append({"cls": tuple(int(x) for x in r[:4]), "cl": int(r[4]), "grid": int(r[5]),
                        "tasks": int(r[6]), "exchanged": int(r[7]), "acc": int(r[8]), "rot": int(r[9]),
                        "ms": float(ms[k])})
        return out

    def save_plan(self, path: str) -> None:
        """Write the current plan records (e.g. after autotune) as JSON."""
        import json
        with open(path, "w") as f:
            json.dump([dict(p, cls=list(p["cls"])) for p in self.plan()], f, indent=1)

    def load_plan(self, path: str) -> None:
        """Apply plan records written by save_plan (same molecules)."""
        import json
        with open(path) as f:
            recs = json.load(f)
        self.set_plan([dict(p, cls=tuple(p["cls"])) for p in recs])

    def set_plan(self, plan: list) -> None:
        """Apply plan records (as returned by ``plan``) to their classes."""
        rec = np.zeros(10 * max(len(plan), 1), np.int32)
        for k, p in enumerate(plan):
            rec[10 * k:10 * k + 10] = [*p["cls"], p["cl"], p["grid"], p.get("tasks", 0), p.get("exchanged", 0),
                                       p.get("acc", -1), p.get("rot", 0)]
        _check(lib().cq_plan_set(self.h, len(plan), rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().cq_basis_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def schwarz(self, stream=None):
        import torch
        if self.batch:
            raise ValueError("schwarz() returns the single-molecule [nshell, nshell] matrix")
        Q = torch.empty((self.nshell, self.nshell), dtype=torch.float64, device="cuda")
        _check(lib().cq_schwarz(self.h, _ptr(Q), _stream(stream)))
        return Q

    def jk(self, P, sym=None, want_j=True, want_k=True, th: Thresholds | None = None, out=None, stream=None,
           noalloc: bool = False):
        """J[X_m], K[X_m] for a list of densities (device float64 [nbf, nbf]).
        ``want_j`` / ``want_k``: bool or per-density list of bools.
        ``noalloc``: cq_jk_build_noalloc (static scratch, no device allocation)."""
        import torch
        Ps = list(P) if isinstance(P, (list, tuple)) else [P]
        n = len(Ps)
        sym = [1] * n if sym is None else list(sym)
        wj = [want_j] * n if isinstance(want_j, bool) else list(want_j)
        wk = [want_k] * n if isinstance(want_k, bool) else list(want_k)
        for p in Ps:
            _req_dev(p, torch.float64, (self.nel,) if self.batch else (self.nbf, self.nbf))
        if out is None:
            J = [torch.empty_like(Ps[m]) if wj[m] else None for m in range(n)]
            K = [torch.empty_like(Ps[m]) if wk[m] else None for m in range(n)]
        else:
            J, K = out
        arr = ctypes.c_void_p * max(n, 1)
        pP = arr(*[p.data_ptr() for p in Ps])
        pJ = arr(*[(j.data_ptr() if j is not None else 0) for j in J])
        pK = arr(*[(k.data_ptr() if k is not None else 0) for k in K])
        psym = (ctypes.c_int * n)(*sym)
        thp = ctypes.byref(th) if th is not None else None
        fn = lib().cq_jk_build_noalloc if noalloc else lib().cq_jk_build
        _check(fn(self.h, n, pP, psym, pJ, pK, thp, _stream(stream)))
        return JKResult(J, K)

    def fock2e_2c(self, P2c, th: Thresholds | None = None, out=None, stream=None):
        """G^{2C} (complex128 [2nbf, 2nbf]) of a spin-blocked density."""
        import torch
        _req_dev(P2c, torch.complex128, (2 * self.nbf, 2 * self.nbf))
        G = torch.empty_like(P2c) if out is None else out
        thp = ctypes.byref(th) if th is not None else None
        _check(lib().cq_fock2e_2c(self.h, _ptr(P2c), _ptr(G), thp, _stream(stream)))
        return G

    def one_electron(self, kind: str, direction: int = 2, origin=(0.0, 0.0, 0.0), charges=None,
                     centers=None, stream=None):
        """S, T, V or a dipole component as a device float64 [nbf, nbf]."""
        import torch
        k = {"overlap": 0, "kinetic": 1, "dipole": 2, "nuclear": 3}[kind]
        out = torch.empty((self.nbf, self.nbf), dtype=torch.float64, device="cuda")
        dp = ctypes.POINTER(ctypes.c_double)
        org = np.ascontiguousarray(origin, dtype=np.float64)
        if k == 3:
            Z = np.ascontiguousarray(charges, dtype=np.float64)
            C = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1)
            nz = int(Z.size)
            zp, cp = Z.ctypes.data_as(dp), C.ctypes.data_as(dp)
        else:
            nz, zp, cp = 0, None, None
        _check(lib().cq_one_electron(self.h, k, int(direction), org.ctypes.data_as(dp), nz, zp, cp,
                                     _ptr(out), _stream(stream)))
        return out

    def quartet_counts(self) -> dict:
        """{(la, lb, lc, ld): unique shell quartets of an unscreened build}."""
        n = ctypes.c_int()
        cls = (ctypes.c_int * 512)()
        cnt = (ctypes.c_longlong * 128)()
        _check(lib().cq_quartet_counts(self.h, 128, cls, cnt, ctypes.byref(n)))
        return {tuple(cls[4 * k: 4 * k + 4]): int(cnt[k]) for k in range(n.value)}

    def prim_quartet_counts(self) -> dict:
        """{(la, lb, lc, ld): primitive quartets above the primitive cut in
        the class's unique shell quartets}."""
        n = ctypes.c_int()
        cls = (ctypes.c_int * 512)()
        cnt = (ctypes.c_longlong * 128)()
        _check(lib().cq_prim_quartet_counts(self.h, 128, cls, cnt, ctypes.byref(n)))
        return {tuple(cls[4 * k: 4 * k + 4]): int(cnt[k]) for k in range(n.value)}

    def sync_status(self, stream=None) -> int:
        """cq_sync_status: CQ_OK, or CQ_ENONFINITE if a density of a build since
        the last call held a non-finite element (the word is cleared)."""
        return int(lib().cq_sync_status(self.h, _stream(stream)))

    def build_stats(self, stream=None) -> dict:
        """Quartets of the last build: evaluated in FP64 / FP32, skipped."""
        out = (ctypes.c_ulonglong * 3)()
        _check(lib().cq_build_stats(self.h, out, _stream(stream)))
        return {"fp64": int(out[0]), "fp32": int(out[1]), "skipped": int(out[2])}

    def profile(self, enable: bool = True, reset: bool = False):
        _check(lib().cq_profile(self.h, 2 if (enable and reset) else int(enable)))

    def trace(self, enable: bool = True):
        """Print "[cq] class (ab|cd) done" to stderr as each class of a build finishes."""
        _check(lib().cq_trace(self.h, int(enable)))

    def profile_read(self) -> dict:
        """{(la, lb, lc, ld): (total kernel ms, launches)} from HIP events."""
        n = ctypes.c_int()
        cls = (ctypes.c_int * 256)()
        ms = (ctypes.c_double * 64)()
        cnt = (ctypes.c_longlong * 64)()
        _check(lib().cq_profile_read(self.h, 64, cls, ms, cnt, ctypes.byref(n)))
        return {tuple(cls[4 * k: 4 * k + 4]): (float(ms[k]), int(cnt[k])) for k in range(n.value)}

    def eri_quartet(self, a, b, c, d, stream=None) -> np.ndarray:
        n = [(int(self.shell_l[s]) + 1) * (int(self.shell_l[s]) + 2) // 2 for s in (a, b, c, d)]
        out = np.zeros(n)
        _check(lib().cq_eri_quartet(self.h, int(a), int(b), int(c), int(d),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(stream)))
        return out


def boys(mmax: int, T, fp32: bool = False, stream=None):
    """F_m(T), m = 0..mmax, for a device float64 vector T -> [n, mmax+1]
    (fp32: the evaluation of the precision-routed FP32 kernels)."""
    import torch
    _req_dev(T, torch.float64)
    F = torch.empty((T.numel(), mmax + 1), dtype=torch.float64, device=T.device)
    _check(lib().cq_boys(int(mmax), int(T.numel()), _ptr(T), _ptr(F), int(bool(fp32)), _stream(stream)))
    return F


RT_EM2, RT_MIDPOINT, RT_LEARNED, RT_MMUT = 0, 1, 2, 3
MLP_PARAMS = 354


class RT:
    """Real-time propagator handle (cq_rt_*)."""

    def __init__(self, basis: "Basis", h, X, Dz, P0, dt: float, mode: int = RT_EM2, stream=None):
        import torch
        n = basis.nbf
        for m in (h, X, Dz):
            _req_dev(m, torch.float64, (n, n))
        _req_dev(P0, torch.complex128, (n, n))
        self.basis = basis
        self.n = n
        self._keep = (h, X, Dz, P0)
        hdl = ctypes.c_void_p()
        _check(lib().cq_rt_create(basis.h, _ptr(h), _ptr(X), _ptr(Dz), _ptr(P0), float(dt), int(mode),
                                  _stream(stream), ctypes.byref(hdl)))
        self.h = hdl

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().cq_rt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_mode(self, mode: int):
        _check(lib().cq_rt_set_mode(self.h, int(mode)))

    def set_params(self, sc_tol=1e-10, max_iter=30, accept_tol=None):
        """accept_tol: first-iterate acceptance (default: sc_tol)."""
        acc = sc_tol if accept_tol is None else accept_tol
        _check(lib().cq_rt_set_params(self.h, float(sc_tol), int(max_iter), float(acc)))

    def set_restart(self, period: int):
        """MMUT: EM2 seed/restart every `period` steps."""
        _check(lib().cq_rt_set_restart(self.h, int(period)))

    FIELD_ENVELOPES = {"none": 0, "step": 1, "ramp": 2, "plane_wave": 3, "gaussian": 4}

    def set_field(self, envelope: str = "none", kappa: float = 0.0, param: float = 0.0, t_on: float = 0.0,
                  t_off: float = float("inf")):
        """External perturbation f(t) Dz (see cq_rt_set_field)."""
        _check(lib().cq_rt_set_field(self.h, self.FIELD_ENVELOPES[envelope], float(kappa), float(param),
                                     float(t_on), float(t_off)))

    def step(self, nsteps: int, energy: bool = False, dipole: bool = True):
        E = np.zeros(nsteps)
        mu = np.zeros(nsteps)
        nb = np.zeros(nsteps, dtype=np.int32)
        dp, ip = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
        _check(lib().cq_rt_step(self.h, int(nsteps), E.ctypes.data_as(dp) if energy else None,
                                mu.ctypes.data_as(dp) if dipole else None, nb.ctypes.data_as(ip)))
        return E, mu, nb

    def density(self, stream=None):
        import torch
        P = torch.empty((self.n, self.n), dtype=torch.complex128, device="cuda")
        _check(lib().cq_rt_density(self.h, _ptr(P), _stream(stream)))
        return P

    def stats(self) -> dict:
        out = (ctypes.c_longlong * 4)()
        _check(lib().cq_rt_stats(self.h, out))
        return {"steps": out[0], "builds": out[1], "accepted": out[2], "fallbacks": out[3]}

    def record(self, enable=True, samples_per_step=4096, seed=1):
        _check(lib().cq_rt_record(self.h, int(enable), int(samples_per_step), int(seed)))

    def train(self, epochs: int, lr: float = 1e-3) -> float:
        loss = ctypes.c_float()
        _check(lib().cq_rt_train(self.h, int(epochs), float(lr), ctypes.byref(loss)))
        return float(loss.value)

    def weights(self, set_=None):
        fp = ctypes.POINTER(ctypes.c_float)
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        if set_ is not None:
            w = np.ascontiguousarray(set_, dtype=np.float32)
            _check(lib().cq_rt_mlp_weights(self.h, w.ctypes.data_as(fp), out.ctypes.data_as(fp)))
        else:
            _check(lib().cq_rt_mlp_weights(self.h, None, out.ctypes.data_as(fp)))
        return out


def _rt_scales(self):
    fp = ctypes.POINTER(ctypes.c_float)
    xs = np.zeros(8, dtype=np.float32)
    ys = ctypes.c_double()
    _check(lib().cq_rt_mlp_scales(self.h, xs.ctypes.data_as(fp), ctypes.byref(ys)))
    return xs, float(ys.value)


RT.scales = _rt_scales


def expm(H, dt: float, stream=None):
    """exp(-i dt H) for a device complex128 Hermitian H."""
    import torch
    _req_dev(H, torch.complex128)
    U = torch.empty_like(H)
    _check(lib().cq_expm(int(H.shape[0]), _ptr(H), float(dt), _ptr(U), _stream(stream)))
    return U


def zgemm(A, B, conj_b: bool = False, stream=None):
    """A @ B (or A @ B^H) for device complex128 square matrices (cq_zgemm)."""
    import torch
    _req_dev(A, torch.complex128)
    _req_dev(B, torch.complex128, tuple(A.shape))
    C = torch.empty_like(A)
    _check(lib().cq_zgemm(int(A.shape[0]), _ptr(A), _ptr(B), int(bool(conj_b)), _ptr(C), _stream(stream)))
    return C


def mlp_eval(w, X, Y, stream=None):
    """Loss and gradient of the midpoint MLP on device FP32 samples."""
    import torch
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(lib().cq_mlp_eval(_ptr(w), _ptr(X), _ptr(Y), int(X.shape[0]), _ptr(g), _ptr(loss), _stream(stream)))
    return loss, g


def mlp_adam(w, g, m, v, lr: float, step: int, stream=None):
    _check(lib().cq_mlp_adam(_ptr(w), _ptr(g), _ptr(m), _ptr(v), float(lr), int(step), _stream(stream)))
