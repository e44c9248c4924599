"""Spherical-harmonic shells and general contraction for the oracle.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no
code, table or constant with the HIP path.

The paper builds its one-particle basis from contracted Gaussians with
either segmented or general contraction (Introduction).  Both are reduced
here to the oracle's segmented Cartesian shells by their definitions:

* A generally contracted shell with ``ncontr`` contractions over one set of
  ``nprim`` exponents is ``ncontr`` function sets that share the exponents:
  contraction k is the segmented shell with coefficients ``coef[k]``.  Its
  functions are listed contraction by contraction.
* A spherical shell of angular momentum l spans the 2l+1 real solid
  harmonics r^l Y_lm(r - A) times the contracted radial part, m = -l..l
  (sine-type for m < 0, cosine-type for m > 0).  Their polynomials are
  generated from the standard expansion of the regular solid harmonics,
  (x +/- i y)^|m| times the z, r^2 polynomial of the associated Legendre
  function, and expressed on the oracle's unit-normalized Cartesian
  functions through the closed-form angular norms of the monomials.  For
  l <= 1 the flag changes nothing (s; p kept as x, y, z).

Each matrix of the spherical basis is T M T^T with the block-diagonal T of
the shells (nbf_sph x nbf_cart); a density enters as T^T X T.
"""
from __future__ import annotations

from math import comb, factorial

import numpy as np

from . import Basis


def cart_components(l: int) -> list[tuple[int, int, int]]:
    """x^a y^b z^c, a descending, then b descending (the oracle's order)."""
    return [(a, b, l - a - b) for a in range(l, -1, -1) for b in range(l - a, -1, -1)]


def _dfact(n: int) -> int:
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def _mul(p: dict, q: dict) -> dict:
    out: dict = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = (ea[0] + eb[0], ea[1] + eb[1], ea[2] + eb[2])
            out[e] = out.get(e, 0) + ca * cb
    return {e: c for e, c in out.items() if c != 0}


def _pow(p: dict, n: int) -> dict:
    out = {(0, 0, 0): 1}
    for _ in range(n):
        out = _mul(out, p)
    return out


def solid_harmonics(l: int) -> list[dict]:
    """Real regular solid harmonics of degree l as {(a, b, c): coefficient}
    polynomials (unnormalized), ordered m = -l..l."""
    r2 = {(2, 0, 0): 1, (0, 2, 0): 1, (0, 0, 2): 1}
    cos_part, sin_part = [], []
    for m in range(l + 1):
        # (x + i y)^m = C_m + i S_m
        C: dict = {}
        S: dict = {}
        for k in range(m + 1):
            e = (m - k, k, 0)
            c = comb(m, k)
            if k % 2 == 0:
                C[e] = C.get(e, 0) + c * (-1) ** (k // 2)
            else:
                S[e] = S.get(e, 0) + c * (-1) ** ((k - 1) // 2)
        # z, r^2 polynomial of degree l - m
        Pi: dict = {}
        for k in range((l - m) // 2 + 1):
            c = (-1) ** k * comb(l, k) * comb(2 * l - 2 * k, l) * factorial(l - 2 * k) // factorial(l - 2 * k - m)
            for e, v in _mul({(0, 0, l - 2 * k - m): 1}, _pow(r2, k)).items():
                Pi[e] = Pi.get(e, 0) + c * v
        cos_part.append(_mul(Pi, C))
        sin_part.append(_mul(Pi, S) if m > 0 else {})
    return [sin_part[m] for m in range(l, 0, -1)] + [cos_part[m] for m in range(l + 1)]


def _angular_gram(l: int) -> np.ndarray:
    """Overlaps of the unit-normalized Cartesian functions of one shell
    (common radial part): <x^a..|x^a'..> is proportional to
    (a+a'-1)!!(b+b'-1)!!(c+c'-1)!! when every sum is even, else 0."""
    comps = cart_components(l)
    n = np.array([_dfact(2 * a - 1) * _dfact(2 * b - 1) * _dfact(2 * c - 1) for a, b, c in comps], float)
    G = np.zeros((len(comps), len(comps)))
    for i, (a, b, c) in enumerate(comps):
        for j, (a2, b2, c2) in enumerate(comps):
            if (a + a2) % 2 or (b + b2) % 2 or (c + c2) % 2:
                continue
            G[i, j] = _dfact(a + a2 - 1) * _dfact(b + b2 - 1) * _dfact(c + c2 - 1) / np.sqrt(n[i] * n[j])
    return G


def sph_transform(l: int) -> np.ndarray:
    """(2l+1) x ncart(l) coefficients of the unit-normalized real solid
    harmonics on the unit-normalized Cartesian functions of one shell."""
    comps = cart_components(l)
    idx = {e: i for i, e in enumerate(comps)}
    G = _angular_gram(l)
    T = np.zeros((2 * l + 1, len(comps)))
    for m, poly in enumerate(solid_harmonics(l)):
        for (a, b, c), v in poly.items():
            # x^a y^b z^c g = phi_abc * ||x^a y^b z^c g||, norm ~ sqrt((2a-1)!!(2b-1)!!(2c-1)!!)
            T[m, idx[(a, b, c)]] += v * np.sqrt(_dfact(2 * a - 1) * _dfact(2 * b - 1) * _dfact(2 * c - 1))
        T[m] /= np.sqrt(T[m] @ G @ T[m])
    return T


class SphericalBasis:
    """A basis of segmented or generally contracted shells, each Cartesian or
    spherical, reduced to an oracle ``Basis`` of segmented Cartesian shells.

    coef: per shell, ``ncontr`` rows of ``nprim`` raw coefficients
    (contraction-major), shells one after another.
    """

    def __init__(self, shell_xyz, shell_l, nprim, ncontr, pure, alpha, coef):
        xyz = np.asarray(shell_xyz, float).reshape(-1, 3)
        ls = np.asarray(shell_l, int)
        npr = np.asarray(nprim, int)
        nco = np.asarray(ncontr, int)
        pu = np.asarray(pure, int)
        alpha = np.asarray(alpha, float)
        coef = np.asarray(coef, float)
        ex_xyz, ex_l, ex_np, ex_a, ex_c, ex_pure = [], [], [], [], [], []
        pa = pc = 0
        for s in range(ls.size):
            n = npr[s]
            for k in range(nco[s]):
                ex_xyz.append(xyz[s])
                ex_l.append(ls[s])
                ex_np.append(n)
                ex_a.append(alpha[pa:pa + n])
                ex_c.append(coef[pc + k * n:pc + (k + 1) * n])
                ex_pure.append(bool(pu[s]) and ls[s] >= 2)
            pa += n
            pc += n * nco[s]
        self.cart = Basis(np.array(ex_xyz), np.array(ex_l, np.int32), np.array(ex_np, np.int32),
                          np.concatenate(ex_a), np.concatenate(ex_c))
        self.shell_l = np.array(ex_l)
        self.shell_pure = np.array(ex_pure)
        blocks, off = [], [0]
        for L, p in zip(ex_l, ex_pure):
            blocks.append(sph_transform(L) if p else np.eye((L + 1) * (L + 2) // 2))
            off.append(off[-1] + blocks[-1].shape[0])
        self.offsets = np.array(off)
        self.nbf = off[-1]
        self.nshell = len(ex_l)
        T = np.zeros((self.nbf, self.cart.nbf))
        co = self.cart.offsets
        for s, blk in enumerate(blocks):
            T[off[s]:off[s + 1], co[s]:co[s + 1]] = blk
        self.T = T

    @classmethod
    def from_molecule(cls, mol) -> "SphericalBasis":
        n = mol.nshell
        nco = mol.ncontr if getattr(mol, "ncontr", None) is not None else np.ones(n, int)
        pu = mol.pure if getattr(mol, "pure", None) is not None else np.zeros(n, int)
        return cls(mol.shell_xyz, mol.shell_l, mol.nprim, nco, pu, mol.alpha, mol.coef)

    def to_cart(self, X: np.ndarray) -> np.ndarray:
        return self.T.T @ X @ self.T

    def from_cart(self, M: np.ndarray) -> np.ndarray:
        return self.T @ M @ self.T.T

    def one_electron(self, kind: str, **kw) -> np.ndarray:
        return self.from_cart(self.cart.one_electron(kind, **kw))

    def overlap(self) -> np.ndarray:
        return self.one_electron("overlap")

    def _apply(self, fn, X, want_j=True, want_k=True):
        X = np.asarray(X, float)
        single = X.ndim == 2
        Xs = X[None] if single else X
        J, K = fn(np.array([self.to_cart(x) for x in Xs]), want_j, want_k)
        J = np.array([self.from_cart(m) for m in J]) if want_j else None
        K = np.array([self.from_cart(m) for m in K]) if want_k else None
        if single:
            J = J[0] if want_j else None
            K = K[0] if want_k else None
        return J, K

    def jk(self, X, want_j=True, want_k=True):
        """J[X] and K[X] through the Cartesian oracle (canonical quartets)."""
        return self._apply(self.cart.jk, X, want_j, want_k)

    def jk_full(self, X, want_j=True, want_k=True):
        """J[X] and K[X] through the Cartesian oracle's plain definition."""
        return self._apply(self.cart.jk_full, X, want_j, want_k)

    def j_block(self, a: int, b: int, X) -> np.ndarray:
        """Rows of expanded shell a, columns of expanded shell b of J[X]."""
        Xc = np.asarray([self.to_cart(x) for x in (X[None] if np.ndim(X) == 2 else X)])
        blk = self.cart.j_block(a, b, Xc)
        o = self.offsets
        co = self.cart.offsets
        Ta = self.T[o[a]:o[a + 1], co[a]:co[a + 1]]
        Tb = self.T[o[b]:o[b + 1], co[b]:co[b + 1]]
        return np.einsum("ij,mjk,lk->mil", Ta, blk, Tb)

    def k_block(self, a: int, c: int, X) -> np.ndarray:
        """Rows of expanded shell a, columns of expanded shell c of K[X]."""
        Xc = np.asarray([self.to_cart(x) for x in (X[None] if np.ndim(X) == 2 else X)])
        blk = self.cart.k_block(a, c, Xc)
        o = self.offsets
        co = self.cart.offsets
        Ta = self.T[o[a]:o[a + 1], co[a]:co[a + 1]]
        Tc = self.T[o[c]:o[c + 1], co[c]:co[c + 1]]
        return np.einsum("ij,mjk,lk->mil", Ta, blk, Tc)
