"""Algorithmic FP64 operation counts of the generated kernels.

The per-unit figures are one primitive quartet and one contracted shell
quartet of a class (la lb|lc ld): a launch does prim x (its primitive
quartets above the primitive cut) + fixed x (its shell quartets).  Counts follow the
emitted recurrences exactly: every VRR node's expression, one add per
contraction target and primitive quartet, two operations per horizontal
transfer node, and the digestion dot products (per density: 4 nv for a
Coulomb matrix, 8 nv for an exchange matrix, nv = functions in the quartet).
Per primitive quartet, fixed setup (Gaussian product, reduced exponent,
argument, prefactors, W-P and W-Q) and the Boys evaluation (Chebyshev
Clenshaw sum of degree 9, exp counted as one operation, downward
recursion) are counted as listed in SETUP and boys_ops().
"""
from __future__ import annotations

import os
import sys

_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
if _CSRC not in sys.path:
    sys.path.insert(0, _CSRC)

import gen_eri  # noqa: E402

# pq, rsqrt, inv, 3 PQ, rho (2), T (5), pref (2), oo2pq, WP (6)+rp2 (2), WQ (6)+rq2 (2)
SETUP = {"base": 1 + 1 + 1 + 3 + 2 + 5 + 2}


def boys_ops(L: int) -> int:
    cheb = 2 + 9 * 3 + 2           # argument map, Clenshaw steps, final step
    return cheb + (1 + 1 + 3 * L if L > 0 else 0)   # exp, 2T, L fma+mul


def _count_expr(line: str) -> int:
    rhs = line.split("=", 1)[1]
    return rhs.count("*") + rhs.count("+") + rhs.count(" - ")


def per_quartet(la, lb, lc, ld, nprim2_bra=9, nprim2_ket=9, nJ=1, nK=1) -> float:
    prim, fixed = parts(la, lb, lc, ld, nJ, nK)
    return float(nprim2_bra * nprim2_ket * prim + fixed)


def parts(la, lb, lc, ld, nJ=1, nK=1) -> tuple[int, int]:
    """(operations per primitive quartet, operations per contracted shell
    quartet): a class's work is prim x (primitive quartets) + fixed x
    (shell quartets)."""
    L = la + lb + lc + ld
    em = gen_eri.Emitter("")
    vrr = gen_eri.VRR(em, L)
    es, fs = gen_eri.targets(la, lb, lc, ld)
    for e in es:
        for f in fs:
            vrr.get(e, f, 0)
    vrr_ops = sum(_count_expr(x) for x in em.lines)
    setup = SETUP["base"] + (L + 1)
    if L > 0:
        setup += 1 + (8 if la + lb > 0 else 0) + (8 if lc + ld > 0 else 0)
        # recurrence coefficients premultiplied by their integer factors
        setup += 2 * max(la + lb - 1, 0) + 2 * max(lc + ld - 1, 0) + (la + lb if lc + ld > 0 else 0)
    prim = setup + boys_ops(L) + vrr_ops + len(es) * len(fs)
    # horizontal transfers: 2 ops per emitted node
    em2 = gen_eri.Emitter("")
    gen_eri.emit_eri_body(em2, la, lb, lc, ld)
    hrr_nodes = sum(1 for x in em2.lines if x.strip().startswith("const double hb") or x.strip().startswith("const double hk"))
    nv = gen_eri.ncart(la) * gen_eri.ncart(lb) * gen_eri.ncart(lc) * gen_eri.ncart(ld)
    dig = nJ * 4 * nv + nK * 8 * nv
    return prim, 2 * hrr_nodes + nv + dig


if __name__ == "__main__":
    for cls in gen_eri.all_classes(2)[1]:
        print(cls, per_quartet(*cls, nJ=1, nK=8))
