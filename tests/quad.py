"""Independent numerical-quadrature references used to pin the oracle.

Nothing here evaluates a Boys function or a recurrence: overlaps and
electron-repulsion integrals are obtained by Gauss-Hermite quadrature of the
Gaussian integrands, and the Coulomb operator by
1/r12 = (2/sqrt(pi)) int_0^inf exp(-t^2 r12^2) dt with adaptive quadrature
in t (scipy.integrate.quad)."""
from __future__ import annotations

import numpy as np
from numpy.polynomial.hermite import hermgauss
from scipy.integrate import quad

_GH_X, _GH_W = hermgauss(24)


def cart_components(l: int) -> list[tuple[int, int, int]]:
    out = []
    for i in range(l, -1, -1):
        for j in range(l - i, -1, -1):
            out.append((i, j, l - i - j))
    return out


def _pair_1d(i, a, A, j, b, B):
    """(x-A)^i (x-B)^j exp(-a(x-A)^2 - b(x-B)^2) = K exp(-p (x-P)^2) * poly."""
    p = a + b
    P = (a * A + b * B) / p
    K = np.exp(-a * b / p * (A - B) ** 2)
    return p, P, K


def overlap_1d(i, a, A, j, b, B) -> float:
    p, P, K = _pair_1d(i, a, A, j, b, B)
    x = P + _GH_X / np.sqrt(p)
    f = (x - A) ** i * (x - B) ** j
    return float(K * np.sum(_GH_W * f) / np.sqrt(p))


def overlap_prim(ea, a, A, eb, b, B) -> float:
    return float(np.prod([overlap_1d(ea[k], a, A[k], eb[k], b, B[k]) for k in range(3)]))


def _coulomb_axis(t, i, a, A, j, b, B, k, c, C, l, d, D) -> float:
    """int int g_ab(x1) g_cd(x2) exp(-t^2 (x1-x2)^2) dx1 dx2 by 2-D Gauss-Hermite
    after completing the square of the quadratic form."""
    p, P, K1 = _pair_1d(i, a, A, j, b, B)
    q, Q, K2 = _pair_1d(k, c, C, l, d, D)
    t2 = t * t
    dlt = P - Q
    M = np.array([[p + t2, -t2], [-t2, q + t2]])
    bvec = t2 * dlt * np.array([1.0, -1.0])
    ustar = -np.linalg.solve(M, bvec)
    const = t2 * dlt * dlt - bvec @ np.linalg.solve(M, bvec)
    Lc = np.linalg.cholesky(M)
    LinvT = np.linalg.inv(Lc).T
    V1, V2 = np.meshgrid(_GH_X, _GH_X, indexing="ij")
    W = np.outer(_GH_W, _GH_W)
    U = ustar[:, None, None] + np.einsum("ab,bij->aij", LinvT, np.stack([V1, V2]))
    x1 = U[0] + P
    x2 = U[1] + Q
    f = (x1 - A) ** i * (x1 - B) ** j * (x2 - C) ** k * (x2 - D) ** l
    return float(K1 * K2 * np.exp(-const) / np.prod(np.diag(Lc)) * np.sum(W * f))


def eri_prim(ea, a, A, eb, b, B, ec, c, C, ed, d, D) -> float:
    def integrand(t):
        r = 1.0
        for k in range(3):
            r *= _coulomb_axis(t, ea[k], a, A[k], eb[k], b, B[k], ec[k], c, C[k], ed[k], d, D[k])
        return r
    val, _ = quad(integrand, 0.0, np.inf, epsabs=0.0, epsrel=1e-13, limit=400)
    return float(2.0 / np.sqrt(np.pi) * val)


# ---------------------------------------------------------------- one-electron
def _gh_gauss(ws, xs, f) -> float:
    """int f(x) exp(-sum_i w_i (x - X_i)^2) dx for a polynomial f, by
    Gauss-Hermite quadrature about the combined centre."""
    p = float(sum(ws))
    P = sum(w * X for w, X in zip(ws, xs)) / p
    c = 0.0
    for i in range(len(ws)):
        for j in range(i + 1, len(ws)):
            c += ws[i] * ws[j] * (xs[i] - xs[j]) ** 2
    x = P + _GH_X / np.sqrt(p)
    return float(np.exp(-c / p) * np.sum(_GH_W * f(x)) / np.sqrt(p))


def _dpoly(i, a, A):
    """d/dx of (x-A)^i exp(-a (x-A)^2) divided by the Gaussian."""
    return lambda x: (i * (x - A) ** (i - 1) if i > 0 else 0.0) - 2.0 * a * (x - A) ** (i + 1)


def kinetic_prim(ea, a, A, eb, b, B) -> float:
    """-1/2 <a|lap|b> = 1/2 int grad(a) . grad(b) (integration by parts),
    each axis by Gauss-Hermite quadrature."""
    S = [overlap_1d(ea[k], a, A[k], eb[k], b, B[k]) for k in range(3)]
    tot = 0.0
    for k in range(3):
        da, db = _dpoly(ea[k], a, A[k]), _dpoly(eb[k], b, B[k])
        D = _gh_gauss([a, b], [A[k], B[k]], lambda x: da(x) * db(x))
        tot += D * np.prod([S[m] for m in range(3) if m != k])
    return 0.5 * tot


def dipole_prim(ea, a, A, eb, b, B, origin, direction) -> float:
    """<a| r_dir - origin_dir |b> by Gauss-Hermite quadrature."""
    r = 1.0
    for k in range(3):
        i, j = ea[k], eb[k]
        if k == direction:
            f = lambda x, i=i, j=j, k=k: (x - A[k]) ** i * (x - B[k]) ** j * (x - origin[k])
            r *= _gh_gauss([a, b], [A[k], B[k]], f)
        else:
            r *= overlap_1d(i, a, A[k], j, b, B[k])
    return r


def nuclear_prim(ea, a, A, eb, b, B, C) -> float:
    """<a| 1/|r - C| |b> from 1/r = (2/sqrt(pi)) int_0^inf exp(-t^2 r^2) dt:
    each axis a three-centre Gaussian integral by Gauss-Hermite quadrature,
    the t integral adaptive."""
    def integrand(t):
        r = 1.0
        for k in range(3):
            i, j = ea[k], eb[k]
            f = lambda x, i=i, j=j, k=k: (x - A[k]) ** i * (x - B[k]) ** j
            r *= _gh_gauss([a, b, t * t], [A[k], B[k], C[k]], f)
        return r

    # t = sqrt(p) u / sqrt(1 - u^2) maps [0, inf) onto [0, 1) and removes the
    # slow t^-3 tail (a change of variables only)
    sp = np.sqrt(a + b)

    def in_u(u):
        w = 1.0 - u * u
        return integrand(sp * u / np.sqrt(w)) * sp / w ** 1.5

    val, _ = quad(in_u, 0.0, 1.0, epsabs=1e-14, epsrel=1e-12, limit=400)
    return float(2.0 / np.sqrt(np.pi) * val)
