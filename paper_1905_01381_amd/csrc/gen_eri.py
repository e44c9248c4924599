"""Generate the per-class electron-repulsion kernels (build step).

For every class (la lb|lc ld) with la >= lb, lc >= ld and bra class >= ket
class, this script emits straight-line HIP for the Head-Gordon-Pople scheme:

1. Obara-Saika vertical recurrence (VRR) per primitive quartet, built on
   the bra center A and the ket center C:
     [e+1_i,0|f0]^(m) = PA_i [e0|f0]^(m) + WP_i [e0|f0]^(m+1)
                        + e_i/(2p) ([e-1_i,0|f0]^(m) - rho/p [e-1_i,0|f0]^(m+1))
                        + f_i/(2(p+q)) [e0|f-1_i,0]^(m+1)
     [e0|f+1_i,0]^(m) = QC_i [e0|f0]^(m) + WQ_i [e0|f0]^(m+1)
                        + f_i/(2q) ([e0|f-1_i,0]^(m) - rho/q [e0|f-1_i,0]^(m+1))
                        + e_i/(2(p+q)) [e-1_i,0|f0]^(m+1)
   from [00|00]^(m) = 2 pi^{5/2}/(p q sqrt(p+q)) K_ab K_cd F_m(rho |PQ|^2);
2. contraction of the targets [e0|f0] (la <= |e| <= la+lb, lc <= |f| <= lc+ld)
   over primitive quartets;
3. horizontal recurrence (HRR) on the contracted integrals, bra then ket:
     (a, b+1_i| = (a+1_i, b| + AB_i (a, b|,   |c, d+1_i) = |c+1_i, d) + CD_i |c, d);
4. digestion into the Coulomb / exchange partial sums.

The recurrences are the published Obara-Saika (1986) and Head-Gordon-Pople
(1988) relations; every node of the recursion is generated on demand from the
targets, so no unused intermediate is emitted.  Cartesian components are in
lexicographic order (xx, xy, xz, yy, yz, zz).

Usage: python gen_eri.py OUTDIR [--lmax 2]  (writes eri_<class>.hip and eri_registry.hpp)
"""
from __future__ import annotations

import argparse
import os
import sys

DIRS = "xyz"

# Arithmetic type of the code being emitted: "double" (FP64 path) or "float"
# (the precision-routed FP32 path).  Set through set_prec().
PREC = {"T": "double"}


def set_prec(t: str) -> None:
    PREC["T"] = t


def T_() -> str:
    return PREC["T"]


# Trip counts of the primitive-pair loops.  The J/K kernels run each loop to
# the largest count of primitive pairs above the primitive cut among the
# wave's active lanes (a wave-uniform bound, nkp / nkq, computed per step);
# the block kernel, whose tail lanes have returned, runs every record.
LOOP = {"kp": "bra.nprim2", "kq": "ket.nprim2"}


def lit(x) -> str:
    """A numeric literal of the current precision."""
    v = repr(float(x))
    return v + "f" if PREC["T"] == "float" else v


# Task tile of the kernel being emitted: ROWS bra shells b by COLS = 64 / ROWS
# ket shells d, lane = COLS * i + j.
TILE = {"rows": 8}


def set_tile(rows: int) -> None:
    TILE["rows"] = rows


def rows_() -> int:
    return TILE["rows"]


def cols_() -> int:
    return 64 // TILE["rows"]


def red(name: str) -> str:
    """Lane sums: red_j over the COLS lanes of a row, red_i over the ROWS
    lanes of a column."""
    f = "f" if PREC["T"] == "float" else ""
    if name == "red_j":
        return f"red_cols{f}<{cols_()}>"
    if name == "red_i":
        return f"red_rows{f}<{cols_()}>"
    return name + f


def cvx(expr: str) -> str:
    """A double-valued load converted to the current precision."""
    return f"(float){expr}" if PREC["T"] == "float" else expr


def comps(l):
    return [(i, j, l - i - j) for i in range(l, -1, -1) for j in range(l - i, -1, -1)]


def ncart(l):
    return (l + 1) * (l + 2) // 2


def tag(v):
    return "".join(str(x) for x in v)


def sub(v, i, k=1):
    w = list(v)
    w[i] -= k
    return tuple(w)


def add(v, i, k=1):
    w = list(v)
    w[i] += k
    return tuple(w)


class Emitter:
    def __init__(self, ind="    "):
        self.lines: list[str] = []
        self.ind = ind

    def __call__(self, s=""):
        self.lines.append(self.ind + s if s else "")

    def text(self):
        return "\n".join(self.lines)


# --------------------------------------------------------------------------
# VRR
# --------------------------------------------------------------------------
class VRR:
    """Demand-driven Obara-Saika VRR for one primitive quartet."""

    def __init__(self, out: Emitter, L: int):
        self.out = out
        self.memo: dict = {}
        self.L = L
        self.count = 0

    def name(self, e, f, m):
        return f"r{tag(e)}_{tag(f)}_{m}"

    def get(self, e, f, m):
        if min(e) < 0 or min(f) < 0:
            return None
        key = (e, f, m)
        if key in self.memo:
            return self.memo[key]
        nm = self.name(e, f, m)
        if sum(e) == 0 and sum(f) == 0:
            self.memo[key] = f"ss{m}"
            return f"ss{m}"
        terms = []
        if sum(f) > 0:
            i = next(k for k in range(3) if f[k] > 0)
            f1 = sub(f, i)
            a = self.get(e, f1, m)
            b = self.get(e, f1, m + 1)
            terms.append(f"QC{DIRS[i]} * {a}")
            terms.append(f"WQ{DIRS[i]} * {b}")
            if f1[i] > 0:
                f2 = sub(f1, i)
                c = self.get(e, f2, m)
                d = self.get(e, f2, m + 1)
                terms.append(f"cq{f1[i]} * {c} - dq{f1[i]} * {d}")
            if e[i] > 0:
                g = self.get(sub(e, i), f1, m + 1)
                terms.append(f"cx{e[i]} * {g}")
        else:
            i = next(k for k in range(3) if e[k] > 0)
            e1 = sub(e, i)
            a = self.get(e1, f, m)
            b = self.get(e1, f, m + 1)
            terms.append(f"PA{DIRS[i]} * {a}")
            terms.append(f"WP{DIRS[i]} * {b}")
            if e1[i] > 0:
                e2 = sub(e1, i)
                c = self.get(e2, f, m)
                d = self.get(e2, f, m + 1)
                terms.append(f"cp{e1[i]} * {c} - dp{e1[i]} * {d}")
        self.out(f"const {T_()} {nm} = " + " + ".join(terms) + ";")
        self.count += 1
        self.memo[key] = nm
        return nm


def class_name(la, lb, lc, ld):
    s = "spdfg"
    return f"{s[la]}{s[lb]}{s[lc]}{s[ld]}"


def targets(la, lb, lc, ld):
    es = [e for l in range(la, la + lb + 1) for e in comps(l)]
    fs = [f for l in range(lc, lc + ld + 1) for f in comps(l)]
    return es, fs


def emit_prim_header(out: Emitter, la, lb, lc, ld):
    """Open the primitive-quartet loops and emit the per-primitive setup:
    Gaussian-product data, the Boys function F_0..F_L and the VRR
    coefficients (the loops are closed by the caller)."""
    L = la + lb + lc + ld
    T = T_()
    out(f"for (int kp = 0; kp < {LOOP['kp']}; ++kp) {{")
    out("  const double2* br = (const double2*)(bra.rec + ((size_t)ib * bra.nprim2 + kp) * 10);")
    out("  const double2 b0 = br[0];")
    out(f"  const {T} p = b0.x;")
    out(f"  const {T} Kab = b0.y;")
    out("  if (Kab == 0) continue;")
    out("  const double2 b1 = br[1], b2 = br[2];")
    out(f"  const {T} oo2p = b1.x;")
    out(f"  const {T} Px = b1.y, Py = b2.x, Pz = b2.y;")
    if la + lb > 0:
        out("  const double2 b3 = br[3], b4 = br[4];")
        out(f"  const {T} PAx = b3.x, PAy = b3.y, PAz = b4.x;")
    out(f"  for (int kq = 0; kq < {LOOP['kq']}; ++kq) {{")
    out("    const double2* kr = (const double2*)(ket.rec + ((size_t)jk * ket.nprim2 + kq) * 10);")
    out("    const double2 k0 = kr[0], k1 = kr[1], k2 = kr[2];")
    out(f"    const {T} q = k0.x;")
    out(f"    const {T} Kcd = k0.y;")
    out(f"    const {T} oo2q = k1.x;")
    out(f"    const {T} Qx = k1.y, Qy = k2.x, Qz = k2.y;")
    if lc + ld > 0:
        out("    const double2 k3 = kr[3], k4 = kr[4];")
        out(f"    const {T} QCx = k3.x, QCy = k3.y, QCz = k4.x;")
    out(f"    const {T} pq = p + q;")
    out(f"    const {T} rs = {'rsqrt_f64' if T == 'double' else 'rsqrt_f32'}(pq);")
    out(f"    const {T} inv = rs * rs;")
    out(f"    const {T} PQx = Px - Qx, PQy = Py - Qy, PQz = Pz - Qz;")
    out(f"    const {T} rho = p * q * inv;")
    out(f"    const {T} T = rho * (PQx * PQx + PQy * PQy + PQz * PQz);")
    out(f"    {T} F[{L + 1}];")
    out(f"    {'boys_fp64_tab' if T == 'double' else 'boys_fp32_tab'}<{L}>(T, s_boys, F);")
    out(f"    const {T} pref = Kab * Kcd * rs;")
    for m in range(L + 1):
        out(f"    const {T} ss{m} = pref * F[{m}];")
    if L > 0:
        out(f"    const {T} oo2pq = {lit(0.5)} * inv;")
        if la + lb > 0:
            out(f"    const {T} WPx = -q * inv * PQx, WPy = -q * inv * PQy, WPz = -q * inv * PQz;")
            out(f"    const {T} rp2 = q * inv * oo2p;")
        if lc + ld > 0:
            out(f"    const {T} WQx = p * inv * PQx, WQy = p * inv * PQy, WQz = p * inv * PQz;")
            out(f"    const {T} rq2 = p * inv * oo2q;")
        # recurrence coefficients premultiplied by the integer factors they
        # take (k / 2p, k rho / 2p^2, k / 2(p+q), ...): every VRR node is then
        # one multiply and a chain of fused multiply-adds
        for k in range(1, la + lb):
            out(f"    const {T} cp{k} = {lit(k)} * oo2p, dp{k} = {lit(k)} * rp2;")
        for k in range(1, lc + ld):
            out(f"    const {T} cq{k} = {lit(k)} * oo2q, dq{k} = {lit(k)} * rq2;")
        for k in range(1, la + lb + 1 if lc + ld > 0 else 1):
            out(f"    const {T} cx{k} = {lit(k)} * oo2pq;")


def emit_boys_lds(o: Emitter, L: int, f32: bool):
    """Kernel prologue: copy the Boys coefficients of order L into LDS (FP32
    ones for the FP32 path below L = 6, FP64 ones otherwise)."""
    if f32 and L < 6:
        o("  __shared__ float s_boys[BOYS_TAB_L];")
        o(f"  {{ const float* src = (const float*)(boys_tab + BOYS_TAB_DOUBLES) + {L} * BOYS_TAB_L;")
    else:
        o("  __shared__ double s_boys[BOYS_TAB_L];")
        o(f"  {{ const double* src = boys_tab + {L} * BOYS_TAB_L;")
    o("    for (int i = threadIdx.x; i < BOYS_TAB_L; i += blockDim.x) s_boys[i] = src[i]; }")
    o("  __syncthreads();")


def emit_eri_body(out: Emitter, la, lb, lc, ld, prec="double"):
    """Emit: accumulators, primitive loop (Boys + VRR + contraction), HRR.
    Leaves v[NV] (raw contracted (ab|cd), layout [a][b][c][d]) defined."""
    L = la + lb + lc + ld
    es, fs = targets(la, lb, lc, ld)
    eidx = {e: k for k, e in enumerate(es)}
    fidx = {f: k for k, f in enumerate(fs)}
    nE, nF = len(es), len(fs)
    T = T_()
    if T == "float":
        out(f"float acc32[{nE * nF}], cmp32[{nE * nF}];")
        out(f"#pragma unroll")
        out(f"for (int t = 0; t < {nE * nF}; ++t) acc32[t] = cmp32[t] = 0;")
    else:
        out(f"double acc[{nE * nF}];")
        out(f"#pragma unroll")
        out(f"for (int t = 0; t < {nE * nF}; ++t) acc[t] = 0;")
    emit_prim_header(out, la, lb, lc, ld)
    inner = Emitter("    ")
    vrr = VRR(inner, L)
    for e in es:
        for f in fs:
            vrr.get(e, f, 0)
    out.lines.extend(inner.lines)
    for e in es:
        for f in fs:
            k = eidx[e] * nF + fidx[f]
            if T == "float":
                out(f"    kahan_add(acc32[{k}], cmp32[{k}], {vrr.memo[(e, f, 0)]});")
            else:
                out(f"    acc[{k}] += {vrr.memo[(e, f, 0)]};")
    out("  }")
    out("}")
    if T == "float":
        # fold the compensated FP32 sums into FP64; the horizontal transfer
        # and the digestion run in FP64
        out(f"double acc[{nE * nF}];")
        out(f"#pragma unroll")
        out(f"for (int t = 0; t < {nE * nF}; ++t) acc[t] = (double)acc32[t] - (double)cmp32[t];")
        set_prec("double")
        T = "double"
    # HRR bra: (a,b|f] for every ket target f
    A_, B_, C_, D_ = comps(la), comps(lb), comps(lc), comps(ld)
    hb: dict = {}

    def bra(a, b, f):
        key = (a, b, f)
        if key in hb:
            return hb[key]
        if sum(b) == 0:
            nm = f"acc[{eidx[a] * nF + fidx[f]}]"
            hb[key] = nm
            return nm
        i = next(k for k in range(3) if b[k] > 0)
        x = bra(add(a, i), sub(b, i), f)
        y = bra(a, sub(b, i), f)
        nm = f"hb{tag(a)}_{tag(b)}_{tag(f)}"
        out(f"const {T} {nm} = {x} + AB{DIRS[i]} * {y};")
        hb[key] = nm
        return nm

    hk: dict = {}

    def ket(a, b, c, d):
        key = (a, b, c, d)
        if key in hk:
            return hk[key]
        if sum(d) == 0:
            nm = bra(a, b, c)
            hk[key] = nm
            return nm
        i = next(k for k in range(3) if d[k] > 0)
        x = ket(a, b, add(c, i), sub(d, i))
        y = ket(a, b, c, sub(d, i))
        nm = f"hk{tag(a)}_{tag(b)}_{tag(c)}_{tag(d)}"
        out(f"const {T} {nm} = {x} + CD{DIRS[i]} * {y};")
        hk[key] = nm
        return nm

    nv = len(A_) * len(B_) * len(C_) * len(D_)
    out(f"{T} v[{nv}];")
    n = 0
    for a in A_:
        for b in B_:
            for c in C_:
                for d in D_:
                    out(f"v[{n}] = {ket(a, b, c, d)};")
                    n += 1
    return nv, vrr.count


def emit_digest(out: Emitter, la, lb, lc, ld):
    """Digestion of one step of a task: the wave holds the 64 quartets
    (a b_i | c d_j), lane = 8 i + j, with v[] already weighted by the
    permutational degeneracy.  Partial sums are reduced across the lanes
    that share a destination before the single atomic flush:
      J'_ab += 2 v X_cd   (same b: reduce over j)
      J'_cd += 2 v X_ab   (same d: reduce over i)
      K'_ac += v X_bd     (one destination per wave: reduce over all lanes)
      K'_ad += v X_bc     (reduce over i)
      K'_bc += v X_ad     (reduce over j)
      K'_bd += v X_ac     (one destination per lane)."""
    na, nb, nc, nd = ncart(la), ncart(lb), ncart(lc), ncart(ld)

    def V(i, j, k, l):
        return f"v[{((i * nb + j) * nc + k) * nd + l}]"

    out("for (int m = 0; m < dg.nX; ++m) {")
    out("  const int js = dg.jslot[m], ks = dg.kslot[m];")
    out("  if (js >= 0) {")
    for k in range(nc):
        for l in range(nd):
            out(f"    const {T_()} xcd{k}{l} = {cvx(f'ld_x(dg, mc, fc + {k}, fd + {l}, m)')};")
    for i in range(na):
        for j in range(nb):
            out(f"    const {T_()} xab{i}{j} = {cvx(f'ld_x(dg, mc, fa + {i}, fb + {j}, m)')};")
    for i in range(na):
        for j in range(nb):
            s = " + ".join(f"{V(i, j, k, l)} * xcd{k}{l}" for k in range(nc) for l in range(nd))
            out(f"    {{ const {T_()} s = {red('red_j')}({lit(2)} * ({s}));")
            out(f"      if (dg.acc_lvl) {{ if (dj == 0) s_jab[(js * {na * nb} + {i * nb + j}) * {rows_()} + bi] += s; }}")
            out(f"      else if (dj == 0 && rowv) acc_j(mc, jidx(dg, mc, fa + {i}, fb + {j}, js), s); }}")
    for k in range(nc):
        for l in range(nd):
            s = " + ".join(f"{V(i, j, k, l)} * xab{i}{j}" for i in range(na) for j in range(nb))
            out(f"    {{ const {T_()} s = {red('red_i')}({lit(2)} * ({s})); if (bi == 0 && colv) acc_j(mc, jidx(dg, mc, fc + {k}, fd + {l}, js), s); }}")
    out("  }")
    out("  if (ks >= 0) {")
    for j in range(nb):
        for l in range(nd):
            out(f"    const {T_()} xbd{j}{l} = {cvx(f'ld_x(dg, mc, fb + {j}, fd + {l}, m)')};")
    for j in range(nb):
        for k in range(nc):
            out(f"    const {T_()} xbc{j}{k} = {cvx(f'ld_x(dg, mc, fb + {j}, fc + {k}, m)')};")
    for i in range(na):
        for l in range(nd):
            out(f"    const {T_()} xad{i}{l} = {cvx(f'ld_x(dg, mc, fa + {i}, fd + {l}, m)')};")
    for i in range(na):
        for k in range(nc):
            out(f"    const {T_()} xac{i}{k} = {cvx(f'ld_x(dg, mc, fa + {i}, fc + {k}, m)')};")
    for i in range(na):
        for k in range(nc):
            s = " + ".join(f"{V(i, j, k, l)} * xbd{j}{l}" for j in range(nb) for l in range(nd))
            out(f"    {{ const {T_()} s = {red('red_i')}({red('red_j')}({s})); if (lane == 0) acc_k(mc, kidx(dg, mc, fa + {i}, fc + {k}, ks), s); }}")
    for i in range(na):
        for l in range(nd):
            s = " + ".join(f"{V(i, j, k, l)} * xbc{j}{k}" for j in range(nb) for k in range(nc))
            out(f"    {{ const {T_()} s = {red('red_i')}({s});")
            out(f"      if (dg.acc_lvl) {{ if (bi == 0) s_kad[(ks * {na * nd} + {i * nd + l}) * {cols_()} + dj] += s; }}")
            out(f"      else if (bi == 0 && colv) acc_k(mc, kidx(dg, mc, fa + {i}, fd + {l}, ks), s); }}")
    for j in range(nb):
        for k in range(nc):
            s = " + ".join(f"{V(i, j, k, l)} * xad{i}{l}" for i in range(na) for l in range(nd))
            out(f"    {{ const {T_()} s = {red('red_j')}({s}); if (dj == 0 && rowv) acc_k(mc, kidx(dg, mc, fb + {j}, fc + {k}, ks), s); }}")
    # K'_bd does not depend on c: it accumulates per lane in LDS over the
    # task's c range and is flushed once per task (acc_flush); J'_ab and K'_ad
    # (above) likewise, one entry per row / column
    for j in range(nb):
        for l in range(nd):
            s = " + ".join(f"{V(i, j, k, l)} * xac{i}{k}" for i in range(na) for k in range(nc))
            out(f"    {{ const {T_()} s = {s};")
            out(f"      if (dg.acc_lvl < 2) {{ if (active) acc_k(mc, kidx(dg, mc, fb + {j}, fd + {l}, ks), s); }}")
            out(f"      else s_kbd[(ks * {nb * nd} + {j * nd + l}) * 64 + lane] += s; }}")
    out("  }")
    out("}")



# --------------------------------------------------------------------------
# Staged variant for high angular momentum: the contracted intermediates do
# not fit one lane's registers, so the VRR runs in passes over subsets of
# targets (each pass re-runs the primitive loop for its own subset), and the contracted [e0|f0], the bra-transferred (ab|f] and the
# final (ab|cd) go through a per-wave global stage laid out [index][lane]
# (coalesced, private to the wave).
# --------------------------------------------------------------------------

# Per-class staging: (targets per pass, waves per SIMD the kernel is
# compiled for).  Smaller passes re-run more of the VRR but free registers
# for a second wave per SIMD; larger ones re-run less at one wave, which
# leaves the FP64 pipeline partly idle.  Each class takes the measured
# faster side on MI355X.  At one wave, (dd|pp) and (dd|dp) keep whole bra
# groups per pass (7 and 3 bra components with every ket target) and (dd|ds)
# runs four greedy passes.
STAGE_CFG = {
    (2, 1, 1, 1): (40, 2),
    (2, 1, 2, 1): (32, 2),
    (2, 2, 1, 1): (63, 1),
    (2, 2, 2, 0): (48, 1),
    (2, 2, 2, 1): (48, 1),
    (2, 2, 2, 2): (48, 1),
}

# Unstaged classes whose register count sits just above an occupancy step:
# a minimum of waves per SIMD makes the compiler fit that step (a few bytes
# of spill outside the primitive loop).  (ps|ps) goes from 2 to 3 waves and
# (ps|ss) from 3 to 4, 17 % and 8 % faster on MI355X; (pp|ss) at 3 waves
# was slower, and classes further from a step spill inside the loop.
# (ss|ss) and (ds|ps) sit a few registers above 5 and 2 waves with the
# fixed-point flushes and the LDS task accumulators.  (pp|ps) needs 270
# registers at one wave; at two it spills 56 bytes per lane, all of it at
# the task and step level, and went from 58.3 to 47.7 ms per launch on the
# 40-atom 3s2p1d two-component build.
UNSTAGED_WAVES = {
    (0, 0, 0, 0): 5,
    (1, 0, 1, 0): 3,
    (1, 0, 0, 0): 4,
    (2, 0, 1, 0): 2,
    (1, 1, 1, 0): 2,
}


def is_staged(la, lb, lc, ld):
    return (la, lb, lc, ld) in STAGE_CFG


def stage_cap(la, lb, lc, ld):
    return STAGE_CFG[(la, lb, lc, ld)][0]


def waves_per_simd(la, lb, lc, ld):
    if is_staged(la, lb, lc, ld):
        return STAGE_CFG[(la, lb, lc, ld)][1]
    return UNSTAGED_WAVES.get((la, lb, lc, ld), 1)


def _vrr_ancestors(la, lb, lc, ld):
    """For every contraction target [e0|f0]: the VRR nodes it needs and the
    operation count of each node."""
    L = la + lb + lc + ld
    es, fs = targets(la, lb, lc, ld)
    em = Emitter("")
    full = VRR(em, L)
    for e in es:
        for f in fs:
            full.get(e, f, 0)
    ops = {}
    for line in em.lines:
        lhs, rhs = line.split("=", 1)
        ops[lhs.split()[-1]] = rhs.count("*") + rhs.count("+") + rhs.count(" - ")
    keys = sorted(full.memo)
    col = {k: i for i, k in enumerate(keys)}
    w = [ops.get(full.memo[k], 0) for k in keys]
    anc = {}
    for e in es:
        for f in fs:
            v = VRR(Emitter(""), L)
            v.get(e, f, 0)
            anc[(e, f)] = sorted(col[k] for k in v.memo)
    return anc, w


PASS_OVERHEAD = 150


def _pass_cost(la, lb, lc, ld, subsets):
    """VRR operations of a pass plan (each pass re-runs its ancestors)."""
    anc, w = _vrr_ancestors(la, lb, lc, ld)
    return sum(sum(w[k] for k in set().union(*(anc[t] for t in sub))) for sub in subsets)


def stage_subsets(la, lb, lc, ld, cap=None):
    """Split the targets into passes of <= cap targets; every pass re-runs
    the VRR for the ancestors of its own targets.  Two plans are costed by
    the VRR operations they re-run and the cheaper is kept: passes over a
    few bra targets e with every ket target f (the recursion builds f on top
    of a fixed e, so those share most ancestors), and greedy filling (seed
    with the most expensive remaining target, then add the target that
    brings the fewest new operations)."""
    if cap is None:
        cap = stage_cap(la, lb, lc, ld)
    es, fs = targets(la, lb, lc, ld)
    plans = [_greedy_subsets(la, lb, lc, ld, cap)]
    k = cap // len(fs)
    if k >= 1:
        plans.append([[(e, f) for e in es[i:i + k] for f in fs] for i in range(0, len(es), k)])
    # each pass also repeats the primitive setup, the Boys function and the
    # primitive-pair loads: about PASS_OVERHEAD operations per primitive
    return min(plans, key=lambda pl: (_pass_cost(la, lb, lc, ld, pl) + PASS_OVERHEAD * len(pl), len(pl)))


def _greedy_subsets(la, lb, lc, ld, cap):
    import numpy as np
    anc, w = _vrr_ancestors(la, lb, lc, ld)
    tg = sorted(anc)
    M = np.zeros((len(tg), len(w)), dtype=bool)
    for r, t in enumerate(tg):
        M[r, anc[t]] = True
    W = np.asarray(w, dtype=np.int64)
    cost = M.astype(np.int64) @ W
    left = np.ones(len(tg), dtype=bool)
    out = []
    while left.any():
        seed = int(np.flatnonzero(left)[np.argmax(cost[left])])
        cur, have = [seed], M[seed].copy()
        left[seed] = False
        while len(cur) < cap and left.any():
            idx = np.flatnonzero(left)
            extra = (M[idx] & ~have).astype(np.int64) @ W
            pick = int(idx[np.argmin(extra)])
            cur.append(pick)
            have |= M[pick]
            left[pick] = False
        out.append([tg[r] for r in sorted(cur)])
    return out


def stage_layout(la, lb, lc, ld):
    es, fs = targets(la, lb, lc, ld)
    nE, nF = len(es), len(fs)
    nab = ncart(la) * ncart(lb)
    ncd = ncart(lc) * ncart(ld)
    G0, HB0 = 0, nE * nF
    V0 = HB0 + nab * nF
    return G0, HB0, V0, V0 + nab * ncd


def emit_staged_eri(out: Emitter, la, lb, lc, ld):
    L = la + lb + lc + ld
    es, fs = targets(la, lb, lc, ld)
    eidx = {e: k for k, e in enumerate(es)}
    fidx = {f: k for k, f in enumerate(fs)}
    nF = len(fs)
    G0, HB0, V0, _ = stage_layout(la, lb, lc, ld)
    nodes = 0
    for sub_ in stage_subsets(la, lb, lc, ld):
        out("{")
        out(f"  {T_()} acc[{len(sub_)}];")
        out(f"  #pragma unroll")
        out(f"  for (int t = 0; t < {len(sub_)}; ++t) acc[t] = 0;")
        if T_() == "float":
            out(f"  float cmp[{len(sub_)}];")
            out(f"  #pragma unroll")
            out(f"  for (int t = 0; t < {len(sub_)}; ++t) cmp[t] = 0;")
            store = lambda k: f"(double)acc[{k}] - (double)cmp[{k}]"
        else:
            store = lambda k: f"acc[{k}]"
        hdr = Emitter(out.ind + "  ")
        emit_prim_header(hdr, la, lb, lc, ld)
        out.lines.extend(hdr.lines)
        inner = Emitter(out.ind + "      ")
        vrr = VRR(inner, L)
        for (e, f) in sub_:
            vrr.get(e, f, 0)
        nodes += vrr.count
        out.lines.extend(inner.lines)
        for k, (e, f) in enumerate(sub_):
            if T_() == "float":
                out(f"      kahan_add(acc[{k}], cmp[{k}], {vrr.memo[(e, f, 0)]});")
            else:
                out(f"      acc[{k}] += {vrr.memo[(e, f, 0)]};")
        out("    }")
        out("  }")
        for k, (e, f) in enumerate(sub_):
            out(f"  STS({G0 + eidx[e] * nF + fidx[f]}, {store(k)});")
        out("}")
        out("stage_fence();")
    A_, B_, C_, D_ = comps(la), comps(lb), comps(lc), comps(ld)
    set_prec("double")  # transfers and digestion in FP64 in both paths
    # bra transfer, one ket target f at a time
    for f in fs:
        out("{")
        needed = set()

        def collect(a, b):
            if sum(b) == 0:
                needed.add(a)
                return
            i = next(k for k in range(3) if b[k] > 0)
            collect(add(a, i), sub(b, i))
            collect(a, sub(b, i))

        for a in A_:
            for b in B_:
                collect(a, b)
        for e in sorted(needed, key=lambda x: eidx[x]):
            out(f"  const {T_()} g{tag(e)} = STL({G0 + eidx[e] * nF + fidx[f]});")
        memo = {}

        def bra(a, b):
            if (a, b) in memo:
                return memo[(a, b)]
            if sum(b) == 0:
                memo[(a, b)] = f"g{tag(a)}"
                return memo[(a, b)]
            i = next(k for k in range(3) if b[k] > 0)
            x = bra(add(a, i), sub(b, i))
            y = bra(a, sub(b, i))
            nm = f"h{tag(a)}_{tag(b)}"
            out(f"  const {T_()} {nm} = {x} + AB{DIRS[i]} * {y};")
            memo[(a, b)] = nm
            return nm

        for ia, a in enumerate(A_):
            for ib_, b in enumerate(B_):
                out(f"  STS({HB0 + (ia * len(B_) + ib_) * nF + fidx[f]}, {bra(a, b)});")
        out("}")
    out("stage_fence();")
    # ket transfer, one bra function pair at a time; weight by degeneracy
    ncd = len(C_) * len(D_)
    for ab in range(len(A_) * len(B_)):
        out("{")
        needed = set()

        def collectk(c, d):
            if sum(d) == 0:
                needed.add(c)
                return
            i = next(k for k in range(3) if d[k] > 0)
            collectk(add(c, i), sub(d, i))
            collectk(c, sub(d, i))

        for c in C_:
            for d in D_:
                collectk(c, d)
        for f in sorted(needed, key=lambda x: fidx[x]):
            out(f"  const {T_()} q{tag(f)} = STL({HB0 + ab * nF + fidx[f]});")
        memo = {}

        def ket(c, d):
            if (c, d) in memo:
                return memo[(c, d)]
            if sum(d) == 0:
                memo[(c, d)] = f"q{tag(c)}"
                return memo[(c, d)]
            i = next(k for k in range(3) if d[k] > 0)
            x = ket(add(c, i), sub(d, i))
            y = ket(c, sub(d, i))
            nm = f"k{tag(c)}_{tag(d)}"
            out(f"  const {T_()} {nm} = {x} + CD{DIRS[i]} * {y};")
            memo[(c, d)] = nm
            return nm

        for ic, c in enumerate(C_):
            for id_, d in enumerate(D_):
                out(f"  STS({V0 + ab * ncd + ic * len(D_) + id_}, deg * {ket(c, d)});")
        out("}")
    out("stage_fence();")
    return nodes


# Integrals a staged digestion group keeps in registers (measured per class:
# larger groups share more density gathers until the kernel starts to
# spill in the primitive loop).  The one-wave classes have up to 512
# registers per lane and take larger groups.
DIGEST_VALUES = 54
DIGEST_VALUES_CLASS = {(2, 2, 1, 1): 108, (2, 2, 2, 0): 108, (2, 2, 2, 1): 108, (2, 2, 2, 2): 144}


def emit_staged_digest(out: Emitter, la, lb, lc, ld):
    """Digestion reading (ab|cd) from the stage: for every group of output
    elements the contributing integrals are loaded once, then the loop over
    densities gathers each X element once for the whole group (lane
    reductions and flush as in emit_digest)."""
    na, nb, nc, nd = ncart(la), ncart(lb), ncart(lc), ncart(ld)
    _, _, V0, _ = stage_layout(la, lb, lc, ld)

    def Vi(i, j, k, l):
        return V0 + ((i * nb + j) * nc + k) * nd + l

    # (name, output index pairs, summed index pairs, V index fn, X row/col, dest, reduction, guard, scale, slot)
    specs = [
        ("J_ab", [(i, j) for i in range(na) for j in range(nb)], [(k, l) for k in range(nc) for l in range(nd)],
         lambda o, s: Vi(o[0], o[1], s[0], s[1]), ("fc", "fd"), ("J", "fa", "fb", "js"), "red_j", "dj == 0 && rowv", "2.0 * "),
        ("J_cd", [(k, l) for k in range(nc) for l in range(nd)], [(i, j) for i in range(na) for j in range(nb)],
         lambda o, s: Vi(s[0], s[1], o[0], o[1]), ("fa", "fb"), ("J", "fc", "fd", "js"), "red_i", "bi == 0 && colv", "2.0 * "),
        ("K_ac", [(i, k) for i in range(na) for k in range(nc)], [(j, l) for j in range(nb) for l in range(nd)],
         lambda o, s: Vi(o[0], s[0], o[1], s[1]), ("fb", "fd"), ("K", "fa", "fc", "ks"), "red_all", "lane == 0", ""),
        ("K_ad", [(i, l) for i in range(na) for l in range(nd)], [(j, k) for j in range(nb) for k in range(nc)],
         lambda o, s: Vi(o[0], s[0], s[1], o[1]), ("fb", "fc"), ("K", "fa", "fd", "ks"), "red_i", "bi == 0 && colv", ""),
        ("K_bc", [(j, k) for j in range(nb) for k in range(nc)], [(i, l) for i in range(na) for l in range(nd)],
         lambda o, s: Vi(s[0], o[0], o[1], s[1]), ("fa", "fd"), ("K", "fb", "fc", "ks"), "red_j", "dj == 0 && rowv", ""),
        ("K_bd", [(j, l) for j in range(nb) for l in range(nd)], [(i, k) for i in range(na) for k in range(nc)],
         lambda o, s: Vi(s[0], o[0], s[1], o[1]), ("fa", "fc"), ("K", "fb", "fd", "ks"), "none", "active", ""),
    ]
    # J'_ab, K'_ad and K'_bd do not depend on c: they are summed over the
    # task's c walk in the wave's own stage region (each entry read and
    # written by one lane only, so in a fixed order) and added to J'/K' once
    # per task (emit_staged_acc_flush) instead of every step
    nb_nd, na_nb = nb * nd, na * nb
    sacc_entry = {"J_ab": lambda o: nb_nd + o[0] * nb + o[1],
                  "K_ad": lambda o: nb_nd + na_nb + o[0] * nd + o[1],
                  "K_bd": lambda o: o[0] * nd + o[1]}
    sacc_guard = {"J_ab": "dj == 0", "K_ad": "bi == 0", "K_bd": None}
    for (name, outs, sums, vfn, (xr, xc), (arr, dr, dc, slot), rd, guard, scale) in specs:
        isJ = arr == "J"
        # outputs in groups of g: the group's integrals stay in registers and
        # each density's X block is gathered once per group, not per output
        g = max(1, DIGEST_VALUES_CLASS.get((la, lb, lc, ld), DIGEST_VALUES) // len(sums))
        for c0 in range(0, len(outs), g):
            grp = outs[c0:c0 + g]
            out("{")
            for u, o in enumerate(grp):
                for t, sidx in enumerate(sums):
                    out(f"  const {T_()} w{u}_{t} = STL({vfn(o, sidx)});")
            out("  for (int m = 0; m < dg.nX; ++m) {")
            out(f"    const int {slot} = dg.{'jslot' if isJ else 'kslot'}[m];")
            out(f"    if ({slot} < 0) continue;")
            for t, sidx in enumerate(sums):
                out(f"    const {T_()} x{t} = {cvx(f'ld_x(dg, mc, {xr} + {sidx[0]}, {xc} + {sidx[1]}, m)')};")
            idxf = "jidx" if isJ else "kidx"
            for u, o in enumerate(grp):
                terms = " + ".join(f"w{u}_{t} * x{t}" for t in range(len(sums)))
                sc = f"{lit(2)} * " if scale else ""
                val = f"{sc}({terms})"
                if rd == "red_all":
                    val = f"{red('red_i')}({red('red_j')}({val}))"
                elif rd != "none":
                    val = f"{red(rd)}({val})"
                out(f"    {{ const {T_()} s = {val};")
                if name in sacc_entry and (la, lb, lc, ld) in STAGE_ACC_CLASSES:
                    e = f"SACC(m, {sacc_entry[name](o)})"
                    g_ = sacc_guard[name]
                    upd = f"STS({e}, STL({e}) + (double)s);"
                    out(f"      {'if (' + g_ + ') ' if g_ else ''}{upd} }}")
                else:
                    out(f"      if ({guard}) acc_{arr.lower()}(mc, {idxf}(dg, mc, {dr} + {o[0]}, {dc} + {o[1]}, {slot}), s); }}")
            out("  }")
            out("}")


def all_classes(lmax):
    pcls = [(a, b) for a in range(lmax + 1) for b in range(a + 1)]
    out = []
    for i, P in enumerate(pcls):
        for Q in pcls[: i + 1]:
            out.append((P[0], P[1], Q[0], Q[1]))
    return pcls, out


HEADER = """// Generated by gen_eri.py -- do not edit.  Per-class Obara-Saika /
// Head-Gordon-Pople electron-repulsion kernels (one thread per contracted
// shell quartet) with Coulomb/exchange digestion."""


# Staged classes that sum J'_ab, K'_ad and K'_bd over a task in their stage
# region.  Measured on the 40-atom 3s2p1d two-component build: (dp|pp)
# 110.8 -> 82.0 ms and (dp|dp) 84.5 -> 83.1 ms (two waves per SIMD); the
# one-wave classes, which cannot hide the read-modify-write latency behind
# another wave, were 3-8 % slower and keep the per-step flush; longer c
# ranges (4 to 32 steps per task, fewer flushes per quartet) did not bring
# them back to the per-step flush either ((dd|dp): 105 ms at the default
# range, 98 ms at 16 steps, against 97 ms without the accumulators).
STAGE_ACC_CLASSES = {(2, 1, 1, 1), (2, 1, 2, 1)}


def staged_acc_doubles(la, lb, lc, ld):
    """Stage-region doubles per lane and density slot for the task
    accumulators of a staged class: K'_bd, J'_ab, K'_ad (in that order)."""
    if (la, lb, lc, ld) not in STAGE_ACC_CLASSES:
        return 0
    na, nb, nd = ncart(la), ncart(lb), ncart(ld)
    return nb * nd + na * nb + na * nd


def emit_staged_acc_zero(o: Emitter, la, lb, lc, ld):
    o(f"    for (int t = 0; t < {staged_acc_doubles(la, lb, lc, ld)} * dg.nX; ++t) STS(SACC(0, t), 0.0);")


def emit_staged_acc_flush(o: Emitter, la, lb, lc, ld):
    """Once per task: add the stage accumulators to J' and K' (fixed point)."""
    na, nb, nd = ncart(la), ncart(lb), ncart(ld)
    o("    stage_fence();")
    o("    for (int m = 0; m < dg.nX; ++m) {")
    o("      const int js = dg.jslot[m], ks = dg.kslot[m];")
    o("      if (js >= 0 && dj == 0 && rowv) {")
    for i in range(na):
        for j in range(nb):
            o(f"        {{ const double s = STL(SACC(m, {nb * nd + i * nb + j}));")
            o(f"          if (s != 0.0) acc_j(mc, jidx(dg, mc, fa + {i}, fb + {j}, js), s); }}")
    o("      }")
    o("      if (ks >= 0 && bi == 0 && fdv >= 0) {")
    for i in range(na):
        for l in range(nd):
            o(f"        {{ const double s = STL(SACC(m, {nb * nd + na * nb + i * nd + l}));")
            o(f"          if (s != 0.0) acc_k(mc, kidx(dg, mc, fa + {i}, fdv + {l}, ks), s); }}")
    o("      }")
    o("      if (ks >= 0 && rowv && fdv >= 0) {")
    for j in range(nb):
        for l in range(nd):
            o(f"        {{ const double s = STL(SACC(m, {j * nd + l}));")
            o(f"          if (s != 0.0) acc_k(mc, kidx(dg, mc, fb + {j}, fdv + {l}, ks), s); }}")
    o("      }")
    o("    }")
    o("    stage_fence();")


def acc_doubles(la, lb, lc, ld):
    """LDS doubles per density slot for the task accumulator of K'_bd (one
    per lane and element; unstaged classes only)."""
    return 0 if is_staged(la, lb, lc, ld) else 64 * ncart(lb) * ncart(ld)


# Rows of the task tile per unstaged class (default 8: 8 b x 8 d).  Fewer
# rows (R b x 64/R d) flush fewer K'_bc lanes per step (R nb nc nK) and more
# J'_cd lanes (64/R nc nd nJ).  Measured on the 40-atom two-component build
# (nK = 8, nJ = 1), every class tried was slower with fewer rows: (dp|ps)
# 77.6 -> 84.4 ms and (dp|ds) 89.1 -> 96.4 ms at R = 2, (ps|ps) 30.6 -> 32.6
# and (ds|ps) 52.7 -> 55.3 ms at R = 4, (ds|ds) 35.2 -> 37.9 ms at R = 2.
# More rows were slower too, even with each a's b partners ordered by their
# surviving primitive pairs (16 b x 4 d): (ps|ss) 26.7 -> 30.1 ms, (pp|ss)
# 15.6 -> 21.3, (ss|ss) 6.6 -> 8.6.  So every class keeps R = 8.
TILE_ROWS = {}


def tile_rows(la, lb, lc, ld):
    if is_staged(la, lb, lc, ld):
        return 8
    return TILE_ROWS.get((la, lb, lc, ld), 8)


def acc8_doubles(la, lb, lc, ld):
    """LDS doubles per density slot for the task accumulators of J'_ab (one
    per wave row) and K'_ad (one per wave column); unstaged classes only."""
    r = tile_rows(la, lb, lc, ld)
    return 0 if is_staged(la, lb, lc, ld) else r * ncart(la) * ncart(lb) + (64 // r) * ncart(la) * ncart(ld)


def emit_acc_zero(o: Emitter, la, lb, lc, ld):
    """Each accumulator entry is zeroed, summed and flushed by its own lane,
    so no cross-lane ordering is needed."""
    kbd = acc_doubles(la, lb, lc, ld) // 64
    nab, nad = ncart(la) * ncart(lb), ncart(la) * ncart(ld)
    o("    if (dg.acc_lvl >= 2)")
    o(f"      for (int t = 0; t < {kbd} * dg.nK; ++t) s_kbd[t * 64 + lane] = 0.0;")
    o("    if (dg.acc_lvl) {")
    o(f"      if (dj == 0) for (int t = 0; t < {nab} * dg.nJ; ++t) s_jab[t * {rows_()} + bi] = 0.0;")
    o(f"      if (bi == 0) for (int t = 0; t < {nad} * dg.nK; ++t) s_kad[t * {cols_()} + dj] = 0.0;")
    o("    }")


def emit_acc_flush(o: Emitter, la, lb, ld):
    """Once per task: add the LDS accumulators to J' and K'."""
    na, nb, nd = ncart(la), ncart(lb), ncart(ld)
    o("    if (dg.acc_lvl) {")
    o("      for (int m = 0; m < dg.nX; ++m) {")
    o("        const int js = dg.jslot[m], ks = dg.kslot[m];")
    o("        if (js >= 0 && dj == 0 && rowv) {")
    for i in range(na):
        for j in range(nb):
            o(f"          {{ const double s = s_jab[(js * {na * nb} + {i * nb + j}) * {rows_()} + bi];")
            o(f"            if (s != 0.0) acc_j(mc, jidx(dg, mc, fa + {i}, fb + {j}, js), s); }}")
    o("        }")
    o("        if (ks >= 0 && bi == 0 && fdv >= 0) {")
    for i in range(na):
        for l in range(nd):
            o(f"          {{ const double s = s_kad[(ks * {na * nd} + {i * nd + l}) * {cols_()} + dj];")
            o(f"            if (s != 0.0) acc_k(mc, kidx(dg, mc, fa + {i}, fdv + {l}, ks), s); }}")
    o("        }")
    o("      }")
    o("    }")
    o("    if (dg.acc_lvl >= 2 && rowv && dval && fdv >= 0) {")
    o("      for (int m = 0; m < dg.nX; ++m) {")
    o("        const int ks = dg.kslot[m];")
    o("        if (ks < 0) continue;")
    for j in range(nb):
        for l in range(nd):
            o(f"        {{ const double s = s_kbd[(ks * {nb * nd} + {j * nd + l}) * 64 + lane];")
            o(f"          if (s != 0.0) acc_k(mc, kidx(dg, mc, fb + {j}, fdv + {l}, ks), s); }}")
    o("      }")
    o("    }")


def emit_jk_kernel(la, lb, lc, ld, prec: str) -> tuple[str, int, int]:
    """One J/K kernel of a class in one precision.  Without screening or
    routing the FP64 kernel walks every task; otherwise each kernel walks the
    task list and step masks of its own precision that the build's
    classification pass wrote."""
    cn = class_name(la, lb, lc, ld)
    L = la + lb + lc + ld
    staged = is_staged(la, lb, lc, ld)
    nv = ncart(la) * ncart(lb) * ncart(lc) * ncart(ld)
    set_prec(prec)
    set_tile(tile_rows(la, lb, lc, ld))
    body = Emitter("    ")
    dig = Emitter("    ")
    LOOP.update(kp="nkp", kq="nkq")
    if staged:
        nvrr = emit_staged_eri(body, la, lb, lc, ld)
    else:
        _, nvrr = emit_eri_body(body, la, lb, lc, ld)
    LOOP.update(kp="bra.nprim2", kq="ket.nprim2")
    set_prec("double")
    if staged:
        emit_staged_digest(dig, la, lb, lc, ld)
    else:
        emit_digest(dig, la, lb, lc, ld)
    stage_n = stage_layout(la, lb, lc, ld)[3] if staged else 0
    f32 = prec == "float"
    kname = f"eri_jk{'32' if f32 else ''}_{cn}"
    o = Emitter("")
    o(f"// ({cn}) L={L}: {nv} integrals, {nvrr} VRR nodes per primitive quartet, {prec}")
    same_ab = int(la == lb)
    same_cd = int(lc == ld)
    same_cls = int((la, lb) == (lc, ld))
    wpe = waves_per_simd(la, lb, lc, ld)
    lb_ = f"__launch_bounds__(64, {wpe})" if wpe > 1 else "__launch_bounds__(64)"
    o(f"__global__ {lb_} void {kname}(const PairSet bra, const PairSet ket, const TaskMap tm, const Digest dg, const double* __restrict__ boys_tab)")
    o("{")
    if f32:
        o("  if (dg.mode != 1) return;")
    emit_boys_lds(o, L, f32)
    kbd = acc_doubles(la, lb, lc, ld)
    if kbd:
        # task accumulators, sized at launch by the Coulomb / exchange slots of
        # the build: K'_bd [nK][nbd][64 lanes] (level 2), then
        # J'_ab [nJ][nab][8 rows] and K'_ad [nK][nad][8 columns] (level >= 1)
        o("  extern __shared__ double s_acc[];")
        o(f"  double* const s_kbd = s_acc;")
        o(f"  double* const s_jab = s_acc + (dg.acc_lvl >= 2 ? {kbd} * dg.nK : 0);")
        o(f"  double* const s_kad = s_jab + {ncart(la) * ncart(lb) * rows_()} * dg.nJ;")
    o("  const int lane = threadIdx.x;")
    o(f"  const int bi = lane >> {cols_().bit_length() - 1}, dj = lane & {cols_() - 1};")
    sacc = staged_acc_doubles(la, lb, lc, ld)
    if staged:
        # per-wave region: the integral stage, then the task accumulators
        # ([density slot][entry] per lane)
        o(f"  const int sreg = {stage_n} + {sacc} * dg.nX;")
        o(f"  const stage_rsrc srs = stage_make(dg.stage + (size_t)blockIdx.x * ((size_t)sreg * 64), sreg * 512);")
        o("  const int svo = lane * 8;")
        o("#define STL(i) stage_load(srs, svo, (i))")
        o("#define STS(i, x) stage_store(srs, svo, (i), (x))")
        o(f"#define SACC(m, e) ({stage_n} + (m) * {sacc} + (e))")
    # With screening or routing, the build's classification pass lists the
    # tasks that have steps of this kernel's precision and marks those steps
    # (bit c - c_lo of the task's mask); the kernel walks only them.
    # With bit 1 of dg.rot (and a grid that is a multiple of 8) the tasks are
    # dealt in runs of 8 consecutive tasks per XCD (the workgroups go to the
    # 8 XCDs round robin): a run shares bra shells and density rows in one
    # XCD's L2, and the runs stay short enough to keep the longest-first
    # order balanced across the XCDs.
    o("  const bool listed = tm.list != nullptr;")
    o("  const int ntk = listed ? *tm.list_n : tm.ntask;")
    o("  const bool xo = (dg.rot & 2) && (gridDim.x & 7) == 0;")
    o("  const int nit = xo ? (ntk + 63) & ~63 : ntk;")
    o("  for (int it = blockIdx.x; it < nit; it += gridDim.x) {")
    o("    // it = 64 g + 8 q + x (x: the XCD) -> task 64 g + 8 x + q")
    o("    const int itx = xo ? (it & ~63) + ((it & 7) << 3) + ((it >> 3) & 7) : it;")
    o("    if (itx >= ntk) continue;")
    o("    const int task = listed ? tm.list[itx] : itx;")
    o(f"    const unsigned long long smask = listed ? tm.masks[2 * task + {1 if f32 else 0}] : ~0ull;")
    o("    const int4 tk = tm.tasks[task];")
    o("    const int4 tk2 = tm.tasks2[task];")
    o("    const MolView mc = mol_view(dg, tm, tk2.z);")
    o("    const int a_idx = tk.x, b_idx = tk.y + bi, d_idx = tk.z + dj;")
    o("    const bool rowv = b_idx < tk2.x;")
    o("    const bool dval = d_idx < tk2.y;")
    o("    const int a = tm.shl_a[a_idx];")
    o("    const int b = tm.shl_b[rowv ? b_idx : tk.y];")
    o("    const int d = tm.shl_d[dval ? d_idx : tk.z];")
    o("    const int ib = mc.ppos[spair(mc, a, b)];")
    o("    const int fa = bra.fa[ib], fb = bra.fb[ib];")
    t = "double"
    if lb > 0:
        o(f"    const {t} ABx = bra.ABx[ib], ABy = bra.ABy[ib], ABz = bra.ABz[ib];")
    o("    const int c_lo = tk.w, c_hi = tk2.w;")
    if kbd:
        emit_acc_zero(o, la, lb, lc, ld)
    if sacc:
        emit_staged_acc_zero(o, la, lb, lc, ld)
    if kbd or sacc:
        o("    int fdv = -1;  // first function of d (valid once a step with this d ran)")
    # With bit 0 of dg.rot the walk over the c range starts at step (task mod length)
    # and wraps around, so that tasks sharing a bra shell a do not flush the
    # same K'_ac elements at the same time; the steps and their sums are the
    # same in either order.
    o("    const int n_st = c_hi - c_lo + 1;")
    o("    const int rot0 = (dg.rot & 1) ? task % n_st : 0;")
    o("    for (int st = 0; st < n_st; ++st) {")
    o("      int s_i = st + rot0;")
    o("      if (s_i >= n_st) s_i -= n_st;")
    o("      if (!((smask >> s_i) & 1ull)) continue;")
    o("      const int c_idx = c_lo + s_i;")
    o("      const int c = tm.shl_c[c_idx];")
    o(f"      const bool colv = dval{' && d_idx <= c_idx' if same_cd else ''};")
    o("      bool active = rowv && colv;")
    if same_cls:
        o("      if (c_idx == a_idx) active = active && b >= d;  // shell numbers: the b list is ordered per a")
    o(f"      const int jk = mc.ppos[spair(mc, c, colv ? d : {'c' if same_cd else 'd'})];")
    o("      const int fc = ket.fa[jk], fd = ket.fb[jk];")
    if kbd or sacc:
        o("      if (colv) fdv = fd;")
    o("      if (dg.skip > 0.0 && active) active = quartet_bound(mc, bra.Q[ib], ket.Q[jk], a, b, c, d) >= dg.skip;")
    o("      if (!__any(active)) continue;")
    if ld > 0:
        o(f"      const {t} CDx = ket.ABx[jk], CDy = ket.ABy[jk], CDz = ket.ABz[jk];")
    o("      double deg = active ? 1.0 : 0.0;")
    if same_ab:
        o("      if (a == b) deg *= 0.5;")
    if same_cd:
        o("      if (c == d) deg *= 0.5;")
    if same_cls:
        o("      if (a == c && b == d) deg *= 0.5;")
    o("      const int nkp = wave_max_bound(active ? bra.nsig[ib] : 0, bra.nprim2);")
    o("      const int nkq = wave_max_bound(active ? ket.nsig[jk] : 0, ket.nprim2);")
    body.lines = ["  " + x if x else x for x in body.lines]
    o(body.text())
    if not staged:
        o(f"      #pragma unroll")
        o(f"      for (int t = 0; t < {nv}; ++t) v[t] *= deg;")
    dig.lines = ["  " + x if x else x for x in dig.lines]
    o(dig.text())
    o("    }")
    if kbd:
        emit_acc_flush(o, la, lb, ld)
    if sacc:
        emit_staged_acc_flush(o, la, lb, lc, ld)
    o("  }")
    if staged:
        o("#undef STL")
        o("#undef STS")
        o("#undef SACC")
    o("}")
    o("")
    return o.text(), nvrr, stage_n


# Classes also generated with bra and ket exchanged, (lc ld|la lb): the same
# unique quartets with the wave's loop running over the other pair's first
# shell.  A step's flushes are J'_cd, K'_ac and K'_bc (eight rows of K'_bc
# per step); exchanged, K'_bc becomes the original K'_ad, so for classes
# with ncart(la) ncart(ld) < ncart(lb) ncart(lc) the exchange flushes fewer
# exchange partial sums per step.  The build picks an orientation per class
# (cq_autotune times both).
SWAP_CLASSES = [(1, 1, 1, 0), (2, 1, 1, 0), (2, 1, 2, 0), (2, 2, 1, 0)]


def gen(lmax: int) -> dict:
    pcls, classes = all_classes(lmax)
    files = {}
    stats = []
    stage_sizes = {}
    swapped = {}
    for (la, lb, lc, ld) in classes:
        cn = class_name(la, lb, lc, ld)
        nv = ncart(la) * ncart(lb) * ncart(lc) * ncart(ld)
        k64, nvrr, stage_n = emit_jk_kernel(la, lb, lc, ld, "double")
        k32, _, _ = emit_jk_kernel(la, lb, lc, ld, "float")
        stage_sizes[(la, lb, lc, ld)] = stage_n
        stats.append((cn, nv, nvrr))
        o = Emitter("")
        o(HEADER)
        o('#include "eri_common.hpp"')
        o("")
        o.lines.append(k64)
        if (la, lb, lc, ld) in SWAP_CLASSES and (la, lb, lc, ld) in classes:
            s64, _, _ = emit_jk_kernel(lc, ld, la, lb, "double")
            s32, _, _ = emit_jk_kernel(lc, ld, la, lb, "float")
            o.lines.append(s64)
            swapped[(la, lb, lc, ld)] = s32
        # block kernel (tests and Schwarz): quartet list -> raw blocks, FP64
        body2 = Emitter("  ")
        emit_eri_body(body2, la, lb, lc, ld)
        o(f"__global__ __launch_bounds__(64) void eri_block_{cn}(const PairSet bra, const PairSet ket, const int* __restrict__ qlist, int nq, double* __restrict__ out, const double* __restrict__ boys_tab)")
        o("{")
        emit_boys_lds(o, la + lb + lc + ld, False)
        o("  const int t = blockIdx.x * blockDim.x + threadIdx.x;")
        o("  if (t >= nq) return;")
        o("  const int ib = qlist[2 * t], jk = qlist[2 * t + 1];")
        if lb > 0:
            o("  const double ABx = bra.ABx[ib], ABy = bra.ABy[ib], ABz = bra.ABz[ib];")
        if ld > 0:
            o("  const double CDx = ket.ABx[jk], CDy = ket.ABy[jk], CDz = ket.ABz[jk];")
        o(body2.text())
        o(f"  #pragma unroll")
        o(f"  for (int u = 0; u < {nv}; ++u) out[(long long)t * {nv} + u] = v[u];")
        o("}")
        files[f"eri_{cn}.hip"] = o.text() + "\n"
        o = Emitter("")
        o(HEADER)
        o('#include "eri_common.hpp"')
        o("")
        o.lines.append(k32)
        if (la, lb, lc, ld) in swapped:
            o.lines.append(swapped[(la, lb, lc, ld)])
        files[f"eri_{cn}_f32.hip"] = o.text() + "\n"
    o = Emitter("")
    o(HEADER)
    o("#pragma once")
    o('#include "eri_common.hpp"')
    for (la, lb, lc, ld) in classes:
        cn = class_name(la, lb, lc, ld)
        o(f"__global__ void eri_jk_{cn}(const PairSet bra, const PairSet ket, const TaskMap tm, const Digest dg, const double* __restrict__ boys_tab);")
        o(f"__global__ void eri_jk32_{cn}(const PairSet bra, const PairSet ket, const TaskMap tm, const Digest dg, const double* __restrict__ boys_tab);")
        o(f"__global__ void eri_block_{cn}(const PairSet bra, const PairSet ket, const int* __restrict__ qlist, int nq, double* __restrict__ out, const double* __restrict__ boys_tab);")
        if (la, lb, lc, ld) in swapped:
            sn = class_name(lc, ld, la, lb)
            o(f"__global__ void eri_jk_{sn}(const PairSet bra, const PairSet ket, const TaskMap tm, const Digest dg, const double* __restrict__ boys_tab);")
            o(f"__global__ void eri_jk32_{sn}(const PairSet bra, const PairSet ket, const TaskMap tm, const Digest dg, const double* __restrict__ boys_tab);")
    # dispatch tables
    o("typedef void (*eri_jk_fn)(PairSet, PairSet, TaskMap, Digest, const double*);")
    o("// jks / jk32s: the kernels of the exchanged orientation (lc ld|la lb), or NULL; acc_s / acc8_s their")
    o("// LDS accumulator sizes; sacc: stage-region task accumulator doubles per lane and density slot;")
    o("// rows / rows_s: bra shells per task tile (64 / rows ket shells) of each orientation")
    o("struct EriClassEntry { int la, lb, lc, ld; int nv; int stage; int acc; int acc8; eri_jk_fn jk; eri_jk_fn jk32; void (*blk)(PairSet, PairSet, const int*, int, double*, const double*); eri_jk_fn jks; eri_jk_fn jk32s; int acc_s, acc8_s; int sacc; int rows, rows_s; };")
    o(f"static const int kNumEriClasses = {len(classes)};")
    o("static const EriClassEntry kEriClasses[] = {")
    for (la, lb, lc, ld) in classes:
        cn = class_name(la, lb, lc, ld)
        nv = ncart(la) * ncart(lb) * ncart(lc) * ncart(ld)
        if (la, lb, lc, ld) in swapped:
            sn = class_name(lc, ld, la, lb)
            sw = f"eri_jk_{sn}, eri_jk32_{sn}, {acc_doubles(lc, ld, la, lb)}, {acc8_doubles(lc, ld, la, lb)}"
            rs = tile_rows(lc, ld, la, lb)
        else:
            sw = "nullptr, nullptr, 0, 0"
            rs = 8
        o(f"  {{{la}, {lb}, {lc}, {ld}, {nv}, {stage_sizes[(la, lb, lc, ld)]}, {acc_doubles(la, lb, lc, ld)}, {acc8_doubles(la, lb, lc, ld)}, eri_jk_{cn}, eri_jk32_{cn}, eri_block_{cn}, {sw}, {staged_acc_doubles(la, lb, lc, ld)}, {tile_rows(la, lb, lc, ld)}, {rs}}},")
    o("};")
    for cn, nv, nvrr in stats:
        print(f"{cn}: nv={nv} vrr_nodes={nvrr}", file=sys.stderr)
    files["eri_registry.hpp"] = o.text() + "\n"
    return files


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("outdir")
    ap.add_argument("--lmax", type=int, default=2)
    a = ap.parse_args()
    os.makedirs(a.outdir, exist_ok=True)
    for name, src in gen(a.lmax).items():
        path = os.path.join(a.outdir, name)
        old = open(path).read() if os.path.exists(path) else None
        if old != src:
            with open(path, "w") as f:
                f.write(src)


if __name__ == "__main__":
    main()
