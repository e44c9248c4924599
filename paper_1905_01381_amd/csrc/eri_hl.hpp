// Electron-repulsion classes with an f shell (every shell l <= 3): one
// workgroup per contracted shell quartet, the recurrences laid out in LDS.
#pragma once
#include "eri_common.hpp"

#define HL_LMAX 3            // highest shell angular momentum of this path
#define HL_THREADS_MAX 1024  // threads of one workgroup, at most
#define HL_LDS_STATIC 2048   // bytes of static LDS the kernel keeps besides the layout

// threads per workgroup for a class: wide workgroups for the large classes
// (their recurrence levels hold thousands of entries), one wave for the
// small ones (most of a wider group would idle at every barrier)
__host__ __device__ inline int hl_threads(int total_doubles)
{
    return total_doubles > 8192 ? 1024 : (total_doubles > 2048 ? 256 : 64);
}

// LDS layout of one class (in doubles).  V: the bra table [e|00]^(m) and
// three ket-level slots (level f in slot f mod 3); after the primitive loop
// the same region stages the six density blocks of the digestion.  Then the
// per-axis transfer coefficients of the bra and the ket primitive pair, the
// ket-transferred [e|cd) of one chunk of ket components and the chunk of
// (ab|cd) summed over primitives.  The ket components cd are taken in
// chunks of `ch` so that the whole fits the device's LDS.
struct HlLayout {
    int la, lb, lc, ld;
    int Lt, Eb, Fk;   // la+lb+lc+ld, la+lb, lc+ld
    int ne;           // components of degree 0..Eb
    int nab, ncd, nOUT, nXS;
    int t0[8];        // offset of degree l in the bra table ([ci][m], m <= Lt - l)
    int oS[3];        // ket-level slots
    int nV;           // bra table + slots, at least nXS
    int oEA, oEC, oECD, oOUT;
    int ch, nch;      // ket components per chunk, chunks
    int total;
};

__host__ __device__ inline int hl_nc(int l) { return (l + 1) * (l + 2) / 2; }
// components of every degree below l
__host__ __device__ inline int hl_cum(int l) { return l * (l + 1) * (l + 2) / 6; }

// maxd: the device's LDS per workgroup in doubles; ch = 0 if even one ket
// component per chunk does not fit.
__host__ __device__ inline HlLayout hl_layout(int la, int lb, int lc, int ld, int maxd)
{
    HlLayout L{};
    L.la = la;
    L.lb = lb;
    L.lc = lc;
    L.ld = ld;
    L.Eb = la + lb;
    L.Fk = lc + ld;
    L.Lt = L.Eb + L.Fk;
    L.ne = hl_cum(L.Eb + 1);
    const int na = hl_nc(la), nb = hl_nc(lb), nc = hl_nc(lc), nd = hl_nc(ld);
    L.nab = na * nb;
    L.ncd = nc * nd;
    L.nOUT = L.nab * L.ncd;
    L.nXS = na * nb + nc * nd + na * nc + na * nd + nb * nc + nb * nd;
    int o = 0;
    for (int l = 0; l < 8; ++l) {
        L.t0[l] = o;
        if (l <= L.Eb) o += hl_nc(l) * (L.Lt - l + 1);
    }
    int slot[3] = {0, 0, 0};
    for (int f = 1; f <= L.Fk; ++f) {
        const int v = L.ne * hl_nc(f) * (L.Fk - f + 1);
        slot[f % 3] = v > slot[f % 3] ? v : slot[f % 3];
    }
    for (int k = 0; k < 3; ++k) {
        L.oS[k] = o;
        o += slot[k];
    }
    L.nV = o > L.nXS ? o : L.nXS;
    L.oEA = L.nV;
    L.oEC = L.oEA + 3 * (la + 1) * (lb + 1) * (L.Eb + 1);
    L.oECD = L.oEC + 3 * (lc + 1) * (ld + 1) * (L.Fk + 1);
    const int fixed = L.oECD;
    const int per = L.ne + L.nab;
    int ch = (maxd - fixed) / per;
    ch = ch > L.ncd ? L.ncd : ch;
    L.ch = ch > 0 ? ch : 0;
    L.nch = L.ch ? (L.ncd + L.ch - 1) / L.ch : 0;
    L.oOUT = L.oECD + L.ne * L.ch;
    L.total = L.oOUT + L.nab * L.ch;
    return L;
}

// One launch of one class.  Digest mode (out == nullptr): task t covers the
// bra pair tasks[t].x and the ket pairs tasks[t].y .. tasks[t].z - 1 of
// molecule tasks[t].w, adds J'/K' and, in screened or routed builds, counts
// quartets.  Block mode (out != nullptr): task t is one quartet
// (tasks[t].x, tasks[t].y) and its raw contracted block goes to
// out[t * nab * ncd ...] in (a b c d) order, no screening.
struct HlArgs {
    PairSet bra, ket;
    const int4* tasks;
    int ntask;
    int same;  // bra and ket pairs from one pair class (the canonical half q <= p)
    HlLayout lay;
    TaskMap tm;  // mols and ppos only
    Digest dg;
    const double* boys;
    double* out;
};

// The kernel of class (la lb|lc ld) (la = 3, the bra pair class at or above
// the ket's), or NULL for any other class.  Launch with hl_threads(total)
// threads and total * 8 bytes of dynamic LDS.
typedef void (*hl_kernel_fn)(HlArgs);
hl_kernel_fn hl_kernel_for(int la, int lb, int lc, int ld);
