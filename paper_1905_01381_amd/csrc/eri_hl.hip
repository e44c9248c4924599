// Electron-repulsion integrals and J/K digestion for the classes that hold
// an f shell (shells up to l = 3; paper: Introduction, contracted Gaussian
// basis functions of any angular momentum).  The generated per-class
// kernels keep one quartet per lane in registers, which does not scale to
// the 10^4 integrals of an (ff|ff) block; here one workgroup (64 to 1024
// threads by the size of the class) owns one contracted shell quartet and
// lays the recurrences out in LDS.
//
// Per primitive quartet, the Obara-Saika recurrence runs about the Gaussian
// product centres P and Q (the vertical recurrence with A = P and C = Q):
//   [e+1_i|00]^(m) = WP_i [e|00]^(m+1) + e_i/(2p) ([e-1_i|00]^(m) - rho/p [e-1_i|00]^(m+1))
//   [e|f+1_i]^(m)  = WQ_i [e|f]^(m+1) + f_i/(2q) ([e|f-1_i]^(m) - rho/q [e|f-1_i]^(m+1))
//                    + e_i/(2(p+q)) [e-1_i|f]^(m+1)
// from [0|0]^(m) = K_ab K_cd / sqrt(p+q) F_m(T); [e|f] is the integral of
// (x1-P)^e (x2-Q)^f times the two Gaussian products.  The Cartesian
// functions follow from x - A = (x - P) + (P - A) per axis:
//   (x-A)^a (x-B)^b = sum_e E^{ab}_e (x-P)^e,
//   E^{ab}_e = sum_{i+j=e} C(a,i) C(b,j) PA^(a-i) PB^(b-j),
// so (ab|cd) = sum_e sum_f E^{ab}_e E^{cd}_f [e|f], applied per primitive
// quartet (ket side level by level as the recurrence produces it, bra side
// once per bra primitive pair) and summed over primitives.  Centring on P
// keeps every intermediate of the size of the final integrals; expanding
// about A instead (the vertical recurrence on A and a horizontal transfer of
// contracted integrals) loses up to 8 digits for (ff|ff) with diffuse
// primitives, where [e0| about A reaches 10^6 times the result.
//
// The ket components cd are taken in chunks that fit the device's LDS; the
// digestion of each chunk adds its partial sums with the same exact
// fixed-point accumulation as the generated kernels (8-fold scatter, same
// degeneracy weights), so J'/K' do not depend on the order of the adds.
#include "eri_hl.hpp"

namespace {

// position of x^i y^j z^k in its degree's list (x descending, then y)
__device__ __forceinline__ int cidx(int j, int k)
{
    const int s = j + k;
    return s * (s + 1) / 2 + k;
}

// Components of every degree 0..6 in order (global index g), packed as
// x | y << 4 | z << 8 | degree << 12; filled once per workgroup.
#define HL_NCOMP 84
__shared__ int s_comp[HL_NCOMP];

__device__ void fill_comps()
{
    for (int g = threadIdx.x; g < HL_NCOMP; g += blockDim.x) {
        int l = 0;
        while (hl_cum(l + 1) <= g) ++l;
        const int ci = g - hl_cum(l);
        int t = 0;
        while ((t + 1) * (t + 2) / 2 <= ci) ++t;
        const int z = ci - t * (t + 1) / 2;
        s_comp[g] = (l - t) | ((t - z) << 4) | (z << 8) | (l << 12);
    }
    __syncthreads();
}

// degree and exponents of global component index g
__device__ __forceinline__ int gexps(int g, int e[3])
{
    const int v = s_comp[g];
    e[0] = v & 15;
    e[1] = (v >> 4) & 15;
    e[2] = (v >> 8) & 15;
    return v >> 12;
}

// exponents of component ci of degree l
__device__ __forceinline__ void exps(int l, int ci, int e[3]) { gexps(hl_cum(l) + ci, e); }

__device__ __forceinline__ int gdeg(int g) { return s_comp[g] >> 12; }

// Exponent pairs of the bra components ab and of one chunk's ket components
// (c | d << 12, each x | y << 4 | z << 8), filled per workgroup / chunk.
#define HL_NPAIR 100
__shared__ int s_ab[HL_NPAIR];
__shared__ int s_cd[HL_NPAIR];

__device__ __forceinline__ int pack3(const int e[3]) { return e[0] | (e[1] << 4) | (e[2] << 8); }
__device__ __forceinline__ void unpack3(int v, int e[3])
{
    e[0] = v & 15;
    e[1] = (v >> 4) & 15;
    e[2] = (v >> 8) & 15;
}

// s_tab[k] for k < n: components (k / n2 of degree l1, k % n2 of degree l2), pair index offset k0
__device__ __forceinline__ void fill_pairs(int* tab, int l1, int l2, int k0, int n)
{
    const int n2 = hl_nc(l2);
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        int a[3], b[3];
        exps(l1, (k0 + k) / n2, a);
        exps(l2, (k0 + k) % n2, b);
        tab[k] = pack3(a) | (pack3(b) << 12);
    }
}

__device__ __forceinline__ int gidx(int x, int y, int z) { return hl_cum(x + y + z) + cidx(y, z); }

__device__ __forceinline__ int first_dir(const int e[3]) { return e[0] > 0 ? 0 : (e[1] > 0 ? 1 : 2); }

__device__ __forceinline__ double binom3(int n, int k)
{
    // 0 <= k <= n <= 3
    return n == 3 ? ((k == 0 || k == 3) ? 1.0 : 3.0) : (n == 2 ? (k == 1 ? 2.0 : 1.0) : 1.0);
}

__device__ __forceinline__ double ipow(double x, int n)
{
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

// The workgroup walks n1 x n2 entries (i1 slow, i2 fast).  With n2 <= the
// group size, thread t keeps i2 = t mod n2 and steps i1 by group / n2 (one
// division per walk instead of one per entry); otherwise entries are dealt
// in flat order.  Either way a given entry always falls to the same thread.
template <class F>
__device__ __forceinline__ void for_pairs(int n1, int n2, F&& body)
{
    const int nth = blockDim.x, tid = threadIdx.x;
    if (n2 <= nth) {
        const int groups = nth / n2, i2 = tid % n2, g = tid / n2;
        if (g < groups)
            for (int i1 = g; i1 < n1; i1 += groups) body(i1, i2);
    } else {
        for (int x = tid; x < n1 * n2; x += nth) {
            const int i1 = x / n2;
            body(i1, x - i1 * n2);
        }
    }
}

// bra table entry (degree l, global index g, order m)
__device__ __forceinline__ int t0i(const HlLayout& L, int l, int g, int m)
{
    return L.t0[l] + (g - hl_cum(l)) * (L.Lt - l + 1) + m;
}

// ket level g >= 1 entry (global e index, f component, order m)
__device__ __forceinline__ int levi(const HlLayout& L, int g, int eg, int fc, int m)
{
    return L.oS[g % 3] + (eg * hl_nc(g) + fc) * (L.Fk - g + 1) + m;
}

// level g at (e of degree le with global index eg, f component fc, order m)
__device__ __forceinline__ double lev(const double* s, const HlLayout& L, int g, int le, int eg, int fc, int m)
{
    return g == 0 ? s[t0i(L, le, eg, m)] : s[levi(L, g, eg, fc, m)];
}

// Per-axis coefficients E_e of (x-P)^e in (x-A)^u (x-B)^v, u <= lu, v <= lv,
// e <= lu + lv: tab[((k (lu+1) + u) (lv+1) + v) (lu+lv+1) + e], axis k.
__device__ __forceinline__ void etable(double* tab, int lu, int lv, const double PA[3], const double PB[3])
{
    const int ne = lu + lv + 1, n = 3 * (lu + 1) * (lv + 1) * ne;
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
        const int e = x % ne, r = x / ne;
        const int v = r % (lv + 1), r2 = r / (lv + 1);
        const int u = r2 % (lu + 1), k = r2 / (lu + 1);
        double t = 0.0;
        const int i0 = e - v > 0 ? e - v : 0, i1 = u < e ? u : e;
        for (int i = i0; i <= i1; ++i)
            t += binom3(u, i) * binom3(v, e - i) * ipow(PA[k], u - i) * ipow(PB[k], v - (e - i));
        tab[x] = t;
    }
}

// Ket transfer of level f (values at order 0) into the chunk's [e|cd):
// ECD[eg cdn + r] += sum over f components of E^{cd}_f [e|f].  Index
// arithmetic is hoisted: per entry the three per-axis coefficient rows and
// the level row of e, per f_x the component offset of the (f_y, f_z) block.
__device__ __forceinline__ void ket_transfer(const HlLayout& L, double* s, int f, int cd0, int cdn)
{
    const double* EC = s + L.oEC;
    double* ECD = s + L.oECD;
    const int ne1 = L.Fk + 1, stride_v = ne1, stride_u = (L.ld + 1) * ne1, stride_k = (L.lc + 1) * stride_u;
    const int nfc = hl_nc(f), nm = L.Fk - f + 1;
    for_pairs(L.ne, cdn, [&](int eg, int r) {
        int c[3], d[3];
        unpack3(s_cd[r], c);
        unpack3(s_cd[r] >> 12, d);
        const double* ex = EC + c[0] * stride_u + d[0] * stride_v;
        const double* ey = EC + stride_k + c[1] * stride_u + d[1] * stride_v;
        const double* ez = EC + 2 * stride_k + c[2] * stride_u + d[2] * stride_v;
        // level f row of e: component fc at row[fc * nm] (order 0)
        const double* row = f == 0 ? s + t0i(L, gdeg(eg), eg, 0) : s + L.oS[f % 3] + eg * nfc * nm;
        const int mx = c[0] + d[0], my = c[1] + d[1], mz = c[2] + d[2];
        double t = 0.0;
        for (int fx = 0; fx <= (mx < f ? mx : f); ++fx) {
            const int sy = f - fx;              // f_y + f_z
            const int cb = sy * (sy + 1) / 2;   // first component with this f_y + f_z
            const double wx = ex[fx];
            const int fy0 = sy - mz > 0 ? sy - mz : 0, fy1 = my < sy ? my : sy;
            for (int fy = fy0; fy <= fy1; ++fy) {
                const int fz = sy - fy;
                t += wx * ey[fy] * ez[fz] * row[(cb + fz) * nm];
            }
        }
        ECD[eg * cdn + r] += t;
    });
}

// One chunk of ket components [cd0, cd0 + cdn) of the quartet (bra pair p,
// ket pair q), summed over primitive quartets into OUT[ab cdn + r].
__device__ __forceinline__ void chunk(const HlArgs& a, const HlLayout& L, int p, int q, int cd0, int cdn, double* s)
{
    const int tid = threadIdx.x, nth = blockDim.x;
    double* EA = s + L.oEA;
    double* EC = s + L.oEC;
    double* ECD = s + L.oECD;
    double* OUT = s + L.oOUT;
    for (int x = tid; x < L.nab * cdn; x += nth) OUT[x] = 0.0;
    fill_pairs(s_cd, L.lc, L.ld, cd0, cdn);
    const double AB[3] = {a.bra.ABx[p], a.bra.ABy[p], a.bra.ABz[p]};
    const double CD[3] = {a.ket.ABx[q], a.ket.ABy[q], a.ket.ABz[q]};
    for (int kp = 0; kp < a.bra.nprim2; ++kp) {
        const double* rb = a.bra.rec + ((size_t)p * a.bra.nprim2 + kp) * 10;
        const double Kab = rb[1];
        if (Kab == 0.0) continue;
        const double pe = rb[0], oo2p = rb[2];
        const double P[3] = {rb[3], rb[4], rb[5]}, PA[3] = {rb[6], rb[7], rb[8]};
        const double PB[3] = {PA[0] + AB[0], PA[1] + AB[1], PA[2] + AB[2]};
        __syncthreads();  // the previous bra transfer has read EA and ECD
        etable(EA, L.la, L.lb, PA, PB);
        for (int x = tid; x < L.ne * cdn; x += nth) ECD[x] = 0.0;
        for (int kq = 0; kq < a.ket.nprim2; ++kq) {
            const double* rk = a.ket.rec + ((size_t)q * a.ket.nprim2 + kq) * 10;
            const double Kcd = rk[1];
            if (Kcd == 0.0) continue;
            const double qe = rk[0], oo2q = rk[2];
            const double Q[3] = {rk[3], rk[4], rk[5]}, QC[3] = {rk[6], rk[7], rk[8]};
            const double QD[3] = {QC[0] + CD[0], QC[1] + CD[1], QC[2] + CD[2]};
            const double inv = 1.0 / (pe + qe);
            const double PQ[3] = {P[0] - Q[0], P[1] - Q[1], P[2] - Q[2]};
            const double rho = pe * qe * inv;
            const double T = rho * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]);
            const double WP[3] = {-qe * inv * PQ[0], -qe * inv * PQ[1], -qe * inv * PQ[2]};
            const double WQ[3] = {pe * inv * PQ[0], pe * inv * PQ[1], pe * inv * PQ[2]};
            const double rp2 = qe * inv * oo2p;  // (rho / p) / (2p)
            const double rq2 = pe * inv * oo2q;  // (rho / q) / (2q)
            const double oo2pq = 0.5 * inv;
            __syncthreads();  // the previous primitive quartet's readers are done
            etable(EC, L.lc, L.ld, QC, QD);
            if (tid == 0) {
                double F[13];
                boys_fp64<12>(T, a.boys, F);
                const double pref = Kab * Kcd * sqrt(inv);
#pragma unroll
                for (int m = 0; m <= 12; ++m)
                    if (m <= L.Lt) s[L.t0[0] + m] = pref * F[m];
            }
            __syncthreads();
            for (int l = 1; l <= L.Eb; ++l) {
                const int nm = L.Lt - l + 1, n = hl_nc(l) * nm;
                for (int x = tid; x < n; x += nth) {
                    const int ci = x / nm, m = x % nm;
                    int e[3];
                    exps(l, ci, e);
                    const int i = first_dir(e);
                    e[i] -= 1;
                    const int g1 = gidx(e[0], e[1], e[2]);
                    double v = WP[i] * s[t0i(L, l - 1, g1, m + 1)];
                    if (e[i] > 0) {
                        const int k = e[i];
                        e[i] -= 1;
                        const int g2 = gidx(e[0], e[1], e[2]);
                        v += k * (oo2p * s[t0i(L, l - 2, g2, m)] - rp2 * s[t0i(L, l - 2, g2, m + 1)]);
                    }
                    s[L.t0[l] + x] = v;
                }
                __syncthreads();
            }
            ket_transfer(L, s, 0, cd0, cdn);
            for (int f = 1; f <= L.Fk; ++f) {
                // one (e, f component) per thread, all its orders m in turn
                // (orders are contiguous in every level)
                const int nfc = hl_nc(f), nm = L.Fk - f + 1;
                for_pairs(L.ne, nfc, [&](int eg, int fc) {
                    int fe[3], e[3];
                    exps(f, fc, fe);
                    const int le = gexps(eg, e);
                    const int i = first_dir(fe);
                    fe[i] -= 1;
                    const int f1 = cidx(fe[1], fe[2]);
                    const double* A1 = s + (f == 1 ? t0i(L, le, eg, 0) : levi(L, f - 1, eg, f1, 0));
                    const int k2 = fe[i];
                    const double* A2 = A1;
                    if (k2 > 0) {
                        fe[i] -= 1;
                        const int f2 = cidx(fe[1], fe[2]);
                        A2 = s + (f == 2 ? t0i(L, le, eg, 0) : levi(L, f - 2, eg, f2, 0));
                    }
                    const int k3 = e[i];
                    const double* A3 = A1;
                    if (k3 > 0) {
                        e[i] -= 1;
                        const int eg1 = gidx(e[0], e[1], e[2]);
                        A3 = s + (f == 1 ? t0i(L, le - 1, eg1, 0) : levi(L, f - 1, eg1, f1, 0));
                    }
                    double* dst = s + levi(L, f, eg, fc, 0);
                    const double c2 = k2 * oo2q, d2 = k2 * rq2, c3 = k3 * oo2pq;
                    for (int m = 0; m < nm; ++m) {
                        double v = WQ[i] * A1[m + 1];
                        if (k2 > 0) v += c2 * A2[m] - d2 * A2[m + 1];
                        if (k3 > 0) v += c3 * A3[m + 1];
                        dst[m] = v;
                    }
                });
                __syncthreads();
                ket_transfer(L, s, f, cd0, cdn);
            }
        }
        __syncthreads();  // ECD complete
        // bra transfer: OUT[ab, r] += sum_e E^{ab}_e [e|cd)
        const int ne1 = L.Eb + 1, stride_u = (L.lb + 1) * ne1, stride_k = (L.la + 1) * stride_u;
        for_pairs(L.nab, cdn, [&](int ab, int r) {
            int ea[3], eb[3];
            unpack3(s_ab[ab], ea);
            unpack3(s_ab[ab] >> 12, eb);
            const double* wxr = EA + ea[0] * stride_u + eb[0] * ne1;
            const double* wyr = EA + stride_k + ea[1] * stride_u + eb[1] * ne1;
            const double* wzr = EA + 2 * stride_k + ea[2] * stride_u + eb[2] * ne1;
            const double* col = ECD + r;
            double t = 0.0;
            for (int ex = 0; ex <= ea[0] + eb[0]; ++ex) {
                const double wx = wxr[ex];
                for (int ey = 0; ey <= ea[1] + eb[1]; ++ey) {
                    const double wy = wx * wyr[ey];
                    // components with e_x = ex, e_y = ey in order of e_z: global
                    // index cum(ex + ey + ez) + cidx(ey, ez)
                    for (int ez = 0; ez <= ea[2] + eb[2]; ++ez)
                        t += wy * wzr[ez] * col[gidx(ex, ey, ez) * cdn];
                }
            }
            OUT[ab * cdn + r] += t;
        });
    }
    __syncthreads();
}

// 8-fold scatter of v = deg (ab|cd) over the chunk's ket components
// (v = OUT[ab cdn + r], cd = cd0 + r):
//   J'_ab += 2 v X_cd, J'_cd += 2 v X_ab,
//   K'_ac += v X_bd, K'_ad += v X_bc, K'_bc += v X_ad, K'_bd += v X_ac;
// each destination's partial sum over the chunk is one fixed-point add.
__device__ __forceinline__ void digest(const HlArgs& a, const HlLayout& L, const MolView& mc, int p, int q, double deg, int cd0,
                       int cdn, double* s)
{
    const int tid = threadIdx.x, nth = blockDim.x;
    const Digest& dg = a.dg;
    const int na = hl_nc(L.la), nb = hl_nc(L.lb), nc = hl_nc(L.lc), nd = hl_nc(L.ld);
    const int fa = a.bra.fa[p], fb = a.bra.fb[p], fc = a.ket.fa[q], fd = a.ket.fb[q];
    const double* v = s + L.oOUT;
    double* xab = s;  // the recurrence region, free after the primitive loop
    double* xcd = xab + na * nb;
    double* xac = xcd + nc * nd;
    double* xad = xac + na * nc;
    double* xbc = xad + na * nd;
    double* xbd = xbc + nb * nc;
    const int k0 = cd0 / nd, k1 = (cd0 + cdn - 1) / nd;  // c components the chunk touches
    for (int m = 0; m < dg.nX; ++m) {
        const int js = dg.jslot[m], ks = dg.kslot[m];
        if (js < 0 && ks < 0) continue;
        for (int x = tid; x < L.nXS; x += nth) {
            int r = x, mu, nu;
            if (r < na * nb) { mu = fa + r / nb; nu = fb + r % nb; }
            else if ((r -= na * nb) < nc * nd) { mu = fc + r / nd; nu = fd + r % nd; }
            else if ((r -= nc * nd) < na * nc) { mu = fa + r / nc; nu = fc + r % nc; }
            else if ((r -= na * nc) < na * nd) { mu = fa + r / nd; nu = fd + r % nd; }
            else if ((r -= na * nd) < nb * nc) { mu = fb + r / nc; nu = fc + r % nc; }
            else { r -= nb * nc; mu = fb + r / nd; nu = fd + r % nd; }
            xab[x] = ld_x(dg, mc, mu, nu, m);
        }
        __syncthreads();
        const int nj = js >= 0 ? na * nb + cdn : 0;
        const int nk = ks >= 0 ? na * nc + na * nd + nb * nc + nb * nd : 0;
        for (int x = tid; x < nj + nk; x += nth) {
            double t = 0.0;
            int r = x;
            if (r < nj) {
                if (r < na * nb) {
                    for (int k = 0; k < cdn; ++k) t += v[r * cdn + k] * xcd[cd0 + k];
                    acc_j(mc, jidx(dg, mc, fa + r / nb, fb + r % nb, js), 2.0 * deg * t);
                } else {
                    r -= na * nb;
                    for (int k = 0; k < na * nb; ++k) t += v[k * cdn + r] * xab[k];
                    const int cd = cd0 + r;
                    acc_j(mc, jidx(dg, mc, fc + cd / nd, fd + cd % nd, js), 2.0 * deg * t);
                }
                continue;
            }
            r -= nj;
            if (r < na * nc) {  // K'_ac(i, k): b and the chunk's d of c = k
                const int i = r / nc, k = r % nc;
                if (k < k0 || k > k1) continue;
                const int lo = k * nd - cd0 > 0 ? k * nd - cd0 : 0;
                const int hi = (k + 1) * nd - cd0 < cdn ? (k + 1) * nd - cd0 : cdn;
                for (int j = 0; j < nb; ++j)
                    for (int rr = lo; rr < hi; ++rr) t += v[(i * nb + j) * cdn + rr] * xbd[j * nd + (cd0 + rr) % nd];
                acc_k(mc, kidx(dg, mc, fa + i, fc + k, ks), deg * t);
            } else if ((r -= na * nc) < na * nd) {  // K'_ad(i, l): b and the chunk's c of d = l
                const int i = r / nd, l = r % nd;
                int r0 = (l - cd0 % nd + nd) % nd;
                if (r0 >= cdn) continue;
                for (int j = 0; j < nb; ++j)
                    for (int rr = r0; rr < cdn; rr += nd) t += v[(i * nb + j) * cdn + rr] * xbc[j * nc + (cd0 + rr) / nd];
                acc_k(mc, kidx(dg, mc, fa + i, fd + l, ks), deg * t);
            } else if ((r -= na * nd) < nb * nc) {  // K'_bc(j, k): a and the chunk's d of c = k
                const int j = r / nc, k = r % nc;
                if (k < k0 || k > k1) continue;
                const int lo = k * nd - cd0 > 0 ? k * nd - cd0 : 0;
                const int hi = (k + 1) * nd - cd0 < cdn ? (k + 1) * nd - cd0 : cdn;
                for (int i = 0; i < na; ++i)
                    for (int rr = lo; rr < hi; ++rr) t += v[(i * nb + j) * cdn + rr] * xad[i * nd + (cd0 + rr) % nd];
                acc_k(mc, kidx(dg, mc, fb + j, fc + k, ks), deg * t);
            } else {  // K'_bd(j, l): a and the chunk's c of d = l
                r -= nb * nc;
                const int j = r / nd, l = r % nd;
                int r0 = (l - cd0 % nd + nd) % nd;
                if (r0 >= cdn) continue;
                for (int i = 0; i < na; ++i)
                    for (int rr = r0; rr < cdn; rr += nd) t += v[(i * nb + j) * cdn + rr] * xac[i * nc + (cd0 + rr) / nd];
                acc_k(mc, kidx(dg, mc, fb + j, fd + l, ks), deg * t);
            }
        }
        __syncthreads();
    }
}

// The kernel body for one class; L's class-dependent fields are
// compile-time constants in every instantiation below.
__device__ __forceinline__ void hl_body(const HlArgs& a, const HlLayout& L)
{
    extern __shared__ double s[];
    const int t = blockIdx.x;
    if (t >= a.ntask) return;
    fill_comps();
    fill_pairs(s_ab, L.la, L.lb, 0, L.nab);  // visible after the first barrier of a chunk
    const int4 tk = a.tasks[t];
    const int p = tk.x;
    if (a.out) {
        const int q = tk.y;
        double* dst = a.out + (size_t)t * L.nOUT;
        for (int ck = 0; ck < L.nch; ++ck) {
            const int cd0 = ck * L.ch, cdn = L.ncd - cd0 < L.ch ? L.ncd - cd0 : L.ch;
            chunk(a, L, p, q, cd0, cdn, s);
            for (int x = threadIdx.x; x < L.nab * cdn; x += blockDim.x)
                dst[(x / cdn) * L.ncd + cd0 + x % cdn] = s[L.oOUT + x];
            __syncthreads();
        }
        return;
    }
    const MolView mc = mol_view(a.dg, a.tm, tk.w);
    const int sa = a.bra.sa[p], sb = a.bra.sb[p];
    const bool classify = a.dg.skip > 0.0 || a.dg.mode == 1;
    unsigned long long nrun = 0, nskip = 0;
    for (int q = tk.y; q < tk.z; ++q) {
        const int sc = a.ket.sa[q], sd = a.ket.sb[q];
        if (a.dg.skip > 0.0 && quartet_bound(mc, a.bra.Q[p], a.ket.Q[q], sa, sb, sc, sd) < a.dg.skip) {
            ++nskip;
            continue;
        }
        ++nrun;
        double deg = 1.0;
        if (sa == sb) deg *= 0.5;
        if (sc == sd) deg *= 0.5;
        if (a.same && p == q) deg *= 0.5;
        for (int ck = 0; ck < L.nch; ++ck) {
            const int cd0 = ck * L.ch, cdn = L.ncd - cd0 < L.ch ? L.ncd - cd0 : L.ch;
            chunk(a, L, p, q, cd0, cdn, s);
            digest(a, L, mc, p, q, deg, cd0, cdn, s);
        }
    }
    if (classify && threadIdx.x == 0) {
        if (nrun) atomicAdd(a.dg.counts, nrun);
        if (nskip) atomicAdd(a.dg.counts + 2, nskip);
    }
}

}  // namespace

// One instantiation per class: the angular momenta fix every size, offset,
// loop bound and stride of the recurrences at compile time (the runtime
// index arithmetic of a class-generic kernel dominated its issue slots);
// only the ket chunking, which depends on the device's LDS, comes from the
// launch.
template <int LA, int LB, int LC, int LD>
__global__ __launch_bounds__(HL_THREADS_MAX) void eri_hl_t(HlArgs a)
{
    HlLayout L = hl_layout(LA, LB, LC, LD, 0);
    L.ch = a.lay.ch;
    L.nch = a.lay.nch;
    L.oOUT = a.lay.oOUT;
    L.total = a.lay.total;
    hl_body(a, L);
}

#define HL_CASE(A, B, C, D) \
    if (la == A && lb == B && lc == C && ld == D) return eri_hl_t<A, B, C, D>;

hl_kernel_fn hl_kernel_for(int la, int lb, int lc, int ld)
{
    HL_CASE(3, 0, 0, 0)
    HL_CASE(3, 0, 1, 0)
    HL_CASE(3, 0, 1, 1)
    HL_CASE(3, 0, 2, 0)
    HL_CASE(3, 0, 2, 1)
    HL_CASE(3, 0, 2, 2)
    HL_CASE(3, 0, 3, 0)
    HL_CASE(3, 1, 0, 0)
    HL_CASE(3, 1, 1, 0)
    HL_CASE(3, 1, 1, 1)
    HL_CASE(3, 1, 2, 0)
    HL_CASE(3, 1, 2, 1)
    HL_CASE(3, 1, 2, 2)
    HL_CASE(3, 1, 3, 0)
    HL_CASE(3, 1, 3, 1)
    HL_CASE(3, 2, 0, 0)
    HL_CASE(3, 2, 1, 0)
    HL_CASE(3, 2, 1, 1)
    HL_CASE(3, 2, 2, 0)
    HL_CASE(3, 2, 2, 1)
    HL_CASE(3, 2, 2, 2)
    HL_CASE(3, 2, 3, 0)
    HL_CASE(3, 2, 3, 1)
    HL_CASE(3, 2, 3, 2)
    HL_CASE(3, 3, 0, 0)
    HL_CASE(3, 3, 1, 0)
    HL_CASE(3, 3, 1, 1)
    HL_CASE(3, 3, 2, 0)
    HL_CASE(3, 3, 2, 1)
    HL_CASE(3, 3, 2, 2)
    HL_CASE(3, 3, 3, 0)
    HL_CASE(3, 3, 3, 1)
    HL_CASE(3, 3, 3, 2)
    HL_CASE(3, 3, 3, 3)
    return nullptr;
}
