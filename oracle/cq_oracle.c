/*
 * cq_oracle.c -- plain, slow, obviously-correct CPU FP64 reference for the
 * integral-direct Coulomb/exchange build.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * constant with the HIP path, and uses a different integral algorithm
 * (McMurchie-Davidson Hermite expansion) and a different Boys-function method
 * (all-positive power series / erf) than the GPU kernels (Obara-Saika /
 * Head-Gordon-Pople with a Chebyshev Boys table).
 *
 * What it computes (paper: "Reference Wave Functions", Eq. 2c_fock, and the
 * direct-SCF statement after it):
 *   J[X]_{mn} = sum_{ls} (mn|ls) X_{ls}
 *   K[X]_{mn} = sum_{ls} (ml|ns) X_{ls}
 * over contracted Cartesian Gaussian shells (paper: Introduction, LCAO over
 * contracted Gaussian-type orbitals).  No screening is ever applied here.
 *
 * Everything is FP64 (long double inside the Boys series).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORA_LMAX 4          /* shells up to g (tests use <= d) */
#define ORA_RMAX (4 * ORA_LMAX + 4)

static const double ORA_PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------ */
/* Boys function  F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt               */
/* ------------------------------------------------------------------ */
/* T <= 50: F_m(T) = exp(-T) * sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)),
 *          an all-positive series (no cancellation), summed in long double.
 * T  > 50: F_0 = sqrt(pi/T) erf(sqrt T) / 2 and the upward recursion
 *          F_{m+1} = ((2m+1) F_m - exp(-T)) / (2T), stable for large T. */
double ora_boys(int m, double T)
{
    if (T <= 50.0) {
        long double term = 1.0L / (2 * m + 1);
        long double sum = term;
        for (int k = 1; k < 2000; ++k) {
            term *= (2.0L * T) / (long double)(2 * m + 2 * k + 1);
            sum += term;
            if (term < sum * 1e-22L) break;
        }
        return (double)(expl(-(long double)T) * sum);
    }
    double f = 0.5 * sqrt(ORA_PI / T) * erf(sqrt(T));
    double e = exp(-T);
    for (int k = 0; k < m; ++k) f = ((2 * k + 1) * f - e) / (2.0 * T);
    return f;
}

void ora_boys_vec(int mmax, int n, const double* T, double* F)
{
    for (int i = 0; i < n; ++i)
        for (int m = 0; m <= mmax; ++m) F[i * (mmax + 1) + m] = ora_boys(m, T[i]);
}

/* ------------------------------------------------------------------ */
/* Cartesian components, lexicographic: x^i y^j z^k with i descending, */
/* then j descending (l=2: xx xy xz yy yz zz).                          */
/* ------------------------------------------------------------------ */
static int ora_ncart(int l) { return (l + 1) * (l + 2) / 2; }

static void ora_cart(int l, int idx, int* c)
{
    int n = 0;
    for (int i = l; i >= 0; --i)
        for (int j = l - i; j >= 0; --j) {
            if (n == idx) { c[0] = i; c[1] = j; c[2] = l - i - j; return; }
            ++n;
        }
}

static double ora_dfact(int n) /* (n)!! with (-1)!! = 1 */
{
    double r = 1.0;
    for (int k = n; k > 1; k -= 2) r *= k;
    return r;
}

/* ------------------------------------------------------------------ */
/* Basis                                                              */
/* ------------------------------------------------------------------ */
typedef struct {
    int nshell, nbf;
    double* xyz;   /* [nshell][3] */
    int* l;
    int* nprim;
    int* poff;     /* first primitive of each shell */
    int* foff;     /* first function of each shell */
    double* alpha; /* [nprim total] */
    double* coef;  /* normalized, includes the primitive x^l norm */
    double* cnorm; /* per function: Cartesian component factor */
} ora_basis;

/* Primitive normalization of x^l exp(-a r^2) along one axis-power pattern:
 * N(a,l) = (2a/pi)^{3/4} (4a)^{l/2} / sqrt((2l-1)!!).  The contraction is
 * then rescaled so that <x^l|x^l> = 1, and each Cartesian component gets
 * sqrt((2l-1)!! / ((2i-1)!!(2j-1)!!(2k-1)!!)) so that every component has
 * unit self-overlap. */
void* ora_basis_create(int nshell, const double* xyz, const int* l, const int* nprim,
                       const double* alpha, const double* coef)
{
    ora_basis* b = (ora_basis*)calloc(1, sizeof(ora_basis));
    b->nshell = nshell;
    b->xyz = (double*)malloc(sizeof(double) * 3 * nshell);
    memcpy(b->xyz, xyz, sizeof(double) * 3 * nshell);
    b->l = (int*)malloc(sizeof(int) * nshell);
    b->nprim = (int*)malloc(sizeof(int) * nshell);
    b->poff = (int*)malloc(sizeof(int) * (nshell + 1));
    b->foff = (int*)malloc(sizeof(int) * (nshell + 1));
    int np = 0, nf = 0;
    for (int s = 0; s < nshell; ++s) {
        b->l[s] = l[s]; b->nprim[s] = nprim[s];
        b->poff[s] = np; b->foff[s] = nf;
        np += nprim[s]; nf += ora_ncart(l[s]);
    }
    b->poff[nshell] = np; b->foff[nshell] = nf;
    b->nbf = nf;
    b->alpha = (double*)malloc(sizeof(double) * np);
    b->coef = (double*)malloc(sizeof(double) * np);
    memcpy(b->alpha, alpha, sizeof(double) * np);
    for (int s = 0; s < nshell; ++s) {
        int L = l[s], p0 = b->poff[s], n = nprim[s];
        for (int i = 0; i < n; ++i) {
            double a = alpha[p0 + i];
            b->coef[p0 + i] = coef[p0 + i] * pow(2.0 * a / ORA_PI, 0.75) * pow(4.0 * a, 0.5 * L)
                              / sqrt(ora_dfact(2 * L - 1));
        }
        /* self overlap of the contracted x^l function */
        double ss = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double p = alpha[p0 + i] + alpha[p0 + j];
                ss += b->coef[p0 + i] * b->coef[p0 + j] * pow(ORA_PI / p, 1.5)
                      * ora_dfact(2 * L - 1) / pow(2.0 * p, L);
            }
        double r = 1.0 / sqrt(ss);
        for (int i = 0; i < n; ++i) b->coef[p0 + i] *= r;
    }
    b->cnorm = (double*)malloc(sizeof(double) * nf);
    for (int s = 0; s < nshell; ++s) {
        int L = l[s];
        for (int c = 0; c < ora_ncart(L); ++c) {
            int e[3] = {0, 0, 0}; ora_cart(L, c, e);
            b->cnorm[b->foff[s] + c] = sqrt(ora_dfact(2 * L - 1) /
                (ora_dfact(2 * e[0] - 1) * ora_dfact(2 * e[1] - 1) * ora_dfact(2 * e[2] - 1)));
        }
    }
    return b;
}

void ora_basis_destroy(void* h)
{
    ora_basis* b = (ora_basis*)h;
    if (!b) return;
    free(b->xyz); free(b->l); free(b->nprim); free(b->poff); free(b->foff);
    free(b->alpha); free(b->coef); free(b->cnorm); free(b);
}

int ora_nbf(void* h) { return ((ora_basis*)h)->nbf; }
void ora_shell_offsets(void* h, int* off)
{
    ora_basis* b = (ora_basis*)h;
    memcpy(off, b->foff, sizeof(int) * (b->nshell + 1));
}

/* ------------------------------------------------------------------ */
/* McMurchie-Davidson Hermite expansion                                */
/* ------------------------------------------------------------------ */
/* E^{ij}_t for one Cartesian direction, Gaussians with exponents a, b at
 * A, B.  E^{00}_0 = exp(-ab/(a+b) X_AB^2);
 * E^{i+1,j}_t = E^{ij}_{t-1}/(2p) + X_PA E^{ij}_t + (t+1) E^{ij}_{t+1};
 * E^{i,j+1}_t = E^{ij}_{t-1}/(2p) + X_PB E^{ij}_t + (t+1) E^{ij}_{t+1}. */
#define EDIM (ORA_LMAX + 3)
static void ora_hermite_E(int imax, int jmax, double a, double b, double A, double B,
                          double E[EDIM][EDIM][2 * EDIM + 1])
{
    double p = a + b, mu = a * b / p, P = (a * A + b * B) / p;
    double XPA = P - A, XPB = P - B, XAB = A - B;
    memset(E, 0, sizeof(double) * EDIM * EDIM * (2 * EDIM + 1));
    E[0][0][0] = exp(-mu * XAB * XAB);
    for (int i = 0; i <= imax; ++i)
        for (int j = 0; j <= jmax; ++j) {
            if (i == 0 && j == 0) continue;
            for (int t = 0; t <= i + j; ++t) {
                double v;
                if (i > 0) {
                    v = XPA * E[i - 1][j][t];
                    if (t > 0) v += E[i - 1][j][t - 1] / (2.0 * p);
                    if (t + 1 <= i - 1 + j) v += (t + 1) * E[i - 1][j][t + 1];
                } else {
                    v = XPB * E[i][j - 1][t];
                    if (t > 0) v += E[i][j - 1][t - 1] / (2.0 * p);
                    if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
                }
                E[i][j][t] = v;
            }
        }
}

/* Hermite Coulomb integrals R_{tuv}(alpha, PQ) for t+u+v <= L:
 * R^n_{000} = (-2 alpha)^n F_n(alpha |PQ|^2),
 * R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X_PQ R^{n+1}_{t,u,v} (same for u, v). */
#define RD (ORA_RMAX + 1)
typedef struct { double v[RD][RD][RD]; } ora_R;

static void ora_hermite_R(int L, double alpha, double X, double Y, double Z, ora_R* out)
{
    static __thread double R[RD][RD][RD][RD];
    double T = alpha * (X * X + Y * Y + Z * Z);
    for (int n = L; n >= 0; --n) {
        R[n][0][0][0] = pow(-2.0 * alpha, n) * ora_boys(n, T);
        for (int s = 1; s <= L - n; ++s)
            for (int t = s; t >= 0; --t)
                for (int u = s - t; u >= 0; --u) {
                    int v = s - t - u;
                    double r;
                    if (t > 0) {
                        r = X * R[n + 1][t - 1][u][v];
                        if (t > 1) r += (t - 1) * R[n + 1][t - 2][u][v];
                    } else if (u > 0) {
                        r = Y * R[n + 1][t][u - 1][v];
                        if (u > 1) r += (u - 1) * R[n + 1][t][u - 2][v];
                    } else {
                        r = Z * R[n + 1][t][u][v - 1];
                        if (v > 1) r += (v - 1) * R[n + 1][t][u][v - 2];
                    }
                    R[n][t][u][v] = r;
                }
    }
    for (int t = 0; t <= L; ++t)
        for (int u = 0; u <= L - t; ++u)
            for (int v = 0; v <= L - t - u; ++v) out->v[t][u][v] = R[0][t][u][v];
}

/* Unnormalized primitive ERI over x^i y^j z^k exp(-a r^2) Gaussians:
 * (ab|cd) = 2 pi^{5/2} / (p q sqrt(p+q)) sum_{tuv} E^{ab}_{tuv}
 *           sum_{tau nu phi} (-1)^{tau+nu+phi} E^{cd}_{tau nu phi} R_{t+tau,u+nu,v+phi}. */
double ora_eri_prim(const int* ea, double a, const double* A,
                    const int* eb, double b, const double* B,
                    const int* ec, double c, const double* C,
                    const int* ed, double d, const double* D)
{
    static __thread double Eab[3][EDIM][EDIM][2 * EDIM + 1];
    static __thread double Ecd[3][EDIM][EDIM][2 * EDIM + 1];
    static __thread ora_R R;
    double p = a + b, q = c + d, alpha = p * q / (p + q);
    double P[3], Q[3];
    for (int k = 0; k < 3; ++k) {
        ora_hermite_E(ea[k], eb[k], a, b, A[k], B[k], Eab[k]);
        ora_hermite_E(ec[k], ed[k], c, d, C[k], D[k], Ecd[k]);
        P[k] = (a * A[k] + b * B[k]) / p;
        Q[k] = (c * C[k] + d * D[k]) / q;
    }
    int L = ea[0] + ea[1] + ea[2] + eb[0] + eb[1] + eb[2] + ec[0] + ec[1] + ec[2] + ed[0] + ed[1] + ed[2];
    ora_hermite_R(L, alpha, P[0] - Q[0], P[1] - Q[1], P[2] - Q[2], &R);
    double sum = 0.0;
    for (int t = 0; t <= ea[0] + eb[0]; ++t)
        for (int u = 0; u <= ea[1] + eb[1]; ++u)
            for (int v = 0; v <= ea[2] + eb[2]; ++v) {
                double e1 = Eab[0][ea[0]][eb[0]][t] * Eab[1][ea[1]][eb[1]][u] * Eab[2][ea[2]][eb[2]][v];
                if (e1 == 0.0) continue;
                for (int tt = 0; tt <= ec[0] + ed[0]; ++tt)
                    for (int uu = 0; uu <= ec[1] + ed[1]; ++uu)
                        for (int vv = 0; vv <= ec[2] + ed[2]; ++vv) {
                            double e2 = Ecd[0][ec[0]][ed[0]][tt] * Ecd[1][ec[1]][ed[1]][uu]
                                        * Ecd[2][ec[2]][ed[2]][vv];
                            double sgn = ((tt + uu + vv) & 1) ? -1.0 : 1.0;
                            sum += e1 * sgn * e2 * R.v[t + tt][u + uu][v + vv];
                        }
            }
    return 2.0 * pow(ORA_PI, 2.5) / (p * q * sqrt(p + q)) * sum;
}

/* Contracted, normalized shell-quartet block, layout [na][nb][nc][nd].
 * Per primitive quartet the Hermite tables E^{ab}, E^{cd} and R are built
 * once, the ket Hermite sum is taken first,
 *   G_{tuv}(kl) = sum_{tau nu phi} (-1)^{tau+nu+phi} E^{cd}_{tau nu phi} R_{t+tau,u+nu,v+phi},
 * and then the bra sum (ij|kl) += pref * sum_{tuv} E^{ab}_{tuv} G_{tuv}(kl):
 * the same double sum as ora_eri_prim, summed in two steps. */
void ora_eri_shell(void* h, int sa, int sb, int sc, int sd, double* out)
{
    ora_basis* B = (ora_basis*)h;
    int la = B->l[sa], lb = B->l[sb], lc = B->l[sc], ld = B->l[sd];
    int na = ora_ncart(la), nb = ora_ncart(lb), nc = ora_ncart(lc), nd = ora_ncart(ld);
    int tot = na * nb * nc * nd;
    for (int i = 0; i < tot; ++i) out[i] = 0.0;
    int Lab = la + lb, Lcd = lc + ld, L = Lab + Lcd;
    int H = Lab + 1;
    double* G = (double*)malloc(sizeof(double) * nc * nd * H * H * H);
    static __thread double Eab[3][EDIM][EDIM][2 * EDIM + 1];
    static __thread double Ecd[3][EDIM][EDIM][2 * EDIM + 1];
    static __thread ora_R R;
    const double* A = B->xyz + 3 * sa; const double* Bc = B->xyz + 3 * sb;
    const double* C = B->xyz + 3 * sc; const double* D = B->xyz + 3 * sd;
    for (int pa = 0; pa < B->nprim[sa]; ++pa)
    for (int pb = 0; pb < B->nprim[sb]; ++pb)
    for (int pc = 0; pc < B->nprim[sc]; ++pc)
    for (int pd = 0; pd < B->nprim[sd]; ++pd) {
        int ia = B->poff[sa] + pa, ib = B->poff[sb] + pb;
        int ic = B->poff[sc] + pc, id = B->poff[sd] + pd;
        double a = B->alpha[ia], b = B->alpha[ib], c = B->alpha[ic], d = B->alpha[id];
        double cc = B->coef[ia] * B->coef[ib] * B->coef[ic] * B->coef[id];
        double p = a + b, q = c + d, alpha = p * q / (p + q);
        double P[3], Q[3];
        for (int k = 0; k < 3; ++k) {
            ora_hermite_E(la, lb, a, b, A[k], Bc[k], Eab[k]);
            ora_hermite_E(lc, ld, c, d, C[k], D[k], Ecd[k]);
            P[k] = (a * A[k] + b * Bc[k]) / p;
            Q[k] = (c * C[k] + d * D[k]) / q;
        }
        ora_hermite_R(L, alpha, P[0] - Q[0], P[1] - Q[1], P[2] - Q[2], &R);
        double pref = cc * 2.0 * pow(ORA_PI, 2.5) / (p * q * sqrt(p + q));
        for (int k = 0; k < nc; ++k)
            for (int l = 0; l < nd; ++l) {
                int e2[3] = {0, 0, 0}, e3[3] = {0, 0, 0};
                ora_cart(lc, k, e2); ora_cart(ld, l, e3);
                double* g = G + (size_t)(k * nd + l) * H * H * H;
                for (int t = 0; t <= Lab; ++t)
                    for (int u = 0; u <= Lab - t; ++u)
                        for (int v = 0; v <= Lab - t - u; ++v) {
                            double s = 0.0;
                            for (int tt = 0; tt <= e2[0] + e3[0]; ++tt)
                                for (int uu = 0; uu <= e2[1] + e3[1]; ++uu)
                                    for (int vv = 0; vv <= e2[2] + e3[2]; ++vv) {
                                        double e = Ecd[0][e2[0]][e3[0]][tt] * Ecd[1][e2[1]][e3[1]][uu]
                                                   * Ecd[2][e2[2]][e3[2]][vv];
                                        double sgn = ((tt + uu + vv) & 1) ? -1.0 : 1.0;
                                        s += sgn * e * R.v[t + tt][u + uu][v + vv];
                                    }
                            g[(t * H + u) * H + v] = s;
                        }
            }
        for (int i = 0; i < na; ++i)
            for (int j = 0; j < nb; ++j) {
                int e0[3] = {0, 0, 0}, e1[3] = {0, 0, 0};
                ora_cart(la, i, e0); ora_cart(lb, j, e1);
                for (int k = 0; k < nc; ++k)
                    for (int l = 0; l < nd; ++l) {
                        const double* g = G + (size_t)(k * nd + l) * H * H * H;
                        double s = 0.0;
                        for (int t = 0; t <= e0[0] + e1[0]; ++t)
                            for (int u = 0; u <= e0[1] + e1[1]; ++u)
                                for (int v = 0; v <= e0[2] + e1[2]; ++v)
                                    s += Eab[0][e0[0]][e1[0]][t] * Eab[1][e0[1]][e1[1]][u]
                                         * Eab[2][e0[2]][e1[2]][v] * g[(t * H + u) * H + v];
                        out[((i * nb + j) * nc + k) * nd + l] += pref * s;
                    }
            }
    }
    free(G);
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j)
            for (int k = 0; k < nc; ++k)
                for (int l = 0; l < nd; ++l)
                    out[((i * nb + j) * nc + k) * nd + l] *=
                        B->cnorm[B->foff[sa] + i] * B->cnorm[B->foff[sb] + j]
                        * B->cnorm[B->foff[sc] + k] * B->cnorm[B->foff[sd] + l];
}

/* ------------------------------------------------------------------ */
/* One-electron integrals (setup for the real-time path)               */
/* ------------------------------------------------------------------ */
/* kind 0: overlap  S = <a|b>
 * kind 1: kinetic  T = -1/2 <a|lap|b>
 * kind 2: dipole   <a| r_dir - origin_dir |b>   (dir = extra)
 * kind 3: nuclear  V = -sum_C Z_C <a| 1/|r-C| |b> */
static double ora_1e_prim(int kind, int dir, const int* ea, double a, const double* A,
                          const int* eb, double b, const double* B,
                          const double* origin, int ncharge, const double* Z, const double* Cxyz)
{
    double E[3][EDIM][EDIM][2 * EDIM + 1];
    double p = a + b, P[3];
    for (int k = 0; k < 3; ++k) {
        ora_hermite_E(ea[k], eb[k] + 2, a, b, A[k], B[k], E[k]);
        P[k] = (a * A[k] + b * B[k]) / p;
    }
    double s1 = sqrt(ORA_PI / p);
    if (kind == 0) return E[0][ea[0]][eb[0]][0] * E[1][ea[1]][eb[1]][0] * E[2][ea[2]][eb[2]][0] * s1 * s1 * s1;
    if (kind == 1) {
        double S[3], D2[3];
        for (int k = 0; k < 3; ++k) {
            int i = ea[k], j = eb[k];
            S[k] = E[k][i][j][0] * s1;
            double d2 = 4.0 * b * b * E[k][i][j + 2][0] - 2.0 * b * (2 * j + 1) * E[k][i][j][0];
            if (j >= 2) d2 += (double)j * (j - 1) * E[k][i][j - 2][0];
            D2[k] = d2 * s1;
        }
        return -0.5 * (D2[0] * S[1] * S[2] + S[0] * D2[1] * S[2] + S[0] * S[1] * D2[2]);
    }
    if (kind == 2) {
        double r = s1 * s1 * s1;
        for (int k = 0; k < 3; ++k) {
            if (k == dir) r *= E[k][ea[k]][eb[k]][1] + (P[k] - origin[k]) * E[k][ea[k]][eb[k]][0];
            else r *= E[k][ea[k]][eb[k]][0];
        }
        return r;
    }
    /* nuclear attraction: -Z_C (2 pi / p) sum_tuv E_tuv R_tuv(p, P - C) */
    int L = ea[0] + ea[1] + ea[2] + eb[0] + eb[1] + eb[2];
    ora_R R;
    double tot = 0.0;
    for (int c = 0; c < ncharge; ++c) {
        ora_hermite_R(L, p, P[0] - Cxyz[3 * c], P[1] - Cxyz[3 * c + 1], P[2] - Cxyz[3 * c + 2], &R);
        double s = 0.0;
        for (int t = 0; t <= ea[0] + eb[0]; ++t)
            for (int u = 0; u <= ea[1] + eb[1]; ++u)
                for (int v = 0; v <= ea[2] + eb[2]; ++v)
                    s += E[0][ea[0]][eb[0]][t] * E[1][ea[1]][eb[1]][u] * E[2][ea[2]][eb[2]][v] * R.v[t][u][v];
        tot += -Z[c] * 2.0 * ORA_PI / p * s;
    }
    return tot;
}

void ora_one_electron(void* h, int kind, int dir, const double* origin,
                      int ncharge, const double* Z, const double* Cxyz, double* out)
{
    ora_basis* B = (ora_basis*)h;
    int nbf = B->nbf;
    double o[3] = {0, 0, 0};
    if (origin) { o[0] = origin[0]; o[1] = origin[1]; o[2] = origin[2]; }
    #pragma omp parallel for schedule(dynamic)
    for (int sa = 0; sa < B->nshell; ++sa)
        for (int sb = 0; sb < B->nshell; ++sb)
            for (int i = 0; i < ora_ncart(B->l[sa]); ++i)
                for (int j = 0; j < ora_ncart(B->l[sb]); ++j) {
                    int e0[3] = {0, 0, 0}, e1[3] = {0, 0, 0};
                    ora_cart(B->l[sa], i, e0); ora_cart(B->l[sb], j, e1);
                    double s = 0.0;
                    for (int pa = 0; pa < B->nprim[sa]; ++pa)
                        for (int pb = 0; pb < B->nprim[sb]; ++pb) {
                            int ia = B->poff[sa] + pa, ib = B->poff[sb] + pb;
                            s += B->coef[ia] * B->coef[ib]
                                 * ora_1e_prim(kind, dir, e0, B->alpha[ia], B->xyz + 3 * sa,
                                               e1, B->alpha[ib], B->xyz + 3 * sb, o, ncharge, Z, Cxyz);
                        }
                    int mu = B->foff[sa] + i, nu = B->foff[sb] + j;
                    out[mu * nbf + nu] = s * B->cnorm[mu] * B->cnorm[nu];
                }
}

/* ------------------------------------------------------------------ */
/* Coulomb / exchange                                                  */
/* ------------------------------------------------------------------ */
/* Apply one ordered shell quartet block v[(i,j,k,l)] = (ab|cd):
 *   J_{ab} += v X_{cd};  K_{ac} += v X_{bd}  for every density. */
static void ora_apply(const ora_basis* B, int sa, int sb, int sc, int sd, const double* v,
                      int nmat, const double* X, double* J, double* K)
{
    int nbf = B->nbf;
    int na = ora_ncart(B->l[sa]), nb = ora_ncart(B->l[sb]);
    int nc = ora_ncart(B->l[sc]), nd = ora_ncart(B->l[sd]);
    int fa = B->foff[sa], fb = B->foff[sb], fc = B->foff[sc], fd = B->foff[sd];
    size_t mm = (size_t)nbf * nbf;
    for (int m = 0; m < nmat; ++m) {
        const double* x = X + m * mm;
        double* j_ = J ? J + m * mm : NULL;
        double* k_ = K ? K + m * mm : NULL;
        for (int i = 0; i < na; ++i)
            for (int j = 0; j < nb; ++j)
                for (int k = 0; k < nc; ++k)
                    for (int l = 0; l < nd; ++l) {
                        double val = v[((i * nb + j) * nc + k) * nd + l];
                        if (j_) j_[(fa + i) * nbf + fb + j] += val * x[(fc + k) * nbf + fd + l];
                        if (k_) k_[(fa + i) * nbf + fc + k] += val * x[(fb + j) * nbf + fd + l];
                    }
    }
}

static int ora_maxblock(const ora_basis* B)
{
    int lm = 0;
    for (int s = 0; s < B->nshell; ++s) if (B->l[s] > lm) lm = B->l[s];
    int n = ora_ncart(lm);
    return n * n * n * n;
}

/* Plain definition: every ordered shell quartet, no symmetry.
 * X, J, K: [nmat][nbf][nbf] row-major; J or K may be NULL. */
void ora_jk_full(void* h, int nmat, const double* X, double* J, double* K)
{
    ora_basis* B = (ora_basis*)h;
    int ns = B->nshell, nbf = B->nbf;
    size_t tot = (size_t)nmat * nbf * nbf;
    if (J) memset(J, 0, sizeof(double) * tot);
    if (K) memset(K, 0, sizeof(double) * tot);
    int nth = omp_get_max_threads();
    double* Jt = J ? (double*)calloc((size_t)nth * tot, sizeof(double)) : NULL;
    double* Kt = K ? (double*)calloc((size_t)nth * tot, sizeof(double)) : NULL;
    int mb = ora_maxblock(B);
    #pragma omp parallel
    {
        int t = omp_get_thread_num();
        double* blk = (double*)malloc(sizeof(double) * mb);
        #pragma omp for schedule(static)
        for (int ab = 0; ab < ns * ns; ++ab) {
            int sa = ab / ns, sb = ab % ns;
            for (int sc = 0; sc < ns; ++sc)
                for (int sd = 0; sd < ns; ++sd) {
                    ora_eri_shell(B, sa, sb, sc, sd, blk);
                    ora_apply(B, sa, sb, sc, sd, blk, nmat, X,
                              Jt ? Jt + t * tot : NULL, Kt ? Kt + t * tot : NULL);
                }
        }
        free(blk);
    }
    for (int t = 0; t < nth; ++t)
        for (size_t i = 0; i < tot; ++i) {
            if (J) J[i] += Jt[t * tot + i];
            if (K) K[i] += Kt[t * tot + i];
        }
    free(Jt); free(Kt);
}

/* The same sum taken over canonical quartets a>=b, c>=d, (ab)>=(cd): each
 * canonical block is computed once and applied through every DISTINCT
 * shell-level image among the eight index permutations (duplicates found by
 * comparing shell tuples, so no degeneracy factors are derived by hand). */
static void ora_permute_block(const ora_basis* B, const int* sh, const double* v, int perm,
                              int* osh, double* w)
{
    /* perm k maps (i,j,k,l) -> image index order */
    static const int P[8][4] = {
        {0, 1, 2, 3}, {1, 0, 2, 3}, {0, 1, 3, 2}, {1, 0, 3, 2},
        {2, 3, 0, 1}, {3, 2, 0, 1}, {2, 3, 1, 0}, {3, 2, 1, 0}};
    int n[4];
    for (int k = 0; k < 4; ++k) n[k] = ora_ncart(B->l[sh[k]]);
    for (int k = 0; k < 4; ++k) osh[k] = sh[P[perm][k]];
    int on[4];
    for (int k = 0; k < 4; ++k) on[k] = n[P[perm][k]];
    int idx[4];
    for (idx[0] = 0; idx[0] < n[0]; ++idx[0])
        for (idx[1] = 0; idx[1] < n[1]; ++idx[1])
            for (idx[2] = 0; idx[2] < n[2]; ++idx[2])
                for (idx[3] = 0; idx[3] < n[3]; ++idx[3]) {
                    int o[4];
                    for (int k = 0; k < 4; ++k) o[k] = idx[P[perm][k]];
                    w[((o[0] * on[1] + o[1]) * on[2] + o[2]) * on[3] + o[3]] =
                        v[((idx[0] * n[1] + idx[1]) * n[2] + idx[2]) * n[3] + idx[3]];
                }
}

void ora_jk_sym(void* h, int nmat, const double* X, double* J, double* K)
{
    ora_basis* B = (ora_basis*)h;
    int ns = B->nshell, nbf = B->nbf;
    size_t tot = (size_t)nmat * nbf * nbf;
    if (J) memset(J, 0, sizeof(double) * tot);
    if (K) memset(K, 0, sizeof(double) * tot);
    int nth = omp_get_max_threads();
    double* Jt = J ? (double*)calloc((size_t)nth * tot, sizeof(double)) : NULL;
    double* Kt = K ? (double*)calloc((size_t)nth * tot, sizeof(double)) : NULL;
    int npair = ns * (ns + 1) / 2;
    int mb = ora_maxblock(B);
    #pragma omp parallel
    {
        int t = omp_get_thread_num();
        double* blk = (double*)malloc(sizeof(double) * mb);
        double* w = (double*)malloc(sizeof(double) * mb);
        #pragma omp for schedule(dynamic, 1)
        for (int ab = 0; ab < npair; ++ab) {
            int sa = 0;
            while ((sa + 1) * (sa + 2) / 2 <= ab) ++sa;
            int sb = ab - sa * (sa + 1) / 2;
            for (int cd = 0; cd <= ab; ++cd) {
                int sc = 0;
                while ((sc + 1) * (sc + 2) / 2 <= cd) ++sc;
                int sd = cd - sc * (sc + 1) / 2;
                int sh[4] = {sa, sb, sc, sd};
                ora_eri_shell(B, sa, sb, sc, sd, blk);
                int seen[8][4], nseen = 0;
                for (int p = 0; p < 8; ++p) {
                    int osh[4];
                    ora_permute_block(B, sh, blk, p, osh, w);
                    int dup = 0;
                    for (int q = 0; q < nseen; ++q)
                        if (seen[q][0] == osh[0] && seen[q][1] == osh[1] &&
                            seen[q][2] == osh[2] && seen[q][3] == osh[3]) dup = 1;
                    if (dup) continue;
                    memcpy(seen[nseen++], osh, sizeof(osh));
                    ora_apply(B, osh[0], osh[1], osh[2], osh[3], w, nmat, X,
                              Jt ? Jt + t * tot : NULL, Kt ? Kt + t * tot : NULL);
                }
            }
        }
        free(blk); free(w);
    }
    for (int t = 0; t < nth; ++t)
        for (size_t i = 0; i < tot; ++i) {
            if (J) J[i] += Jt[t * tot + i];
            if (K) K[i] += Kt[t * tot + i];
        }
    free(Jt); free(Kt);
}

/* Sampled blocks straight from the definition (no symmetry):
 *   J block (sa,sb):  J_{mn} = sum over all shells c,d of (ab|cd) X_cd
 *   K block (sa,sc):  K_{mn} = sum over all shells b,d of (ab|cd) X_bd
 * out: [nmat][na][nb] (J) or [nmat][na][nc] (K). */
void ora_j_block(void* h, int sa, int sb, int nmat, const double* X, double* out)
{
    ora_basis* B = (ora_basis*)h;
    int ns = B->nshell, nbf = B->nbf;
    int na = ora_ncart(B->l[sa]), nb = ora_ncart(B->l[sb]);
    size_t mm = (size_t)nbf * nbf;
    int nth = omp_get_max_threads();
    double* acc = (double*)calloc((size_t)nth * nmat * na * nb, sizeof(double));
    int mb = ora_maxblock(B);
    #pragma omp parallel
    {
        int t = omp_get_thread_num();
        double* blk = (double*)malloc(sizeof(double) * mb);
        double* a = acc + (size_t)t * nmat * na * nb;
        #pragma omp for schedule(static)
        for (int cd = 0; cd < ns * ns; ++cd) {
            int sc = cd / ns, sd = cd % ns;
            int nc = ora_ncart(B->l[sc]), nd = ora_ncart(B->l[sd]);
            int fc = B->foff[sc], fd = B->foff[sd];
            ora_eri_shell(B, sa, sb, sc, sd, blk);
            for (int m = 0; m < nmat; ++m)
                for (int i = 0; i < na; ++i)
                    for (int j = 0; j < nb; ++j)
                        for (int k = 0; k < nc; ++k)
                            for (int l = 0; l < nd; ++l)
                                a[(m * na + i) * nb + j] += blk[((i * nb + j) * nc + k) * nd + l]
                                                            * X[m * mm + (size_t)(fc + k) * nbf + fd + l];
        }
        free(blk);
    }
    memset(out, 0, sizeof(double) * nmat * na * nb);
    for (int t = 0; t < nth; ++t)
        for (int i = 0; i < nmat * na * nb; ++i) out[i] += acc[(size_t)t * nmat * na * nb + i];
    free(acc);
}

void ora_k_block(void* h, int sa, int sc, int nmat, const double* X, double* out)
{
    ora_basis* B = (ora_basis*)h;
    int ns = B->nshell, nbf = B->nbf;
    int na = ora_ncart(B->l[sa]), nc = ora_ncart(B->l[sc]);
    size_t mm = (size_t)nbf * nbf;
    int nth = omp_get_max_threads();
    double* acc = (double*)calloc((size_t)nth * nmat * na * nc, sizeof(double));
    int mb = ora_maxblock(B);
    #pragma omp parallel
    {
        int t = omp_get_thread_num();
        double* blk = (double*)malloc(sizeof(double) * mb);
        double* a = acc + (size_t)t * nmat * na * nc;
        #pragma omp for schedule(static)
        for (int bd = 0; bd < ns * ns; ++bd) {
            int sb = bd / ns, sd = bd % ns;
            int nb = ora_ncart(B->l[sb]), nd = ora_ncart(B->l[sd]);
            int fb = B->foff[sb], fd = B->foff[sd];
            ora_eri_shell(B, sa, sb, sc, sd, blk);
            for (int m = 0; m < nmat; ++m)
                for (int i = 0; i < na; ++i)
                    for (int j = 0; j < nb; ++j)
                        for (int k = 0; k < nc; ++k)
                            for (int l = 0; l < nd; ++l)
                                a[(m * na + i) * nc + k] += blk[((i * nb + j) * nc + k) * nd + l]
                                                            * X[m * mm + (size_t)(fb + j) * nbf + fd + l];
        }
        free(blk);
    }
    memset(out, 0, sizeof(double) * nmat * na * nc);
    for (int t = 0; t < nth; ++t)
        for (int i = 0; i < nmat * na * nc; ++i) out[i] += acc[(size_t)t * nmat * na * nc + i];
    free(acc);
}

/* Schwarz factors Q_ab = sqrt(max_{m in a, n in b} (mn|mn)), [nshell][nshell]. */
void ora_schwarz(void* h, double* Q)
{
    ora_basis* B = (ora_basis*)h;
    int ns = B->nshell;
    int mb = ora_maxblock(B);
    #pragma omp parallel
    {
        double* blk = (double*)malloc(sizeof(double) * mb);
        #pragma omp for schedule(dynamic)
        for (int ab = 0; ab < ns * ns; ++ab) {
            int sa = ab / ns, sb = ab % ns;
            int na = ora_ncart(B->l[sa]), nb = ora_ncart(B->l[sb]);
            ora_eri_shell(B, sa, sb, sa, sb, blk);
            double mx = 0.0;
            for (int i = 0; i < na; ++i)
                for (int j = 0; j < nb; ++j) {
                    double v = blk[((i * nb + j) * na + i) * nb + j];
                    if (v > mx) mx = v;
                }
            Q[ab] = sqrt(mx);
        }
        free(blk);
    }
}

int ora_num_threads(void) { return omp_get_max_threads(); }
void ora_set_threads(int n) { omp_set_num_threads(n); }

/* Normalized primitive coefficients (incl. the x^l primitive factor) and the
 * per-function Cartesian component factors, for independent checks. */
void ora_basis_coefs(void* h, double* coef, double* cnorm)
{
    ora_basis* b = (ora_basis*)h;
    memcpy(coef, b->coef, sizeof(double) * b->poff[b->nshell]);
    memcpy(cnorm, b->cnorm, sizeof(double) * b->nbf);
}
