// One-electron integrals over the library's normalized Cartesian shells:
// overlap, kinetic energy, nuclear attraction (point charges) and a dipole
// component.  They set up the real-time propagation (core Hamiltonian,
// metric and the field/observable operator; paper: "Real-Time Electronic
// Dynamics", Eqs. td_pert and td_expectation) and the S-orthonormal
// densities of the synthetic workloads.  Obara-Saika recurrences:
//   overlap (per axis):  S_{i+1,j} = X_PA S_ij + (i S_{i-1,j} + j S_{i,j-1}) / (2p)
//   kinetic (per axis):  T_ij = -1/2 (4 b^2 S_{i,j+2} - 2 b (2j+1) S_ij + j(j-1) S_{i,j-2})
//   moment  (per axis):  <i|x - O|j> = S_{i,j+1} + (B - O) S_ij
//   nuclear: [a+1_i|b]^(m) = PA_i [a|b]^(m) - PC_i [a|b]^(m+1)
//                            + a_i/(2p) ([a-1_i|b]^(m) - [a-1_i|b]^(m+1))
//            from [0|0]^(m) = 2 pi / p exp(-mu AB^2) F_m(p |PC|^2), then
//            the horizontal transfer (a, b+1_i) = (a+1_i, b) + AB_i (a, b).
#include "eri_common.hpp"
#include "one_electron.hpp"

namespace {

__device__ int cart_index(int l, int i, int j)
{
    // position of x^i y^j z^(l-i-j) in the lexicographic list of degree l
    const int x = l - i;  // components before x^i start: 0 + 1 + ... + (l - i)
    return x * (x + 1) / 2 + (l - i - j);
}

__device__ void overlap_1d(double p, double PA, double PB, int imax, int jmax, double S[5][7])
{
    for (int i = 0; i <= imax; ++i)
        for (int j = 0; j <= jmax; ++j) {
            double v;
            if (i == 0 && j == 0) v = 1.0;
            else if (i > 0) {
                v = PA * S[i - 1][j];
                if (i > 1) v += (i - 1) * S[i - 2][j] / (2 * p);
                if (j > 0) v += j * S[i - 1][j - 1] / (2 * p);
            } else {
                v = PB * S[i][j - 1];
                if (j > 1) v += (j - 1) * S[i][j - 2] / (2 * p);
            }
            S[i][j] = v;
        }
}

}  // namespace

// One thread per ordered shell pair (a, b); writes the full block.
__global__ void one_electron_kernel(OneEArgs g, const double* __restrict__ boys_tab)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.nshell * g.nshell) return;
    const int sa = t / g.nshell, sb = t % g.nshell;
    const int la = g.l[sa], lb = g.l[sb];
    const double A[3] = {g.xyz[3 * sa], g.xyz[3 * sa + 1], g.xyz[3 * sa + 2]};
    const double B[3] = {g.xyz[3 * sb], g.xyz[3 * sb + 1], g.xyz[3 * sb + 2]};
    const int na = (la + 1) * (la + 2) / 2, nb = (lb + 1) * (lb + 2) / 2;
    double out[100];  // shells up to f
    for (int k = 0; k < 100; ++k) out[k] = 0.0;
    const double AB2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
    for (int pa = 0; pa < g.nprim[sa]; ++pa)
        for (int pb = 0; pb < g.nprim[sb]; ++pb) {
            const double al = g.alpha[g.poff[sa] + pa], be = g.alpha[g.poff[sb] + pb];
            const double cc = g.coef[g.poff[sa] + pa] * g.coef[g.poff[sb] + pb];
            const double p = al + be, mu = al * be / p;
            double P[3], PA[3], PB[3];
            for (int k = 0; k < 3; ++k) {
                P[k] = (al * A[k] + be * B[k]) / p;
                PA[k] = P[k] - A[k];
                PB[k] = P[k] - B[k];
            }
            const double Kab = exp(-mu * AB2);
            if (g.kind != 3) {
                double S[3][5][7];
                for (int k = 0; k < 3; ++k) overlap_1d(p, PA[k], PB[k], la, lb + 2, S[k]);
                const double s1 = sqrt(3.14159265358979323846 / p);
                const double pre = cc * Kab * s1 * s1 * s1;
                for (int i = 0; i < na; ++i)
                    for (int j = 0; j < nb; ++j) {
                        int ea[3], eb[3];
                        cart_exps(la, i, ea);
                        cart_exps(lb, j, eb);
                        double v;
                        if (g.kind == 0) {
                            v = S[0][ea[0]][eb[0]] * S[1][ea[1]][eb[1]] * S[2][ea[2]][eb[2]];
                        } else if (g.kind == 1) {
                            double Sx[3], Tx[3];
                            for (int k = 0; k < 3; ++k) {
                                const int ii = ea[k], jj = eb[k];
                                Sx[k] = S[k][ii][jj];
                                double d2 = 4 * be * be * S[k][ii][jj + 2] - 2 * be * (2 * jj + 1) * S[k][ii][jj];
                                if (jj >= 2) d2 += jj * (jj - 1) * S[k][ii][jj - 2];
                                Tx[k] = -0.5 * d2;
                            }
                            v = Tx[0] * Sx[1] * Sx[2] + Sx[0] * Tx[1] * Sx[2] + Sx[0] * Sx[1] * Tx[2];
                        } else {
                            v = 1.0;
                            for (int k = 0; k < 3; ++k) {
                                if (k == g.dir) v *= S[k][ea[k]][eb[k] + 1] + (B[k] - g.origin[k]) * S[k][ea[k]][eb[k]];
                                else v *= S[k][ea[k]][eb[k]];
                            }
                        }
                        out[i * nb + j] += pre * v;
                    }
            } else {
                // nuclear attraction: vertical recurrence on a up to la+lb, then
                // the horizontal transfer to (a, b)
                const int L = la + lb;
                for (int c = 0; c < g.ncharge; ++c) {
                    const double C[3] = {g.cxyz[3 * c], g.cxyz[3 * c + 1], g.cxyz[3 * c + 2]};
                    const double PC[3] = {P[0] - C[0], P[1] - C[1], P[2] - C[2]};
                    const double T = p * (PC[0] * PC[0] + PC[1] * PC[1] + PC[2] * PC[2]);
                    double F[7];
                    boys_fp64<6>(T, boys_tab, F);
                    // V[e][m]: e over all components of degree 0..L (<= 84), m <= L
                    double V[84][7];
                    const double base = 2 * 3.14159265358979323846 / p * Kab;
                    for (int m = 0; m <= L; ++m) V[0][m] = base * F[m];
                    const int off[8] = {0, 1, 4, 10, 20, 35, 56, 84};
                    for (int le = 1; le <= L; ++le)
                        for (int ci = 0; ci < (le + 1) * (le + 2) / 2; ++ci) {
                            int e[3];
                            cart_exps(le, ci, e);
                            const int i = e[0] > 0 ? 0 : (e[1] > 0 ? 1 : 2);
                            int e1[3] = {e[0], e[1], e[2]};
                            e1[i] -= 1;
                            const int i1 = off[le - 1] + cart_index(le - 1, e1[0], e1[1]);
                            for (int m = 0; m <= L - le; ++m) {
                                double v = PA[i] * V[i1][m] - PC[i] * V[i1][m + 1];
                                if (e1[i] > 0) {
                                    int e2[3] = {e1[0], e1[1], e1[2]};
                                    e2[i] -= 1;
                                    const int i2 = off[le - 2] + cart_index(le - 2, e2[0], e2[1]);
                                    v += e1[i] / (2 * p) * (V[i2][m] - V[i2][m + 1]);
                                }
                                V[off[le] + ci][m] = v;
                            }
                        }
                    // horizontal transfer: (a, b) from (e, 0), e = a + part of b
                    for (int i = 0; i < na; ++i)
                        for (int j = 0; j < nb; ++j) {
                            int ea[3], eb[3];
                            cart_exps(la, i, ea);
                            cart_exps(lb, j, eb);
                            // expand prod_k (x_A + AB_k)^{b_k} binomially
                            double v = 0.0;
                            for (int tx = 0; tx <= eb[0]; ++tx)
                                for (int ty = 0; ty <= eb[1]; ++ty)
                                    for (int tz = 0; tz <= eb[2]; ++tz) {
                                        const int ex = ea[0] + tx, ey = ea[1] + ty, ez = ea[2] + tz;
                                        const int le = ex + ey + ez;
                                        const double w = binom(eb[0], tx) * binom(eb[1], ty) * binom(eb[2], tz)
                                                         * ipow(A[0] - B[0], eb[0] - tx) * ipow(A[1] - B[1], eb[1] - ty)
                                                         * ipow(A[2] - B[2], eb[2] - tz);
                                        v += w * V[off[le] + cart_index(le, ex, ey)][0];
                                    }
                            out[i * nb + j] += -g.Z[c] * cc * v;
                        }
                }
            }
        }
    const int fa = g.foff[sa], fb = g.foff[sb];
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nb; ++j)
            g.out[(long long)(fa + i) * g.nbf + fb + j] = out[i * nb + j] * g.cnorm[fa + i] * g.cnorm[fb + j];
}
