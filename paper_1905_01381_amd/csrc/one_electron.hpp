// Arguments of the one-electron integral kernel (see one_electron.hip).
#pragma once
#include <hip/hip_runtime.h>

struct OneEArgs {
    int nshell, nbf, kind, dir, ncharge, pad_;
    const int* l;
    const int* nprim;
    const int* poff;
    const int* foff;
    const double* xyz;
    const double* alpha;
    const double* coef;   // primitive coefficients incl. the x^l normalization
    const double* cnorm;  // per-function component factors
    const double* Z;      // point charges
    const double* cxyz;   // their positions
    double origin[3];
    double* out;          // [nbf][nbf]
};

__device__ __forceinline__ void cart_exps(int l, int idx, int* e)
{
    int n = 0;
    for (int i = l; i >= 0; --i)
        for (int j = l - i; j >= 0; --j) {
            if (n == idx) {
                e[0] = i;
                e[1] = j;
                e[2] = l - i - j;
                return;
            }
            ++n;
        }
    e[0] = e[1] = e[2] = 0;
}

__device__ __forceinline__ double binom(int n, int k)
{
    double r = 1.0;
    for (int t = 1; t <= k; ++t) r = r * (n - k + t) / t;
    return r;
}

__device__ __forceinline__ double ipow(double x, int n)
{
    double r = 1.0;
    for (int t = 0; t < n; ++t) r *= x;
    return r;
}

__global__ void one_electron_kernel(OneEArgs g, const double* __restrict__ boys_tab);
