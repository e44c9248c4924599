// Device-side types and helpers shared by the generated electron-repulsion
// kernels and the hand-written support kernels of libcq.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define CQ_MAX_MAT 16

// ---------------------------------------------------------------------------
// Boys function F_m(T), m = 0..L, FP64.
// T < BOYS_TC: F_L from a Chebyshev interpolant on intervals of width
// BOYS_H (degree BOYS_NC-1), then the downward recursion
// F_m = (2T F_{m+1} + exp(-T)) / (2m+1), which is stable.
// T >= BOYS_TC: F_0 = sqrt(pi/T)/2 (erf(sqrt T) = 1 to 2e-17 there) and the
// upward recursion F_{m+1} = ((2m+1) F_m - exp(-T)) / (2T), stable for T > m.
// ---------------------------------------------------------------------------
#define BOYS_TC 36.0
#define BOYS_H 0.5
#define BOYS_NINT 72
#define BOYS_NC 10
#define BOYS_LMAX 16

__device__ __forceinline__ double rsqrt_f64(double x) { return rsqrt(x); }
__device__ __forceinline__ float rsqrt_f32(float x) { return rsqrtf(x); }

#define BOYS_TAB_L (BOYS_NINT * BOYS_NC)  // coefficients of one order F_L

// tabL: the BOYS_NINT x BOYS_NC coefficients of order L (device or LDS).
template <int L>
__device__ __forceinline__ void boys_fp64_tab(double T, const double* __restrict__ tabL, double* F)
{
    if (T < BOYS_TC) {
        int k = (int)(T * (1.0 / BOYS_H));
        k = k < 0 ? 0 : (k > BOYS_NINT - 1 ? BOYS_NINT - 1 : k);
        const double x = (T - k * BOYS_H) * (2.0 / BOYS_H) - 1.0;
        const double* c = tabL + k * BOYS_NC;
        double b1 = 0.0, b2 = 0.0;
#pragma unroll
        for (int j = BOYS_NC - 1; j >= 1; --j) {
            const double b0 = fma(2.0 * x, b1, c[j] - b2);
            b2 = b1;
            b1 = b0;
        }
        F[L] = fma(x, b1, c[0] - b2);
        if (L > 0) {
            const double e = exp(-T);
            const double t2 = 2.0 * T;
#pragma unroll
            for (int m = L - 1; m >= 0; --m) F[m] = fma(t2, F[m + 1], e) * (1.0 / (2 * m + 1));
        }
    } else {
        F[0] = 0.88622692545275801365 * rsqrt_f64(T);  // sqrt(pi)/2 / sqrt(T)
        if (L > 0) {
            const double e = exp(-T);
            const double h = 0.5 / T;
#pragma unroll
            for (int m = 0; m < L; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) * h;
        }
    }
}

// tab: the whole table, orders 0..BOYS_LMAX.
template <int L>
__device__ __forceinline__ void boys_fp64(double T, const double* __restrict__ tab, double* F)
{
    boys_fp64_tab<L>(T, tab + (size_t)L * BOYS_TAB_L, F);
}

// FP32 Boys function for the precision-routed path.  The table of FP32
// Chebyshev coefficients follows the FP64 table in the same allocation.
// Large arguments (T >= BOYS_TC) and high orders (L >= 6) are evaluated in
// FP64 and rounded, so only the low-order, small-argument part runs in FP32.
#define BOYS_TAB_DOUBLES ((BOYS_LMAX + 1) * BOYS_NINT * BOYS_NC)

// tabL: for L < 6 the FP32 coefficients of order L; for L >= 6 the FP64
// coefficients of order L (only the FP64 evaluation uses a table then; the
// large-argument branch uses none).
template <int L>
__device__ __forceinline__ void boys_fp32_tab(float T, const void* __restrict__ tabL, float* F)
{
    if (L >= 6 || !(T < (float)BOYS_TC)) {
        double Fd[L + 1];
        boys_fp64_tab<L>((double)T, (const double*)tabL, Fd);
#pragma unroll
        for (int m = 0; m <= L; ++m) F[m] = (float)Fd[m];
        return;
    }
    int k = (int)(T * (1.0f / (float)BOYS_H));
    k = k < 0 ? 0 : (k > BOYS_NINT - 1 ? BOYS_NINT - 1 : k);
    const float x = (T - k * (float)BOYS_H) * (2.0f / (float)BOYS_H) - 1.0f;
    const float* c = (const float*)tabL + k * BOYS_NC;
    float b1 = 0.0f, b2 = 0.0f;
#pragma unroll
    for (int j = BOYS_NC - 1; j >= 1; --j) {
        const float b0 = fmaf(2.0f * x, b1, c[j] - b2);
        b2 = b1;
        b1 = b0;
    }
    F[L] = fmaf(x, b1, c[0] - b2);
    if (L > 0) {
        const float e = expf(-T);
        const float t2 = 2.0f * T;
#pragma unroll
        for (int m = L - 1; m >= 0; --m) F[m] = fmaf(t2, F[m + 1], e) * (1.0f / (2 * m + 1));
    }
}

// Compensated (Kahan) FP32 accumulation: s + c carries the running sum.
__device__ __forceinline__ void kahan_add(float& s, float& c, float x)
{
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// ---------------------------------------------------------------------------
// Shell-pair data of one pair class (la >= lb).  Pair-level arrays are
// [npair]; the primitive-pair data of a pair is one contiguous run of
// records, so a lane fetches a primitive pair with a few wide loads (a wave
// touches at most eight distinct ket pairs per step).
// ---------------------------------------------------------------------------
struct PairSet {
    int npair, nprim2, stride, pad_;  // stride: unused (kept for layout)
    const int* sa;   // first shell (angular momentum la)
    const int* sb;   // second shell
    const int* fa;   // first function of sa, counted from its molecule's first
    const int* fb;
    const double* ABx;  // A - B
    const double* ABy;
    const double* ABz;
    const double* Q;    // Schwarz factor of the pair (raw components)
    // Primitive-pair records [npair][nprim2][10]: p, K, 1/(2p), Px, Py, Pz,
    // PAx, PAy, PAz, 0 (one lane reads its record with five 16-byte loads).
    const double* rec;  // K = c_a c_b exp(-alpha beta/p |AB|^2) sqrt(2) pi^{5/4} / p
    // Records of a pair with K != 0 (above the primitive cut); they come
    // first, so records nsig .. nprim2-1 of the pair all have K = 0.
    const int* nsig;
};

// One molecule of a basis (a batch holds many): its shells and functions are
// contiguous; shell-pair tables (ppos, block maxima) and the packed densities
// and partial sums are block-diagonal, one block per molecule.
struct MolInfo {
    long long xoff;   // first element of the molecule's [nbf][nbf] block
    long long soff;   // first element of its [ns][ns] shell-pair block
    int f0, nbf;      // first function, functions
    int s0, ns;       // first shell, shells
};

// Work of one class (la lb|lc ld): one task per (molecule, a, R consecutive
// b, 64/R consecutive d, a range of c), R the class's tile rows (8 unless the
// generator says otherwise); the wave loops over c.  Lane (64/R) i + j holds
// the quartet (a b_i | c d_j).  Shells of each angular momentum are
// listed molecule by molecule in index order (shl_*); ppos maps an oriented
// shell pair (higher l first; a >= b for equal l) of one molecule to its
// position in its pair class.
struct TaskMap {
    const int4* tasks;  // (a index, first b index, first d index, first c index)
    const int4* tasks2; // (end of b range, end of d range, molecule, last c index)
    const int* ppos;    // block-diagonal [ns][ns] per molecule
    const int* shl_a;
    const int* shl_b;
    const int* shl_c;
    const int* shl_d;
    const MolInfo* mols;
    int ntask, pad_;
    // screened or routed builds: the tasks of one precision (list[0 ..
    // *list_n)) and per task the steps of each precision (masks[2 t] FP64,
    // masks[2 t + 1] FP32; bit k = step c_lo + k).  list = NULL: every task,
    // every step (c ranges are at most 64 steps).
    const int* list;
    const int* list_n;
    const unsigned long long* masks;
};

// Sums over the C lanes of a tile row (lanes C i .. C i + C - 1) / over the
// 64 / C lanes of a tile column (lane = C i + j).
template <int C>
__device__ __forceinline__ double red_cols(double v)
{
#pragma unroll
    for (int o = 1; o < C; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <int C>
__device__ __forceinline__ double red_rows(double v)
{
#pragma unroll
    for (int o = C; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <int C>
__device__ __forceinline__ float red_colsf(float v)
{
#pragma unroll
    for (int o = 1; o < C; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <int C>
__device__ __forceinline__ float red_rowsf(float v)
{
#pragma unroll
    for (int o = C; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}


// Densities and outputs of one build, interleaved [mu][nu][slot] within each
// molecule's block.
struct Digest {
    const double* X;  // per molecule [nbf][nbf][nX], scaled by component factors
    double* J;        // per molecule [nbf][nbf][nJ] partial sums J' (two fixed-point words each)
    double* K;        // per molecule [nbf][nbf][nK] partial sums K'
    int nbf, nX, nJ, nK;
    int jslot[CQ_MAX_MAT];
    int kslot[CQ_MAX_MAT];
    double skip;          // density-weighted Schwarz threshold (0: none)
    const double* pmax;   // block-diagonal [ns][ns] per molecule: max |X| per shell block
    int nshell;
    int rot;              // bit 0: each task starts its c walk at step (task mod length);
                          // bit 1: tasks dealt to the 8 XCDs in contiguous eighths
    double* stage;        // per-wave private stage, [wave][class stage size][64]
    size_t stage_bytes;   // bytes of the stage workspace (caps the grid of staged classes)
    int mode;             // 0: FP64 everywhere; 1: precision-routed
    int acc_lvl;          // task-invariant partial sums kept in LDS over a task: 0 none (straight to
                          // J'/K'), 1 J'_ab and K'_ad, 2 also K'_bd (unstaged classes)
    double fp32_below;    // routed mode: a wave step whose largest bound is below this runs in FP32
    unsigned long long* counts;  // [3]: quartets evaluated in FP64, in FP32, skipped by screening
    // J' and K' hold each element as two 64-bit integers, the fixed-point
    // limbs of fx_add, side by side; fx[0] = 2^S is the build's fixed-point
    // scale (computed on the device from the inputs), fx[1] = 2^-S.
    const double* fx;
};

// One molecule's blocks as seen by a task: uniform base pointers plus
// 32-bit offsets (function indices are local to the molecule; a molecule
// holds at most 16383 functions, so [nbf][nbf][8] offsets fit in 32 bits).
struct MolView {
    const double* X;
    double* J;
    double* K;
    const int* ppos;
    const double* pmax;
    int nbf, s0, ns;
    double fxs;  // fixed-point scale 2^S
};

__device__ __forceinline__ MolView mol_view(const Digest& dg, const TaskMap& tm, int m)
{
    const MolInfo mi = tm.mols[m];
    MolView v;
    v.X = dg.X + mi.xoff * dg.nX;
    v.J = dg.J + 2 * mi.xoff * dg.nJ;
    v.K = dg.K + 2 * mi.xoff * dg.nK;
    v.ppos = tm.ppos + mi.soff;
    v.pmax = dg.pmax + mi.soff;
    v.nbf = mi.nbf;
    v.s0 = mi.s0;
    v.ns = mi.ns;
    v.fxs = dg.fx[0];
    return v;
}
__device__ __forceinline__ double ld_x(const Digest& dg, const MolView& mc, int mu, int nu, int m)
{
    return mc.X[(mu * mc.nbf + nu) * dg.nX + m];
}
__device__ __forceinline__ int jidx(const Digest& dg, const MolView& mc, int mu, int nu, int s)
{
    return (mu * mc.nbf + nu) * dg.nJ + s;
}
__device__ __forceinline__ int kidx(const Digest& dg, const MolView& mc, int mu, int nu, int s)
{
    return (mu * mc.nbf + nu) * dg.nK + s;
}
// offset of the oriented shell pair (a, b) (global shell indices) in the
// molecule's [ns][ns] tables
__device__ __forceinline__ int spair(const MolView& mc, int a, int b) { return (a - mc.s0) * mc.ns + (b - mc.s0); }

// Accumulation by exact fixed-point integers, so that results do not depend
// on the order in which waves add (the technique of reproducible GPU force
// summation, e.g. Le Grand, Goetz and Walker's SPFP, Comput. Phys. Commun.
// 184, 374 (2013), taken to two limbs): a contribution x becomes the integer
// w = rint(x 2^S), |w| < 2^91, split as w = hi 2^31 + lo with
// 0 <= lo < 2^31.  hi adds into the element's first 64-bit word and lo into
// the second, with no carries between them; integer addition is associative,
// so every sum is the same whatever the order.  The low word takes up to
// 2^32 contributions per element.
__device__ __forceinline__ void fx_add(double* p, double x, double scale)
{
    const double w = rint(x * scale);
    const double t = floor(w * 0x1p-31);   // hi as an integer-valued double, |t| < 2^60
    const double lo = w - t * 0x1p31;       // exact, in [0, 2^31)
    const double th = floor(t * 0x1p-32);
    const double tl = t - th * 0x1p32;      // exact, in [0, 2^32)
    const unsigned long long hi =
        ((unsigned long long)(long long)(int)th << 32) | (unsigned long long)(unsigned)tl;
    atomicAdd((unsigned long long*)p, hi);
    atomicAdd((unsigned long long*)p + 1, (unsigned long long)(unsigned)lo);
}

// Value of element i of a J'/K' buffer of fixed-point limb pairs
// (inv = 2^-S).
__device__ __forceinline__ double partial_value(const double* A, long long i, double inv)
{
    const long long hi = ((const long long*)A)[2 * i];
    const long long lo = ((const long long*)A)[2 * i + 1];
    return fma((double)hi, 0x1p31, (double)lo) * inv;
}

// Flush one partial sum into J' / K' (element index from jidx / kidx, below
// 2^31 by the build's size check, so 2 idx fits 32 unsigned bits).
__device__ __forceinline__ void acc_j(const MolView& mc, int idx, double v)
{
    fx_add(mc.J + 2u * (unsigned)idx, v, mc.fxs);
}
__device__ __forceinline__ void acc_k(const MolView& mc, int idx, double v)
{
    fx_add(mc.K + 2u * (unsigned)idx, v, mc.fxs);
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// min(cap, largest v over the 64 lanes), read into a scalar register so that
// a loop bounded by it is wave-uniform.  Every lane of the wave must be
// active.
__device__ __forceinline__ int wave_max_bound(int v, int cap)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return __builtin_amdgcn_readfirstlane(v < cap ? v : cap);
}


__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Per-wave stage of the staged kernels, addressed through a buffer resource:
// element i of lane l lives at byte 512 i + 8 l of the wave's region, so one
// VGPR (8 l) and a uniform scalar offset (512 i) address every element and
// no per-element address registers are kept live.
typedef __amdgpu_buffer_rsrc_t stage_rsrc;
typedef unsigned int stage_u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ stage_rsrc stage_make(double* base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ double stage_load(stage_rsrc r, int voff, int i)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, i * 512, 0));
}
__device__ __forceinline__ void stage_store(stage_rsrc r, int voff, int i, double x)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(stage_u32x2, x), r, voff, i * 512, 0);
}

// Compiler-only barrier between the phases of the staged kernels: values
// written to the per-wave stage are re-read from memory instead of being
// forwarded in registers (which would defeat the staging).
__device__ __forceinline__ void stage_fence() { __asm__ volatile("" ::: "memory"); }

__device__ __forceinline__ double quartet_bound(const MolView& mc, double qab, double qcd, int a, int b, int c, int d)
{
    const double* pm = mc.pmax;
    double m = fmax(fmax(pm[spair(mc, a, b)], pm[spair(mc, c, d)]), fmax(pm[spair(mc, a, c)], pm[spair(mc, a, d)]));
    m = fmax(m, fmax(pm[spair(mc, b, c)], pm[spair(mc, b, d)]));
    return qab * qcd * m;
}
