/*
 * cq.h -- C ABI of libcq, the MI355X (gfx950) integral-direct Coulomb /
 * exchange build.
 *
 * What is computed (paper: "Reference Wave Functions", Eq. 2c_fock, and the
 * integral-direct statement that follows it; "General Infrastructure for the
 * Unified Treatment of Electronic Spin", Eqs. pauli_sep, spin_generalization,
 * 2c_expectation):
 *
 *   J[X]_{mn} = sum_{ls} (mn|ls) X_{ls}          K[X]_{mn} = sum_{ls} (ml|ns) X_{ls}
 *
 * with (mn|ls) the electron-repulsion integrals over contracted Cartesian
 * Gaussian shells (paper: Introduction, LCAO over contracted Gaussian-type
 * orbitals), recomputed on every call (direct SCF) and never stored.
 *
 * Conventions for every entry point
 * - Units: bohr, hartree, atomic units of time.
 * - Matrices are contiguous row-major double [nbf][nbf] in DEVICE memory,
 *   owned by the caller; the library never frees them.  Outputs must not
 *   alias inputs.
 * - Functions are ordered shell by shell in the order given to
 *   cq_basis_create; within a shell, Cartesian components are lexicographic
 *   (l=1: x y z; l=2: xx xy xz yy yz zz; l=3: xxx xxy xxz xyy xyz xzz yyy
 *   yyz yzz zzz), each normalized to unit self-overlap.  Bases made by
 *   cq_basis_create_general may also hold spherical d and f shells and
 *   generally contracted shells (see there); nbf then counts the caller's
 *   functions.
 * - Work is enqueued on the given stream (NULL = the default stream) and is
 *   asynchronous unless stated.  A handle must not be used from two streams
 *   at the same time.
 * - Every function returns a cq_status; on failure, cq_last_error() gives a
 *   message (thread-local).  Argument errors are detected before any work
 *   is enqueued.
 */
#ifndef CQ_H
#define CQ_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CQ_OK = 0,
    CQ_EINVAL = 1,        /* invalid argument */
    CQ_ENOMEM = 2,        /* device or host allocation failed */
    CQ_EHIP = 3,          /* a HIP runtime call failed */
    CQ_EUNSUPPORTED = 4,  /* angular momentum above f, or a feature not built */
    CQ_ENONFINITE = 5,    /* a non-finite value was found in an input density */
    CQ_ENOTCONV = 6       /* an iterative step did not converge */
} cq_status;

typedef struct cq_basis_s* cq_basis;

/* Thresholds of one build (NULL = exact FP64, deterministic, overwrite).
 *   skip:       quartets whose bound Q_ab Q_cd max|X| (Schwarz factors times
 *               the largest density element of the six shell blocks the
 *               quartet touches, maximized over all densities; the paper's
 *               LinK-like screening, "Reference Wave Functions") is below
 *               this value are not evaluated.  0 = no screening (exact).
 *   fp32_below: in mode 1, a batch of 64 quartets (one wave step: one bra
 *               shell a, eight b, one c, eight d) whose largest bound is below
 *               this value is evaluated in FP32: FP32 recurrences with
 *               compensated (Kahan) accumulation over primitives, FP32 partial
 *               sums folded into the FP64 J and K; the Boys function for
 *               T >= 36 or order >= 6 stays FP64.  Other batches run in FP64.
 *   mode:       0 = FP64 throughout; 1 = precision-routed.
 *   flags:      CQ_ACCUMULATE adds into J/K instead of overwriting them.
 *               CQ_DETERMINISTIC (accepted, always in effect): partial sums
 *               are accumulated as exact fixed-point integers (a scale 2^S
 *               chosen per build from a bound of the sums, two 64-bit words
 *               per element), so two builds of the same inputs give bitwise
 *               equal J and K whatever the order of the device's additions.
 *               Other bits: CQ_EINVAL. */
typedef struct {
    double skip;
    double fp32_below;
    int mode;
    unsigned flags;
} cq_thresholds;

#define CQ_ACCUMULATE 1u
#define CQ_DETERMINISTIC 2u
#define CQ_MAX_DENSITIES 16

/* Thread-local message describing the last failure ("" if none). */
const char* cq_last_error(void);

/* Create a basis from host arrays (copied; the caller keeps ownership).
 *   nshell          number of shells (>= 1)
 *   xyz[nshell*3]   shell centers (bohr)
 *   l[nshell]       angular momentum, 0..3 (classes with an f shell run one
 *                   workgroup per shell quartet with its recurrences in LDS;
 *                   CQ_EUNSUPPORTED if the device's LDS per workgroup cannot
 *                   hold one ket component of a class)
 *   nprim[nshell]   primitives per shell, 1..8
 *   alpha[], coef[] exponents and raw contraction coefficients, concatenated
 *                   shell by shell (sum(nprim) entries)
 * Each contracted function is normalized (paper: Introduction, contracted
 * Gaussian-type orbitals): primitives carry (2a/pi)^{3/4}(4a)^{l/2}/sqrt((2l-1)!!),
 * the contraction is rescaled to unit self-overlap of x^l, and each Cartesian
 * component x^i y^j z^k gets sqrt((2l-1)!!/((2i-1)!!(2j-1)!!(2k-1)!!)).
 * Allocates library-owned device memory; synchronizes `stream`.  The Schwarz
 * factors are computed here (see cq_schwarz). */
cq_status cq_basis_create(int nshell, const double* xyz, const int* l, const int* nprim,
                          const double* alpha, const double* coef, hipStream_t stream,
                          cq_basis* out);

/* A batch of independent molecules in one handle (the batched uneven
 * launch: one integral pass serves every molecule, each class in a single
 * launch whose tasks span all molecules; quartets never mix molecules).
 *   nmol             number of molecules, >= 1
 *   nshell_mol[nmol] host, shells of each molecule (>= 1 each); the shell
 *                    arrays (xyz, l, nprim, alpha, coef: as in
 *                    cq_basis_create) list molecule 0's shells, then
 *                    molecule 1's, ...
 * Matrices of a batch handle (densities, J, K, cq_schwarz output) are the
 * concatenation of the molecules' row-major [nbf_m][nbf_m] blocks, molecule
 * m starting at element sum_{k<m} nbf_k^2.  Shell-pair quantities
 * (cq_schwarz) are concatenated [ns_m][ns_m] blocks likewise.  The
 * two-component, one-electron and real-time entry points take
 * single-molecule handles only (CQ_EUNSUPPORTED otherwise).  Allocates and
 * synchronizes like cq_basis_create. */
cq_status cq_basis_create_batch(int nmol, const int* nshell_mol, const double* xyz, const int* l,
                                const int* nprim, const double* alpha, const double* coef,
                                hipStream_t stream, cq_basis* out);

/* A basis of segmented or generally contracted shells, each Cartesian or
 * spherical (paper: Introduction, contracted Gaussian basis functions with
 * general or segmented contraction).  Arguments as in
 * cq_basis_create_batch (nmol = 1 for one molecule), plus, per shell:
 *   ncontr[nshell]  host, contractions over the shell's nprim exponents
 *                   (1 = segmented, up to 64)
 *   pure[nshell]    host, 1 = spherical, 0 = Cartesian; for l <= 1 the two
 *                   are the same (p stays x, y, z)
 *   coef[]          per shell ncontr rows of nprim raw coefficients
 *                   (contraction-major), shells one after another
 *                   (sum nprim * ncontr entries; alpha has sum nprim)
 * A shell with ncontr contractions contributes its functions contraction by
 * contraction: contraction k is the segmented shell with coefficient row k,
 * normalized as in cq_basis_create.  A spherical d shell has 5 functions,
 * the unit-normalized real solid harmonics m = -2..2: xy, yz,
 * (3z^2 - r^2), xz, (x^2 - y^2) (each as a combination of the normalized
 * Cartesian xx..zz of the same contraction); a spherical f shell has 7,
 * m = -3..3: y(3x^2 - y^2), xyz, y(4z^2 - x^2 - y^2), z(2z^2 - 3x^2 - 3y^2),
 * x(4z^2 - x^2 - y^2), z(x^2 - y^2), x(x^2 - 3y^2).  Every matrix of the
 * handle (densities, J, K, one-electron integrals, cq_fock2e_2c's spin
 * blocks, the real-time matrices) is in these functions; internally the
 * integrals run over Cartesian segmented shells and densities pass through
 * the shell transformations on the way in, results on the way out.
 * Shell-level outputs (cq_schwarz, cq_eri_quartet, cq_basis_nshell) refer
 * to the expanded Cartesian segmented shells.  l = 4 and above:
 * CQ_EUNSUPPORTED.
 * Allocates and synchronizes like cq_basis_create. */
cq_status cq_basis_create_general(int nmol, const int* nshell_mol, const double* xyz, const int* l,
                                  const int* nprim, const int* ncontr, const int* pure, const double* alpha,
                                  const double* coef, hipStream_t stream, cq_basis* out);

/* Molecules in a handle (1 for cq_basis_create; -1 on NULL) and the basis
 * functions of each, written to HOST nbf_mol[nmol]. */
int cq_basis_nmol(cq_basis b);
cq_status cq_basis_mol_nbf(cq_basis b, int* nbf_mol);

/* Release a basis and all of its device memory (synchronizes the device). */
cq_status cq_basis_destroy(cq_basis b);

/* Number of basis functions (the caller's) / shells (after expanding
 * general contractions) of a basis (-1 on a NULL handle). */
int cq_basis_nbf(cq_basis b);
int cq_basis_nshell(cq_basis b);

/* Schwarz factors Q_ab = sqrt(max_{m in a, n in b} (mn|mn)) (paper:
 * "Reference Wave Functions", integral screening).  Computed once at basis
 * creation and cached.  If Q is not NULL, the [nshell][nshell] matrix (for
 * a batch: the per-molecule [ns_m][ns_m] blocks, concatenated) is copied to
 * the DEVICE buffer Q (stream-ordered). */
cq_status cq_schwarz(cq_basis b, double* Q, hipStream_t stream);

/* Size limit of the build kernels, which address a molecule's interleaved
 * [nbf][nbf][slots] blocks with 32-bit element offsets: returns CQ_OK if
 * nbf^2 * max(nx, nj, nk) < 2^31, else CQ_EUNSUPPORTED (CQ_EINVAL for
 * negative arguments).  nbf is the largest molecule's function count; nx, nj,
 * nk are the density, Coulomb and exchange slots of one integral pass
 * (cq_jk_build: nmat and the non-NULL J / K entries; cq_fock2e_2c: 8, 1, 8).
 * Host only.  cq_jk_build, cq_fock2e_2c and cq_autotune apply it to their own
 * arguments before any work is enqueued. */
cq_status cq_jk_size_check(int nbf, int nx, int nj, int nk);

/* Device status of a basis: synchronizes `stream`, then returns
 * CQ_ENONFINITE if a density packed by a build on this basis since the last
 * call held a NaN or infinity (the packing kernels set a device status word;
 * J and K of such a build are not meaningful), CQ_OK otherwise.  Reading
 * clears the word. */
cq_status cq_sync_status(cq_basis b, hipStream_t stream);

/* Coulomb and exchange matrices of nmat densities in one integral pass.
 *   nmat        1..CQ_MAX_DENSITIES internal slots (see sym)
 *   P[nmat]     host array of device pointers to the densities X_m
 *               (nbf x nbf row-major; for a batch handle, the concatenated
 *               per-molecule blocks described at cq_basis_create_batch)
 *   sym[nmat]   +1 if X_m is symmetric, -1 if antisymmetric (only that part
 *               of X_m is used; e.g. the imaginary part of a Hermitian
 *               density is antisymmetric, paper: the remark on the
 *               symmetry of X^I after Eq. spin_generalization), 0 for a
 *               general real matrix with no symmetry, such as the transition
 *               densities of the direct response sigma-vectors (paper:
 *               "Residue Methods"); it is split into its symmetric and
 *               antisymmetric parts, takes two of the CQ_MAX_DENSITIES
 *               internal slots, and J[X] = J[X_s], K[X] = K[X_s] + K[X_a]
 *   J[nmat]     host array of device output pointers; an entry may be NULL
 *               (no Coulomb matrix wanted); must be NULL where sym = -1
 *               (J of an antisymmetric density vanishes).  J itself may be
 *               NULL (no Coulomb matrices at all).
 *   K[nmat]     same for exchange; K may be NULL.
 *   th          thresholds (NULL = exact FP64, overwrite)
 * No Fock factors are applied: J and K are the bare contractions above.
 * Asynchronous on `stream`. */
cq_status cq_jk_build(cq_basis b, int nmat, const double* const* P, const int* sym,
                      double* const* J, double* const* K, const cq_thresholds* th,
                      hipStream_t stream);

/* cq_jk_build for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, results and errors as cq_jk_build (results are bitwise
 * equal to it in the default deterministic mode), except:
 * - All scratch (packed densities, partial sums, block maxima, counters and
 *   the stage regions of the high angular momentum classes) comes from one
 *   static device array of 512 MiB that every GPU the library runs on holds
 *   until the process ends.  No hipMalloc, hipFree or allocating library
 *   routine is called.  The basis handle (created beforehand) and the
 *   caller's P, J, K are used as they are.
 * - The scratch must hold the densities and partial sums, about
 *   nel * 8 * (nmat + 2 (nJ + nK)) bytes for nel = sum of nbf_m^2 (e.g. nbf 600
 *   with 8 densities, 1 J and 8 K: 75 MB), plus one stage region of the largest
 *   angular momentum class present (1.7 MB for (dd|dd)); larger builds return
 *   CQ_ENOMEM before any work is enqueued.  The rest of the array holds stage
 *   regions, which caps the grid of those classes.
 * - The classes run one after another on `stream` (no internal streams or
 *   events).
 * - Every call on a GPU shares that GPU's array and leaves its contents
 *   behind; each call clears what it needs.  Calls that overlap in time on
 *   one GPU (other streams, other threads) race and must not be issued. */
cq_status cq_jk_build_noalloc(cq_basis b, int nmat, const double* const* P, const int* sym,
                              double* const* J, double* const* K, const cq_thresholds* th,
                              hipStream_t stream);

/* Two-electron part of the two-component (generalized spin) Fock matrix
 * (paper: Eq. pauli_sep and Eq. 2c_fock, with G^0 = 2 J[P^0] - K[P^0] and
 * G^k = -K[P^k]; the factor 2 follows from the 1/2 in Eq. pauli_sep):
 *   P2c   device, complex Hermitian spin-blocked density [[aa, ab],[ba, bb]],
 *         2nbf x 2nbf, interleaved (re, im) doubles, row-major
 *   G2c   device output, same layout: sum_I sigma_I (x) G^I
 * P2c is split into the real symmetric Re P^I and antisymmetric Im P^I
 * (I = 0..3); J is formed for Re P^0 and K for all eight in one integral
 * pass.  Asynchronous on `stream`. */
cq_status cq_fock2e_2c(cq_basis b, const double* P2c, double* G2c, const cq_thresholds* th,
                       hipStream_t stream);


/* One-electron integrals over the basis, written to the DEVICE matrix out
 * [nbf][nbf] (setup of the real-time path; paper: "Real-Time Electronic
 * Dynamics", Eqs. td_pert / td_expectation use a core Hamiltonian, a metric
 * and one-body field / observable operators):
 *   kind 0  overlap      S_mn = <m|n>
 *   kind 1  kinetic      T_mn = -1/2 <m|lap|n>
 *   kind 2  dipole       <m| r_dir - origin_dir |n>, dir = 0,1,2 (x,y,z)
 *   kind 3  nuclear      V_mn = -sum_C Z_C <m| 1/|r - R_C| |n>
 * origin (host, 3 doubles) may be NULL (= 0); Z[ncharge] and cxyz[3*ncharge]
 * are host arrays used only by kind 3.  Asynchronous on `stream` except for
 * kind 3, which synchronizes it. */
cq_status cq_one_electron(cq_basis b, int kind, int dir, const double* origin, int ncharge,
                          const double* Z, const double* cxyz, double* out, hipStream_t stream);

/* Number of unique contracted shell quartets per class for an unscreened
 * build (bra pair >= ket pair; la>=lb, lc>=ld).  For entry k < maxn:
 * cls[4k..4k+3] = (la, lb, lc, ld), count[k]; *n = number of classes (the
 * generated s-d classes, then the classes with an f shell that the basis
 * holds; at most 55). */
cq_status cq_quartet_counts(cq_basis b, int maxn, int* cls, long long* count, int* n);

/* As cq_quartet_counts, but count[k] is the number of primitive quartets
 * those shell quartets hold once primitive pairs below the cut are dropped
 * (sum over the quartets of the surviving primitive pairs of the bra pair
 * times those of the ket pair).  A primitive pair is dropped when its
 * prefactor |c_a c_b| exp(-alpha beta/p |AB|^2) sqrt(2) pi^{5/4} / p is below
 * 1e-30 of the largest in the basis: its contribution to any integral is
 * below FP64 resolution.  The kernels skip those primitive pairs.  This is
 * the algorithmic primitive work of an unscreened build. */
cq_status cq_prim_quartet_counts(cq_basis b, int maxn, int* cls, long long* count, int* n);

/* Quartet counts of the most recent cq_jk_build / cq_fock2e_2c on this
 * basis, written to HOST out3: [0] evaluated in FP64, [1] evaluated in FP32
 * (precision-routed mode), [2] removed by screening.  Synchronizes `stream`. */
cq_status cq_build_stats(cq_basis b, unsigned long long* out3, hipStream_t stream);

/* Autotuner for the electron-repulsion launches of this handle: for every
 * class it times, with HIP events, each `reps` times (1..100), on a
 * synthetic density of nmat slots:
 *   1. orientations (as generated, and with bra and ket exchanged where
 *      that kernel exists) x task shapes (length of the c range one wave
 *      walks: the default, half, twice and four times it, at most 64) x grid
 *      caps (one wave per task, or 2048 waves looping over tasks);
 *   2. at the fastest of those, the task order flags (bit 0: tasks start
 *      their c walk at step task mod length, spreading the flushes of tasks
 *      that share a bra shell; bit 1: the task list is dealt to the 8 XCDs
 *      in runs of 8 consecutive tasks, so that tasks sharing shells share
 *      an L2) and
 *      every LDS accumulator level below the highest that fits (less LDS
 *      per wave, more resident waves, more flushes);
 * and keeps the fastest for every later build on the handle.  Classes with
 * an f shell have one fixed launch form and are not tuned.  Every plan is
 * deterministic; two plans agree to rounding only (the FP64 partial sums a
 * wave forms before its exact fixed-point additions depend on the plan).
 * Synchronizes `stream`; overwrites the handle's work buffers only. */
cq_status cq_autotune(cq_basis b, int nmat, int reps, hipStream_t stream);

/* The launch plan per class (tuned, set or default): for k < cap,
 * rec[10k..10k+9] = (la, lb, lc, ld, c-range length, grid cap or 0, tasks,
 * exchanged, LDS level or -1, task order flags) and ms[k] = best time measured by
 * cq_autotune (0 if not tuned); *n = classes with work.  exchanged = 1: the
 * class runs with bra and ket pairs exchanged, (lc ld|la lb), which loops
 * over the other pair's first shell and flushes fewer exchange partial sums
 * per step (built for (pp|ps), (dp|ps), (dp|ds) and (dd|ps)).  LDS level -1:
 * the highest that fits for the build's density count (0: none, 1: J'_ab and
 * K'_ad, 2: also K'_bd).  Host arrays. */
cq_status cq_autotune_read(cq_basis b, int cap, int* rec, float* ms, int* n);

/* Set the launch plan of n classes from records laid out as
 * cq_autotune_read writes them (the tasks field is ignored), e.g. a plan
 * tuned earlier on the same molecules.  Every record is checked first
 * (class with work on this basis, c-range length 1..64, grid cap >= 0,
 * exchanged 0/1 and built, LDS level -1..2, task order flags 0..3; CQ_EINVAL
 * otherwise, nothing changed).  Re-uploads the classes' task lists
 * (allocates); not stream-ordered: no build may be in flight on the handle. */
cq_status cq_plan_set(cq_basis b, int n, const int* rec);

/* Per-class launch timing with HIP events recorded on the launch stream
 * (tracing aid).  enable: 0 off, 1 on, 2 on and reset the totals.  Builds
 * normally run the classes concurrently on internal streams forked from the
 * caller's stream; with timing on they run one after another on the
 * caller's stream, so each time is one kernel's own.
 * cq_profile_read synchronizes on the recorded events and returns, per class
 * that ran (classes with an f shell included), cls[4k..4k+3], the summed
 * kernel time ms[k] and launch count count[k]; *n = number of such classes. */
cq_status cq_profile(cq_basis b, int enable);

/* Progress trace (tracing aid): with enable != 0, every build on this handle
 * prints "[cq] class (ab|cd) done" to stderr as each class's kernels finish
 * (a host function enqueued on the launch stream after them).  Off by
 * default; adds one host callback per class and build. */
cq_status cq_trace(cq_basis b, int enable);
cq_status cq_profile_read(cq_basis b, int maxn, int* cls, double* ms, long long* count, int* n);

/* ---- real-time propagation (paper: "Real-Time Electronic Dynamics") ---- */

typedef struct cq_rt_s* cq_rt;

#define CQ_RT_EM2 0       /* explicit 2nd-order Magnus (the paper's EM2), 2 builds/step */
#define CQ_RT_MIDPOINT 1  /* self-consistent midpoint Magnus-2 corrector */
#define CQ_RT_LEARNED 2   /* MLP midpoint proposal, corrector as fallback */
#define CQ_RT_MMUT 3      /* the paper's leap-frog MMUT, EM2 seed / restart, 1 build/step */

/* Propagator for a closed-shell density (P per spin, total 2P) in the
 * Loewdin orthonormal basis.  All matrix arguments are DEVICE buffers,
 * row-major [nbf][nbf], copied at creation:
 *   h   real core Hamiltonian (AO)        X   real S^{-1/2} (AO)
 *   Dz  real dipole-length operator <m|z - origin|n> (AO)
 *   P0  complex orthonormal-basis density P'(t0) = S^{1/2} P S^{1/2},
 *       interleaved (re, im)
 * F(P) = h + 2 J[Re P] - K[Re P] - i K[Im P] (Eq. 2c_fock, scalar part,
 * reading A1); the field-free propagation uses U = exp(-i dt F') with
 * F' = X F X (Taylor degree 16 with scaling and squaring).  The first three
 * steps of the midpoint and learned modes use EM2 (the paper's seed step).
 * Work runs on `stream` (kept by the handle). */
cq_status cq_rt_create(cq_basis b, const double* h, const double* X, const double* Dz, const double* P0,
                       double dt, int mode, hipStream_t stream, cq_rt* out);
cq_status cq_rt_destroy(cq_rt rt);
cq_status cq_rt_set_mode(cq_rt rt, int mode);
/* Midpoint convergence: max |P_mid^(i+1) - P_mid^(i)| < sc_tol within
 * max_iter builds (else CQ_ENOTCONV).  The first iterate of a midpoint or
 * learned step (the extrapolated guess, or the learned proposal) is accepted
 * when max |(P_k + P_{k+1})/2 - P_mid^(0)| < accept_tol (default 1e-10 =
 * the default sc_tol); both modes use the same acceptance, so their builds
 * per step compare at one tolerance. */
cq_status cq_rt_set_params(cq_rt rt, double sc_tol, int max_iter, double accept_tol);
/* MMUT (paper: "Real-Time Electronic Dynamics", the MMUT equation and the
 * EM2 seed / restart paragraph): P_{k+1} = U P_{k-1} U^dagger with
 * U = exp(-2 i dt F'(P_k)).  Step n of the handle (counted from creation) is
 * an EM2 step from P_k when n % period == 0 or no P_{k-1} exists yet, a
 * leap-frog step otherwise.  period >= 1 (default 1000). */
cq_status cq_rt_set_restart(cq_rt rt, int period);
/* External one-body perturbation (paper: "Real-Time Electronic Dynamics",
 * Eq. td_pert and the envelope list after it): F(P, t) = F_0(P) + f(t) V with
 * V the dipole matrix Dz given to cq_rt_create (a length-gauge electric
 * field along that operator) and
 *   f(t) = kappa g(t - t_on) for t_on <= t < t_off, 0 otherwise,
 *   g = 1 (envelope 1, step), u (2, linear ramp), cos(param u) (3, plane
 *   wave, param = omega), exp(-param u^2) (4, Gaussian, param = alpha);
 * envelope 0 removes the field (default).  Time t = (steps taken) x dt from
 * creation.  The Fock matrix of a density is taken at its own time: EM2 at
 * t_k and t_k + dt, the midpoint at t_k + dt/2, MMUT at t_k.  The energy
 * observable includes the interaction, Re Tr P (h + f V + F).  A delta kick
 * is applied by the caller to P0 before cq_rt_create.  CQ_EINVAL for an
 * envelope outside 0..4, non-finite kappa or param, or t_off < t_on. */
cq_status cq_rt_set_field(cq_rt rt, int envelope, double kappa, double param, double t_on, double t_off);
/* Advance nsteps steps; per step (HOST arrays, each may be NULL): the
 * electronic energy Re Tr[P(h + F)] (costs one extra, uncounted build),
 * the electronic dipole -2 Re Tr[D_z P] (Eq. td_expectation), and the
 * number of Fock builds the step used.  Synchronizes the stream. */
cq_status cq_rt_step(cq_rt rt, int nsteps, double* energy, double* dipole, int* builds);
/* Current orthonormal density (DEVICE complex [nbf][nbf]). */
cq_status cq_rt_density(cq_rt rt, double* P, hipStream_t stream);
/* out4 (HOST): steps, builds, accepted learned proposals, fallbacks. */
cq_status cq_rt_stats(cq_rt rt, long long* out4);
/* Learned proposal: record (features, converged midpoint) samples at
 * samples_per_step fixed random elements of every midpoint step while
 * enabled.  Proposal baseline B = (P_k + U_prev P_k U_prev^dagger)/2 with
 * the previous step's propagator; features per element: B - P_k,
 * P_k - P_{k-1}, P_{k-1} - P_{k-2}, B - P_k - (P_k - P_{k-1})/2 (re, im);
 * target: converged midpoint - B; all scaled by their RMS over the samples;
 * train the pointwise MLP (8 -> 32 tanh -> 2, FP32) with Adam on
 * the GPU for `epochs` passes (one mini-batch per recorded step, learning
 * rate lr; feature / target scales from the recorded samples); set / get
 * the 354 FP32 weights [W1 32x8, b1 32, W2 2x32, b2 2] (HOST). */
cq_status cq_rt_record(cq_rt rt, int enable, int samples_per_step, unsigned seed);
cq_status cq_rt_recorded(cq_rt rt, int* nsteps);
cq_status cq_rt_train(cq_rt rt, int epochs, float lr, float* loss);
cq_status cq_rt_mlp_weights(cq_rt rt, const float* set354, float* get354);
cq_status cq_rt_mlp_scales(cq_rt rt, float* feature_scale8, double* out_scale);

/* Test exports: U = exp(-i dt H) for a Hermitian DEVICE complex H [n][n];
 * MLP loss 1/(2N) sum |y - t|^2 and its gradient for DEVICE weights w354,
 * samples X [ns][8], targets Y [ns][2]; one Adam step (beta 0.9/0.999,
 * eps 1e-8) on DEVICE w, g, m, v (354 each). */
cq_status cq_expm(int n, const double* H, double dt, double* U, hipStream_t stream);
/* C = A op(B) for DEVICE row-major complex n x n matrices (interleaved re,
 * im), op(B) = B (conjB = 0) or B^H (conjB = 1): the complex GEMM of every
 * real-time product, on the FP64 matrix cores.  C must not alias A or B
 * (CQ_EINVAL).  Asynchronous on `stream`. */
cq_status cq_zgemm(int n, const double* A, const double* B, int conjB, double* C, hipStream_t stream);
cq_status cq_mlp_eval(const float* w354, const float* X, const float* Y, int ns, float* grad, float* loss,
                      hipStream_t stream);
cq_status cq_mlp_adam(float* w, const float* g, float* m, float* v, float lr, int step, hipStream_t stream);

/* ---- test-only exports ------------------------------------------------ */

/* Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt for m = 0..mmax
 * (mmax <= 16) at n points.  T: device [n]; F: device [n][mmax+1] (FP64).
 * fp32 = 0: the FP64 evaluation of the FP64 kernels; fp32 = 1: the one of
 * the precision-routed FP32 kernels (T rounded to FP32; FP32 Chebyshev table
 * and recursion for mmax < 6 and T < 36, FP64 rounded to FP32 otherwise),
 * widened to FP64.  Asynchronous on `stream`. */
cq_status cq_boys(int mmax, int n, const double* T, double* F, int fp32, hipStream_t stream);

/* One contracted, normalized shell-quartet block (ab|cd), layout
 * [na][nb][nc][nd], written to HOST memory `out` (synchronizes `stream`). */
cq_status cq_eri_quartet(cq_basis b, int a, int bsh, int c, int d, double* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* CQ_H */
