/*
 * jk.h -- C ABI of the MI355X (gfx950) Coulomb/exchange matrix library.
 *
 * The library builds, for one or more symmetric density matrices D^s,
 *
 *     J^s_ij = sum_kl (ij|kl) D^s_kl          K^s_ik = sum_jl (ij|kl) D^s_jl
 *
 * (paper Section 2, eq. jk), where (ij|kl) are electron repulsion integrals
 * over contracted Cartesian Gaussian shells (Section 2, eq. rys0), evaluated
 * by Rys quadrature (Section 2, eqs. rys1 and rys2) on the GPU, over the
 * shell quartets that pass the Schwarz test Q_IJ * Q_KL >= cutoff with
 * Q_IJ = sqrt(max_{a in I, b in J} |(ab|ab)|) (Section 2, eq. schwartz).
 * Only unique quartets are evaluated (the eight-fold permutational symmetry
 * of Section 2).
 *
 * Conventions shared by every entry point:
 *   - Basis: see jk_basis.  coefs multiply raw primitives
 *     x^ax y^ay z^az exp(-alpha r^2) centred on the shell's atom.
 *   - Cartesian components in reversed lexicographic order (xx, xy, xz, yy,
 *     yz, zz for d; Section 2's index function).  Spherical shells are real
 *     solid harmonics m = -l..l (l = 1 stays x, y, z), normalised like the
 *     Cartesian x^l component.
 *   - Matrices are FP64, row-major [nset][nao][nao], nao counting spherical
 *     functions when the basis is spherical.
 *   - Device pointers are HIP device memory on the current device.  Streams
 *     are hipStream_t passed as void* (NULL = the null stream).
 *   - Every function returns 0 (JK_OK) or a negative JK_E* code and never
 *     aborts; jk_last_error() gives a thread-local message.  Errors raised
 *     by work already enqueued on a stream surface from a later call that
 *     synchronises (jk_build, jk_plan_create, jk_eri_block) as JK_EDEVICE.
 */
#ifndef JK_H
#define JK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    JK_OK = 0,
    JK_EINVAL = -1,        /* bad argument: sizes, ranges, non-finite values */
    JK_EUNSUPPORTED = -2,  /* valid but not built: a shell with l above the
                              built maximum (JK_LMAX_BUILT), too many quartets */
    JK_ENOMEM = -3,        /* device or host allocation failed */
    JK_EDEVICE = -4        /* a HIP call failed */
};

/* Arithmetic of the integral evaluation (Table 1's DataType). */
enum {
    JK_FP64 = 0,   /* every quartet in FP64 */
    JK_MIXED = 1,  /* every quartet whose bound Q_IJ Q_KL max|D_block| (FP64, the
                      largest |D| over the six blocks the quartet touches and over
                      the densities) is below mix_threshold runs in FP32, the rest
                      in FP64, in every angular class; accumulation always FP64 */
    JK_FP32 = 2    /* every quartet in FP32, FP64 accumulation */
};

/* jk_execute flags (Table 1's do_j / do_k). */
enum {
    JK_DO_J = 1,
    JK_DO_K = 2,
    JK_ACCUMULATE = 4,     /* add into J/K instead of overwriting them */
    JK_CHECK_SYMMETRY = 8, /* check on the device that every D is finite and
                              symmetric (max|D - D^T| <= 1e-12 max|D|) before the
                              build; JK_EINVAL otherwise.  Synchronises the stream */
    JK_DETERMINISTIC = 16  /* bitwise the same J and K on every run, every stream
                              count and every launch order: each addition into
                              J', K' and the pair-ordered J' is split exactly into
                              three 64-bit integer limbs (2^-16, 2^-56 and a
                              rounded 2^-96 part) added with integer atomics, and
                              the limbs are summed in a fixed order at the end.
                              Every class runs as tiles (no row mode).  Needs
                              |addend| < 2^24 and at most 2^23 additions per
                              element; takes 9 x max(nset nao_cart^2, nset x the
                              pair-block elements) more doubles of plan scratch
                              and is slower than the default.  jk_execute only
                              (jk_execute_noalloc returns JK_EINVAL) */
};

#define JK_LMAX 4       /* highest angular momentum the basis format admits (g) */
#define JK_LMAX_BUILT 4 /* highest one with built kernels (g) */
#define JK_MAXPRIM 16   /* most primitives per shell */

/* Basis description, host memory, owned by the caller, read only during the
 * call that takes it. */
typedef struct {
    int32_t nshell;
    int32_t natom;
    int32_t spherical;      /* 0 Cartesian, 1 real solid harmonics */
    const int32_t *l;       /* [nshell] 0..JK_LMAX (l > JK_LMAX: JK_EINVAL) */
    const int32_t *nprim;   /* [nshell] 1..JK_MAXPRIM */
    const int32_t *atom;    /* [nshell] 0..natom-1 */
    const double *exps;     /* [sum nprim] > 0, grouped by shell in shell order */
    const double *coefs;    /* [sum nprim] finite, primitive normalisation folded in */
    const double *coords;   /* [natom][3] bohr */
} jk_basis;

typedef struct jk_plan jk_plan;
typedef struct jk_batch jk_batch;

/* Statistics of a plan (host copy). */
typedef struct {
    int64_t nquartets;          /* significant unique shell quartets */
    int64_t nprim_quartets;     /* primitive quartets inside them */
    int64_t nquartets_fp32;     /* quartets the last build ran in FP32 (JK_MIXED: those
                                   below the threshold; JK_FP32: all evaluated) */
    int32_t nclasses;           /* (bra pair type, ket pair type) launches */
    int32_t npairs;             /* shell pairs kept after screening */
    double setup_ms;            /* jk_plan_create wall time */
    double model_flops;         /* algorithmic FLOPs of one build with nset = 1 */
    int64_t nquartets_evaluated; /* quartets the last build evaluated (nquartets less
                                    those dropped by density screening) */
} jk_stats;

/*
 * Build a plan for one geometry (Section 3: the molecule is the dynamic
 * input; angular momenta and contraction patterns select the kernels).
 * Validates the basis, copies it to the device, builds the primitive shell-
 * pair data, the Schwarz table (on the GPU) and the screened, sorted task
 * lists.  cutoff: Schwarz threshold (>= 0).  Synchronous; uses the null
 * stream.  On error *out is NULL.
 */
int jk_plan_create(const jk_basis *basis, double cutoff, jk_plan **out);
void jk_plan_destroy(jk_plan *plan);

/* nao: size of D/J/K rows (spherical count when spherical); nao_cart: the
 * Cartesian count the kernels work in. */
int jk_plan_info(const jk_plan *plan, int32_t *nao, int32_t *nao_cart);
int jk_plan_stats(const jk_plan *plan, jk_stats *stats);

/* Copy the Schwarz table Q_IJ [nshell][nshell] to host memory. */
int jk_plan_schwarz(const jk_plan *plan, double *Q_host);

/*
 * One J/K build.  D, J, K: device FP64 [nset][nao][nao]; D must be
 * symmetric (the kernels read both triangles and assume D_kl = D_lk).
 * J and K are overwritten unless JK_ACCUMULATE; either may be NULL when the
 * matching JK_DO_* flag is clear.  precision: JK_FP64 / JK_MIXED / JK_FP32;
 * mix_threshold: bound below which JK_MIXED uses FP32 (ignored otherwise).
 * omega selects the operator (the range-separation parameter of Table 2,
 * rys_type of Table 1): 0 the Coulomb operator 1/r, > 0 the long-range
 * erf(omega r)/r, < 0 the short-range erfc(|omega| r)/r; the screening uses
 * the Coulomb Schwarz factors in every case (they bound both parts); non-
 * finite omega -> JK_EINVAL.  Asynchronous on
 * stream (unless JK_CHECK_SYMMETRY); D/J/K must stay valid until the stream
 * reaches this point.  nset >= 1.  Scratch (Cartesian J', K', density, the
 * block maxima) is allocated by the plan at the first call that needs it
 * and reused; calls on one plan must be ordered.  The class kernels run on
 * stream and on up to three more streams of the plan (JK_STREAMS=n in the
 * environment at plan creation sets the total, 1 to 8, default 4), forked
 * from stream by an event and joined back into it before J and K are
 * written, so the build stays ordered on stream (also under graph capture).
 */
int jk_execute(jk_plan *plan, const double *D, int32_t nset, int32_t flags, int32_t precision,
               double mix_threshold, double omega, double *J, double *K, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * build as jk_execute, with the same arguments and results, but its scratch
 * (Cartesian J', K' and density, the pair-ordered J' buffer, the block
 * maxima, the counters) taken from one fixed device array of
 * JK_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from load until
 * the process ends.  Calls no allocating routine.  A build that needs more
 * scratch than the array holds (8 bytes x (nset nao_cart^2 (2 + spherical)
 * + nset x the pair-block elements + nshell^2) + 64 x classes, each part
 * rounded to 256 bytes) returns JK_EINVAL before anything runs.  Every
 * call on one GPU shares that GPU's array and leaves its contents there:
 * calls that overlap on one GPU race (order them on one stream), and
 * jk_plan_stats after such a call reads the counters the last call on that
 * GPU wrote.  Each call clears what it accumulates into.  Per-kernel
 * profiling (jk_plan_profile) does not apply to it, and JK_DETERMINISTIC
 * (whose limbs the array does not hold) returns JK_EINVAL.
 */
#define JK_NOALLOC_SCRATCH_BYTES (128u << 20)
int jk_execute_noalloc(jk_plan *plan, const double *D, int32_t nset, int32_t flags, int32_t precision,
                       double mix_threshold, double omega, double *J, double *K, void *stream);

/*
 * Density screening for direct SCF (Section 2: the screening of the J and K
 * changes by the density change, at shell-pair level).  With threshold > 0,
 * later jk_execute calls on this plan drop every quartet with
 *   Q_IJ Q_KL max(Dm_IJ, Dm_KL, Dm_IK, Dm_IL, Dm_JK, Dm_JL) < threshold,
 * Dm_XY the largest |D| over the densities and the Cartesian components of
 * block (X, Y) (double precision), so each dropped contribution to any J or
 * K element is below the threshold.  Passing the density change Delta D with
 * JK_ACCUMULATE builds the incremental J += Delta J, K += Delta K.
 * threshold = 0 turns it off (the default).  JK_EINVAL for a NULL plan or a
 * negative / non-finite threshold.
 */
int jk_plan_set_density_screening(jk_plan *plan, double threshold);

/* One-shot: plan_create + execute (J and K) + synchronise + destroy. */
int jk_build(const jk_basis *basis, const double *D, int32_t nset, double cutoff, int32_t precision,
             double *J, double *K, void *stream);

/*
 * Batched builds over many plans (molecules), the same two-index
 * contraction (Section 2, eq. jk) per molecule.  Per angular class and
 * kernel family one launch covers the tiles of every molecule (heaviest
 * molecule first); transforms, clearing and finalisation are batched
 * kernels over all molecules; the whole build is recorded into a hipGraph
 * at the first jk_batch_execute and replayed on later calls.
 *   plans[nmol]: plans created on the current device; they must outlive the
 *                batch (the batch reads their device arrays).
 *   nset:        densities per molecule; precision / mix_threshold as in
 *                jk_execute (J and K are always built and overwritten).
 *   D[m], J[m], K[m]: device FP64 [nset][nao_m][nao_m] of molecule m; D[m]
 *                symmetric.  Pointers may change between calls (a small
 *                host-to-device update on the stream precedes the replay).
 * Scratch (Cartesian D, J', K', block maxima, counters) is owned by the
 * batch and shared by its calls: calls on one batch must be ordered (same
 * stream, or the caller synchronises); concurrent calls race.  Errors:
 * JK_EINVAL for NULL or mismatched arguments (checked before anything
 * changes), JK_ENOMEM, JK_EDEVICE.
 * jk_batch_stats: quartets the last execute evaluated over all molecules,
 * and how many of them in FP32 (mixed precision); synchronises the device.
 */
int jk_batch_create(jk_plan *const *plans, int32_t nmol, int32_t nset, int32_t precision,
                    double mix_threshold, jk_batch **out);
int jk_batch_execute(jk_batch *batch, const double *const *D, double *const *J, double *const *K,
                     void *stream);
int jk_batch_stats(const jk_batch *batch, int64_t *nquartets, int64_t *nquartets_fp32);
void jk_batch_destroy(jk_batch *batch);

/*
 * Test hook: contracted Cartesian block (IJ|KL) of shells I, J, K, L
 * (indices into the basis), computed by the same GPU kernels as the build,
 * copied to host_out [nI][nJ][nK][nL] (Cartesian counts).  Synchronous.
 */
int jk_eri_block(jk_plan *plan, int32_t I, int32_t J, int32_t K, int32_t L, int32_t precision,
                 double *host_out);

/*
 * Test hook: n-point Rys roots (t^2) and weights as the kernels evaluate
 * them, for count values of T (host arrays); roots/weights [count][n].
 * precision JK_FP64 or JK_FP32.  Synchronous.
 */
int jk_rys_eval(int32_t n, const double *T_host, int32_t count, int32_t precision, double *roots_host,
                double *weights_host);

/* Test hook: Boys F_0..F_m at count values of T as the kernels evaluate
 * them (table + downward recursion), out [count][m+1].  m <= 1.  Synchronous. */
int jk_boys_eval(int32_t m, const double *T_host, int32_t count, int32_t precision, double *out_host);

/*
 * Per-kernel timing (measurement support).  While enabled, jk_execute
 * launches every class kernel on its stream, one after another, records a
 * HIP event on that stream before and after every class-kernel launch, waits for the last one before returning, and adds each launch's
 * duration to the running total of its (class, precision, kind) entry.
 * jk_plan_profile(plan, 1) resets the totals; jk_plan_timings copies up to
 * cap entries (those that ran) and stores the number available in *count.
 */
typedef struct {
    int32_t li, lj, lk, ll;     /* angular momenta of the class */
    int32_t npb, npk;           /* primitive pairs per bra / ket pair */
    int32_t precision;          /* JK_FP64 or JK_FP32 */
    int32_t launches;           /* launches summed into ms (one per build) */
    int32_t family;             /* kernel family (1, 2 or 3) */
    int32_t kind;               /* 0 tiles, 1 row mode (long bras, 256-lane workgroups), 3 row mode
                                   (short bras, 64-lane workgroups); 2 is not used */
    int64_t nquartets;          /* quartets evaluated, summed over the launches (after the mixed
                                   split and density screening) */
    double model_flops;         /* their algorithmic FLOPs (nset = 1), summed likewise */
    double ms;                  /* summed kernel time */
} jk_class_timing;

int jk_plan_profile(jk_plan *plan, int32_t enable);
int jk_plan_timings(const jk_plan *plan, jk_class_timing *out, int32_t cap, int32_t *count);

/*
 * Kernel tuning table (the per-device heuristics database of Section 3).
 * Every canonical angular class (li >= lj, lk >= ll, (lk,ll) <= (li,lj))
 * has up to three kernel families: 1 = one lane per quartet with the
 * integral block in registers; 2 = a lane group per quartet with the 2-D
 * integrals of all roots in LDS; 3 = a lane per Cartesian component of the
 * bra's first shell, its elements in registers and only the vertical
 * recurrence tables in LDS (row mode only: bras with short ket prefixes run
 * as tiles of family 2, or 1 where 2 is not built).  jk_tune_set picks the
 * family for one class and precision (JK_FP64 or JK_FP32; family 0
 * restores the built-in default); plans read the table when they are
 * created.  jk_tune_set_row controls row mode for one class and precision
 * (0 default = 1; 1 bras with long ket prefixes; 2 off; 3 every bra, the
 * short ones in 64-lane workgroups): in row mode a workgroup walks (a chunk
 * of) one bra's ket prefix and keeps the bra's K rows in LDS, so most J/K
 * updates stay out of global atomics; batched builds run every bra of a
 * class as 64-lane row tasks unless its setting is 2.  At load time the
 * library reads tune_gfx950.txt next to itself (or the file named by
 * JK_TUNE_DB): one "li lj lk ll precision family [row]" line per entry,
 * "shape ..." lines (jk_tune_set_shape), '#' comments.
 * jk_tune_get reports the family a new plan would use and a bit mask of
 * the built families (1: family 1, 2: family 2, 4: family 3).
 */
int jk_tune_set(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t precision, int32_t family);
int jk_tune_set_row(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t precision, int32_t row);
int jk_tune_get(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t precision, int32_t *family,
                int32_t *available);
/* Task shape of one class (the fragmentation of Section 3.2), read by plans
 * created afterwards: bras with at least min_kets kets run in row mode
 * (default 192) and one row task covers at most chunk kets of a bra (default:
 * 2048 for family 1, 256 wave steps for families 2 and 3); 0 restores a
 * default.  Table lines "shape li lj lk ll min_kets chunk". */
int jk_tune_set_shape(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t min_kets, int32_t chunk);
/* Mixed-precision split of one class, read by plans created afterwards
 * (Section 4.3 leaves the split open; JK_MIXED applies it per quartet):
 * 1 (the default) splits the class's quartets by their bound against the
 * threshold; 0 runs the whole class in double precision in JK_MIXED builds,
 * for classes whose single-precision kernels are no faster on the device
 * (the split would only add a second pass; double precision is never less
 * accurate).  Table lines "split li lj lk ll s".  JK_EINVAL for a class
 * that is not canonical or built, or s not 0 or 1. */
int jk_tune_set_split(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t split);
int jk_tune_load(const char *path);

const char *jk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* JK_H */
