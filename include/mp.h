/*
 * mp.h -- C ABI of the MI355X (gfx950) Matching Pursuit decoder, libmp.so.
 *
 * The decoder recovers a sparse x from y = Psi x, given y and the N x M
 * dictionary Psi with unit-norm columns (Section 2, eqs. 2-4), by the Matching
 * Pursuit iteration of Section 3 (eqs. 8-12):
 *
 *     t = 0, x~ = 0, r = y
 *     while ||r||_2 > eps ||y||_2 and t < T:
 *         i    = argmax_m |<r, psi_m>|   (smallest index on ties, as the
 *                                          i?amax kernel of eq. 16)
 *         x~_i += <r, psi_i>
 *         r    -= <r, psi_i> psi_i
 *         t    += 1
 *
 * Conventions shared by every entry point
 *  - Indices are 0-based.
 *  - Matrices are column-major: element (row n, column m) of a matrix with
 *    leading dimension ld is at offset n + m * ld.  A dictionary column psi_m
 *    is therefore contiguous.
 *  - Pointers documented as "device" must point to memory of the current HIP
 *    device; "host" pointers to ordinary host memory.  The library never
 *    frees caller memory and never keeps a caller pointer past the call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *    is ordered on that stream; an mp_solve* call returns only after its
 *    decode has finished (the host reads the device's stop flag to know when
 *    to stop issuing iterations), except a decode with MP_SOLVE_ASYNC, which
 *    is only enqueued (its result comes from mp_solve_result).
 *  - Errors are reported by return code only; nothing aborts the process.
 *    mp_last_error(ctx) returns a human-readable detail for the last failed
 *    call on a context.
 *  - A context is not thread-safe: one call at a time per context.
 *
 * Stopping rule (the pseudo-code's test, on squared norms in FP64): the loop
 * continues while ||r||^2 > eps^2 ||y||^2 and t < max_iters; it is tested
 * before every step, so `iters` counts the updates done.  y = 0 takes no step
 * (MP_STOP_ZERO_INPUT); a largest |<r, psi_m>| of exactly 0 ends the run
 * without an update (MP_STOP_STALLED).
 */
#ifndef MP_H_
#define MP_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mp_status {
    MP_OK = 0,
    MP_EINVAL = 1,        /* an argument is out of range or NULL where not allowed */
    MP_ENOTNORM = 2,      /* a dictionary column's L2 norm is not 1 within 1e-4 */
    MP_ENONFINITE = 3,    /* NaN or Inf in the dictionary or in y */
    MP_ENOMEM = 4,        /* a device or pinned-host allocation failed */
    MP_EDEVICE = 5,       /* no usable HIP device, or a HIP runtime call failed */
    MP_EUNSUPPORTED = 6   /* the request is valid but this build/device cannot do it */
} mp_status;

/* Storage of the dictionary copy the correlation pass streams. */
typedef enum mp_dtype {
    MP_F32 = 0,           /* FP32, as given */
    MP_BF16 = 1,          /* BF16, round to nearest even from FP32 */
    MP_FP8_E4M3 = 2,      /* OCP FP8 E4M3 (e4m3fn) with one FP32 scale per column:
                             s_m = fp32(max_n |psi_nm| / 448) (1 for a zero column),
                             code = RNE-saturate(fp32(psi_nm / s_m)) */
    MP_F64 = 3,           /* FP64 dictionary and FP64 decode (mp_create_f64 /
                             mp_solve_f64 only) */
    MP_SIGN1 = 4          /* one sign bit per entry, psi_nm = (1 - 2 b_nm) / sqrt(N):
                             the Bernoulli dictionary of eq. 13 (mp_create_signs) */
} mp_dtype;

/* Why a decode stopped (mp_result.stop_reason). */
enum {
    MP_STOP_CONVERGED = 0,   /* ||r||^2 <= eps^2 ||y||^2 */
    MP_STOP_MAX_ITERS = 1,   /* t reached max_iters */
    MP_STOP_STALLED = 2,     /* max_m |<r, psi_m>| == 0 with r != 0 */
    MP_STOP_ZERO_INPUT = 3   /* y == 0 */
};

/* mp_create flags */
#define MP_SKIP_NORM_CHECK 0x1u   /* do not verify ||psi_m|| = 1 (finiteness is still checked) */

typedef struct mp_ctx mp_ctx;

typedef struct mp_opts {
    double eps;           /* relative tolerance, >= 0 and finite */
    int64_t max_iters;    /* iteration cap T, >= 0 */
    int32_t rescore_k;    /* reduced-precision storage: how many best candidates of
                             each pass are re-scored against the FP32 columns (1..8;
                             0 means 8).  Ignored for MP_F32 storage. */
    uint32_t flags;       /* 0, or MP_SOLVE_STEP_LAUNCHES (mp_solve, mp_solve_f64 and
                             mp_solve_omp) and MP_SOLVE_ASYNC (mp_solve and
                             mp_solve_noalloc); 0 for the others */
} mp_opts;

/* mp_opts.flags: decode with one kernel launch per step even where the whole
   decode fits one persistent launch (the one-bit form MP_SIGN1, and MP_F32
   contexts whose dictionary fits the LDS of at most 32 workgroups); the same
   results bit for bit; no effect on the other forms. */
#define MP_SOLVE_STEP_LAUNCHES 0x1u

/* mp_opts.flags: a stream-ordered decode (mp_solve and mp_solve_noalloc on
   MP_F32, MP_BF16 and MP_FP8_E4M3 contexts).  The call enqueues the whole
   decode on its stream and returns without waiting for the device: x~, r and
   the trace are final once the stream reaches the point of the call, and the
   result (iterations, norms, stop reason, and the errors only the device can
   find: non-finite y, a wait that gave up) is collected with mp_solve_result.
   res must be NULL.  Since the host cannot see when the decode stops, it
   enqueues every launch the cap allows (max_iters + 1; the one launch of a
   decode held in LDS); a launch past the stop returns at once, costing its
   dispatch only (about 4 us at N=8192, M=32768), so a cap far above the steps
   needed costs that per spare step.  Decodes on different contexts overlap
   on different streams; a context holds one stream-ordered decode at a time
   (every decode call on it returns MP_EINVAL until mp_solve_result).
   mp_solve_noalloc decodes all use the library's one static scratch per
   GPU, so stream-ordered ones must not overlap either: issue them on one
   stream. */
#define MP_SOLVE_ASYNC 0x2u

typedef struct mp_result {
    int64_t iters;        /* updates performed */
    double yy;            /* ||y||^2, FP64 */
    double rr;            /* ||r||^2 at exit, FP64 (from the FP32 residual) */
    int32_t stop_reason;  /* MP_STOP_* */
    int32_t persistent;   /* 1: the decode ran as one persistent launch (one-bit form) */
} mp_result;

/* Optional per-step record, all arrays device memory of `cap` entries.
   Step t (0-based) writes idx[t], coef[t] (the FP32 coefficient added to
   x~), rr[t] (||r||^2 after the step, FP64) while t < cap; any array may be
   NULL.  r, if not NULL, receives the whole residual after each step
   (eq. 11's r_{t+1}): rows 0..N-1 of step t at r + t * ldr, ldr >= N, so
   r must hold cap * ldr floats (the batched and ragged decodes: signal or
   instance b's step t at r + (b * cap + t) * ldr, ldr >= every N).  Rows
   N..ldr-1 are left unwritten.  The one-bit form stores its FP64 residual
   rounded to FP32.  Writing it costs N floats of traffic per step; it is
   meant for checking a decode step by step, not for timing one. */
typedef struct mp_trace {
    int32_t* idx;
    float* coef;
    double* rr;
    int64_t cap;
    float* r;
    int64_t ldr;
} mp_trace;

/* The same record for an FP64 decode: coef[t] is the FP64 coefficient and
   r (cap * ldr doubles, or NULL) the FP64 residual after each step. */
typedef struct mp_trace_f64 {
    int32_t* idx;
    double* coef;
    double* rr;
    int64_t cap;
    double* r;
    int64_t ldr;
} mp_trace_f64;

/*
 * mp_create -- take the dictionary Psi (Section 2, eqs. 3-4) and prepare it
 * for decoding.  The one-time host-to-device dictionary set-up that every
 * later decode reuses (the paper uploads the dictionary once for all signals).
 *
 *   out      host: receives the new context (set to NULL on failure)
 *   psi      device: FP32 N x M column-major dictionary, leading dimension ld
 *   n, m     rows N >= 1 and columns M >= 1 (M < 2^31, N <= 16384)
 *   ld       leading dimension, ld >= n
 *   storage  which copy the correlation pass streams (mp_dtype).  MP_BF16 and
 *            MP_FP8_E4M3 keep an FP32 master as well, for re-scoring and the
 *            residual update: each pass keeps the 8 best reduced-precision
 *            candidates, re-computes up to opts.rescore_k of them in FP32 and
 *            selects the best re-computed one (smallest index on ties).
 *   flags    MP_SKIP_NORM_CHECK or 0
 *   stream   hipStream_t as void*
 *
 * The context copies psi (re-laid out with a padded leading dimension), so
 * the caller may free psi when mp_create returns.
 * Errors: MP_EINVAL (NULL, n < 1, m < 1, ld < n, size limits, unknown storage
 * or flags), MP_ENONFINITE, MP_ENOTNORM, MP_ENOMEM, MP_EDEVICE,
 * MP_EUNSUPPORTED (the device is not gfx950, or it has more than 256 compute
 * units).
 */
mp_status mp_create(mp_ctx** out, const float* psi, int64_t n, int64_t m, int64_t ld,
                    mp_dtype storage, uint32_t flags, void* stream);

/*
 * mp_solve -- decode one signal: the Section 3 loop, run entirely on the
 * device (correlation, argmax, coefficient and residual update, FP64 stop
 * test), with no host round trip per iteration.
 *
 *   ctx      from mp_create
 *   y        device: N floats, not modified
 *   x        device: M floats, overwritten with x~ (FP32)
 *   r        device: N floats or NULL; receives the final residual (FP32)
 *   opts     host: tolerance, cap, re-score count, flags (0 or
 *            MP_SOLVE_STEP_LAUNCHES)
 *   res      host or NULL: iteration count, norms, stop reason, and whether
 *            the decode ran as one persistent launch
 *   trace    host struct of device arrays, or NULL (see mp_trace)
 *   stream   hipStream_t as void*
 *
 * An MP_F32 context whose dictionary, split into shares of whole columns,
 * fits the LDS of at most 32 workgroups beside r (at most 150 KB each, e.g.
 * N = 256 with M up to 4608) decodes in one persistent launch, each
 * workgroup keeping its share in LDS and exchanging its best key with the
 * others through device memory each step (bit-identical to one launch per
 * step, which MP_SOLVE_STEP_LAUNCHES selects).  That launch needs every
 * workgroup resident at once: run it on a device no other kernel holds; a
 * wait between its workgroups that exceeds the poll limit (2^22, or the
 * non-negative integer in the environment variable MP_SMALL_SPIN_LIMIT, read
 * at each decode; 0 gives up at the first wait) ends the decode with
 * MP_EDEVICE.
 *
 * y, x and r must not overlap.  Errors: MP_EINVAL (NULL ctx/y/x/opts, eps < 0
 * or not finite, max_iters < 0, unknown flags, rescore_k outside 0..8),
 * MP_ENONFINITE (y holds NaN/Inf; x and r are then unspecified), MP_EDEVICE.
 */
mp_status mp_solve(mp_ctx* ctx, const float* y, float* x, float* r, const mp_opts* opts,
                   mp_result* res, const mp_trace* trace, void* stream);

/*
 * mp_solve_result -- wait for the stream-ordered decode (MP_SOLVE_ASYNC) last
 * issued on ctx and return its result: the same result and errors mp_solve
 * gives for that decode.  The context can then decode again.
 *
 *   res      host or NULL: as for mp_solve
 * Errors: MP_EINVAL (NULL ctx, or no stream-ordered decode pending), and the
 * decode's own: MP_ENONFINITE, MP_EDEVICE.
 */
mp_status mp_solve_result(mp_ctx* ctx, mp_result* res);

/*
 * mp_solve_noalloc -- mp_solve for callers that cannot allocate memory while
 * they decode: code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, results and errors as mp_solve for
 * an MP_F32, MP_BF16 or MP_FP8_E4M3 context from mp_create (the same kernels,
 * bit-identical results), but the decode's device work buffers (state,
 * residual double buffer, per-workgroup keys, column-share state) live in
 * a static array of 256 KiB that the library holds on each GPU it runs on
 * until the process ends (the decode always takes one launch per step), and
 * the call allocates nothing (no hipMalloc,
 * hipFree or allocating library call; the pinned state slots and events it
 * uses were made by mp_create).
 *
 * Limits: N <= 16384 (the residual double buffer), at most 256 correlation
 * workgroups (MP_EINVAL otherwise; mp_create's own limits already imply
 * both on an MI355X).  Every call on one GPU shares that GPU's array and
 * leaves its contents behind: calls that overlap on one GPU (other streams,
 * other threads, other contexts) race and must not be issued.  Nothing in
 * the array needs to start at zero: each decode writes its state and
 * buffers before reading them, and the column shares left by an earlier
 * call only guide the work split, never the results.
 * Errors: as mp_solve, plus MP_EINVAL for a ragged, MP_F64 or MP_SIGN1
 * context.
 */
mp_status mp_solve_noalloc(mp_ctx* ctx, const float* y, float* x, float* r, const mp_opts* opts,
                           mp_result* res, const mp_trace* trace, void* stream);

/*
 * mp_solve_batched -- decode B signals that share the context's dictionary
 * (the paper encodes and decodes every signal with one dictionary,
 * Section 4).  Each signal runs its own Section 3 loop; the correlations of
 * all still-active signals are computed together as one BF16 matrix product
 * Psi^T R on the matrix cores (FP32 accumulate), the 8 best candidates of
 * each signal are re-scored against the FP32 columns, and signals drop out
 * of later products as soon as they stop.  A context created with MP_F32 or
 * MP_FP8_E4M3 storage gets a BF16 copy of its dictionary on first use.
 *
 *   Y         device: N x B, column b = y of signal b, leading dimension ldy >= N
 *   X         device: M x B, overwritten with the x~ columns, ldx >= M
 *   R         device: N x B or NULL, receives the final residuals, ldr >= N
 *   opts      host: eps and rescore_k apply to every signal; max_iters is the
 *             cap unless max_iters_b is given
 *   max_iters_b  host: B per-signal caps, or NULL
 *   res       host: B results, or NULL
 *   trace     host struct of device arrays of B * cap entries, or NULL; signal
 *             b's step t goes to index b * cap + t
 *
 * Errors: MP_EINVAL (NULL ctx/Y/X/opts, B < 0 or >= 2^30, a leading
 * dimension too small, eps/max_iters/rescore_k/flags as for mp_solve, a
 * negative max_iters_b entry), MP_ENONFINITE (a column of Y holds NaN/Inf;
 * the other signals are still decoded), MP_ENOMEM, MP_EDEVICE.  B = 0 is a
 * no-op.
 */
mp_status mp_solve_batched(mp_ctx* ctx, const float* Y, int64_t ldy, int64_t B, float* X,
                           int64_t ldx, float* R, int64_t ldr, const mp_opts* opts,
                           const int64_t* max_iters_b, mp_result* res, const mp_trace* trace,
                           void* stream);

/* Tile of the batched product by the number of signals still active (chosen
   by the autotuner; results do not depend on it beyond which 8 candidates of
   each signal reach the FP32 re-score, and the selection is the re-scored
   one): 128 atoms x 64 signals per workgroup while more than atoms128_above
   signals are active, 64 atoms while more than atoms64_above, 32 while more
   than atoms32_above, else 16 (more workgroups for a small product; the 32-
   and 16-atom tiles give the same products).  The 128- and 64-atom forms that
   stage the residuals in LDS need the padded column length to be a multiple
   of 256 (otherwise 64 atoms without staging), and a 128- or 64-atom tile
   gives way to the next smaller one where its grid, ceil(M / atoms) x
   ceil(active / 64) workgroups, would not cover every compute unit.
   Default {2^31 - 1, 96, 0}: no 128-atom and no 16-atom tile. */
typedef struct mp_batched_config {
    int32_t atoms128_above;
    int32_t atoms64_above;
    int32_t atoms32_above;
} mp_batched_config;

/* mp_batched_set_config / mp_batched_get_config -- the product tile rule of
   mp_solve_batched on this context (the Section 4 setting of one dictionary
   for every signal).  Errors: MP_EINVAL (NULL, a ragged, MP_F64 or MP_SIGN1
   context, a negative count). */
mp_status mp_batched_set_config(mp_ctx* ctx, const mp_batched_config* cfg);
mp_status mp_batched_get_config(const mp_ctx* ctx, mp_batched_config* cfg);

/*
 * mp_create_f64 -- mp_create for an FP64 dictionary: the double-precision
 * configuration of the decoder (the paper times single- and double-precision
 * builds of the same loop, Section 4).  The correlation pass streams the FP64
 * copy (8 bytes per element) and every inner product, coefficient, residual
 * and norm is FP64.  The context has storage MP_F64 and is decoded only with
 * mp_solve_f64 (mp_solve and mp_solve_batched return MP_EINVAL for it).
 *
 *   out      host: receives the new context (set to NULL on failure)
 *   psi      device: FP64 N x M column-major dictionary, leading dimension ld
 *   n, m     1 <= N <= 16384, 1 <= M < 2^31
 *   ld       leading dimension, ld >= n
 *   flags    MP_SKIP_NORM_CHECK or 0
 *   stream   hipStream_t as void*
 *
 * The context copies psi (padded leading dimension); the caller may free it
 * when the call returns.  Errors: as mp_create.
 */
mp_status mp_create_f64(mp_ctx** out, const double* psi, int64_t n, int64_t m, int64_t ld,
                        uint32_t flags, void* stream);

/*
 * mp_solve_f64 -- decode one signal on an MP_F64 context: the Section 3 loop
 * in FP64 on the device, as mp_solve.
 *
 *   y        device: N doubles, not modified
 *   x        device: M doubles, overwritten with x~
 *   r        device: N doubles or NULL; receives the final residual
 *   opts     host: eps, max_iters (rescore_k is ignored), flags 0 (or
 *            MP_SOLVE_STEP_LAUNCHES, which has no effect here)
 *   res      host or NULL (rr is the FP64 norm of the FP64 residual)
 *   trace    host struct of device arrays, or NULL (see mp_trace_f64)
 *
 * y, x and r must not overlap.  Errors: MP_EINVAL (not an MP_F64 context,
 * NULL ctx/y/x/opts, bad opts), MP_ENONFINITE (y holds NaN/Inf),
 * MP_EDEVICE.
 */
mp_status mp_solve_f64(mp_ctx* ctx, const double* y, double* x, double* r, const mp_opts* opts,
                       mp_result* res, const mp_trace_f64* trace, void* stream);

/*
 * mp_create_signs -- a context for the paper's own dictionary, the Bernoulli
 * matrix of eq. 13 (entries +-1/sqrt(N), every column of unit norm), held as
 * one sign bit per entry: psi_nm = (1 - 2 b_nm) / sqrt(N).  Decoded with
 * mp_solve (FP32 y, x~ and r, as for MP_F32 storage).  The decode is the
 * Section 3 loop with the correlations carried from step to step: two
 * columns' inner product is (N - 2 popcount(b_i XOR b_m)) / N, exact, so
 * after selecting (i, c*) every c_m drops by c* <psi_i, psi_m> (eq. 9 applied
 * to eq. 11's r).  The correlations and r are kept in FP64 (c at the start is
 * Psi^T y in FP64), so the selections follow the exact iteration closely;
 * x~ accumulates fp32(c*) and r is returned rounded to FP32.  A pass reads
 * N/8 bytes per column instead of 4N.  Where the device can keep one
 * workgroup per compute unit resident with its share of the bits in LDS
 * (the share at most 150 KB, e.g. N = 8192 with M up to 32768 on 256 CUs),
 * mp_solve runs the whole decode as one persistent launch that keeps the
 * bits on chip and exchanges each step's candidates between workgroups
 * through device memory; otherwise, or with MP_SOLVE_STEP_LAUNCHES, one
 * launch per step.  Both give the same results bit for bit.  The persistent
 * launch needs every workgroup resident at once: run it on a device no other
 * kernel is holding.  A wait between its workgroups that exceeds the poll
 * limit (2^22, or the positive integer in the environment variable
 * MP_SIGN_SPIN_LIMIT, read at each decode) ends the decode with MP_EDEVICE
 * (r then holds each workgroup's rows as of its last step, x~ is partial).  The context has
 * storage MP_SIGN1; mp_solve_batched and mp_solve_omp return MP_EINVAL for
 * it.
 *
 *   out      host: receives the new context (set to NULL on failure)
 *   signs    device: packed bits, column m in words [m ldw, m ldw + ldw);
 *            bit q of word w is b_nm for row n = 32 w + q (1: -1/sqrt(N),
 *            0: +1/sqrt(N)); bits of rows n >= N are ignored
 *   n, m     1 <= N <= 16384; 1 <= M <= 131072 for N <= 8192, M <= 65536
 *            above (MP_EUNSUPPORTED beyond: a workgroup scores at most 128,
 *            or 64, columns and a launch holds at most 1024 workgroups)
 *   ldw      words per column, ldw >= ceil(N / 32)
 *   flags    0 or MP_SKIP_NORM_CHECK (no effect: the columns have unit norm
 *            by construction)
 *   stream   hipStream_t as void*
 *
 * The context keeps its own copy of the bits; the caller may free signs when
 * the call returns.  mp_get_storage returns the bits in the packed form above
 * with ldw = ceil(N / 32).  Errors: MP_EINVAL (NULL, n or m out of range, ldw
 * too small, unknown flags), MP_ENOMEM, MP_EDEVICE, MP_EUNSUPPORTED (not a
 * gfx950 device, or M above the limit for N).
 */
mp_status mp_create_signs(mp_ctx** out, const uint32_t* signs, int64_t n, int64_t m, int64_t ldw,
                          uint32_t flags, void* stream);

/*
 * mp_solve_omp -- decode one signal with Orthogonal Matching Pursuit, the
 * refinement of MP the paper names as its next target: each iteration selects
 * an atom exactly as mp_solve does (eq. 9, smallest index on ties as eq. 16),
 * then re-fits all selected atoms by least squares, so r stays orthogonal to
 * every selected atom:  x~_S = argmin ||y - Psi_S x~_S||_2,  r = y - Psi_S x~_S.
 * The fit is kept as a QR factorisation of the selected atoms grown by one
 * column per iteration (classical Gram-Schmidt run twice), FP32 with FP64
 * norms; x~_S is solved at the end in FP64.
 *
 *   ctx      from mp_create with MP_F32 storage
 *   y, x, r  as mp_solve (x~ is nonzero only on the selected atoms)
 *   opts     eps, max_iters (at most min(max_iters, N) atoms are selected),
 *            rescore_k ignored, flags 0 (or MP_SOLVE_STEP_LAUNCHES, no effect)
 *   res      host or NULL
 *   trace    host struct of device arrays, or NULL: idx[t] the atom selected
 *            at step t, coef[t] its correlation <r, psi_idx>, rr[t] ||r||^2
 *            after the re-fit
 *
 * A selection that repeats an atom, or a new atom that is a combination of
 * the selected ones to FP32 accuracy (||w||^2 <= 1e-10), ends the run with
 * MP_STOP_STALLED.  Work buffers of min(max_iters, N) x ld and
 * min(max_iters, N)^2 floats are kept by the context.  Errors: MP_EINVAL
 * (not an MP_F32 context, NULL ctx/y/x/opts, bad opts), MP_ENONFINITE,
 * MP_ENOMEM, MP_EDEVICE.
 */
mp_status mp_solve_omp(mp_ctx* ctx, const float* y, float* x, float* r, const mp_opts* opts,
                       mp_result* res, const mp_trace* trace, void* stream);

/* One problem of a ragged set: its own dictionary (device, FP32, column-major
   N x M with leading dimension ld). */
typedef struct mp_instance {
    const float* psi;
    int64_t n, m, ld;
} mp_instance;

/* Launch shape of the ragged decode (chosen by the autotuner). */
typedef struct mp_ragged_config {
    int32_t threads;        /* workgroup size: 256, 512 or 1024 */
    int32_t cols_per_wave;  /* columns one wave streams at once: 1, 2 or 4 */
    int32_t wgs_per_cu;     /* persistent workgroups per compute unit: 1..8 */
    int32_t split;          /* most parts one instance is cut into, 1..8 (0: the default,
                               3).  An instance whose estimated work (n^2 m) exceeds the
                               average per workgroup of the launch is decoded by up to
                               `split` workgroups at once, each streaming a share of its
                               columns; the parts exchange their candidates every step. */
} mp_ragged_config;

/*
 * mp_create_ragged -- take `count` independent problems of uneven size, each
 * with its own dictionary (Section 2, eqs. 3-4, per instance), for decoding
 * together with mp_solve_ragged.  Each dictionary is copied (padded leading
 * dimension), checked for finite unit-norm columns like mp_create, and with
 * MP_BF16 storage also kept as BF16 for the correlation pass (re-scored in
 * FP32 as for mp_create).
 *
 *   inst     host: count descriptors; psi pointers are device memory, may be
 *            freed after the call; 1 <= n <= 8192, ld >= n, 1 <= m < 2^31
 *   count    1 <= count < 2^30
 *   storage  MP_F32 or MP_BF16
 * Errors: MP_EINVAL (bad arguments, naming the instance), MP_ENONFINITE,
 * MP_ENOTNORM, MP_ENOMEM, MP_EDEVICE, MP_EUNSUPPORTED (MP_FP8_E4M3, or the
 * device is not gfx950).
 */
mp_status mp_create_ragged(mp_ctx** out, const mp_instance* inst, int64_t count, mp_dtype storage,
                           uint32_t flags, void* stream);

/*
 * mp_solve_ragged -- decode every instance of a ragged context (the
 * Section 3 loop per instance) in one persistent launch, replayed from a
 * captured HIP graph while the arguments stay the same.  Workgroups take
 * instances largest first; each runs one instance's whole loop, or one part
 * of it for an instance cut into parts (mp_ragged_config.split).  The parts
 * of an instance wait for each other every step: the launch needs at least
 * `split` of its workgroups resident at once (always so on an MI355X), and
 * a wait that exceeds the poll limit (2^22, or the non-negative integer in
 * the environment variable MP_RAGGED_SPIN_LIMIT, read at each call; 0 gives
 * up at the first wait) ends the call with MP_EDEVICE.
 *
 *   Y        device: the y of all instances packed in instance order
 *            (instance i starts at n_0 + ... + n_{i-1})
 *   X        device: the x~ packed the same way by m_i; overwritten
 *   R        device or NULL: final residuals, packed like Y
 *   opts     host: eps, max_iters (unless max_iters is given), rescore_k
 *   max_iters host: count per-instance caps, or NULL
 *   res      host: count results, or NULL
 *   trace    host struct of device arrays of count * cap entries, or NULL;
 *            instance i's step t goes to index i * cap + t
 * Errors: MP_EINVAL (not a ragged context, NULL Y/X/opts, bad opts or caps),
 * MP_ENONFINITE (some y holds NaN/Inf; the others are decoded), MP_EDEVICE.
 */
mp_status mp_solve_ragged(mp_ctx* ctx, const float* Y, float* X, float* R, const mp_opts* opts,
                          const int64_t* max_iters, mp_result* res, const mp_trace* trace,
                          void* stream);

/* mp_ragged_set_config / mp_ragged_get_config -- launch shape of
   mp_solve_ragged (results do not depend on it).  Errors: MP_EINVAL (not a
   ragged context, or a shape outside the listed values). */
mp_status mp_ragged_set_config(mp_ctx* ctx, const mp_ragged_config* cfg);
mp_status mp_ragged_get_config(const mp_ctx* ctx, mp_ragged_config* cfg);

/*
 * mp_destroy -- free everything the context owns.  NULL is a no-op.
 */
void mp_destroy(mp_ctx* ctx);

/* Name of a status code (static string). */
const char* mp_status_str(mp_status s);

/* Detail of the last failed call on ctx ("" if none); the pointer stays valid
   until the next call on ctx.  With ctx == NULL: the last mp_create failure
   of the calling thread. */
const char* mp_last_error(const mp_ctx* ctx);

/*
 * mp_get_storage -- copy out the dictionary copy the correlation pass reads,
 * without its padding: FP64 (8-byte), FP32 (4-byte), BF16 (2-byte) or FP8
 * (1-byte) codes, column-major N x M with leading dimension N, and for
 * MP_FP8_E4M3 the M per-column FP32 scales (scales may be NULL otherwise).
 * For MP_SIGN1 the sign bits in mp_create_signs' packed form, ceil(N/32)
 * 32-bit words per column, bits of rows >= N zero.
 *
 *   codes    device: N*M elements of the storage type's size (MP_SIGN1:
 *            M ceil(N/32) words)
 *   scales   device: M floats, or NULL
 * Errors: MP_EINVAL, MP_EDEVICE.
 */
mp_status mp_get_storage(const mp_ctx* ctx, void* codes, float* scales, void* stream);

/*
 * mp_set_profiling / mp_kernel_time -- per-launch timing of the kernel that
 * makes one MP iteration (the pass over the whole dictionary, eq. 9, with the
 * step of eqs. 10-12 carried into it) during the last mp_solve, or of the
 * matrix-product kernel (the correlations of all active signals) during the
 * last mp_solve_batched, or of the whole persistent launch of the last
 * mp_solve_ragged, measured with HIP events on the decode stream.
 *
 *   every     0: off.  k > 0: mp_solve in FP32, BF16, FP8, FP64 and the sign
 *             form (one launch per iteration) times windows of k consecutive
 *             launches (at most 64) with one event before each window and one
 *             after it, so the timed launches run as untimed ones do and the
 *             average includes the gaps between consecutive launches (the
 *             persistent one-bit decode: its launch, over its t + 2 steps); OMP
 *             times every k-th selection launch on its own; mp_solve_batched
 *             every k-th round's product launch.
 *   avg_ms    host: mean duration of one timed launch in milliseconds
 *   launches  host: number of launches averaged (only launches that performed
 *             an iteration are counted, a window only when all its launches
 *             did; 0 when profiling is off)
 * Errors: MP_EINVAL (NULL ctx or outputs, every < 0), MP_EDEVICE.
 */
mp_status mp_set_profiling(mp_ctx* ctx, int every);
mp_status mp_kernel_time(const mp_ctx* ctx, double* avg_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* MP_H_ */
