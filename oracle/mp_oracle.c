/*
 * Plain double-precision CPU reference of Matching Pursuit.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the decoder itself never calls it, and it
 * shares no code, header or constant with the GPU library.
 *
 * What it computes (Section 3, the MP pseudo-code, eqs. 8-12):
 *   init   t = 0, x~ = 0, r = y                                   (eq. 8)
 *   while  ||r||_2 > eps ||y||_2  and  t < T:                     (step 2)
 *       i   = argmax_m |<r, psi_m>|, smallest index on ties       (eq. 9;
 *             the i?amax semantics of eq. 16)
 *       x~_i += <r, psi_i>                                        (eq. 10)
 *       r    -= <r, psi_i> psi_i                                  (eq. 11)
 *       t    += 1                                                 (eq. 12)
 *   return x~                                                     (step 3)
 *
 * Readings where the paper is loose (each is listed in the design doc):
 *   - The stopping test is the relative one of the pseudo-code, evaluated on
 *     squared norms: continue while sum r^2 > eps^2 * sum y^2, and t < T.
 *     It is tested before every step, so t counts updates done.
 *   - y = 0: no step is taken (stop reason ZERO_INPUT).  If the largest
 *     |<r, psi_m>| is exactly 0 while r != 0, MP cannot progress: stop reason
 *     STALLED, no update.
 *   - The residual is the recursive one of eq. 11 (never recomputed as
 *     y - Psi x~); ||r|| for the stopping test is recomputed from r every
 *     step, as the nrm2 call of the Section 4 kernel list does.
 *   - Columns are used exactly as given (no renormalisation).
 *
 * Everything is FP64.  FP32 inputs are promoted exactly.  Each inner product
 * is a sequential sum over n = 0..N-1, so results do not depend on the
 * OpenMP thread count.
 *
 * Layout: psi is column-major N x M with leading dimension ld >= N, i.e.
 * psi_nm = psi[n + m*ld].
 *
 * Replay mode (mpo_replay_*): the same iteration with the selection of
 * eq. 9 replaced by a given index sequence, so that another decoder's
 * choices can be followed exactly in FP64.  Each step still takes its
 * coefficient as the FP64 inner product <r, psi_i> (eq. 10) and updates r
 * by eq. 11.  With check_ties set, every step also computes all the
 * correlations and records the forced atom's deficit max_m |c_m| - |c_i|,
 * which is 0 when the forced atom is a correct choice of eq. 9 and small
 * when it is a near tie.  Replaying this file's own free-run sequence gives
 * its free run back bit for bit (the coefficient is the same sequential sum
 * in both modes).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { MPO_CONVERGED = 0, MPO_MAX_ITERS = 1, MPO_STALLED = 2, MPO_ZERO_INPUT = 3 };
enum { MPO_OK = 0, MPO_BAD_ARGS = -1, MPO_NO_MEMORY = -2 };

int mpo_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void mpo_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Sum of squares, sequential, in FP64. */
static double sumsq(const double* v, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += v[i] * v[i];
    return s;
}

/* Smallest index of the largest |c_m| (eq. 16); also the runner-up |c|. */
static int64_t argmax_abs(const double* c, int64_t m, double* best, double* second) {
    int64_t bi = 0;
    double b = fabs(c[0]);
    double s = -1.0;
    for (int64_t j = 1; j < m; ++j) {
        double a = fabs(c[j]);
        if (a > b) {
            s = b;
            b = a;
            bi = j;
        } else if (a > s) {
            s = a;
        }
    }
    *best = b;
    *second = s;
    return bi;
}

/*
 * The same algorithm instantiated for FP32 and FP64 dictionaries.
 *   x_out (M), r_out (N): final estimate and residual, FP64.
 *   trace arrays (each of length tr_cap, any may be NULL): per step the
 *   selected index, the coefficient <r, psi_i>, sum r^2 after the update,
 *   and the gap between the largest and second-largest |<r, psi_m>|.
 */
#define MPO_DEFINE_CORRELATE(SUFFIX, T)                                                   \
    void mpo_correlate_##SUFFIX(const T* psi, int64_t n, int64_t m, int64_t ld,          \
                                const double* r, double* c) {                            \
        _Pragma("omp parallel for schedule(static)")                                      \
        for (int64_t j = 0; j < m; ++j) {                                                 \
            const T* col = psi + j * ld;                                                  \
            double s = 0.0;                                                               \
            for (int64_t i = 0; i < n; ++i) s += (double)col[i] * r[i];                   \
            c[j] = s;                                                                     \
        }                                                                                 \
    }

/* The solver for dictionary element type T and y element type YT, whose
   correlation pass is mpo_correlate_SUFFIX; y is promoted exactly to FP64. */
#define MPO_DEFINE_SOLVE(NAME, SUFFIX, T, YT)                                             \
    int NAME(const T* psi, int64_t n, int64_t m, int64_t ld,                              \
             const YT* y, double eps, int64_t max_iters,                                  \
             double* x_out, double* r_out, int64_t* iters_out,                            \
             int32_t* reason_out, double* yy_out, double* rr_out,                         \
             int32_t* tr_idx, double* tr_coef, double* tr_rr,                             \
             double* tr_gap, int64_t tr_cap) {                                            \
        if (!psi || !y || !x_out || !r_out || n < 1 || m < 1 || ld < n || max_iters < 0 \
            || !(eps >= 0.0))                                                             \
            return MPO_BAD_ARGS;                                                          \
        double* c = (double*)malloc(sizeof(double) * (size_t)m);                          \
        if (!c) return MPO_NO_MEMORY;                                                     \
        for (int64_t i = 0; i < n; ++i) r_out[i] = (double)y[i];                          \
        for (int64_t j = 0; j < m; ++j) x_out[j] = 0.0;                                   \
        const double yy = sumsq(r_out, n);                                                \
        const double thr = eps * eps * yy;                                                \
        double rr = yy;                                                                   \
        int64_t t = 0;                                                                    \
        int32_t reason;                                                                   \
        if (yy == 0.0) {                                                                  \
            reason = MPO_ZERO_INPUT;                                                      \
        } else {                                                                          \
            for (;;) {                                                                    \
                if (!(rr > thr)) { reason = MPO_CONVERGED; break; }                       \
                if (t >= max_iters) { reason = MPO_MAX_ITERS; break; }                    \
                mpo_correlate_##SUFFIX(psi, n, m, ld, r_out, c);                          \
                double best, second;                                                      \
                const int64_t i = argmax_abs(c, m, &best, &second);                       \
                const double ci = c[i];                                                   \
                if (ci == 0.0) { reason = MPO_STALLED; break; }                           \
                x_out[i] += ci;                                                           \
                const T* col = psi + i * ld;                                              \
                for (int64_t k = 0; k < n; ++k) r_out[k] -= ci * (double)col[k];          \
                rr = sumsq(r_out, n);                                                     \
                if (t < tr_cap) {                                                         \
                    if (tr_idx) tr_idx[t] = (int32_t)i;                                   \
                    if (tr_coef) tr_coef[t] = ci;                                         \
                    if (tr_rr) tr_rr[t] = rr;                                             \
                    if (tr_gap) tr_gap[t] = (m > 1) ? best - second : best;               \
                }                                                                         \
                ++t;                                                                      \
            }                                                                             \
        }                                                                                 \
        free(c);                                                                          \
        if (iters_out) *iters_out = t;                                                    \
        if (reason_out) *reason_out = reason;                                             \
        if (yy_out) *yy_out = yy;                                                         \
        if (rr_out) *rr_out = rr;                                                         \
        return MPO_OK;                                                                    \
    }

MPO_DEFINE_CORRELATE(f32, float)
MPO_DEFINE_CORRELATE(f64, double)
MPO_DEFINE_SOLVE(mpo_solve_f32, f32, float, float)
MPO_DEFINE_SOLVE(mpo_solve_f64, f64, double, float)
/* FP64 dictionary and FP64 y (the inputs of an FP64 decode) */
MPO_DEFINE_SOLVE(mpo_solve_f64_y64, f64, double, double)

/*
 * Replay: x_out (M), r_out (N) as the solver; per step t < steps (each array
 * may be NULL): the coefficient, sum r^2 after the step, the deficit
 * max |c| - |c_i| before it (check_ties only, else 0), and r after the step
 * (tr_r: steps x N doubles, step t at tr_r + t*N).  An index outside
 * [0, M) is rejected (MPO_BAD_ARGS) before any step is taken.
 */
#define MPO_DEFINE_REPLAY(NAME, SUFFIX, T, YT)                                            \
    int NAME(const T* psi, int64_t n, int64_t m, int64_t ld, const YT* y,                \
             const int32_t* idx, int64_t steps, int check_ties,                          \
             double* x_out, double* r_out, double* tr_coef, double* tr_rr,               \
             double* tr_deficit, double* tr_r) {                                          \
        if (!psi || !y || !x_out || !r_out || n < 1 || m < 1 || ld < n || steps < 0      \
            || (steps > 0 && !idx))                                                       \
            return MPO_BAD_ARGS;                                                          \
        for (int64_t t = 0; t < steps; ++t)                                               \
            if (idx[t] < 0 || idx[t] >= m) return MPO_BAD_ARGS;                           \
        double* c = NULL;                                                                 \
        if (check_ties) {                                                                 \
            c = (double*)malloc(sizeof(double) * (size_t)m);                              \
            if (!c) return MPO_NO_MEMORY;                                                 \
        }                                                                                 \
        for (int64_t i = 0; i < n; ++i) r_out[i] = (double)y[i];                          \
        for (int64_t j = 0; j < m; ++j) x_out[j] = 0.0;                                   \
        for (int64_t t = 0; t < steps; ++t) {                                             \
            const int64_t i = idx[t];                                                     \
            const T* col = psi + i * ld;                                                  \
            double ci, deficit = 0.0;                                                     \
            if (check_ties) {                                                             \
                mpo_correlate_##SUFFIX(psi, n, m, ld, r_out, c);                          \
                double best, second;                                                      \
                (void)argmax_abs(c, m, &best, &second);                                   \
                ci = c[i];                                                                \
                deficit = best - fabs(ci);                                                \
            } else {                                                                      \
                double s = 0.0;                                                           \
                for (int64_t k = 0; k < n; ++k) s += (double)col[k] * r_out[k];           \
                ci = s;                                                                   \
            }                                                                             \
            x_out[i] += ci;                                                               \
            for (int64_t k = 0; k < n; ++k) r_out[k] -= ci * (double)col[k];              \
            if (tr_coef) tr_coef[t] = ci;                                                 \
            if (tr_rr) tr_rr[t] = sumsq(r_out, n);                                        \
            if (tr_deficit) tr_deficit[t] = deficit;                                      \
            if (tr_r) memcpy(tr_r + t * n, r_out, sizeof(double) * (size_t)n);            \
        }                                                                                 \
        free(c);                                                                          \
        return MPO_OK;                                                                    \
    }

MPO_DEFINE_REPLAY(mpo_replay_f32, f32, float, float)
MPO_DEFINE_REPLAY(mpo_replay_f64, f64, double, float)
MPO_DEFINE_REPLAY(mpo_replay_f64_y64, f64, double, double)
