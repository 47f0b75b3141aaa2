/*
 * pks.h -- temporally parallel Kalman filter and Rauch-Tung-Striebel smoother
 *          for AMD MI355X (gfx950).  C ABI of libpks.so.
 *
 * Method: Sarkka & Garcia-Fernandez, "Temporal Parallelization of Bayesian
 * Smoothers".  The filter turns every time step into an element
 * (A_k, b_k, C_k, eta_k, J_k) (Lemma 1) and combines them with the
 * associative operator of Lemma 2 in a forward all-prefix-sums scan
 * (Definition of all-prefix-sums, Theorem 1): the prefix a_1 (x) ... (x) a_k
 * carries the filtering density N(x_k; m_k, P_k).  The smoother turns every
 * step into (E_k, g_k, L_k) (Lemma 3), combined with the operator of Lemma 4
 * in a reverse (suffix) scan (Theorem 2): a_k (x) ... (x) a_n carries the
 * smoothing density N(x_k; ms_k, Ps_k).
 *
 * Model (Section IV, time-invariant case):
 *     x_0 ~ N(m0, P0),
 *     x_k = F x_{k-1} + u + q_{k-1},  q ~ N(0, Q),
 *     y_k = H x_k + d + r_k,          r ~ N(0, R).
 * The first measurement is y_1; the prior sits on x_0 (Lemma 1, k = 1).
 *
 * Conventions for every entry point
 *  - Pointers marked "device" address GPU memory the caller owns (allocated
 *    with hipMalloc or by a framework); "host" pointers address CPU memory.
 *  - Arrays are C-contiguous, row-major.  Row k-1 holds time step k:
 *    y [T][ny], m/ms [T][nx], P/Ps [T][nx][nx] (full symmetric matrices).
 *  - Element type of y and of every output: double for PKS_FP64, float for
 *    PKS_MIXED_FP32.  Model matrices are always double.
 *  - Calls are stream-ordered and asynchronous: they validate their
 *    arguments on the host, enqueue kernels on `stream` (a hipStream_t;
 *    NULL = the default stream) and return.  They allocate no device memory:
 *    all scratch lives in the caller's workspace `ws` of `ws_bytes` bytes,
 *    sized with pks_workspace_bytes().  Two calls that run concurrently need
 *    distinct workspaces.
 *  - Errors: invalid arguments return PKS_E_ARG / PKS_E_UNSUPPORTED /
 *    PKS_E_WORKSPACE and enqueue nothing; a failed HIP launch returns
 *    PKS_E_HIP.  pks_last_error() describes the last failure of the calling
 *    thread.  Numerical failures found on the device (a Cholesky factor of
 *    H Q H^T + R, of H P^-_1 H^T + R, or of F P_k F^T + Q that does not
 *    exist) do not fail the call: they set a flag in `ws` that
 *    pks_read_numeric_status() reports, and the outputs of the affected
 *    sequence are NaN.  NaN or Inf in y propagate into the outputs.
 *  - No exception crosses this interface; the library keeps no state
 *    between calls except a plan (pks_plan_*) and the tuning cache.
 */
#ifndef PKS_H
#define PKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PKS_OK = 0,
    PKS_E_ARG = 1,          /* null pointer, bad size, aliasing, bad enum   */
    PKS_E_UNSUPPORTED = 2,  /* valid request this library does not handle   */
    PKS_E_WORKSPACE = 3,    /* ws_bytes smaller than pks_workspace_bytes()   */
    PKS_E_HIP = 4,          /* a HIP runtime call or kernel launch failed    */
    PKS_E_NUMERIC = 5,      /* reported by pks_read_numeric_status only      */
    PKS_STATUS_RANGE_ = 0x7fffffff  /* not a status: makes every int a valid value */
} pks_status;

typedef enum {
    PKS_FP64 = 0,        /* all arithmetic, inputs and outputs in double              */
    PKS_MIXED_FP32 = 1,  /* float storage and products; the (I + C_i J_j) solves of
                            Lemma 2, the Cholesky solves of Lemmas 1 and 3 and the
                            additions that complete each (exactly symmetric)
                            covariance run in double                                 */
    PKS_PRECISION_RANGE_ = 0x7fffffff  /* not a precision: any int passed here is a valid
                                          value of the type, and is rejected with PKS_E_ARG */
} pks_precision;

/*
 * Time-invariant linear/Gaussian model (Section IV).  All matrix pointers
 * are DEVICE pointers to double arrays:
 *   F [nx][nx], Q [nx][nx] symmetric PSD (Q = 0 allowed),
 *   H [ny][nx], R [ny][ny] symmetric positive definite,
 *   m0 [nx], P0 [nx][nx] symmetric PSD (prior on x_0),
 *   u [nx] and d [ny] may be NULL (zero).
 * per_sequence = 1 (batched calls only): every array holds B models stacked
 * along a leading axis (model b at offset b * size); 0: one shared model.
 * 1 <= nx <= 64 and 1 <= ny <= 64.
 */
typedef struct {
    int32_t nx, ny;
    const double *F, *u, *Q;
    const double *H, *d, *R;
    const double *m0, *P0;
    int32_t per_sequence;
} pks_model;

/*
 * Bytes of device workspace needed by any call on problems with these
 * sizes (an upper bound over every tile configuration the library or the
 * autotuner may pick).  total_steps = T for single-sequence calls, the sum
 * of lengths for batched calls; B = number of sequences (1 for single).
 * Returns 0 for invalid sizes.  Host-only; touches no device.
 */
size_t pks_workspace_bytes(int32_t nx, int32_t ny, int64_t total_steps, int32_t B,
                           pks_precision prec);

/*
 * Parallel Kalman filter (Lemmas 1-2, Theorem 1): writes the filtered means
 * m [T][nx] and covariances P [T][nx][nx] of a single sequence y [T][ny].
 * y, m, P, ws: device.  T = 0 is a no-op.  m and P must not overlap y or
 * each other.
 */
pks_status pks_filter(const pks_model *model, int64_t T, const void *y, void *m, void *P,
                      pks_precision prec, void *ws, size_t ws_bytes, void *stream);

/*
 * Parallel RTS smoother (Lemmas 3-4, Theorem 2): from filtered moments
 * m [T][nx], P [T][nx][nx] (the output of pks_filter, symmetric P) writes the
 * smoothed moments ms [T][nx], Ps [T][nx][nx].  Uses F, u, Q of the model.
 * All arrays and ws: device.  Outputs must not overlap the inputs.
 */
pks_status pks_smooth(const pks_model *model, int64_t T, const void *m, const void *P,
                      void *ms, void *Ps, pks_precision prec, void *ws, size_t ws_bytes,
                      void *stream);

/* pks_filter followed by pks_smooth on the same stream, in one call. */
pks_status pks_filter_smooth(const pks_model *model, int64_t T, const void *y, void *m, void *P,
                             void *ms, void *Ps, pks_precision prec, void *ws, size_t ws_bytes,
                             void *stream);

/*
 * Batched forms: B independent sequences packed back to back.  offsets is a
 * DEVICE int64 array [B+1] with offsets[0] = 0, non-decreasing, offsets[B] =
 * total; sequence b occupies rows offsets[b] .. offsets[b+1]-1 of y/m/P/ms/Ps.
 * Zero-length sequences are allowed.  With model->per_sequence = 1 sequence b
 * uses model b.  The k = 1 element of Lemma 1 and the k = n element of
 * Lemma 3 are applied at every sequence start and end, which separates the
 * sequences inside one scan.  Offsets that break the rules above give
 * undefined (but memory-safe) results.
 */
pks_status pks_filter_batched(const pks_model *model, int32_t B, const int64_t *offsets,
                              int64_t total, const void *y, void *m, void *P,
                              pks_precision prec, void *ws, size_t ws_bytes, void *stream);
/*
 * Checks DEVICE offsets [B+1] against the packing rules above (offsets[0] =
 * 0, non-decreasing, none above total, offsets[B] = total) with a kernel on
 * `stream` and synchronises it.  PKS_OK if they hold; else PKS_E_ARG with
 * *first_bad (host pointer, may be NULL) = the smallest offending index b.
 * Uses the third int of the workspace `ws` (any workspace of this library,
 * at least 256 bytes; the numeric flag is left alone).  B < 1, NULL offsets
 * or ws: PKS_E_ARG without a launch (*first_bad = -1).
 */
pks_status pks_check_offsets(int32_t B, const int64_t *offsets, int64_t total, void *ws, int32_t *first_bad,
                             void *stream);
pks_status pks_smooth_batched(const pks_model *model, int32_t B, const int64_t *offsets,
                              int64_t total, const void *m, const void *P, void *ms, void *Ps,
                              pks_precision prec, void *ws, size_t ws_bytes, void *stream);

/*
 * Marginal likelihood (Section III-C).  From the measurements y [T][ny] and
 * the filtered moments m [T][nx], P [T][nx][nx] that pks_filter wrote for the
 * same model, evaluates every factor of p(y_1:T) = prod_k p(y_k | y_1:k-1):
 *     log p(y_k | y_1:k-1) = log N(y_k; H m^-_k + d, H P^-_k H^T + R),
 *     m^-_k = F m_{k-1} + u,  P^-_k = F P_{k-1} F^T + Q,
 * with m_0 = m0, P_0 = P0 at the first step.  Evaluated in double in both
 * precisions (PKS_MIXED_FP32 widens its float y, m, P); the residual
 * y_k - H m^-_k - d is a compensated sum, so each factor is the factor of the
 * given inputs to about 1e-15 relative of its terms.
 * Accuracy envelope: a factor is as accurate as the moments it is given.  Its
 * first-order sensitivity to them is |v_k|^T |G| |dm_{k-1}| (v_k the whitened
 * residual S_k^-1 r_k, G = H F), so float storage of m (PKS_MIXED_FP32, a
 * relative error of 2^-24) costs about 6e-8 |v_k| |G| |m_{k-1}| nats per
 * factor: negligible for states of order 1e2, about one nat per factor at
 * states of 1e7 (a constant-velocity track of 2^20 steps), where only PKS_FP64
 * moments give a meaningful likelihood.
 *   ll       DEVICE double [T] or NULL: log p(y_k | y_1:k-1) for every k, or,
 *            with cumulative != 0, the partial sums log p(y_1:k).
 *   ll_total DEVICE double [1] or NULL: log p(y_1:T) (0 when T = 0).
 * At least one of ll, ll_total must be given; cumulative != 0 needs ll.
 * Outputs must not overlap the inputs or each other.  The sums are taken in
 * a fixed order (reproducible run to run).  An innovation covariance whose
 * Cholesky factorisation fails sets the numeric flag (see
 * pks_read_numeric_status) and gives NaN for that step and every sum over
 * it; NaN in y gives NaN without the flag.  Same workspace as pks_filter.
 */
pks_status pks_loglik(const pks_model *model, int64_t T, const void *y, const void *m, const void *P,
                      double *ll, double *ll_total, int32_t cumulative, pks_precision prec, void *ws,
                      size_t ws_bytes, void *stream);
/*
 * Batched form: offsets, packing and per-sequence models as in
 * pks_filter_batched; ll [total], ll_total [B] (0 for an empty sequence); the
 * partial sums restart at every sequence start.
 */
pks_status pks_loglik_batched(const pks_model *model, int32_t B, const int64_t *offsets, int64_t total,
                              const void *y, const void *m, const void *P, double *ll, double *ll_total,
                              int32_t cumulative, pks_precision prec, void *ws, size_t ws_bytes,
                              void *stream);
/*
 * Time-varying linear/Gaussian model (Section IV in its general form):
 *     x_k = F_{k-1} x_{k-1} + u_{k-1} + q_{k-1},  q_{k-1} ~ N(0, Q_{k-1}),
 *     y_k = H_k x_k + d_k + r_k,                  r_k ~ N(0, R_k),
 * for k = 1..T, with x_0 ~ N(m0, P0).  Every matrix pointer is a DEVICE
 * pointer to T stacked double matrices; row k-1 holds the step-k quantities:
 *   F [T][nx][nx] (F_{k-1}: the transition INTO step k), Q [T][nx][nx],
 *   u [T][nx] or NULL, H [T][ny][nx], R [T][ny][ny], d [T][ny] or NULL;
 *   m0 [nx], P0 [nx][nx] as for pks_model; per_sequence = 1 (batched calls
 *   only): m0 [B][nx], P0 [B][nx][nx] hold one prior per sequence.
 * The smoothing element of step k (Lemma 3) uses the transition out of it,
 * row k (F_k, Q_k, u_k); row 0 is used by the filter only.  Every step's
 * Lemma 1 element is built from its own rows, so the workspace holds one
 * block of constants per step: size it with pks_workspace_bytes_tv (total
 * steps).  Batched calls pack the sequences' rows like y (row i belongs to
 * the step in row i of y), each sequence starting from its prior.  A failing
 * factorisation flags its sequence and gives NaN outputs from that step on.
 */
typedef struct {
    int32_t nx, ny;
    const double *F, *u, *Q;
    const double *H, *d, *R;
    const double *m0, *P0;
    int32_t per_sequence;
} pks_model_tv;
/* Workspace bytes for the time-varying calls below (T <= 2^31 - 1); 0 if invalid. */
size_t pks_workspace_bytes_tv(int32_t nx, int32_t ny, int64_t T, pks_precision prec);
/* pks_filter, pks_smooth, pks_filter_smooth and pks_loglik for a time-varying
 * model: same arrays, conventions and errors as their time-invariant forms. */
pks_status pks_filter_tv(const pks_model_tv *model, int64_t T, const void *y, void *m, void *P,
                         pks_precision prec, void *ws, size_t ws_bytes, void *stream);
pks_status pks_smooth_tv(const pks_model_tv *model, int64_t T, const void *m, const void *P, void *ms,
                         void *Ps, pks_precision prec, void *ws, size_t ws_bytes, void *stream);
pks_status pks_filter_smooth_tv(const pks_model_tv *model, int64_t T, const void *y, void *m, void *P,
                                void *ms, void *Ps, pks_precision prec, void *ws, size_t ws_bytes,
                                void *stream);
pks_status pks_loglik_tv(const pks_model_tv *model, int64_t T, const void *y, const void *m, const void *P,
                         double *ll, double *ll_total, int32_t cumulative, pks_precision prec, void *ws,
                         size_t ws_bytes, void *stream);
/* Packed time-varying sequences: offsets and outputs as in pks_filter_batched
 * and pks_loglik_batched; the model rows are packed like y. */
pks_status pks_filter_tv_batched(const pks_model_tv *model, int32_t B, const int64_t *offsets, int64_t total,
                                 const void *y, void *m, void *P, pks_precision prec, void *ws, size_t ws_bytes,
                                 void *stream);
pks_status pks_smooth_tv_batched(const pks_model_tv *model, int32_t B, const int64_t *offsets, int64_t total,
                                 const void *m, const void *P, void *ms, void *Ps, pks_precision prec, void *ws,
                                 size_t ws_bytes, void *stream);
pks_status pks_loglik_tv_batched(const pks_model_tv *model, int32_t B, const int64_t *offsets, int64_t total,
                                 const void *y, const void *m, const void *P, double *ll, double *ll_total,
                                 int32_t cumulative, pks_precision prec, void *ws, size_t ws_bytes, void *stream);
/*
 * Plans: the whole filter + smoother of a (batched) problem, with its tile
 * configuration taken from the tuning cache, captured once into a HIP graph
 * bound to these pointers; pks_plan_launch replays it with one
 * hipGraphLaunch.  `tune_cache` names the JSON cache file (NULL: environment
 * variable PKS_TUNE_CACHE, else built-in defaults).  B = 1 with offsets =
 * NULL plans a single sequence of `total` steps.  *plan receives an opaque
 * handle owned by the caller, released with pks_plan_destroy.
 */
pks_status pks_plan_create(const pks_model *model, int32_t B, const int64_t *offsets,
                           int64_t total, const void *y, void *m, void *P, void *ms, void *Ps,
                           pks_precision prec, void *ws, size_t ws_bytes,
                           const char *tune_cache, void *stream, void **plan);
/*
 * The same for a time-varying model (one row of F, u, Q, H, d, R per step, as
 * in pks_filter_tv): the per-step precompute and both passes are captured.
 * B = 1 with offsets = NULL plans one sequence; packed sequences take
 * offsets as in pks_filter_tv_batched.  Workspace: pks_workspace_bytes_tv of
 * `total` steps.  Errors as pks_plan_create; more than 2^31 - 1 steps returns
 * PKS_E_UNSUPPORTED.
 */
pks_status pks_plan_create_tv(const pks_model_tv *model, int32_t B, const int64_t *offsets,
                              int64_t total, const void *y, void *m, void *P, void *ms, void *Ps,
                              pks_precision prec, void *ws, size_t ws_bytes,
                              const char *tune_cache, void *stream, void **plan);
pks_status pks_plan_launch(void *plan, void *stream);
pks_status pks_plan_destroy(void *plan);

/*
 * Autotuner: times the available tile configurations (elements per thread,
 * scan levels) for problems of this shape on the current device with HIP
 * events, using synthetic data in the caller's workspace plus a temporary
 * allocation it frees before returning, and stores the fastest in the JSON
 * cache `cache_path` (NULL: PKS_TUNE_CACHE).  Synchronises `stream`.
 */
pks_status pks_autotune(int32_t nx, int32_t ny, int32_t B, int64_t total, pks_precision prec,
                        const char *cache_path, void *stream);

/*
 * Synchronises `stream` and reads the numeric flag of `ws`: PKS_OK, or
 * PKS_E_NUMERIC with *first_bad_sequence (host pointer, may be NULL) set to
 * the smallest sequence index whose Cholesky factorisation failed.  Clears
 * the flag.
 */
pks_status pks_read_numeric_status(void *ws, int32_t *first_bad_sequence, void *stream);

/*
 * Debug mode: NaN-filled workspaces.  While on, every call that takes a
 * workspace (the noalloc entry point's static one included) first fills its
 * floating-point regions with a pattern that reads as NaN in double and in
 * float, on the call's stream; a kernel that read workspace memory the call
 * has not written would then give NaN outputs.  The numeric flag and the
 * integer tables are not filled, so pks_read_numeric_status keeps working.
 * Results are otherwise unchanged (bitwise); the fill costs one pass over the
 * workspace.  A plan captured while the mode is on fills its workspace at
 * every launch.  Off by default; also switched on when the environment
 * variable PKS_DEBUG_POISON is set to anything but "0" when first queried.
 * pks_set_debug_poison(on): on != 0 switches it on, 0 off (process-wide;
 * always PKS_OK).  pks_debug_poison(): 1 if on, else 0.
 */
pks_status pks_set_debug_poison(int32_t on);
int32_t pks_debug_poison(void);

/*
 * Environment variable PKS_PIVOTED_INVERSE=1 (read at every launch): for
 * time-invariant models with 5 <= nx <= 16 and ny <= 16 (one sequence or
 * packed sequences), the combines of two block elements (Lemma 2) invert
 * I + J_j C_i with partial pivoting straight away.  By default they first invert it without pivoting and keep that
 * inverse when the residual of every entry is below 1e-11, else invert again
 * with pivoting; both give results within the parity tolerances.  For tests.
 */

/*
 * pks_filter_smooth without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * hosts that forbid hipMalloc).  Same arguments, outputs and errors as
 * pks_filter_smooth minus ws / ws_bytes: the workspace is a static device
 * array of pks_noalloc_scratch_bytes() bytes (32 MiB) that every GPU the
 * library runs on holds until the process ends.  The call allocates nothing.
 * A problem whose pks_workspace_bytes(nx, ny, T, 1, prec) exceeds that size
 * returns PKS_E_UNSUPPORTED (about 3.1e5 steps at nx = 4, ny = 2 in FP64,
 * 5.4e5 in PKS_MIXED_FP32).  All calls on one GPU share that GPU's array:
 * calls that overlap on one GPU race (serialise them on one stream), and
 * pks_read_numeric_status is not available for this entry point (its flag
 * lives in the shared array; a failed factorisation still yields NaN).
 */
pks_status pks_filter_smooth_noalloc(const pks_model *model, int64_t T, const void *y, void *m, void *P,
                                     void *ms, void *Ps, pks_precision prec, void *stream);
size_t pks_noalloc_scratch_bytes(void);

/*
 * Discrete-state hidden Markov model: the same parallel filter and smoother
 * with a finite state space, where the integrals of Definitions 1 and 2
 * become sums over the states (the paper's concluding section notes that the
 * framework holds with the counting measure).  Model:
 *     x_0 ~ p0,  p(x_k = j | x_{k-1} = i) = Pi[i][j],  p(y_k | x_k = j) = exp(L[k-1][j]),
 * with the emission log-likelihoods L [T][K] supplied by the caller (any
 * emission model).  Theorem 1: the prefix a_1 (x) ... (x) a_k carries the
 * filtered marginal alpha_k = p(x_k | y_1:k) and p(y_1:k); Theorem 2: the
 * suffix a_k (x) ... (x) a_T carries the smoothed marginal gamma_k =
 * p(x_k | y_1:T).  FP64 throughout.
 *   K      number of states, 1..64
 *   Pi     DEVICE double [K][K], rows summing to one
 *   p0     DEVICE double [K], the distribution of x_0 (the first data are y_1)
 *   L      DEVICE double [T][K]; rows may hold -inf (impossible states); a
 *          step whose data are impossible under the model gives NaN
 *   alpha  DEVICE double [T][K] out (filter) / in (smoother)
 *   logp   DEVICE double [T] out or NULL: log p(y_1:k), the g-part of the prefix
 *   gamma  DEVICE double [T][K] out
 * Workspace: pks_hmm_workspace_bytes(K, T) bytes (0 for invalid sizes).
 * Outputs must not overlap the inputs or each other.  A row of Pi with no
 * way into a state that the filter reaches is fine; a smoothed marginal puts
 * no weight on states the filter cannot reach.
 */
typedef struct {
    int32_t K;
    const double *Pi;
    const double *p0;
} pks_hmm;
size_t pks_hmm_workspace_bytes(int32_t K, int64_t T);
pks_status pks_hmm_filter(const pks_hmm *model, int64_t T, const double *L, double *alpha, double *logp,
                          void *ws, size_t ws_bytes, void *stream);
pks_status pks_hmm_smooth(const pks_hmm *model, int64_t T, const double *alpha, double *gamma, void *ws,
                          size_t ws_bytes, void *stream);
pks_status pks_hmm_filter_smooth(const pks_hmm *model, int64_t T, const double *L, double *alpha,
                                 double *logp, double *gamma, void *ws, size_t ws_bytes, void *stream);

/*
 * Diagnostics: per-kernel timing.  After pks_profile_start(), every call made
 * by this thread brackets each kernel it launches with HIP events recorded on
 * the launch stream.  pks_profile_stop() synchronises the device, stops the
 * recording and reports up to max_kernels distinct kernel names in first-
 * launch order: names (host buffer of max_kernels * 64 chars, NUL-terminated
 * entries), total_ms (host, summed event-to-event milliseconds), launches
 * (host, launch counts) and *n_kernels (host).  Any output pointer may be NULL.
 */
pks_status pks_profile_start(void);
pks_status pks_profile_stop(int32_t max_kernels, char *names, float *total_ms, int32_t *launches,
                            int32_t *n_kernels);

/* Description of the calling thread's last failure ("" if none). */
const char *pks_last_error(void);

/* Library version string. */
const char *pks_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PKS_H */
