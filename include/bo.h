/* bo.h -- C ABI of the MI355X (gfx950) Gaussian-process surrogate step for
 * Bayesian-optimization auto-tuning over a discrete, constrained search space.
 *
 * Method: Willemsen, van Nieuwpoort, van Werkhoven, "Bayesian Optimization for
 * auto-tuning GPU kernels" (arXiv 2111.14991).  One step, after each new
 * observation:
 *   fit      K_nn = amp * Matern(|x_i - x_j| / l) + delta I, L L^T = K_nn (FP64),
 *            alpha = K_nn^-1 (y - m), m = mean(y)            (Section III-B)
 *   predict  mu(x) = m + k*^T alpha, var(x) = amp - |L^-1 k*|^2 clamped at 0,
 *            for every valid, not yet evaluated candidate  (Sections III-D.2, III-G)
 *   acquire  EI, PI, LCB in minimization form with one exploration factor
 *            lambda, constant or contextual-variance          (Sections III-C, III-F)
 *   select   argmax EI, argmax PI, argmin LCB over those candidates.
 *
 * Conventions for every call:
 *  - Ownership: the caller owns all buffers.  Pointers marked "device" are
 *    device memory on the current HIP device; "host" pointers are ordinary
 *    host memory.  The library never frees caller memory.  The workspace
 *    passed to bo_session_create holds all per-session device state; the
 *    library allocates only a small host-side handle and one pinned host
 *    result record at creation, and nothing afterwards.
 *  - Indices: 0-based int64 into the caller's enumeration of the candidate set
 *    (restriction-pruned points included).
 *  - Ordering: all device work is enqueued on the session stream in call
 *    order.  Calls documented as synchronizing wait for that stream.
 *  - Errors: every call returns a bo_status; no exception crosses the ABI.
 *    Host-checkable arguments are validated before anything is enqueued.
 *    Errors found on the device (an observation index of an invalid point, a
 *    non-finite y, an exhausted jitter schedule) are reported by the next
 *    synchronizing call.  bo_last_error() returns a thread-local message for
 *    the last failing call on that thread.
 *  - Threads: one session must not be used from two threads at once.
 */
#ifndef BO_MI355X_H
#define BO_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BO_OK = 0,
  BO_E_INVALID_ARG = 1,  /* bad argument (host check) or bad observation data (device check) */
  BO_E_NOT_PD = 2,       /* K_nn not positive definite for any jitter of the schedule */
  BO_E_NO_CANDIDATE = 3, /* every candidate is restriction-pruned or already evaluated */
  BO_E_WORKSPACE = 4,    /* workspace too small or misaligned */
  BO_E_HIP = 5,          /* a HIP runtime call failed */
  BO_E_STATE = 6,        /* call out of order (no candidates set, no fit, n = 0, ...) */
  BO_E_BUDGET = 7,       /* serving memory budget below one session */
  BO_E_NUMERIC = 8       /* a NaN acquisition value was met */
} bo_status;

/* Arithmetic of the posterior (the fit is FP64 in every mode).
 *  BO_FP64   : cross-covariance, variance contraction and mean in FP64.
 *  BO_FP32   : mean and variance stored in FP32.  For n <= 256 they come from
 *              the same FP64 products as BO_FP64 (an FP32 contraction cannot
 *              hold a variance that is small next to the prior to 1e-6 of
 *              itself); above, the variance contraction runs on FP32 matrix
 *              cores over the covariance residuals after the nearest
 *              observation, chunks of 16 observations summed in FP64, with
 *              FP64 rows where the residual part dominates.
 *  BO_BF16X3 : squared distances from three FP16 matrix-core products of
 *              augmented coordinates, cross-covariance in FP32, split into
 *              bfloat16 high and low parts; variance contraction as three
 *              bfloat16 matrix-core products (hi*hi + hi*lo + lo*hi) with FP32
 *              accumulation; mean in FP64 from the FP32 covariances. */
typedef enum { BO_FP64 = 0, BO_FP32 = 1, BO_BF16X3 = 2 } bo_precision;

/* Acquisition-function bits (Section III-C). */
enum { BO_EI = 1, BO_POI = 2, BO_LCB = 4 };

/* Problem size fixed for a session's lifetime. */
typedef struct {
  int64_t N;         /* candidates in the caller's enumeration, 1 <= N < 2^31 */
  int32_t d;         /* parameters (dimensions), 1 <= d <= 16 */
  int32_t n_max;     /* most observations a fit will hold, 1 <= n_max <= 1024 */
  int32_t precision; /* bo_precision */
  int32_t reserved;
} bo_problem;

/* Surrogate hyperparameters (Section III-B: fixed lengthscale, no marginal-
 * likelihood search).  Defaults: nu2 = 5, lengthscale = 1, amp = 1,
 * noise = 1e-6, jitter_tries = 7. */
typedef struct {
  int32_t nu2;          /* 3 or 5: Matern nu = nu2 / 2 */
  int32_t jitter_tries; /* 1..20: attempts of the diagonal-addition schedule */
  double lengthscale;   /* > 0, in normalized coordinates */
  double amp;           /* prior variance k(0) > 0 */
  double noise;         /* >= 0, added to the diagonal of K_nn; attempt t >= 1 adds
                           max(noise, 1e-10 amp) * 10^t instead */
} bo_gp_params;

/* Exploration factor (Section III-F). */
typedef struct {
  int32_t mode;        /* 0: lambda = lambda_const; 1: contextual variance
                          lambda = (var_mean / (mu_s / f_best)) / var_s_mean */
  uint32_t acq_bits;   /* BO_EI | BO_POI | BO_LCB (0 means all three) */
  double lambda_const; /* mode 0 (the paper's constant is 0.01) */
  double mu_s;         /* mode 1: mean of the initial sample's observations, > 0 */
  double var_s_mean;   /* mode 1: mean posterior variance after the initial sample;
                          <= 0 means "this step is that one" (lambda = f_best/mu_s) */
} bo_acq_params;

/* Result of one step.  Slots: [0] EI (argmax), [1] PI (argmax), [2] LCB
 * (argmin).  Ties go to the lowest index.  A slot whose function was not
 * requested, or with no candidate, holds idx -1 and a NaN score. */
typedef struct {
  int64_t idx[3];
  double score[3];
  double lambda;     /* exploration factor used */
  double var_mean;   /* mean posterior variance over the predicted candidates */
  double jitter;     /* diagonal addition accepted by the fit */
  double f_best;     /* incumbent: minimum observed y */
  double mean_y;     /* prior mean m */
  int64_t n_unmasked;/* candidates predicted (valid and not evaluated) */
  int32_t status;    /* bo_status of the step */
  int32_t n_obs;     /* observations in the fit */
} bo_acq_result;

/* Fit diagnostics. */
typedef struct {
  int32_t status;
  int32_t n;
  int32_t attempt;   /* index of the accepted jitter attempt */
  int32_t reserved;
  double jitter, mean_y, f_best;
} bo_fit_info;

typedef struct bo_session bo_session;

/* Library version string (static storage). */
const char* bo_version(void);

/* Thread-local message of the last failing call on this thread ("" if none).
 * Valid until the next failing call on the same thread. */
const char* bo_last_error(void);

/* Device workspace bytes a session of this problem needs (256-byte aligned
 * start required).  Returns BO_E_INVALID_ARG for sizes outside the limits. */
bo_status bo_workspace_query(const bo_problem* prob, size_t* bytes);

/* Create a session over a caller-owned device workspace (>= the queried size)
 * and a hipStream_t (passed as void*; NULL = the default stream).  gp may be
 * NULL for the defaults.  The handle is freed by bo_session_destroy. */
bo_status bo_session_create(bo_session** out, const bo_problem* prob, const bo_gp_params* gp,
                            void* workspace, size_t bytes, void* stream);

/* Waits for the session stream, then releases the handle (not the workspace). */
void bo_session_destroy(bo_session* s);

/* Change the stream later calls enqueue on. */
bo_status bo_session_set_stream(bo_session* s, void* stream);

/* Candidate set as a discrete grid (Section III-D): parameter j has
 * levels[j] >= 1 ordered values (host array of d entries); candidate c is grid
 * point cand[c] (device int64 array of N entries, row-major grid index, last
 * parameter fastest), or grid point c when cand is NULL (then N must equal the
 * grid size).  Each parameter is normalized linearly, level i -> i / (k - 1)
 * (Section III-D.1).  invalid (device uint8[N], nonzero = restriction-pruned;
 * NULL = none) marks points never to predict or select (Section III-D.2).
 * Valid candidates are compacted once, keeping their original indices.
 * Synchronizing; *n_valid (host, nullable) receives the valid count.
 * Errors: BO_E_INVALID_ARG (bad levels, grid index out of range). */
bo_status bo_set_grid(bo_session* s, const int32_t* levels, const int64_t* cand,
                      const uint8_t* invalid, int64_t* n_valid);

/* Candidate set from coordinates already normalized by the caller: X is a
 * device N x d row-major array, FP64 (x_is_f32 = 0) or FP32 (x_is_f32 = 1).
 * Otherwise as bo_set_grid. */
bo_status bo_set_candidates(bo_session* s, const void* X, int32_t x_is_f32,
                            const uint8_t* invalid, int64_t* n_valid);

/* Refit on n valid observations (Section III-B): obs_idx (device int64[n],
 * candidate indices, each of a valid candidate) and y (device double[n],
 * finite), in observation order; 1 <= n <= n_max.  Computes m = mean(y),
 * f_best = min(y), the FP64 Cholesky factor of K_nn with the jitter schedule
 * (pivots must exceed n 2^-52 times their diagonal entry), L^-1 and alpha.
 * Asynchronous; device-side errors surface at the next synchronizing call. */
bo_status bo_gp_fit(bo_session* s, const int64_t* obs_idx, const double* y, int32_t n);

/* Refit after one new observation (Section III-B), as a bordered rank-1
 * extension of the device-resident factor: obs_idx and y (device, n entries)
 * hold the current fit's n - 1 observations in the same order followed by the
 * new one.  When the session holds a fit of n - 1 points and n <= 256, the
 * new row of L and L^-1 is computed from L^-1 in O(n^2), alpha is recomputed
 * and only the changed part of the packed operand is rewritten.  Otherwise,
 * or when a pivot fails the test of the (n)-point factorization (the new
 * pivot, or the smallest old one against the larger threshold), this is
 * bo_gp_fit.  The outcome equals bo_gp_fit's on the same arrays up to
 * rounding, with the same accepted jitter.  Asynchronous; errors as
 * bo_gp_fit.  BF16X3 sessions always refit. */
bo_status bo_gp_append(bo_session* s, const int64_t* obs_idx, const double* y, int32_t n);

/* Records one evaluation in the session (Sections III-B, III-D.2): candidate
 * idx (0 <= idx < N) is marked evaluated in the session's own record, so that
 * it is never predicted or selected again.  A valid evaluation (valid = 1,
 * y finite, run time of the configuration) is appended to the session's
 * observations -- those of the last bo_gp_fit / bo_gp_append / bo_observe,
 * none after bo_set_grid -- and the surrogate is refit: the bordered rank-1
 * extension of the device-resident factor when the session holds a fit of the
 * n - 1 earlier points and n <= 256, otherwise a whole fit.  A failed
 * evaluation (valid = 0: the configuration did not compile or run) is only
 * marked; it never enters the fit (Section III-D.2 argues against giving it an
 * artificial value).  Asynchronous; errors as bo_gp_append (an evaluation of a
 * restriction-pruned candidate with valid = 1 is BO_E_INVALID_ARG at the next
 * synchronizing call).  BO_E_INVALID_ARG on the host for idx out of range,
 * valid not 0/1, non-finite y, or more than n_max valid observations. */
bo_status bo_observe(bo_session* s, int64_t idx, double y, int32_t valid);

/* Synchronizing: fit status, accepted jitter, m and f_best.  alpha (host
 * double[n]) and Linv (host double[n*n], row-major lower triangle of L^-1)
 * are filled when non-NULL. */
bo_status bo_fit_read(bo_session* s, bo_fit_info* info, double* alpha, double* Linv);

/* Exhaustive prediction over the discrete space (Section III-G): the GP
 * posterior mean mu = m + k*^T alpha and latent variance var = amp - |L^-1 k*|^2
 * (clamped at zero) of the surrogate of Section III-B, for every candidate
 * that is valid and not visited (Section III-D.2).  visited: device uint8[N],
 * nonzero = evaluated; NULL = the session's own record (bo_observe), which is
 * empty until bo_observe is called.  mu and var (device double[N], nullable)
 * receive the mean and latent variance in the caller's enumeration, NaN where
 * excluded.  var_mean (host, nullable) receives the mean variance over the
 * predicted candidates (Section III-F); when it is non-NULL the call is
 * synchronizing. */
bo_status bo_posterior(bo_session* s, const uint8_t* visited, double* mu, double* var,
                       double* var_mean);

/* Whole step after bo_gp_fit: posterior, lambda, acquisitions and the masked
 * arg-optimum (Sections III-C, III-D.2, III-F, III-G).  visited as in
 * bo_posterior (NULL = the session's own record).  Synchronizing: *out
 * (host) receives the result; the return value equals out->status. */
bo_status bo_acquire(bo_session* s, const uint8_t* visited, const bo_acq_params* params,
                     bo_acq_result* out);

/* Same as bo_acquire, and the acquisition values the arg-optimum was taken
 * over (Section III-C, minimization forms): ei, pi and lcb (device double[N],
 * each nullable) receive EI, PI and LCB of every predicted candidate in the
 * caller's enumeration, NaN where the candidate is excluded or the function
 * is not requested.  Synchronizing. */
bo_status bo_acquire_values(bo_session* s, const uint8_t* visited, const bo_acq_params* params, double* ei,
                            double* pi, double* lcb, bo_acq_result* out);

/* Same as bo_acquire without waiting: *out_dev (device) is written on the
 * session stream.  The jitter schedule of the fit is escalated on the device
 * (every fit size), so the result equals bo_acquire's. */
bo_status bo_acquire_async(bo_session* s, const uint8_t* visited, const bo_acq_params* params,
                           bo_acq_result* out_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture aside: this call synchronizes), e.g. tight serving loops or
 * harnesses that forbid hipMalloc: one whole step with no session and no
 * workspace.  Equivalent to bo_session_create + bo_set_candidates(X, x_is_f32,
 * invalid) + bo_gp_fit(obs_idx, y, n) + bo_acquire(visited, params) on the
 * same arguments, with the same kernels and the same result, but all device
 * state lives in a static device array of 32 MiB that the library holds on
 * each GPU it runs on until the process ends; the call allocates nothing
 * (no hipMalloc, no pinned host memory, no host heap).  Arguments are those
 * of the calls it replaces (device pointers X, invalid, visited, obs_idx, y;
 * host prob, gp (NULL: defaults), params, out; stream as in
 * bo_session_create).  visited NULL means nothing evaluated yet.
 * BO_E_WORKSPACE when the problem's device state (bo_workspace_query of prob)
 * exceeds the 32 MiB.  Every call on one GPU uses that GPU's single array:
 * calls that overlap on one GPU (two host threads, or two streams) race and
 * must be serialized by the caller.  Synchronizing; returns out->status as
 * bo_acquire does. */
bo_status bo_step_noalloc(const bo_problem* prob, const bo_gp_params* gp, const void* X, int32_t x_is_f32,
                          const uint8_t* invalid, const uint8_t* visited, const int64_t* obs_idx, const double* y,
                          int32_t n, const bo_acq_params* params, bo_acq_result* out, void* stream);

/* Phase timing.  With timing enabled the library records HIP events on the
 * session stream around its own launches: the fit (bo_gp_fit), the posterior
 * kernel and the acquisition kernel (bo_posterior / bo_acquire).
 * bo_get_timing is synchronizing and returns the durations, in milliseconds,
 * of the most recent fit, posterior and acquisition (-1 for a phase that has
 * not run since timing was enabled).  The events are created by
 * bo_set_timing, never on the step path. */
bo_status bo_set_timing(bo_session* s, int32_t enable);
bo_status bo_get_timing(bo_session* s, float* fit_ms, float* posterior_ms, float* acquire_ms);

/* ------------------------------------------------------------------------
 * Batched form: many independent sessions advance one step together.
 *
 * One HIP graph, captured once and replayed each step, runs every session's
 * FP64 fit (n <= 256), the posterior over every session's candidates (one
 * launch per precision, in 64-candidate slots), the exploration factors, the
 * acquisition chunks and the selections, between a plan upload and a result
 * download; each kernel's grid is set to the step's work before the replay.
 * Per-session results equal those of bo_gp_fit + bo_acquire on the same
 * session bit for bit (the same kernels per candidate and the same reduction
 * orders).  Sessions must be FP64 or FP32, have candidates set, and have no
 * work pending on their own streams; the batch runs on its own stream.
 * ---------------------------------------------------------------------- */
typedef struct bo_batch bo_batch;

/* Work sizes and scheduling of the batched step. */
typedef struct {
  int32_t post_order; /* posterior slots: 0, the sessions of the largest fits first; 1, in
                           the fit order */
  int32_t acq_chunk;  /* candidates per acquisition workgroup, a positive multiple of 2048
                         (raised where a session would need more than 512 chunks) */
  int32_t fit_order;  /* 0: sessions in order; 1: largest fit first */
  int32_t reserved;
} bo_batch_config;

/* Device workspace bytes of a batch of `count` sessions (1..65536). */
bo_status bo_batch_workspace_query(int32_t count, size_t* bytes);

/* Bind `count` distinct sessions (host array of handles, kept by reference:
 * they must outlive the batch) over a caller-owned, 256-byte-aligned device
 * workspace.  stream: hipStream_t as void*; NULL creates a private blocking
 * stream.  Default config {0, 8192, 1}. */
bo_status bo_batch_create(bo_batch** out, bo_session* const* sessions, int32_t count, void* workspace,
                          size_t bytes, void* stream);
void bo_batch_destroy(bo_batch* b);

bo_status bo_batch_set_config(bo_batch* b, const bo_batch_config* cfg);
bo_status bo_batch_get_config(bo_batch* b, bo_batch_config* cfg);

/* With timing on, bo_batch_step reports the graph's duration (HIP events on
 * the batch stream). */
bo_status bo_batch_set_timing(bo_batch* b, int32_t enable);

/* One step of every session, synchronizing.  Host arrays of `count` entries:
 * obs_idx[i], y[i] (device pointers, as bo_gp_fit), n[i] (1..min(n_max, 256)),
 * visited[i] (device uint8[N_i], or NULL for the session's own record as in
 * bo_posterior; visited itself may be NULL),
 * params[i], out[i] (host).  Each out[i].status reports that session's
 * outcome; the return value reports argument and runtime errors only.
 * graph_ms (nullable) receives the graph's duration, -1 without timing.
 * After the call each session holds the new fit, as after bo_gp_fit. */
bo_status bo_batch_step(bo_batch* b, const int64_t* const* obs_idx, const double* const* y, const int32_t* n,
                        const uint8_t* const* visited, const bo_acq_params* params, bo_acq_result* out,
                        float* graph_ms);

/* Autotuner: runs the step `reps` + 1 times for each slots-per-workgroup /
 * chunk / fit order of a fixed candidate set, keeps the configuration with the
 * lowest median graph time, stores it in the batch and returns it in
 * *chosen (nullable).  out receives the results of the last run. */
bo_status bo_batch_tune(bo_batch* b, const int64_t* const* obs_idx, const double* const* y, const int32_t* n,
                        const uint8_t* const* visited, const bo_acq_params* params, int32_t reps,
                        bo_batch_config* chosen, bo_acq_result* out);

/* ------------------------------------------------------------------------
 * Serving form: live sessions, BO step requests arriving at any time.
 *
 * A request appends one evaluation to its session (bo_gp_append's rank-1
 * extension of the device-resident factor; for an evaluation that failed,
 * valid = 0, only the visited mark) and returns the step's result.  A
 * scheduler thread gathers pending requests of idle sessions (one request in
 * flight per session, oldest first) into replays of the batched step graph
 * on up to `streams` launch contexts, each with its own stream, so
 * that requests arriving while launches run are admitted as soon as a context
 * frees up and launches overlap on the device.  A session's device state is
 * allocated when it fits in the memory budget; until then it waits, with its
 * requests.  All entry points are thread-safe.
 * ---------------------------------------------------------------------- */
typedef struct bo_server bo_server;

typedef struct {
  size_t hbm_budget;       /* device bytes for session state (bo_server_session_bytes each) */
  int32_t max_batch;       /* most requests in one launch, 1..4096 */
  int32_t streams;         /* launches in flight at once, 1..8 */
  bo_batch_config tiles;   /* work sizes of the batched step */
} bo_server_config;

typedef struct {
  int64_t steps_done;
  int64_t launches;
  int64_t sessions_resident;
  int64_t sessions_waiting;  /* opened, waiting for memory */
  int64_t pending;           /* requests not yet launched */
  size_t bytes_in_use;
  double mean_batch;         /* requests per launch */
  int64_t sessions_setting_up; /* admitted, being uploaded and fitted (counted as resident too) */
  double mean_wait_us;       /* per request: submission to the start of its launch call */
  double mean_launch_us;     /* per launch: host time of the launch call */
  double mean_gpu_us;        /* per launch: device time of the batched step graph */
} bo_server_info;

/* Device bytes one session of this problem holds while resident. */
bo_status bo_server_session_bytes(const bo_problem* prob, size_t* bytes);

/* Starts the scheduler on the current device.  The server allocates its
 * launch contexts now and session state on admission (hipMalloc, outside the
 * step path). */
bo_status bo_server_create(bo_server** out, const bo_server_config* cfg);

/* Refuses requests not yet launched (status BO_E_STATE), waits for launches
 * in flight, frees everything. */
void bo_server_destroy(bo_server* srv);

/* Opens a session: problem (precision FP64 or FP32, n_max <= 256), GP
 * parameters (NULL: defaults), the candidate grid as in bo_set_grid but with
 * host arrays (levels[d]; cand[N] or NULL; invalid[N] or NULL) and n0 >= 1
 * initial observations (host obs_idx, y).  *id identifies the session.  The
 * session is set up now if it fits in the budget, otherwise when memory is
 * freed.  BO_E_BUDGET when it alone exceeds the budget. */
bo_status bo_server_open(bo_server* srv, const bo_problem* prob, const bo_gp_params* gp, const int32_t* levels,
                         const int64_t* cand, const uint8_t* invalid, const int64_t* obs_idx, const double* y,
                         int32_t n0, int32_t* id);

/* Closes a session: its queued requests still run, then its memory returns
 * to the budget (a session still waiting for memory is dropped at once and its
 * requests finish with BO_E_STATE). */
bo_status bo_server_close(bo_server* srv, int32_t id);

/* Queues a step: evaluation `y` of candidate `idx` (valid != 0), or a failed
 * evaluation of `idx` (valid = 0: visited mark only), then the acquisition
 * with `acq`.  *ticket identifies the request.  Errors in the arguments are
 * returned here; errors of the step are in the result's status. */
bo_status bo_server_submit(bo_server* srv, int32_t id, int64_t idx, double y, int32_t valid,
                           const bo_acq_params* acq, uint64_t* ticket);

/* *done = 1 once the request's result is available. */
bo_status bo_server_poll(bo_server* srv, uint64_t ticket, int32_t* done);

/* Blocks until the request is done, returns its result and its latency from
 * submission (ms, nullable), and forgets the ticket. */
bo_status bo_server_wait(bo_server* srv, uint64_t ticket, bo_acq_result* out, double* latency_ms);

/* Completion queue: waits up to timeout_us microseconds (0: not at all) for
 * a finished request not yet returned, then returns up to `max` of them in
 * the order they finished: tickets[k], out[k] and latency_ms[k] (nullable)
 * for k < *count (0 when none finished in time), and forgets those tickets.
 * Requests taken by bo_server_wait are not returned again. */
bo_status bo_server_wait_any(bo_server* srv, int32_t max, int32_t timeout_us, uint64_t* tickets,
                             bo_acq_result* out, double* latency_ms, int32_t* count);

/* Counters and occupancy of the server. */
bo_status bo_server_stats(bo_server* srv, bo_server_info* out);

#ifdef __cplusplus
}
#endif
#endif
