/*
 * cp_arls_lev.h -- C ABI of the MI355X (gfx950) CP-ARLS-LEV mode-update library.
 *
 * The library runs the per-mode step of CP via alternating randomized least
 * squares with leverage-score sampling (Larsen & Kolda, "Practical
 * Leverage-Based Sampling for Low-Rank Tensor Decomposition", Alg. 3):
 * leverage scores of the factor matrices (Def. 3.4), hybrid deterministic +
 * random sampling of Khatri-Rao-product rows (Alg. 1, Alg. 2, Sec. 4.2-4.3,
 * Sec. 5.3), extraction of the sampled tensor fibers (Sec. 6.3) and the
 * sampled least-squares solve, plus the stratified fit estimate (Sec. 6.4).
 *
 * Conventions
 *  - Pointers are DEVICE pointers unless marked "host".
 *  - Factor matrices are FP64, row-major n_m x R, owned by the caller; the
 *    library reads them and overwrites factors[k] on a mode-k update.
 *  - Tensor coordinates are 0-based int32 in structure-of-arrays layout
 *    coords[m * nnz + e]; coordinates must be distinct.
 *  - Linear index of a KRP row for the update of mode k: the other modes in
 *    ascending order, first other mode fastest (eq. (2.2), 0-based).
 *  - All work is enqueued on the stream given at init; calls are
 *    asynchronous unless stated.  A context is not thread-safe.
 *  - Status codes report argument/state errors synchronously; data-dependent
 *    conditions are reported through cpal_mode_stats.flags in device memory.
 */
#ifndef CP_ARLS_LEV_H
#define CP_ARLS_LEV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cpal_ctx cpal_ctx;

typedef enum {
  CPAL_OK = 0,
  CPAL_E_ARG = 1,      /* invalid argument (null pointer, bad size, bad option)  */
  CPAL_E_NOMEM = 2,    /* device allocation failed                               */
  CPAL_E_DEVICE = 3,   /* a HIP call or kernel launch failed                     */
  CPAL_E_STATE = 4     /* invalid state (e.g. an all-zero factor matrix)          */
} cpal_status;

typedef enum { CPAL_F64 = 0, CPAL_F32 = 1, CPAL_BF16 = 2 } cpal_dtype;

/* Probability of row i of factor m used to sample KRP rows; a KRP row's
 * probability is the product over the other modes (Sec. 5.3 for leverage,
 * App. B for the other two). */
typedef enum {
  CPAL_SAMPLE_LEVERAGE = 0,        /* l_i(A_m) / R (Def. 3.4; the method)              */
  CPAL_SAMPLE_UNIFORM = 1,         /* 1 / n_m                                          */
  CPAL_SAMPLE_LENGTH_SQUARED = 2   /* ||A_m(i,:)||^2 / ||A_m||_F^2                      */
} cpal_sampling;

/* Bits of cpal_mode_stats.flags. */
enum {
  CPAL_FLAG_PINV = 1,       /* a Gram matrix was singular: pseudo-inverse used        */
  CPAL_FLAG_DETCAP = 2,     /* deterministic enumeration exceeded det_enum_cap: the
                               update sampled randomly only (tau treated as 1)        */
  CPAL_FLAG_DET_TRUNC = 4,  /* >= s rows above tau: the s most probable kept          */
  CPAL_FLAG_PDET_ONE = 8,   /* 1 - p_det <= 2^-40: no random rows                     */
  CPAL_FLAG_DRAWCAP = 16,   /* random draws hit 64*s_rnd + 2^20 before s_rnd accepts  */
  CPAL_FLAG_OVERFLOW = 32,  /* the deterministic set exceeded its buffer; the buffer
                               is sized at init from the bound |D| < 1/tau (Sec. 5.3),
                               the largest other-mode KRP row count and det_enum_cap,
                               so this flag marks an internal error                  */
  CPAL_FLAG_STATE = 64      /* a probability vector summed to zero                    */
};

/* Device memory provider (ownership of every buffer the library allocates):
 * alloc(bytes, user) returns `bytes` of device memory on the context's device,
 * 256-byte aligned, or NULL on failure (the call then fails with
 * CPAL_E_NOMEM); free(ptr, user) releases a pointer alloc returned.  Every
 * allocation of a context or batch -- persistent buffers, the temporaries of
 * init, buffers added later by cp_arls_lev_set_gather_config or the
 * autotuner -- goes through it, and cp_arls_lev_destroy (or
 * cp_arls_lev_destroy_batch) returns all of them after synchronizing the
 * streams.  The callbacks are called from the calling host thread only, never
 * from a stream or graph.  A NULL cpal_allocator* selects hipMalloc/hipFree. */
typedef struct {
  void *(*alloc)(size_t bytes, void *user);
  void (*free)(void *ptr, void *user);
  void *user;
} cpal_allocator;

typedef struct {
  int32_t order;             /* D >= 2, <= 8                                           */
  const int64_t *dims;       /* host, order entries; prod(dims) < 2^62                 */
  int64_t nnz;               /* sparse: >= 1, < 2^32; ignored when dense               */
  const int32_t *coords;     /* device, [order][nnz], distinct coordinates; ignored
                                (may be NULL) when dense                             */
  const void *values;        /* device, value_dtype: nnz values (sparse), or
                                prod(dims) values with mode 0 fastest (dense)        */
  int32_t value_dtype;       /* CPAL_F32 or CPAL_F64                                   */
  int32_t dense;             /* 0: COO sparse; 1: every entry stored (the fibers of
                                the sampled rows are whole columns, Sec. 6.3)        */
} cpal_tensor;

typedef struct {
  int32_t rank;              /* R, 1..64                                               */
  int64_t samples;           /* s >= 1 (rows sampled per least-squares problem)        */
  double tau;                /* deterministic threshold in [0,1]; 1 = random only      */
  uint64_t seed;             /* Philox key word 0                                      */
  uint64_t stream_id;        /* Philox key word 1 (e.g. the restart number)            */
  int32_t gather_dtype;      /* CPAL_F64 (parity) or CPAL_F32: precision of the fiber
                                values, the weighted KRP rows and the sampled MTTKRP;
                                CPAL_BF16 (dense tensors only): BF16 fiber values and
                                KRP rows on the matrix cores, FP32 accumulation.
                                Gram matrices, solves and leverage are always FP64   */
  int64_t fit_samples;       /* s_fit for cp_arls_lev_fit_estimate; 0 = no fit sample
                                (must be 0 for a dense tensor)                       */
  double fit_nnz_fraction;   /* alpha in [0,1] (Sec. 6.4), default 0.5                 */
  int64_t det_enum_cap;      /* max candidate combinations examined by the
                                deterministic enumeration; 0 = 2^26                  */
  int32_t sampling;          /* cpal_sampling: CPAL_SAMPLE_LEVERAGE (0, the method),
                                CPAL_SAMPLE_UNIFORM or CPAL_SAMPLE_LENGTH_SQUARED;
                                the scores behind the probabilities are what
                                cp_arls_lev_leverage returns                         */
  int32_t pad;
} cpal_options;

typedef struct {
  int64_t s_det;             /* deterministic rows                                     */
  int64_t s_rnd;             /* accepted random draws                                  */
  int64_t s_bar;             /* rows of the sampled system (s_det + unique random)     */
  int64_t draws;             /* random draws made                                      */
  int64_t gathered_nnz;      /* nonzeros in the sampled fibers                         */
  double p_det;              /* total probability of the deterministic rows            */
  int32_t flags;             /* CPAL_FLAG_* bits                                       */
  int32_t pad;
} cpal_mode_stats;

/* Create a context (Alg. 3 setup): copies X into per-mode fiber indexes
 * (Sec. 6.3: every nonzero keyed by the linear index of its other-mode
 * coordinates, sorted, with a hash table key -> fiber; for a dense X one
 * copy per mode in the gather precision with every mode-m fiber
 * contiguous, prod(dims) * (element size) bytes each), computes the
 * leverage scores of every initial factor (Alg. 3, first loop) and, if
 * fit_samples > 0, draws the stratified fit sample once (Sec. 6.4).
 * factors: host array of `order` device pointers, each n_m x R FP64,
 * caller-owned, must outlive the context.  hip_stream: hipStream_t (may be
 * NULL for the default stream).  alloc: device memory provider (NULL:
 * hipMalloc); it must outlive the context.  Synchronizes the stream before returning;
 * X may be freed afterwards.  Errors: CPAL_E_ARG (bad sizes/options/null),
 * CPAL_E_NOMEM, CPAL_E_DEVICE, CPAL_E_STATE (an all-zero factor). */
cpal_status cp_arls_lev_init(const cpal_tensor *X, const cpal_options *opt,
                             double *const *factors, void *hip_stream,
                             const cpal_allocator *alloc, cpal_ctx **out);

/* One mode update of Alg. 3 for mode `mode`: SkrpLev (Alg. 1) over the
 * cached leverage of the other modes -- deterministic rows with p > tau
 * (Sec. 5.3), random rows by per-mode Philox draws (Lemma 5.3, Alg. 2) with
 * rejection of p > tau, repeats combined (Sec. 4.1, 4.3) -- then the sampled
 * fibers (Sec. 6.3), the weighted normal equations G_s = Z~^T Z~,
 * M = X~^T Z~ and A_k = M G_s^{-1} (pseudo-inverse if singular) written to
 * factors[mode], and the leverage of the new A_k.  The step counter t (the
 * third Philox counter word) increments by one per call.  stats_dev: device
 * pointer to one cpal_mode_stats, or NULL.  Asynchronous; errors:
 * CPAL_E_ARG (mode out of range), CPAL_E_STATE (context failed earlier),
 * CPAL_E_DEVICE. */
cpal_status cp_arls_lev_mode_update(cpal_ctx *ctx, int32_t mode, cpal_mode_stats *stats_dev);

/* Estimated fit 1 - sqrt(F^)/||X|| (Sec. 6.4) with the fit sample drawn at
 * init, from the current factors.  fit_dev: device pointer to one double.
 * CPAL_E_STATE if the context was created with fit_samples = 0. */
cpal_status cp_arls_lev_fit_estimate(cpal_ctx *ctx, double *fit_dev);

/* The output (idx, wgt, s_bar) of SkrpLev (Alg. 1) for the last mode update:
 * linear indices of the sampled KRP rows (eq. (2.2), 0-based), omega
 * (= weight^2, the combined-row weights of Sec. 4.1 and 4.3) and weights;
 * deterministic rows first (ascending), then combined random rows
 * (ascending).  Copies min(s_bar, cap) rows; *count_dev = s_bar.
 * Asynchronous.  CPAL_E_STATE before the first update and after
 * cp_arls_lev_autotune (whose trial samples are not an update's) until the
 * next update.  Exists so that callers can audit the sketch. */
cpal_status cp_arls_lev_samples(const cpal_ctx *ctx, uint64_t *idx_dev, double *omega_dev,
                                double *w_dev, int64_t cap, int64_t *count_dev);

/* Exact fit 1 - ||X - M|| / ||X|| (eq. (6.1)) of the current factors, with
 * ||X - M||^2 = ||X||^2 - 2 <X, M> + sum_{r,r'} prod_m (A_m^T A_m)(r,r'):
 * <X, M> is summed over every stored entry (dense: every entry) from the
 * per-mode copy of the mode with the fewest rows (a dense BF16 context holds
 * only BF16 copies, so its exact fit is that of the BF16-rounded tensor).
 * The sums are blocked in a fixed order, so the result does not vary from
 * run to run.  fit_dev: device pointer to one double.  Asynchronous. */
cpal_status cp_arls_lev_fit_exact(cpal_ctx *ctx, double *fit_dev);

/* Options of the full CP-ARLS-LEV loop (Alg. 3). */
typedef struct {
  int32_t eta;          /* outer iterations per epoch, >= 1 (Alg. 3 default 5)           */
  int32_t pi;           /* consecutive epochs without improvement that end the run, >= 1
                           (default 3)                                                   */
  double tol;           /* an epoch improves when its fit exceeds the best earlier fit by
                           more than tol (>= 0; default 1e-4)                            */
  int32_t max_epochs;   /* upper bound on the epochs run, >= 1                           */
  int32_t exact_fit;    /* 0: the estimated fit of Sec. 6.4 (needs fit_samples > 0);
                           1: the exact fit (cp_arls_lev_fit_exact)                      */
} cpal_run_options;

typedef struct {
  int32_t epochs;          /* epochs run (entries of the fit trace)                      */
  int32_t stopped;         /* 1: pi epochs in a row did not improve; 0: max_epochs hit   */
  double best_fit;         /* largest fit in the trace                                   */
  double final_exact_fit;  /* exact fit of the final factors; with exact_fit = 0, the
                              trace minus (last trace entry - this) is the bias-corrected
                              fit trace of Sec. 7                                        */
} cpal_run_result;

/* CP-ARLS-LEV (Alg. 3) from the context's current state: epochs of eta outer
 * iterations, each iteration one mode update of every mode in ascending
 * order; after each epoch the fit (estimated or exact) is taken and copied to
 * the host; the run ends when pi consecutive epochs fail to improve on the
 * best earlier fit by more than tol, or after max_epochs.  fit_trace_host:
 * host array of max_epochs doubles (the fit after each epoch); res_host: the
 * outcome.  Factors are updated in place; the step counter advances by one
 * per mode update.  Synchronizes the stream once per epoch.  Errors:
 * CPAL_E_ARG (bad options or null pointers), CPAL_E_STATE (estimated fit
 * without a fit sample, or a failed context), CPAL_E_DEVICE. */
cpal_status cp_arls_lev_run(cpal_ctx *ctx, const cpal_run_options *opts, double *fit_trace_host,
                            cpal_run_result *res_host);

/* Copy the cached leverage scores (Def. 3.4) of a mode: n_mode doubles. */
cpal_status cp_arls_lev_leverage(const cpal_ctx *ctx, int32_t mode, double *lev_dev);

/* Recompute the cached leverage of `mode` from the current factors[mode]
 * (call after the caller changed a factor matrix). */
cpal_status cp_arls_lev_refresh(cpal_ctx *ctx, int32_t mode);

/* Get / set the step counter t used in the Philox counter of the next update. */
cpal_status cp_arls_lev_get_step(const cpal_ctx *ctx, uint64_t *t_host);
cpal_status cp_arls_lev_set_step(cpal_ctx *ctx, uint64_t t);

/* Stages of a mode update timed by cp_arls_lev_stage_times. */
enum {
  CPAL_STAGE_SAMPLE = 0,   /* deterministic + random rows, combining (Alg. 1, 2)  */
  CPAL_STAGE_ROWS = 1,     /* weights, KRP rows, fiber probes, G_s partials       */
  CPAL_STAGE_GATHER = 2,   /* fiber gather + sampled MTTKRP (Sec. 6.3)            */
  CPAL_STAGE_SOLVE = 3,    /* G_s factorization and A_k = M G_s^{-1}              */
  CPAL_STAGE_LEVERAGE = 4, /* leverage scores and CDF of the new A_k (Def. 3.4)   */
  CPAL_NSTAGES = 5
};

/* Record HIP events around the stages of each mode update on the context's
 * stream: stage_mask bit s times stage s (CPAL_TIMING_ALL: every stage, 0:
 * none, the default).  Each timed stage adds two event records per update.
 * Profiling aid. */
#define CPAL_TIMING_ALL ((1 << CPAL_NSTAGES) - 1)
cpal_status cp_arls_lev_set_timing(cpal_ctx *ctx, int32_t stage_mask);

/* Synchronizes the stream and returns, per stage, the summed duration in
 * milliseconds (ms_host[CPAL_NSTAGES]) and the number of timed updates
 * (count_host[CPAL_NSTAGES]) since the last reset; reset != 0 clears them. */
cpal_status cp_arls_lev_stage_times(cpal_ctx *ctx, double *ms_host, int64_t *count_host,
                                    int32_t reset);

/* Launch shape of the fiber gather + sampled MTTKRP of mode k (Sec. 6.3):
 * grid = workgroups (0: the library's default), sort_min = the segmented
 * gather (modes of at most 2^20 rows) keeps the nonzeros of a 2048-position
 * chunk in stream order instead of sorting them by row when the chunk spans
 * at most sort_min sampled fibers (0: always sort); sort_min = -1 selects the
 * bucketed gather instead (modes of at most 2^20 rows): the sampled nonzeros
 * are first moved into 4096 buckets of consecutive output rows, so that the
 * adds of different fibers to one row are summed on chip (it allocates 16
 * bytes per stored nonzero plus 48 MB on first use).  sort_min = -2 selects
 * the owner gather (modes of at most 2^20 rows; grid unused): no atomic
 * operation, each workgroup alone forms a block of rows of one of 8 partial
 * copies of M from its part of the sampled fibers, and the copies are added
 * in a fixed order, so the update's result does not depend on timing (it
 * allocates 4 bytes per sample and row block).  sort_min = -3 selects the
 * tile gather (grid unused; modes of 1024 to 2^20 rows cut into 32 to 1023
 * blocks of up to 512 rows): workgroup (row block, fiber part) adds the
 * block's segment of each of its fibers into an FP64 block of M in shared
 * memory and stores the block into one of the 8 copies (it allocates 4 bytes
 * per sample and row block).  sort_min = -4 selects the bucketed gather with
 * shared-memory buckets (grid unused; modes of at least 1024 rows, buckets of
 * up to 512 rows, at most 2048 of them; the bucketed gather's buffers): each bucket's records are
 * added into an FP64 block in shared memory slice by slice, and each slice's
 * block into M.  sort_min = -5 selects the hybrid of the two (grid = the
 * long-fiber factor f in [0, 256], 0: 16; both gathers' limits and
 * buffers): fibers of at least f times the tile gather's row-block count
 * nonzeros go through the tile gather, the others through the shared-block
 * bucketed gather.  FP64 contexts start on the owner gather for every such
 * mode, which makes their updates bit-for-bit reproducible; the segmented,
 * bucketed and tile gathers add with atomics and their sums are in a
 * timing-dependent order.  Dense tensors: grid = workgroups along the
 * sampled fibers of the split contraction (each writes one partial M; at
 * most the default, which get_gather_config reports; sort_min unused).
 * Results do not depend on either beyond the rounding order of the FP32/FP64
 * sums.  Host-side setting, takes effect at the next mode update; grid in
 * [0, 2^20] (dense: [0, default]), sort_min >= -5 (-1 to -5 only for sparse
 * modes within the limits above), else CPAL_E_ARG; CPAL_E_NOMEM if the
 * chosen gather's buffers cannot be allocated. */
cpal_status cp_arls_lev_set_gather_config(cpal_ctx *ctx, int32_t k, int32_t grid,
                                          int32_t sort_min);
/* The launch shape mode k uses (grid_host: the effective workgroup count). */
cpal_status cp_arls_lev_get_gather_config(const cpal_ctx *ctx, int32_t k, int32_t *grid_host,
                                          int32_t *sort_min_host);

/* Autotuner of the gather launch shapes: for every mode, builds the sampled
 * system of an update of that mode at the current step (sampling, KRP rows,
 * fiber probes; the factors, leverage scores and step counter are left as
 * they were), times the gather over a fixed set of grids (and, for the
 * segmented gather, sort thresholds, the bucketed, owner, tile,
 * shared-block bucketed and hybrid (f = 8, 16, 32) gathers, whose buffers it
 * allocates where they fit;
 * for dense tensors the default split of the sampled fibers and 1/2, 1/4,
 * 1/8 of it) with HIP events, best of `reps` runs each (0: 2, at most 16;
 * every candidate once per round, so that clock changes during the trials
 * affect all alike),
 * and keeps the fastest shape for the mode, a later candidate replacing an
 * earlier one only when at least 3% faster (in FP64 contexts a shape other
 * than the owner gather gives up bit-for-bit reproducibility for speed).  Every trial samples at the current step; afterwards the step
 * counter, factors and leverage scores are as before, and
 * cp_arls_lev_samples reports CPAL_E_STATE until the next mode update.
 * Synchronizes the stream and is not graph-capturable. */
cpal_status cp_arls_lev_autotune(cpal_ctx *ctx, int32_t reps);

/* Randomized range finder initialisation (App. F): overwrites every factor
 * matrix (the caller's buffers given at init) with A_k = the sum over s_init
 * draws of a mode-k fiber times that draw's row of omega_dev[k]; the fibers
 * are drawn uniformly with replacement from the fibers holding a nonzero
 * (every fiber of a dense tensor), fiber u being the u-th in ascending
 * linear index of its other-mode coordinates and u = floor(U nfib / 2^128)
 * for the Philox4x64-10 block at counter (j, k << 8 | 3 << 16, 0, 0) under
 * the context's (seed, stream_id).  omega_dev: host array of order device
 * pointers, each an s_init x R FP64 row-major matrix (the caller's Gaussian
 * draws).  The products and sums run through the mode's gather in its
 * precision and launch shape; leverage scores and FP32 mirrors are
 * refreshed, the step counter is unchanged.  Allocates (and frees) the
 * fiber lists of the largest mode through the context's provider and
 * synchronizes the stream.  CPAL_E_ARG: s_init outside [1, samples], null
 * pointers; CPAL_E_NOMEM; CPAL_E_DEVICE. */
cpal_status cp_arls_lev_rrf_init(cpal_ctx *ctx, int64_t s_init, const double *const *omega_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * leverage scores of the rows of an n x R FP64 row-major matrix A_dev (device
 * memory), written to lev_dev (n doubles, device memory), computed by the
 * same kernels and in the same order as the scores a context keeps for its
 * factor matrices (cp_arls_lev_leverage returns the same bits for the same
 * matrix).  No context and no allocation: the kernels' scratch (Gram
 * partials per 256-row block, the decomposition, per-row weights) lives in a
 * static 16 MiB device array per GPU, held until the process ends, whose
 * address is looked up on the first call on each GPU.  Work is enqueued on
 * hip_stream (NULL: the default stream); the caller synchronizes.  Every
 * call on one GPU shares that array, so calls that overlap on one GPU (on
 * different streams or host threads) race and must be serialized by the
 * caller.  CPAL_E_ARG for null pointers, n < 1, R outside [1, 64], or a
 * matrix whose scratch exceeds the array (about 2^17 rows at R = 64, more at
 * smaller R); CPAL_E_DEVICE for a launch failure; the message is available
 * from cp_arls_lev_last_error(NULL) on the calling thread. */
cpal_status cp_arls_lev_leverage_noalloc(const double *A_dev, int64_t n, int32_t R,
                                         double *lev_dev, void *hip_stream);

/* Text of the last error on this context (never NULL); with ctx = NULL, the
 * last error of cp_arls_lev_leverage_noalloc on the calling thread. */
const char *cp_arls_lev_last_error(const cpal_ctx *ctx);

/* Free everything the library allocated for the context (synchronizes). */
void cp_arls_lev_destroy(cpal_ctx *ctx);

/* ---------------------------------------------------------------- batches
 * Many independent decompositions (random restarts, tensors of different
 * shape, order and rank): n decompositions over m tensors, decomposition i
 * of tensor tensor_of[i] with options opts[i] and factors factors[i] (host
 * array of that tensor's order device pointers, as for cp_arls_lev_init).
 * Decompositions of one tensor with the same gather precision share its
 * per-mode fiber index (or dense copies), built once.  The batch runs its
 * decompositions on a few streams of its own (default priority) so that
 * their kernels overlap; every batch call is ordered after the work already
 * enqueued on hip_stream and work enqueued on hip_stream afterwards runs
 * after it.  alloc as for cp_arls_lev_init (every member context and the
 * batch's own buffers use it).  Errors as for cp_arls_lev_init; on error
 * nothing is created. */
typedef struct cpal_batch cpal_batch;

cpal_status cp_arls_lev_init_batch(int32_t m, const cpal_tensor *Xs, int32_t n,
                                   const int32_t *tensor_of, const cpal_options *opts,
                                   double *const *const *factors, void *hip_stream,
                                   const cpal_allocator *alloc, cpal_batch **out);

/* One mode update (cp_arls_lev_mode_update) of mode `mode` in every
 * decomposition whose tensor has more than `mode` modes.  stats_dev: device
 * array of n cpal_mode_stats, or NULL.  Returns the first error met. */
cpal_status cp_arls_lev_mode_step_batch(cpal_batch *batch, int32_t mode,
                                        cpal_mode_stats *stats_dev);

/* cp_arls_lev_fit_estimate of every decomposition into fits_dev[0..n). */
cpal_status cp_arls_lev_fit_estimate_batch(cpal_batch *batch, double *fits_dev);

/* on = 1 or 2: from now on every cp_arls_lev_mode_step_batch of a mode
 * replays one HIP graph holding that mode's update of every decomposition,
 * captured on the first such call (the step counter t lives in device
 * memory, so a replay samples with the next t; statistics are copied to
 * stats_dev after the replay; stage timing is not recorded in replays).
 *   on = 1: each decomposition's kernels as a branch of the graph (the
 *           decompositions spread over the batch's streams);
 *   on = 2: stage-major: the kernels of one stage of all decompositions run
 *           as one launch where the kernel has a batched form (sampling,
 *           KRP rows, gather preparation, segmented gather, Gram matrix
 *           and solve, leverage), each workgroup finding its decomposition
 *           in a table of launch arguments the capture writes to device
 *           memory (allocated with the batch's allocator, freed when the
 *           graph is dropped); other kernels (the bucketed, owner and tile
 *           gathers, dense contractions) run per decomposition beside them.
 *           Results equal those of on = 1 (same kernels, same arguments).
 * on = 0 launches the kernels of every step again.  Changing a
 * decomposition's options afterwards is not supported.  CPAL_E_ARG for
 * other values of on. */
cpal_status cp_arls_lev_batch_set_graphs(cpal_batch *batch, int32_t on);

/* Kernel launches in the captured graph of `mode` (kind 1: graph of
 * branches, kind 2: stage-major), 0 while none is captured. */
cpal_status cp_arls_lev_batch_graph_kernels(const cpal_batch *batch, int32_t kind, int32_t mode,
                                            int64_t *kernels);

/* cp_arls_lev_autotune for the first decomposition of every tensor; the
 * other decompositions of that tensor take its launch shapes.  Then, per
 * mode, the gather stage of all decompositions is timed together as
 * stage-major launches (as the stage-major graph runs it), once with those
 * shapes and once with the shared-block bucketed gather (sort_min -4) in
 * every mode that takes it; the latter is kept when at least 3% faster.  The
 * timing runs one more sampling pass per mode (factors unchanged, step
 * counters restored; cp_arls_lev_samples is invalid until the next mode
 * update).  Graphs captured earlier are dropped (the next graph step
 * captures again).  Synchronizes the batch's streams. */
cpal_status cp_arls_lev_autotune_batch(cpal_batch *batch, int32_t reps);

/* The context of decomposition i (for samples, leverage, step counter and
 * error text); owned by the batch, valid until cp_arls_lev_destroy_batch. */
cpal_status cp_arls_lev_batch_ctx(const cpal_batch *batch, int32_t i, cpal_ctx **ctx);

/* Synchronize the batch's streams and free everything it allocated. */
void cp_arls_lev_destroy_batch(cpal_batch *batch);

#ifdef __cplusplus
}
#endif
#endif /* CP_ARLS_LEV_H */
