/*
 * CPU oracle for the CP-ARLS-LEV mode update (Larsen & Kolda, "Practical
 * Leverage-Based Sampling for Low-Rank Tensor Decomposition").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a slow, plain FP64 reference used by the
 * test-suite, the smoke check and the CPU baseline of the benchmark.  The
 * product library never links, loads or calls it, and it shares no code,
 * header or table with the GPU library.
 *
 * All buffers are host memory.  Matrices are row-major n x R doubles.
 * Tensor coordinates are 0-based int32, structure-of-arrays [order][nnz].
 */
#ifndef CPAL_ORACLE_H
#define CPAL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FLAG_PINV = 1, ORC_FLAG_DETCAP = 2, ORC_FLAG_DET_TRUNC = 4,
       ORC_FLAG_PDET_ONE = 8, ORC_FLAG_DRAWCAP = 16 };

typedef struct {
  int32_t order;
  const int64_t *dims;     /* order entries */
  int64_t nnz;
  const int32_t *coords;   /* [order][nnz] */
  const double *vals;      /* nnz */
} orc_tensor;

typedef struct {
  int32_t rank;
  int64_t samples;
  double tau;
  uint64_t seed;
  uint64_t stream_id;
  int64_t det_cap;
  int32_t sampling;   /* 0 leverage scores, 1 uniform, 2 length squared (App. B) */
  int32_t pad;
} orc_opts;

typedef struct {
  int64_t s_det, s_rnd, s_bar, draws, gathered_nnz;
  double p_det;
  int32_t flags;
  int32_t pad;
} orc_stats;

typedef struct orc_index orc_index;

/* Threads of the oracle's independent loops (default 1); the results do not
 * depend on the thread count. */
void orc_set_threads(int32_t n);
int32_t orc_get_threads(void);

/* Philox4x64-10 block function (Salmon et al., SC'11). */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
/* floor(U * W / 2^128) for U = u1*2^64 + u0. */
uint64_t orc_scale128(uint64_t u0, uint64_t u1, uint64_t W);
/* smallest i with C[i] > v (C nondecreasing, v < C[n-1]). */
int64_t orc_upper_bound(const uint64_t *C, int64_t n, uint64_t v);

/* Gram matrix in the blocked summation order; G is R x R. */
void orc_gram(const double *A, int64_t n, int32_t R, double *G);
/* Leverage scores of A's rows; returns flags (ORC_FLAG_PINV when the
 * pseudo-inverse fallback was used). */
int32_t orc_leverage(const double *A, int64_t n, int32_t R, double *lev);
/* Integer sampling weights, inclusive CDF and probabilities; returns W. */
uint64_t orc_sampling_vectors(const double *lev, int64_t n, int32_t R,
                              uint64_t *w, uint64_t *C, double *q);

/* Row scores of the sampling distributions of App. B: kind 1 uniform (every
 * score 1), kind 2 length squared (||A(i,:)||^2); returns their total
 * (n, or the trace of orc_gram's blocked Gram matrix). */
double orc_scores(const double *A, int64_t n, int32_t R, int32_t kind, double *score);
/* As orc_sampling_vectors with the scores normalised by S instead of R. */
uint64_t orc_sampling_vectors_norm(const double *score, int64_t n, double S,
                                   uint64_t *w, uint64_t *C, double *q);

/* Per-mode fiber index (sorted complement keys). */
orc_index *orc_index_build(const orc_tensor *X);
void orc_index_free(orc_index *ix);

/* Deterministic set for update of mode k from the probability vectors of all
 * modes (q[m] of length dims[m]; q[k] is ignored).  Writes up to cap linear
 * indices (ascending) and their probabilities; returns s_det, sets *p_det and
 * *flags.  A return of -1 means cap was too small. */
int64_t orc_det_set(int32_t order, const int64_t *dims, const double *const *q,
                    int32_t k, int64_t s, double tau, int64_t det_cap,
                    uint64_t *idx, double *p, int64_t cap,
                    double *p_det, int32_t *flags);

/* One mode update.  factors[m] are n_m x R; factors[k] is overwritten.
 * idx/omega/wgt receive the s_bar sampled rows (det ascending, then random
 * unique ascending); raw_rnd (nullable) receives the s_rnd accepted random
 * draws in draw order.  Capacities are samples entries each.
 * Returns 0 on success, nonzero on argument/state error. */
int32_t orc_mode_update(const orc_tensor *X, const orc_index *ix,
                        double *const *factors, const orc_opts *opt,
                        int32_t k, uint64_t t,
                        uint64_t *idx, double *omega, double *wgt,
                        uint64_t *raw_rnd, orc_stats *st);

/* Model entry sum_r prod_m A_m(i_m, r). */
double orc_model_entry(int32_t order, double *const *factors, int32_t R,
                       const int32_t *coord);
/* Exact fit 1 - ||X - M|| / ||X||. */
double orc_fit_exact(const orc_tensor *X, double *const *factors, int32_t R);

/* Randomized range finder initialisation of mode k (App. F): A (n_k x R) =
 * the sum over s_init uniform draws of nonempty mode-k fibers of the fiber
 * times the draw's row of omega (s_init x R).  Returns the number of
 * nonempty mode-k fibers. */
int64_t orc_rrf_init(const orc_tensor *X, const orc_index *ix, int32_t k, int64_t s_init,
                     const double *omega, int32_t R, uint64_t seed, uint64_t stream_id,
                     double *A);
/* Stratified fit sample: fills sc [order][cap] (row stride cap), sx, sphi; returns the number
 * of entries written (n_nz + n_zero) or -1 on error. */
int64_t orc_fit_sample(const orc_tensor *X, uint64_t seed, uint64_t stream_id,
                       int64_t s_fit, double alpha,
                       int32_t *sc, double *sx, double *sphi, int64_t cap,
                       int32_t *flags);
double orc_fit_estimate(int32_t order, int64_t n_fit, const int32_t *sc, int64_t ld,
                        const double *sx, const double *sphi,
                        double *const *factors, int32_t R, double normX);

#ifdef __cplusplus
}
#endif
#endif
