/*
 * CPU oracle for the CP-ARLS-LEV mode update.
 *
 * TEST INFRASTRUCTURE ONLY: a plain, slow FP64 reference, compiled with
 * -O2 -ffp-contract=off so that every multiply and add rounds separately.
 * Only the tests, the smoke check and the benchmark's CPU baseline use it.
 *
 * Each function names the passage of the paper it follows:
 *   Sec. 2, eqs. (2.1)-(2.2)  KRP rows and the multi-index <-> linear index map
 *   Def. 3.1                  weighted random sampling matrix
 *   Def. 3.4                  leverage scores
 *   Sec. 4.1 eq. (4.1)        combining repeated rows
 *   Sec. 4.2-4.3              hybrid deterministic + random sampling
 *   Lemma 5.3                 per-mode sampling of KRP rows
 *   Sec. 5.3                  deterministic-set candidates and enumeration
 *   Alg. 1, Alg. 2            SkrpLev, random KRP indices with rejection
 *   Alg. 3                    the mode update inside CP-ARLS-LEV
 *   Sec. 6.3                  fiber extraction from a COO tensor
 *   Sec. 6.4                  stratified estimate of the fit
 * Readings where the paper is silent (integer CDF, Philox counters, blocked
 * summation order, tie rules) are fixed here and restated in the design notes.
 */
#include "cpal_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define GRAM_BLOCK 256
#define MAXR 64

/* Threads of the loops below whose iterations are independent (rows of the
 * Gram matrix, leverage rows, blocks of draws, sampled rows, solved rows).
 * Every such loop keeps the summation order of the sequential loop it
 * replaces: any thread count gives the same bits as one thread. */
static int g_threads = 1;

void orc_set_threads(int32_t n) { g_threads = n > 1 ? n : 1; }
int32_t orc_get_threads(void) { return g_threads; }

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox4x64-10, written from the published description   */
/* (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,  */
/* 3", SC'11): ten rounds of two 64x64->128 multiplies with key bumps by    */
/* the Weyl constants.                                                      */
/* ------------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k0 += W0; k1 += W1; }
    unsigned __int128 p0 = (unsigned __int128)M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

uint64_t orc_scale128(uint64_t u0, uint64_t u1, uint64_t W) {
  /* U*W/2^128 with U = u1*2^64 + u0, computed with full 192-bit product. */
  unsigned __int128 a = (unsigned __int128)u0 * W;
  unsigned __int128 b = (unsigned __int128)u1 * W;
  unsigned __int128 mid = (b & 0xFFFFFFFFFFFFFFFFULL) + (a >> 64);
  return (uint64_t)(b >> 64) + (uint64_t)(mid >> 64);
}

int64_t orc_upper_bound(const uint64_t *C, int64_t n, uint64_t v) {
  int64_t lo = 0, hi = n;            /* answer in [lo, hi) */
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (C[mid] > v) hi = mid; else lo = mid + 1;
  }
  return lo;
}

/* Counter layout: (draw j, mode | k<<8 | purpose<<16, step t, 0).
 * purpose 0 = KRP row sampling, 1 = fit nonzero sample, 2 = fit zero sample. */
static void draw_words(uint64_t seed, uint64_t stream, uint64_t j, uint64_t word1,
                       uint64_t t, uint64_t out[4]) {
  uint64_t ctr[4] = {j, word1, t, 0};
  uint64_t key[2] = {seed, stream};
  orc_philox4x64_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Leverage scores (Def. 3.4) through the Gram matrix: for full column rank  */
/* A = Q T, l_i = ||Q(i,:)||^2 = a_i^T (A^T A)^{-1} a_i.  A^T A = L L^T by     */
/* Cholesky; l_i = ||L^{-1} a_i||^2.  Rank-deficient A: l_i = a_i^T G^+ a_i  */
/* with G^+ from a Jacobi eigendecomposition (projection onto range(A)).     */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t R;
  int32_t pinv;
  double L[MAXR * MAXR];     /* Cholesky factor, row-major lower */
  double V[MAXR * MAXR];     /* eigenvectors in columns (pinv)   */
  double lam[MAXR];          /* eigenvalues (pinv)               */
  double etol;
} decomp;

void orc_gram(const double *A, int64_t n, int32_t R, double *G) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(g_threads) if (g_threads > 1)
  for (int a = 0; a < R; ++a) {
    for (int b = a; b < R; ++b) {
      double total = 0.0;
      for (int64_t r0 = 0; r0 < n; r0 += GRAM_BLOCK) {
        int64_t r1 = r0 + GRAM_BLOCK < n ? r0 + GRAM_BLOCK : n;
        double part = 0.0;
        for (int64_t r = r0; r < r1; ++r) {
          double prod = A[r * R + a] * A[r * R + b];
          part = part + prod;
        }
        total = total + part;
      }
      G[a * R + b] = total;
      G[b * R + a] = total;
    }
  }
}

static void jacobi_eig(const double *G, int R, decomp *d) {
  double S[MAXR * MAXR];
  memcpy(S, G, sizeof(double) * R * R);
  for (int i = 0; i < R; ++i)
    for (int j = 0; j < R; ++j) d->V[i * R + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < R - 1; ++p) {
      for (int q = p + 1; q < R; ++q) {
        double apq = S[p * R + q];
        if (apq == 0.0) continue;
        double app = S[p * R + p], aqq = S[q * R + q];
        if (fabs(apq) <= 0x1p-53 * sqrt(fabs(app * aqq))) {
          S[p * R + q] = 0.0; S[q * R + p] = 0.0;
          continue;
        }
        /* rotation angle that annihilates S(p,q): cot(2 phi) = theta */
        double theta = (aqq - app) / (2.0 * apq);
        double t;
        if (fabs(theta) > 0x1p500) {
          t = 0.5 / theta;
        } else {
          t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
          if (theta < 0.0) t = -t;
        }
        double c = 1.0 / sqrt(t * t + 1.0);
        double s = t * c;
        for (int r = 0; r < R; ++r) {
          if (r == p || r == q) continue;
          double srp = S[r * R + p], srq = S[r * R + q];
          double np_ = c * srp - s * srq;
          double nq_ = s * srp + c * srq;
          S[r * R + p] = np_; S[p * R + r] = np_;
          S[r * R + q] = nq_; S[q * R + r] = nq_;
        }
        S[p * R + p] = app - t * apq;
        S[q * R + q] = aqq + t * apq;
        S[p * R + q] = 0.0; S[q * R + p] = 0.0;
        for (int r = 0; r < R; ++r) {
          double vrp = d->V[r * R + p], vrq = d->V[r * R + q];
          d->V[r * R + p] = c * vrp - s * vrq;
          d->V[r * R + q] = s * vrp + c * vrq;
        }
        rotated = 1;
      }
    }
    if (!rotated) break;
  }
  double mx = 0.0;
  for (int j = 0; j < R; ++j) {
    d->lam[j] = S[j * R + j];
    if (fabs(d->lam[j]) > mx) mx = fabs(d->lam[j]);
  }
  d->etol = ((double)R * 0x1p-52) * mx;
}

/* Cholesky G = L L^T (columns ascending, inner sums ascending); falls back to
 * the eigendecomposition when a pivot is not above R*2^-52*max diag. */
static void factorize(const double *G, int R, decomp *d) {
  d->R = R;
  d->pinv = 0;
  double maxdiag = 0.0;
  for (int j = 0; j < R; ++j) if (G[j * R + j] > maxdiag) maxdiag = G[j * R + j];
  double tol = ((double)R * 0x1p-52) * maxdiag;
  memset(d->L, 0, sizeof(d->L));
  for (int j = 0; j < R; ++j) {
    double v = G[j * R + j];
    for (int p = 0; p < j; ++p) v = v - d->L[j * R + p] * d->L[j * R + p];
    if (!(v > tol)) { d->pinv = 1; break; }
    double ljj = sqrt(v);
    d->L[j * R + j] = ljj;
    for (int i = j + 1; i < R; ++i) {
      double u = G[i * R + j];
      for (int p = 0; p < j; ++p) u = u - d->L[i * R + p] * d->L[j * R + p];
      d->L[i * R + j] = u / ljj;
    }
  }
  if (d->pinv) jacobi_eig(G, R, d);
}

/* a^T G^{-1} a (or a^T G^+ a) for one row a. */
static double quad_form(const decomp *d, const double *a) {
  int R = d->R;
  double acc = 0.0;
  if (!d->pinv) {
    double y[MAXR];
    for (int j = 0; j < R; ++j) {
      double v = a[j];
      for (int p = 0; p < j; ++p) v = v - d->L[j * R + p] * y[p];
      y[j] = v / d->L[j * R + j];
    }
    for (int j = 0; j < R; ++j) acc = acc + y[j] * y[j];
  } else {
    for (int j = 0; j < R; ++j) {
      if (!(d->lam[j] > d->etol)) continue;
      double y = 0.0;
      for (int p = 0; p < R; ++p) y = y + d->V[p * R + j] * a[p];
      acc = acc + (y * y) / d->lam[j];
    }
  }
  return acc;
}

/* x = G^{-1} m (or G^+ m) for one right-hand side. */
static void solve_row(const decomp *d, const double *m, double *x) {
  int R = d->R;
  if (!d->pinv) {
    double y[MAXR];
    for (int j = 0; j < R; ++j) {
      double v = m[j];
      for (int p = 0; p < j; ++p) v = v - d->L[j * R + p] * y[p];
      y[j] = v / d->L[j * R + j];
    }
    for (int j = R - 1; j >= 0; --j) {
      double v = y[j];
      for (int p = j + 1; p < R; ++p) v = v - d->L[p * R + j] * x[p];
      x[j] = v / d->L[j * R + j];
    }
  } else {
    double c[MAXR];
    for (int j = 0; j < R; ++j) {
      c[j] = 0.0;
      if (!(d->lam[j] > d->etol)) continue;
      double y = 0.0;
      for (int p = 0; p < R; ++p) y = y + d->V[p * R + j] * m[p];
      c[j] = y / d->lam[j];
    }
    for (int r = 0; r < R; ++r) {
      double v = 0.0;
      for (int j = 0; j < R; ++j) {
        if (!(d->lam[j] > d->etol)) continue;
        v = v + c[j] * d->V[r * R + j];
      }
      x[r] = v;
    }
  }
}

/* Fewer rows than columns (n < R): range(A) is all of R^n exactly when A has
 * full row rank, and then every leverage score is 1 (Def. 3.4 with Q = I_n).
 * Full row rank is decided by a Cholesky of K = A A^T (n x n, entries summed
 * over the R columns in ascending order) with the same pivot test as for
 * A^T A.  Returns 1 when that holds. */
static int full_row_rank(const double *A, int64_t n, int32_t R) {
  double K[MAXR * MAXR];
  for (int i = 0; i < n; ++i) {
    for (int j = i; j < n; ++j) {
      double acc = 0.0;
      for (int r = 0; r < R; ++r) acc = acc + A[(int64_t)i * R + r] * A[(int64_t)j * R + r];
      K[i * n + j] = acc;
      K[j * n + i] = acc;
    }
  }
  double maxdiag = 0.0;
  for (int j = 0; j < n; ++j) if (K[j * n + j] > maxdiag) maxdiag = K[j * n + j];
  const double tol = ((double)n * 0x1p-52) * maxdiag;
  double L[MAXR * MAXR];
  memset(L, 0, sizeof(L));
  for (int j = 0; j < n; ++j) {
    double v = K[j * n + j];
    for (int p = 0; p < j; ++p) v = v - L[j * n + p] * L[j * n + p];
    if (!(v > tol)) return 0;
    double ljj = sqrt(v);
    L[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double u = K[i * n + j];
      for (int p = 0; p < j; ++p) u = u - L[i * n + p] * L[j * n + p];
      L[i * n + j] = u / ljj;
    }
  }
  return 1;
}

int32_t orc_leverage(const double *A, int64_t n, int32_t R, double *lev) {
  double G[MAXR * MAXR];
  if (n < R && full_row_rank(A, n, R)) {
    for (int64_t i = 0; i < n; ++i) lev[i] = 1.0;
    return ORC_FLAG_PINV;   /* A^T A is singular */
  }
  decomp *d = (decomp *)malloc(sizeof(decomp));
  orc_gram(A, n, R, G);
  factorize(G, R, d);
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)
  for (int64_t i = 0; i < n; ++i) {
    double l = quad_form(d, A + i * R);
    lev[i] = l > 0.0 ? l : 0.0;
  }
  int32_t flags = d->pinv ? ORC_FLAG_PINV : 0;
  free(d);
  return flags;
}

/* Normalised leverage p_k = l(A_k)/r (Sec. 5.3) held as integers: w_i =
 * floor(2^52 * l_i / R), W = sum w, C = inclusive prefix, q_i = w_i / W. */
uint64_t orc_sampling_vectors(const double *lev, int64_t n, int32_t R,
                              uint64_t *w, uint64_t *C, double *q) {
  return orc_sampling_vectors_norm(lev, n, (double)R, w, C, q);
}

/* The other row distributions of App. B: uniform, and length squared, whose
 * total ||A||_F^2 is the trace of the Gram matrix in orc_gram's order. */
double orc_scores(const double *A, int64_t n, int32_t R, int32_t kind, double *score) {
  if (kind == 1) {
    for (int64_t i = 0; i < n; ++i) score[i] = 1.0;
    return (double)n;
  }
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int c = 0; c < R; ++c) acc = acc + A[i * R + c] * A[i * R + c];
    score[i] = acc;
  }
  double G[MAXR * MAXR];
  orc_gram(A, n, R, G);
  double S = 0.0;
  for (int j = 0; j < R; ++j) S = S + G[j * R + j];
  return S;
}

uint64_t orc_sampling_vectors_norm(const double *lev, int64_t n, double S,
                                   uint64_t *w, uint64_t *C, double *q) {
  uint64_t W = 0;
  for (int64_t i = 0; i < n; ++i) {
    double v = S > 0.0 ? lev[i] / S : 0.0;
    if (!(v > 0.0)) v = 0.0;
    if (v > 1.0) v = 1.0;
    w[i] = (uint64_t)(v * 0x1p52);
    W += w[i];
    C[i] = W;
  }
  for (int64_t i = 0; i < n; ++i) q[i] = W ? (double)w[i] / (double)W : 0.0;
  return W;
}

/* ------------------------------------------------------------------------ */
/* Tensor fibers (Sec. 6.3): for mode k every nonzero gets the linear index */
/* of its other-mode coordinates (eq. (2.2), 0-based, first other mode       */
/* fastest).  The oracle keeps, per mode, the nonzero ids sorted by that key */
/* and finds a fiber by binary search.                                       */
/* ------------------------------------------------------------------------ */
struct orc_index {
  int32_t order;
  int64_t nnz;
  uint64_t *key[16];   /* sorted complement keys per mode */
  int64_t *id[16];     /* nonzero id per sorted position  */
  uint64_t *full;      /* sorted full linear indices      */
};

typedef struct { uint64_t key; int32_t ik; int64_t id; } keyrec;

static int cmp_keyrec(const void *a, const void *b) {
  const keyrec *x = (const keyrec *)a, *y = (const keyrec *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->ik != y->ik) return x->ik < y->ik ? -1 : 1;
  return 0;
}

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

static uint64_t complement_key(const orc_tensor *X, int k, int64_t e) {
  uint64_t key = 0, stride = 1;
  for (int m = 0; m < X->order; ++m) {
    if (m == k) continue;
    key += (uint64_t)X->coords[(int64_t)m * X->nnz + e] * stride;
    stride *= (uint64_t)X->dims[m];
  }
  return key;
}

orc_index *orc_index_build(const orc_tensor *X) {
  if (X->order < 2 || X->order > 16) return NULL;
  orc_index *ix = (orc_index *)calloc(1, sizeof(orc_index));
  ix->order = X->order;
  ix->nnz = X->nnz;
  keyrec *tmp = (keyrec *)malloc(sizeof(keyrec) * (X->nnz ? X->nnz : 1));
  for (int k = 0; k < X->order; ++k) {
    for (int64_t e = 0; e < X->nnz; ++e) {
      tmp[e].key = complement_key(X, k, e);
      tmp[e].ik = X->coords[(int64_t)k * X->nnz + e];
      tmp[e].id = e;
    }
    qsort(tmp, X->nnz, sizeof(keyrec), cmp_keyrec);
    ix->key[k] = (uint64_t *)malloc(sizeof(uint64_t) * (X->nnz ? X->nnz : 1));
    ix->id[k] = (int64_t *)malloc(sizeof(int64_t) * (X->nnz ? X->nnz : 1));
    for (int64_t e = 0; e < X->nnz; ++e) { ix->key[k][e] = tmp[e].key; ix->id[k][e] = tmp[e].id; }
  }
  free(tmp);
  ix->full = (uint64_t *)malloc(sizeof(uint64_t) * (X->nnz ? X->nnz : 1));
  for (int64_t e = 0; e < X->nnz; ++e) {
    uint64_t key = 0, stride = 1;
    for (int m = 0; m < X->order; ++m) {
      key += (uint64_t)X->coords[(int64_t)m * X->nnz + e] * stride;
      stride *= (uint64_t)X->dims[m];
    }
    ix->full[e] = key;
  }
  qsort(ix->full, X->nnz, sizeof(uint64_t), cmp_u64);
  return ix;
}

void orc_index_free(orc_index *ix) {
  if (!ix) return;
  for (int k = 0; k < ix->order; ++k) { free(ix->key[k]); free(ix->id[k]); }
  free(ix->full);
  free(ix);
}

static int64_t lower_bound_u64(const uint64_t *a, int64_t n, uint64_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

/* ------------------------------------------------------------------------ */
/* Deterministic set (Sec. 5.3, and the DetSkrp step of Alg. 1).            */
/* p of a multi-index is the product of the per-mode q's, taken in ascending */
/* mode order.  A row i_m of mode m can belong to a combination with p > tau */
/* only if the product with every other mode at its maximum alpha exceeds   */
/* tau (the paper's test q > tau*alpha_m/alpha_* with both sides multiplied  */
/* by alpha_star over alpha_m; rounding is monotone so the test is exact).  */
/* ------------------------------------------------------------------------ */
typedef struct { uint64_t lin; double p; } detrec;

static int cmp_det_lin(const void *a, const void *b) {
  const detrec *x = (const detrec *)a, *y = (const detrec *)b;
  return x->lin < y->lin ? -1 : (x->lin > y->lin ? 1 : 0);
}
static int cmp_det_p_desc(const void *a, const void *b) {
  const detrec *x = (const detrec *)a, *y = (const detrec *)b;
  if (x->p != y->p) return x->p > y->p ? -1 : 1;
  return x->lin < y->lin ? -1 : (x->lin > y->lin ? 1 : 0);
}

static double blocked_sum(const double *v, int64_t n) {
  double total = 0.0;
  for (int64_t b0 = 0; b0 < n; b0 += GRAM_BLOCK) {
    int64_t b1 = b0 + GRAM_BLOCK < n ? b0 + GRAM_BLOCK : n;
    double part = 0.0;
    for (int64_t i = b0; i < b1; ++i) part = part + v[i];
    total = total + part;
  }
  return total;
}

int64_t orc_det_set(int32_t order, const int64_t *dims, const double *const *q,
                    int32_t k, int64_t s, double tau, int64_t det_cap,
                    uint64_t *idx, double *p, int64_t cap,
                    double *p_det, int32_t *flags) {
  *p_det = 0.0;
  if (!(tau < 1.0)) return 0;
  int O[16], d = 0;
  for (int m = 0; m < order; ++m) if (m != k) O[d++] = m;
  double alpha[16];
  for (int t = 0; t < d; ++t) {
    int m = O[t];
    alpha[t] = 0.0;
    for (int64_t i = 0; i < dims[m]; ++i) if (q[m][i] > alpha[t]) alpha[t] = q[m][i];
  }
  int64_t *cand[16];
  int64_t ncand[16];
  double combos = 1.0;
  for (int t = 0; t < d; ++t) {
    int m = O[t];
    cand[t] = (int64_t *)malloc(sizeof(int64_t) * (dims[m] ? dims[m] : 1));
    ncand[t] = 0;
    for (int64_t i = 0; i < dims[m]; ++i) {
      double b = (t == 0) ? q[m][i] : alpha[0];
      for (int u = 1; u < d; ++u) b = b * ((u == t) ? q[m][i] : alpha[u]);
      if (b > tau) cand[t][ncand[t]++] = i;
    }
    combos *= (double)ncand[t];
  }
  int64_t ndet = 0;
  if (combos > (double)det_cap) {
    *flags |= ORC_FLAG_DETCAP;
    for (int t = 0; t < d; ++t) free(cand[t]);
    return 0;
  }
  int64_t ncombo = (int64_t)combos;
  int64_t reccap = 1024;
  detrec *rec = (detrec *)malloc(sizeof(detrec) * reccap);
  int64_t c[16];
  for (int64_t e = 0; e < ncombo; ++e) {
    int64_t rem = e;
    for (int t = 0; t < d; ++t) { c[t] = rem % ncand[t]; rem /= ncand[t]; }
    double pr = q[O[0]][cand[0][c[0]]];
    for (int t = 1; t < d; ++t) pr = pr * q[O[t]][cand[t][c[t]]];
    if (pr > tau) {
      uint64_t lin = 0, stride = 1;
      for (int t = 0; t < d; ++t) { lin += (uint64_t)cand[t][c[t]] * stride; stride *= (uint64_t)dims[O[t]]; }
      if (ndet == reccap) { reccap *= 2; rec = (detrec *)realloc(rec, sizeof(detrec) * reccap); }
      rec[ndet].lin = lin;
      rec[ndet].p = pr;
      ndet++;
    }
  }
  for (int t = 0; t < d; ++t) free(cand[t]);
  if (ndet >= s) {
    /* more than s rows above tau: keep the s most probable (Alg. 1 notes) */
    qsort(rec, ndet, sizeof(detrec), cmp_det_p_desc);
    ndet = s;
    *flags |= ORC_FLAG_DET_TRUNC;
  }
  qsort(rec, ndet, sizeof(detrec), cmp_det_lin);
  if (ndet > cap) { free(rec); return -1; }
  double *pv = (double *)malloc(sizeof(double) * (ndet ? ndet : 1));
  for (int64_t i = 0; i < ndet; ++i) { idx[i] = rec[i].lin; p[i] = rec[i].p; pv[i] = rec[i].p; }
  *p_det = blocked_sum(pv, ndet);
  free(pv);
  free(rec);
  return ndet;
}

/* ------------------------------------------------------------------------ */
/* One CP-ARLS-LEV mode update (Alg. 3 inner loop body): SkrpLev (Alg. 1,    */
/* Alg. 2, Sec. 4), KrpSamp, TnsrSamp (Sec. 6.3) and the sampled least       */
/* squares solve, here through the weighted normal equations                 */
/*   G_s = sum_j omega_j z_j z_j^T,  M = sum_j omega_j x_j z_j^T,             */
/*   A_k = M G_s^{-1}, with omega_j = wgt_j^2.                               */
/* ------------------------------------------------------------------------ */
/* The sampled normal equations G = sum_j omega_j z_j z_j^T and
 * M = sum_j omega_j X~(j,:)^T z_j^T with several threads and the sums of
 * the sequential loop: the KRP rows and fiber ranges of the sampled rows are
 * found in parallel, every gathered nonzero is listed as (row i_k, sample j,
 * entry), the list is sorted by i_k stably (so j ascends within a row), and
 * each row of M, like each row of G, is summed by one thread in ascending j.
 * Returns nnz(X~). */
static int64_t sampled_system_threads(const orc_tensor *X, const orc_index *ix,
                                      double *const *factors, int k, int R, int d,
                                      const int *O, const uint64_t *idx, const double *omega,
                                      int64_t sb, double *G, double *M) {
  const int64_t nk = X->dims[k];
  double *Z = (double *)malloc(sizeof(double) * (size_t)(sb ? sb : 1) * R);
  int64_t *lo = (int64_t *)malloc(sizeof(int64_t) * (size_t)(sb + 1));
  int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(sb + 1));
#pragma omp parallel for schedule(static) num_threads(g_threads)
  for (int64_t j = 0; j < sb; ++j) {
    uint64_t rem = idx[j];
    int64_t im[16];
    for (int u = 0; u < d; ++u) { im[u] = (int64_t)(rem % (uint64_t)X->dims[O[u]]); rem /= (uint64_t)X->dims[O[u]]; }
    for (int r = 0; r < R; ++r) {
      double v = factors[O[0]][im[0] * R + r];
      for (int u = 1; u < d; ++u) v = v * factors[O[u]][im[u] * R + r];
      Z[j * R + r] = v;
    }
    int64_t pos = lower_bound_u64(ix->key[k], X->nnz, idx[j]);
    int64_t end = pos;
    while (end < X->nnz && ix->key[k][end] == idx[j]) end++;
    lo[j] = pos;
    cnt[j] = end - pos;
  }
  int64_t total = 0;
  for (int64_t j = 0; j < sb; ++j) { int64_t c = cnt[j]; cnt[j] = total; total += c; }
  cnt[sb] = total;
  int64_t *rowof = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total ? total : 1));
  int64_t *jof = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total ? total : 1));
  int64_t *eof = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total ? total : 1));
#pragma omp parallel for schedule(static) num_threads(g_threads)
  for (int64_t j = 0; j < sb; ++j)
    for (int64_t q = cnt[j]; q < cnt[j + 1]; ++q) {
      int64_t e = ix->id[k][lo[j] + (q - cnt[j])];
      rowof[q] = X->coords[(int64_t)k * X->nnz + e];
      jof[q] = j;
      eof[q] = e;
    }
  /* stable counting sort of the list by row */
  int64_t *rstart = (int64_t *)calloc((size_t)nk + 1, sizeof(int64_t));
  for (int64_t q = 0; q < total; ++q) rstart[rowof[q] + 1]++;
  for (int64_t i = 0; i < nk; ++i) rstart[i + 1] += rstart[i];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nk ? nk : 1));
  memcpy(fill, rstart, sizeof(int64_t) * (size_t)nk);
  int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total ? total : 1));
  for (int64_t q = 0; q < total; ++q) order[fill[rowof[q]]++] = q;
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads)
  for (int64_t i = 0; i < nk; ++i)
    for (int64_t u = rstart[i]; u < rstart[i + 1]; ++u) {
      const int64_t q = order[u];
      const double ox = omega[jof[q]] * X->vals[eof[q]];
      const double *z = Z + jof[q] * R;
      for (int r = 0; r < R; ++r) M[i * R + r] = M[i * R + r] + ox * z[r];
    }
#pragma omp parallel for schedule(static) num_threads(g_threads)
  for (int a = 0; a < R; ++a)
    for (int64_t j = 0; j < sb; ++j) {
      const double om = omega[j];
      const double *z = Z + j * R;
      for (int b = 0; b < R; ++b) G[a * R + b] = G[a * R + b] + (om * z[a]) * z[b];
    }
  free(Z); free(lo); free(cnt); free(rowof); free(jof); free(eof);
  free(rstart); free(fill); free(order);
  return total;
}

int32_t orc_mode_update(const orc_tensor *X, const orc_index *ix,
                        double *const *factors, const orc_opts *opt,
                        int32_t k, uint64_t t,
                        uint64_t *idx, double *omega, double *wgt,
                        uint64_t *raw_rnd, orc_stats *st) {
  const int D = X->order;
  const int R = opt->rank;
  const int64_t s = opt->samples;
  if (D < 2 || D > 16 || R < 1 || R > MAXR || s < 1 || k < 0 || k >= D) return 1;
  if (!(opt->tau >= 0.0 && opt->tau <= 1.0)) return 1;
  if (opt->sampling < 0 || opt->sampling > 2) return 1;
  memset(st, 0, sizeof(*st));

  /* leverage and sampling vectors of every other mode (Alg. 3 setup) */
  double *q[16] = {0};
  uint64_t *C[16] = {0};
  uint64_t W[16] = {0};
  for (int m = 0; m < D; ++m) {
    if (m == k) continue;
    int64_t n = X->dims[m];
    double *lev = (double *)malloc(sizeof(double) * n);
    uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * n);
    q[m] = (double *)malloc(sizeof(double) * n);
    C[m] = (uint64_t *)malloc(sizeof(uint64_t) * n);
    if (opt->sampling == 0) {
      st->flags |= orc_leverage(factors[m], n, R, lev);
      W[m] = orc_sampling_vectors(lev, n, R, w, C[m], q[m]);
    } else {
      double S = orc_scores(factors[m], n, R, opt->sampling, lev);
      W[m] = orc_sampling_vectors_norm(lev, n, S, w, C[m], q[m]);
    }
    free(lev);
    free(w);
  }
  int32_t rc = 0;
  for (int m = 0; m < D; ++m) if (m != k && W[m] == 0) rc = 2;

  int O[16], d = 0;
  for (int m = 0; m < D; ++m) if (m != k) O[d++] = m;

  uint64_t *didx = (uint64_t *)malloc(sizeof(uint64_t) * s);
  double *dp = (double *)malloc(sizeof(double) * s);
  uint64_t *acc = (uint64_t *)malloc(sizeof(uint64_t) * s);
  double p_det = 0.0;
  int64_t s_det = 0, s_rnd = 0, draws = 0, nacc = 0;
  if (rc == 0) {
    int32_t fl = 0;
    s_det = orc_det_set(D, X->dims, (const double *const *)q, k, s, opt->tau,
                        opt->det_cap, didx, dp, s, &p_det, &fl);
    st->flags |= fl;
    double tau_eff = (fl & ORC_FLAG_DETCAP) ? 1.0 : opt->tau;
    s_rnd = s - s_det;
    if (s_rnd > 0 && !(1.0 - p_det > 0x1p-40)) { s_rnd = 0; st->flags |= ORC_FLAG_PDET_ONE; }

    /* Alg. 2: draw per-mode indices (Lemma 5.3), reject p > tau, keep the
     * first s_rnd accepted in draw order. */
    /* The draws are made in blocks (each draw depends only on its index),
     * then examined in draw order. */
    int64_t guard = 64 * s_rnd + (1 << 20);
    const int64_t DBLK = 1 << 16;
    uint64_t *blin = (uint64_t *)malloc(sizeof(uint64_t) * DBLK);
    double *bpr = (double *)malloc(sizeof(double) * DBLK);
    while (nacc < s_rnd) {
      if (draws >= guard) { st->flags |= ORC_FLAG_DRAWCAP; break; }
      const int64_t nb = guard - draws < DBLK ? guard - draws : DBLK;
      const int64_t j0 = draws;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)
      for (int64_t b = 0; b < nb; ++b) {
        uint64_t lin = 0, stride = 1;
        double pr = 0.0;
        for (int u = 0; u < d; ++u) {
          int m = O[u];
          uint64_t out[4];
          draw_words(opt->seed, opt->stream_id, (uint64_t)(j0 + b),
                     (uint64_t)m | ((uint64_t)k << 8), t, out);
          uint64_t v = orc_scale128(out[0], out[1], W[m]);
          int64_t i = orc_upper_bound(C[m], X->dims[m], v);
          pr = (u == 0) ? q[m][i] : pr * q[m][i];
          lin += (uint64_t)i * stride;
          stride *= (uint64_t)X->dims[m];
        }
        blin[b] = lin;
        bpr[b] = pr;
      }
      for (int64_t b = 0; b < nb && nacc < s_rnd; ++b) {
        draws++;
        if (bpr[b] <= tau_eff) acc[nacc++] = blin[b];
      }
    }
    free(blin);
    free(bpr);
    if (raw_rnd) memcpy(raw_rnd, acc, sizeof(uint64_t) * nacc);
    int64_t s_rnd_used = nacc;  /* == s_rnd unless the draw guard tripped */

    /* Sec. 4.1/4.3: combine repeats; omega = c (1 - p_det) / (s_rnd p). */
    qsort(acc, nacc, sizeof(uint64_t), cmp_u64);
    int64_t sb = 0;
    for (int64_t i = 0; i < s_det; ++i) { idx[sb] = didx[i]; omega[sb] = 1.0; wgt[sb] = 1.0; sb++; }
    for (int64_t i = 0; i < nacc;) {
      int64_t j = i;
      while (j < nacc && acc[j] == acc[i]) j++;
      uint64_t lin = acc[i];
      uint64_t rem = lin;
      double pr = 0.0;
      for (int u = 0; u < d; ++u) {
        int m = O[u];
        uint64_t im = rem % (uint64_t)X->dims[m];
        rem /= (uint64_t)X->dims[m];
        pr = (u == 0) ? q[m][im] : pr * q[m][im];
      }
      double num = (double)(j - i) * (1.0 - p_det);
      double den = (double)s_rnd_used * pr;
      double om = num / den;
      idx[sb] = lin; omega[sb] = om; wgt[sb] = sqrt(om);
      sb++;
      i = j;
    }
    st->s_det = s_det;
    st->s_rnd = s_rnd_used;
    st->s_bar = sb;
    st->draws = draws;
    st->p_det = p_det;

    /* KrpSamp + TnsrSamp + sampled normal equations */
    const int64_t nk = X->dims[k];
    double *M = (double *)calloc((size_t)nk * R, sizeof(double));
    double G[MAXR * MAXR];
    memset(G, 0, sizeof(G));
    int64_t gathered = 0;
    if (g_threads > 1) {
      gathered = sampled_system_threads(X, ix, factors, k, R, d, O, idx, omega, sb, G, M);
    } else {
      for (int64_t j = 0; j < sb; ++j) {
        double z[MAXR];
        uint64_t rem = idx[j];
        int64_t im[16];
        for (int u = 0; u < d; ++u) { im[u] = (int64_t)(rem % (uint64_t)X->dims[O[u]]); rem /= (uint64_t)X->dims[O[u]]; }
        for (int r = 0; r < R; ++r) {
          double v = factors[O[0]][im[0] * R + r];
          for (int u = 1; u < d; ++u) v = v * factors[O[u]][im[u] * R + r];
          z[r] = v;
        }
        double om = omega[j];
        for (int a = 0; a < R; ++a)
          for (int b = 0; b < R; ++b) G[a * R + b] = G[a * R + b] + (om * z[a]) * z[b];
        int64_t pos = lower_bound_u64(ix->key[k], X->nnz, idx[j]);
        for (; pos < X->nnz && ix->key[k][pos] == idx[j]; ++pos) {
          int64_t e = ix->id[k][pos];
          int64_t ik = X->coords[(int64_t)k * X->nnz + e];
          double ox = om * X->vals[e];
          for (int r = 0; r < R; ++r) M[ik * R + r] = M[ik * R + r] + ox * z[r];
          gathered++;
        }
      }
    }
    st->gathered_nnz = gathered;
    decomp *dc = (decomp *)malloc(sizeof(decomp));
    factorize(G, R, dc);
    if (dc->pinv) st->flags |= ORC_FLAG_PINV;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (g_threads > 1)
    for (int64_t i = 0; i < nk; ++i) solve_row(dc, M + i * R, factors[k] + i * R);
    free(dc);
    free(M);
  }
  free(didx); free(dp); free(acc);
  for (int m = 0; m < D; ++m) { free(q[m]); free(C[m]); }
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Randomized range finder initialisation (App. F): the columns of A_k are  */
/* random linear combinations of mode-k fibers.  s_init fibers are drawn    */
/* uniformly, with replacement, from the fibers holding a nonzero, and      */
/* A_k = sum_j x_{f_j} Omega(j,:) with Omega (s_init x R, Gaussian) given.  */
/* Fiber u is the u-th distinct other-mode linear index in ascending order; */
/* draw j takes u = floor(U nfib / 2^128) from the Philox block at counter  */
/* (j, k << 8 | 3 << 16, 0, 0).  Returns the number of nonempty fibers.     */
/* ------------------------------------------------------------------------ */
int64_t orc_rrf_init(const orc_tensor *X, const orc_index *ix, int32_t k, int64_t s_init,
                     const double *omega, int32_t R, uint64_t seed, uint64_t stream_id,
                     double *A) {
  const int64_t nk = X->dims[k];
  memset(A, 0, sizeof(double) * (size_t)nk * R);
  const int64_t nnz = X->nnz;
  int64_t nfib = 0;
  for (int64_t e = 0; e < nnz; ++e)
    if (e == 0 || ix->key[k][e] != ix->key[k][e - 1]) nfib++;
  if (nfib == 0) return 0;
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nfib + 1));
  int64_t f = 0;
  for (int64_t e = 0; e < nnz; ++e)
    if (e == 0 || ix->key[k][e] != ix->key[k][e - 1]) start[f++] = e;
  start[nfib] = nnz;
  for (int64_t j = 0; j < s_init; ++j) {
    uint64_t out[4];
    draw_words(seed, stream_id, (uint64_t)j, ((uint64_t)k << 8) | (3ull << 16), 0, out);
    const int64_t u = (int64_t)orc_scale128(out[0], out[1], (uint64_t)nfib);
    for (int64_t pos = start[u]; pos < start[u + 1]; ++pos) {
      const int64_t e = ix->id[k][pos];
      const int64_t ik = X->coords[(int64_t)k * nnz + e];
      const double x = X->vals[e];
      for (int r = 0; r < R; ++r) A[ik * R + r] = A[ik * R + r] + x * omega[j * R + r];
    }
  }
  free(start);
  return nfib;
}

/* ------------------------------------------------------------------------ */
/* Fit (Sec. 6.2 eq. (6.1)) and its stratified estimate (Sec. 6.4).         */
/* ------------------------------------------------------------------------ */
double orc_model_entry(int32_t order, double *const *factors, int32_t R,
                       const int32_t *coord) {
  double m = 0.0;
  for (int r = 0; r < R; ++r) {
    double v = factors[0][(int64_t)coord[0] * R + r];
    for (int u = 1; u < order; ++u) v = v * factors[u][(int64_t)coord[u] * R + r];
    m = m + v;
  }
  return m;
}

/* ||X - M||^2 = ||X||^2 - 2<X,M> + ||M||^2 with ||M||^2 the sum over (r,r')
 * of the Hadamard product of the factor Gram matrices. */
double orc_fit_exact(const orc_tensor *X, double *const *factors, int32_t R) {
  const int D = X->order;
  double xx = 0.0, xm = 0.0;
  int32_t coord[16];
  for (int64_t e = 0; e < X->nnz; ++e) {
    for (int m = 0; m < D; ++m) coord[m] = X->coords[(int64_t)m * X->nnz + e];
    double x = X->vals[e];
    xx = xx + x * x;
    xm = xm + x * orc_model_entry(D, factors, R, coord);
  }
  double H[MAXR * MAXR], G[MAXR * MAXR];
  for (int i = 0; i < R * R; ++i) H[i] = 1.0;
  for (int m = 0; m < D; ++m) {
    orc_gram(factors[m], X->dims[m], R, G);
    for (int i = 0; i < R * R; ++i) H[i] = H[i] * G[i];
  }
  double mm = 0.0;
  for (int i = 0; i < R * R; ++i) mm = mm + H[i];
  double f2 = xx - 2.0 * xm + mm;
  if (f2 < 0.0) f2 = 0.0;
  return 1.0 - sqrt(f2) / sqrt(xx);
}

int64_t orc_fit_sample(const orc_tensor *X, uint64_t seed, uint64_t stream_id,
                       int64_t s_fit, double alpha,
                       int32_t *sc, double *sx, double *sphi, int64_t cap,
                       int32_t *flags) {
  const int D = X->order;
  if (s_fit < 1 || !(alpha >= 0.0 && alpha <= 1.0) || X->nnz < 1) return -1;
  int64_t n_nz = (int64_t)ceil(alpha * (double)s_fit);
  int64_t n_z = (int64_t)floor((1.0 - alpha) * (double)s_fit);
  uint64_t total = 1;
  for (int m = 0; m < D; ++m) total *= (uint64_t)X->dims[m];
  uint64_t zeros = total - (uint64_t)X->nnz;
  if (zeros == 0) n_z = 0;
  if (n_nz + n_z > cap) return -1;
  orc_index *ix = orc_index_build(X);
  double phi_nz = n_nz ? (double)X->nnz / (double)n_nz : 0.0;
  for (int64_t j = 0; j < n_nz; ++j) {
    uint64_t out[4];
    draw_words(seed, stream_id, (uint64_t)j, (uint64_t)1 << 16, 0, out);
    int64_t e = (int64_t)orc_scale128(out[0], out[1], (uint64_t)X->nnz);
    for (int m = 0; m < D; ++m) sc[(int64_t)m * cap + j] = X->coords[(int64_t)m * X->nnz + e];
    sx[j] = X->vals[e];
    sphi[j] = phi_nz;
  }
  int64_t got = 0, draws = 0, guard = 64 * n_z + (1 << 20);
  while (got < n_z) {
    if (draws >= guard) { *flags |= ORC_FLAG_DRAWCAP; break; }
    uint64_t key = 0, stride = 1;
    int32_t c[16];
    for (int m = 0; m < D; ++m) {
      uint64_t out[4];
      draw_words(seed, stream_id, (uint64_t)draws, (uint64_t)m | ((uint64_t)2 << 16), 0, out);
      c[m] = (int32_t)orc_scale128(out[0], out[1], (uint64_t)X->dims[m]);
      key += (uint64_t)c[m] * stride;
      stride *= (uint64_t)X->dims[m];
    }
    draws++;
    int64_t pos = lower_bound_u64(ix->full, X->nnz, key);
    if (pos < X->nnz && ix->full[pos] == key) continue;   /* stored: reject */
    int64_t j = n_nz + got;
    for (int m = 0; m < D; ++m) sc[(int64_t)m * cap + j] = c[m];
    sx[j] = 0.0;
    got++;
  }
  /* the zero stratum holds (prod n - nnz) entries represented by the `got`
   * zeros actually drawn (fewer than n_z when the draw guard stopped it) */
  double phi_z = got ? (double)zeros / (double)got : 0.0;
  for (int64_t j = n_nz; j < n_nz + got; ++j) sphi[j] = phi_z;
  orc_index_free(ix);
  return n_nz + got;
}

double orc_fit_estimate(int32_t order, int64_t n_fit, const int32_t *sc, int64_t ld,
                        const double *sx, const double *sphi,
                        double *const *factors, int32_t R, double normX) {
  double F = 0.0;
  int32_t coord[16];
  for (int64_t j = 0; j < n_fit; ++j) {
    for (int m = 0; m < order; ++m) coord[m] = sc[(int64_t)m * ld + j];
    double r = orc_model_entry(order, factors, R, coord) - sx[j];
    F = F + sphi[j] * (r * r);
  }
  return 1.0 - sqrt(F) / normX;
}
