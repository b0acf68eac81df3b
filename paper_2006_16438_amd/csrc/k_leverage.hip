// Leverage scores of a factor matrix (Def. 3.4) and its integer sampling
// distribution (normalized leverage of Sec. 5.3 held as an integer CDF).
//
//   G = A^T A in blocks of 256 rows (rows ascending inside a block, blocks
//   ascending), Cholesky G = L L^T column by column, l_i = ||L^{-1} a_i||^2;
//   a pivot not above R*2^-52*max(diag G) switches to a Jacobi eigen-
//   decomposition and l_i = a_i^T G^+ a_i.  w_i = floor(2^52 * l_i / R),
//   C = inclusive prefix of w, q_i = w_i / W.
//
// Every multiply and add rounds separately (the library is built with
// -ffp-contract=off), so these values are reproducible bit for bit.
#include "cpal_common.h"

namespace cpal {

__device__ __forceinline__ void pair_of(int p, int R, int &a, int &c) {
  int row = 0;
  while (p >= R - row) { p -= R - row; ++row; }
  a = row;
  c = row + p;
}

// part[b][p]: sum over the rows of block b of A(r,a)*A(r,c), pair p = (a<=c).
#define GRAM_THREADS 512
__device__ __forceinline__ void lev_gram_partial_body(Blk bk, const double *__restrict__ A, i64 n,
    int R, double *__restrict__ part, const int *skip) {
  extern __shared__ double sA[];  // CPAL_GRAM_ROWS x R
  if (skip && *skip) return;
  const i64 r0 = (i64)bk.x * CPAL_GRAM_ROWS;
  const int rows = (int)min((i64)CPAL_GRAM_ROWS, n - r0);
  for (int e = threadIdx.x; e < rows * R; e += blockDim.x) sA[e] = A[r0 * R + e];
  __syncthreads();
  const int np = R * (R + 1) / 2;
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    int a, c;
    pair_of(p, R, a, c);
    double acc = 0.0;
    int r = 0;
    for (; r + 8 <= rows; r += 8) {   // products first, then added in row order
      double t[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t[q] = sA[(r + q) * R + a] * sA[(r + q) * R + c];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc = acc + t[q];
    }
    for (; r < rows; ++r) acc = acc + sA[r * R + a] * sA[r * R + c];
    part[(i64)bk.x * np + p] = acc;
  }
}
__global__ void __launch_bounds__(GRAM_THREADS) k_lev_gram_partial(const double *__restrict__ A, i64 n,
                                                          int R, double *__restrict__ part,
                                                          const int *skip) {
  lev_gram_partial_body(CPAL_BLK, A, n, R, part, skip);
}
CPAL_BODY(B_lev_gram_partial, GRAM_THREADS, 1, lev_gram_partial_body);

// Cyclic Jacobi eigendecomposition of the symmetric matrix S (R x R, shared
// memory), one wavefront.  Pairs (p,q) are visited row by row; the rotation
// for (p,q): theta = (S_qq - S_pp) / (2 S_pq), t = sign(theta) / (|theta| +
// sqrt(theta^2 + 1)), c = 1/sqrt(t^2+1), s = t c; an entry with |S_pq| <=
// 2^-53 sqrt|S_pp S_qq| is set to zero without rotating; stop after a sweep
// without rotations or after 64 sweeps.  Every lane derives (t, c, s) from the
// same three entries, then lane r updates row/column r of S and row r of V;
// these updates touch disjoint entries, so the result equals the sequential
// sweep element for element.
__device__ void jacobi_wave(double *S, double *V, int R, Decomp *out) {
  const int lane = threadIdx.x;
  for (int e = lane; e < R * R; e += 64) V[e] = (e / R == e % R) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 64; ++sweep) {
    bool any = false;
    for (int p = 0; p + 1 < R; ++p) {
      for (int q = p + 1; q < R; ++q) {
        const double spq = S[p * R + q];
        if (spq == 0.0) continue;
        const double spp = S[p * R + p], sqq = S[q * R + q];
        if (fabs(spq) <= 0x1p-53 * sqrt(fabs(spp * sqq))) {
          __syncthreads();
          if (lane == 0) { S[p * R + q] = 0.0; S[q * R + p] = 0.0; }
          __syncthreads();
          continue;
        }
        const double theta = (sqq - spp) / (2.0 * spq);
        double t;
        if (fabs(theta) > 0x1p500) {
          t = 0.5 / theta;
        } else {
          t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
          if (theta < 0.0) t = -t;
        }
        const double c = 1.0 / sqrt(t * t + 1.0);
        const double s = t * c;
        __syncthreads();  // every lane has read S_pp, S_qq, S_pq
        if (lane < R && lane != p && lane != q) {
          const double x = S[lane * R + p], y = S[lane * R + q];
          const double xp = c * x - s * y;
          const double yq = s * x + c * y;
          S[lane * R + p] = xp; S[p * R + lane] = xp;
          S[lane * R + q] = yq; S[q * R + lane] = yq;
        }
        if (lane < R) {
          const double x = V[lane * R + p], y = V[lane * R + q];
          V[lane * R + p] = c * x - s * y;
          V[lane * R + q] = s * x + c * y;
        }
        if (lane == 0) {
          S[p * R + p] = spp - t * spq;
          S[q * R + q] = sqq + t * spq;
          S[p * R + q] = 0.0;
          S[q * R + p] = 0.0;
        }
        __syncthreads();
        any = true;
      }
    }
    if (!any) break;
  }
  double mx = 0.0;
  for (int j = 0; j < R; ++j) mx = fmax(mx, fabs(S[j * R + j]));
  for (int e = lane; e < R * R; e += 64) out->V[e] = V[e];
  if (lane < R) out->lam[lane] = S[lane * R + lane];
  if (lane == 0) out->etol = ((double)R * 0x1p-52) * mx;
}

// Right-looking Cholesky of the symmetric matrix S (R x R in shared memory;
// its lower triangle is overwritten by the trailing updates) into L.  Entry
// (i,j) receives the subtractions L(i,p) L(j,p) for p = 0, 1, ..., j-1 in
// that order, then one division by L(j,j) -- the same operations as the
// column-by-column form -- so the factor is identical bit for bit, while
// each column's updates run in parallel.  Returns false when a pivot is not
// above tol.
__device__ bool chol_right(double *S, double *L, int R, double tol, int *fail_sh) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < R * R; e += nt) L[e] = 0.0;
  if (tid == 0) *fail_sh = 0;
  __syncthreads();
  for (int j = 0; j < R; ++j) {
    if (tid == 0) {
      const double v = S[j * R + j];
      if (!(v > tol)) *fail_sh = 1;
      else L[j * R + j] = sqrt(v);
    }
    __syncthreads();
    if (*fail_sh) return false;
    const double ljj = L[j * R + j];
    for (int i = j + 1 + tid; i < R; i += nt) L[i * R + j] = S[i * R + j] / ljj;
    __syncthreads();
    const int m = R - j - 1;
    const int cnt = m * (m + 1) / 2;
    for (int e = tid; e < cnt; e += nt) {
      int a = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
      while (a > 0 && a * (a + 1) / 2 > e) --a;
      while ((a + 1) * (a + 2) / 2 <= e) ++a;
      const int b = e - a * (a + 1) / 2;
      const int i = j + 1 + a, l = j + 1 + b;
      S[i * R + l] = S[i * R + l] - L[i * R + j] * L[l * R + j];
    }
    __syncthreads();
  }
  return true;
}

// Register form of the same right-looking Cholesky for R <= RM <= 32: lane
// i holds row i of the lower triangle of S in registers; column j's pivot is
// read from lane j, and the column entries L(l,j) from lane l.  Every entry
// of the lower triangle sees the same operations in the same order as
// chol_right.  S and L are shared-memory R x R arrays (S read, L written in
// full when the factorization succeeds).  One wavefront.

template <int RM>
__device__ __forceinline__ bool chol_regs(const double *S, double *L, int R, double tol) {
  const int lane = threadIdx.x;
  double g[RM];
#pragma unroll
  for (int l = 0; l < RM; ++l) g[l] = (lane < R && l < R) ? S[lane * R + l] : 0.0;
  double lcol[RM];   // this lane's entries L(lane, j)
#pragma unroll
  for (int j = 0; j < RM; ++j) lcol[j] = 0.0;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    if (j < R && ok) {
      const double piv = lane_value(g[j], j);
      if (!(piv > tol)) {
        ok = false;
      } else {
        const double ljj = sqrt(piv);
        const double lij = (lane == j) ? ljj : ((lane > j && lane < R) ? g[j] / ljj : 0.0);
        lcol[j] = lij;
        // trailing update of every lane's row: entries above the diagonal
        // (lane < l) and rows past R (all zero) are updated too but never read
#pragma unroll
        for (int l = j + 1; l < RM; ++l) {
          if (l < R) {
            const double llj = lane_value(lij, l);
            g[l] = g[l] - lij * llj;
          }
        }
      }
    }
  }
  if (ok) {
#pragma unroll
    for (int j = 0; j < RM; ++j)
      if (lane < R && j < R) L[lane * R + j] = lcol[j];
  }
  return ok;
}

// Branch-free register Cholesky for R <= RM: lane i holds row i of S in
// g[0..RM) with every entry past R (rows and columns) zero, and receives its
// row of L in lcol.  The padded columns see zero pivots and zero updates, so
// every entry of the R x R factor gets the same operations in the same order
// as chol_right (bit for bit), while the straight-line code lets column j's
// trailing update overlap the square root and divisions of column j + 1.
// Returns false when a pivot of the first R columns is not above tol.  One
// wavefront.
template <int RM>
__device__ __forceinline__ bool chol_pad(double (&g)[RM], double (&lcol)[RM], int R, double tol) {
  const int lane = threadIdx.x & 63;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < RM; ++j) {
    const double piv = lane_value(g[j], j);
    ok = ok & ((j >= R) | (piv > tol));
    const double ljj = sqrt(piv);
    const double q = g[j] / ljj;
    const double lij = (lane == j) ? ljj : ((lane > j && lane < R) ? q : 0.0);
    lcol[j] = lij;
#pragma unroll
    for (int l = j + 1; l < RM; ++l) g[l] = g[l] - lij * lane_value(lij, l);
  }
  return ok;
}

// Pair sums of the block partials in block order (pair p of lane + 64 k),
// straight from global memory.  Returns them packed in sG.
template <int KP>
__device__ __forceinline__ void pair_sums(const double *__restrict__ part, int nblk, int np,
                                          double *sG) {
  const int lane = threadIdx.x & 63;
  double acc[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) acc[k] = 0.0;
#pragma unroll 4
  for (int b = 0; b < nblk; ++b) {
    const double *pb = part + (i64)b * np;
#pragma unroll
    for (int k = 0; k < KP; ++k) {
      const int p = lane + 64 * k;
      if (p < np) acc[k] = acc[k] + pb[p];
    }
  }
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    const int p = lane + 64 * k;
    if (p < np) sG[p] = acc[k];
  }
}

// k_decomp for R <= RM <= 32 (one wavefront): pair sums, lane i's row of G
// from the packed sums, the pivot tolerance from the diagonal, chol_pad, and
// the factor written from registers.  On a failed pivot G is unpacked into
// the shared square matrix Gsq for the eigen-decomposition; returns whether
// the Cholesky succeeded.
template <int RM>
__device__ bool decomp_regs(const double *__restrict__ part, int nblk, int R,
                            Decomp *__restrict__ out, double *sG, double *Gsq) {
  const int lane = threadIdx.x & 63;
  const int np = R * (R + 1) / 2;
  pair_sums<(RM * (RM + 1) / 2 + 63) / 64>(part, nblk, np, sG);
  __syncthreads();
  double g[RM];
#pragma unroll
  for (int l = 0; l < RM; ++l) {
    const int a = min(lane, l), c = max(lane, l);
    g[l] = (lane < R && l < R) ? sG[a * R - (a * (a - 1)) / 2 + (c - a)] : 0.0;
  }
  double md = lane < R ? sG[lane * R - (lane * (lane - 1)) / 2] : 0.0;
  for (int off = 32; off > 0; off >>= 1) md = fmax(md, __shfl_xor(md, off, 64));
  const double tol = ((double)R * 0x1p-52) * md;
  double lcol[RM];
  const bool ok = chol_pad<RM>(g, lcol, R, tol);
  if (ok) {
    if (lane < R)
#pragma unroll
      for (int j = 0; j < RM; ++j)
        if (j < R) out->L[lane * R + j] = lcol[j];
  } else {
    for (int e = lane; e < R * R; e += 64) {
      const int r = e / R, q = e - r * R;
      const int a = min(r, q), c = max(r, q);
      Gsq[e] = sG[a * R - (a * (a - 1)) / 2 + (c - a)];
    }
    __syncthreads();
  }
  return ok;
}

// Leverage of a factor with fewer rows than columns (n < R <= 64): if A A^T
// (n x n, each entry summed over the R columns in ascending order) passes the
// Cholesky pivot test, A has full row rank, range(A) = R^n and every
// leverage score is exactly 1; the generic kernels are then skipped (*skip =
// 1).  Otherwise *skip = 0 and the Gram / eigen path runs.  One block.
__device__ __forceinline__ void lev_rowspace_body(Blk bk, const double *__restrict__ A, int n,
    int R, double *__restrict__ lev, u64 *__restrict__ w, u64 *__restrict__ blocksum, int rb,
    int *skip, int *pinv_store) {
  __shared__ double K[CPAL_MAXR * CPAL_MAXR];
  __shared__ double L[CPAL_MAXR * CPAL_MAXR];
  __shared__ double sA[CPAL_MAXR * CPAL_MAXR];   // A, n x R with n < R
  __shared__ int fail;
  const int tid = threadIdx.x;
#pragma unroll 8
  for (int e = tid; e < n * R; e += 64) sA[e] = A[e];
  __syncthreads();
  for (int e = tid; e < n * n; e += 64) {
    const int i = e / n, j = e - i * n;
    if (j > i) continue;
    double acc = 0.0;
    for (int r = 0; r < R; ++r) acc = acc + sA[i * R + r] * sA[j * R + r];
    K[i * n + j] = acc;
    K[j * n + i] = acc;
  }
  __syncthreads();
  double maxdiag = 0.0;
  for (int j = 0; j < n; ++j) maxdiag = fmax(maxdiag, K[j * n + j]);
  const double tol = ((double)n * 0x1p-52) * maxdiag;
  bool ok;
  if (n <= 16) ok = chol_regs<16>(K, L, n, tol);
  else if (n <= 32) ok = chol_regs<32>(K, L, n, tol);
  else ok = chol_right(K, L, n, tol, &fail);
  if (ok) {
    double v = 1.0 / (double)R;
    if (v > 1.0) v = 1.0;
    const u64 wi = (u64)(v * 0x1p52);
    for (int i = tid; i < n; i += 64) { lev[i] = 1.0; w[i] = wi; }
    for (int b = tid; b * rb < n; b += 64) blocksum[b] = wi * (u64)min(rb, n - b * rb);
    if (tid == 0) *pinv_store = 1;
  }
  if (tid == 0) *skip = ok ? 1 : 0;
}
__global__ void __launch_bounds__(64) k_lev_rowspace(const double *__restrict__ A, int n, int R,
                                                     double *__restrict__ lev, u64 *__restrict__ w,
                                                     u64 *__restrict__ blocksum, int rb,
                                                     int *skip, int *pinv_store) {
  lev_rowspace_body(CPAL_BLK, A, n, R, lev, w, blocksum, rb, skip, pinv_store);
}
CPAL_BODY(B_lev_rowspace, 64, 1, lev_rowspace_body);

// Sum the block partials in block order into G, then factor G.  One block of
// 64 threads (one wavefront); lane i owns row i during the Cholesky sweep.
// nrows_dev (nullable) gives the number of partial blocks at run time as
// ceil(*nrows_dev / rows_per_blk).  Partials are staged through shared
// memory in slabs so that each pair's sum stays in block order.
#define DECOMP_SLAB 4096
__device__ __forceinline__ void decomp_body(Blk bk, const double *__restrict__ part, int nblk,
    const i64 *nrows_dev, int rows_per_blk, int R, Decomp *__restrict__ out, int *flag_or,
    int *flag_store, const int *skip) {
  __shared__ double G[CPAL_MAXR * CPAL_MAXR];
  __shared__ double L[CPAL_MAXR * CPAL_MAXR];
  __shared__ double slab[DECOMP_SLAB];
  __shared__ int fail;
  if (skip && *skip) return;
  const int lane = threadIdx.x;
  if (nrows_dev) nblk = (int)((*nrows_dev + rows_per_blk - 1) / rows_per_blk);
  const int np = R * (R + 1) / 2;
  if (R <= 32) {
    bool ok;
    if (R <= 8) ok = decomp_regs<8>(part, nblk, R, out, slab, G);
    else if (R <= 16) ok = decomp_regs<16>(part, nblk, R, out, slab, G);
    else if (R <= 24) ok = decomp_regs<24>(part, nblk, R, out, slab, G);
    else ok = decomp_regs<32>(part, nblk, R, out, slab, G);
    if (ok) {
      if (lane == 0) {
        out->pinv = 0;
        out->R = R;
        if (flag_store) *flag_store = 0;
      }
    } else {
      jacobi_wave(G, L, R, out);
      if (lane == 0) {
        out->pinv = 1;
        out->R = R;
        if (flag_or) atomicOr(flag_or, CPAL_FLAG_PINV);
        if (flag_store) *flag_store = 1;
      }
    }
    return;
  }
  for (int p = lane; p < np; p += 64) G[p] = 0.0;   // running sums, packed by pair
  const int per = max(1, DECOMP_SLAB / np);          // blocks per slab
  for (int b0 = 0; b0 < nblk; b0 += per) {
    const int nb = min(per, nblk - b0);
    __syncthreads();
#pragma unroll 8
    for (int e = lane; e < nb * np; e += 64) slab[e] = part[(i64)b0 * np + e];
    __syncthreads();
    for (int p = lane; p < np; p += 64) {
      double tot = G[p];
      for (int b = 0; b < nb; ++b) tot = tot + slab[b * np + p];
      G[p] = tot;
    }
  }
  __syncthreads();
  // unpack the pair sums into the full symmetric matrix (L as staging); pair
  // (a <= c) sits at a*R - a*(a-1)/2 + (c - a)
  for (int p = lane; p < np; p += 64) L[p] = G[p];
  __syncthreads();
  for (int e = lane; e < R * R; e += 64) {
    const int r = e / R, q = e - r * R;
    const int a = min(r, q), c = max(r, q);
    G[e] = L[a * R - (a * (a - 1)) / 2 + (c - a)];
  }
  __syncthreads();
  double maxdiag = 0.0;
  for (int j = 0; j < R; ++j) maxdiag = fmax(maxdiag, G[j * R + j]);
  const double tol = ((double)R * 0x1p-52) * maxdiag;
  if (R <= 16) {
    for (int e = lane; e < R * R; e += 64) L[e] = 0.0;
    __syncthreads();
    const bool ok = chol_regs<16>(G, L, R, tol);
    if (lane == 0) fail = ok ? 0 : 1;
  } else if (R <= 32) {
    for (int e = lane; e < R * R; e += 64) L[e] = 0.0;
    __syncthreads();
    const bool ok = chol_regs<32>(G, L, R, tol);
    if (lane == 0) fail = ok ? 0 : 1;
  } else {
    for (int e = lane; e < R * R; e += 64) slab[e] = G[e];   // working copy
    __syncthreads();
    chol_right(slab, L, R, tol, &fail);
  }
  __syncthreads();
  if (!fail) {
    for (int e = lane; e < R * R; e += 64) out->L[e] = L[e];
    if (lane == 0) {
      out->pinv = 0;
      out->R = R;
      if (flag_store) *flag_store = 0;
    }
  } else {
    jacobi_wave(G, L, R, out);
    if (lane == 0) {
      out->pinv = 1;
      out->R = R;
      if (flag_or) atomicOr(flag_or, CPAL_FLAG_PINV);
      if (flag_store) *flag_store = 1;
    }
  }
}
__global__ void __launch_bounds__(64) k_decomp(const double *__restrict__ part, int nblk,
                                               const i64 *nrows_dev, int rows_per_blk, int R,
                                               Decomp *__restrict__ out, int *flag_or,
                                               int *flag_store, const int *skip) {
  decomp_body(CPAL_BLK, part, nblk, nrows_dev, rows_per_blk, R, out, flag_or, flag_store, skip);
}
CPAL_BODY(B_decomp, 64, 1, decomp_body);

// Parallel reduction of Gram partials (any order; used for the sampled G_s,
// which is not part of the reproducible sampling state): out[p] = sum_b
// part[b][p] for b < ceil(*nrows_dev / rows_per_blk).
__device__ __forceinline__ void gram_reduce_body(Blk bk, const double *__restrict__ part,
    const i64 *nrows_dev, int rows_per_blk, int np, double *__restrict__ out) {
  __shared__ double red[256];
  const int nblk = (int)((*nrows_dev + rows_per_blk - 1) / rows_per_blk);
  const int p = bk.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 256) acc += part[(i64)b * np + p];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p] = red[0];
}
__global__ void __launch_bounds__(256) k_gram_reduce(const double *__restrict__ part,
                                                     const i64 *nrows_dev, int rows_per_blk,
                                                     int np, double *__restrict__ out) {
  gram_reduce_body(CPAL_BLK, part, nrows_dev, rows_per_blk, np, out);
}
CPAL_BODY(B_gram_reduce, 256, 1, gram_reduce_body);

// Leverage of the rows of A (Def. 3.4): l_i = ||L^{-1} a_i||^2 with the
// Cholesky factor (forward substitution, y_j subtracted in ascending order,
// squares summed in ascending order), or sum over the kept eigenpairs of
// (v_j . a_i)^2 / lambda_j; then w_i = floor(2^52 min(l_i/R, 1)) and the
// block's sum of w.  Lanes = columns, LPN lanes per row (R <= LPN), every
// operation of a row in the same order as the sequential form.  Blocks of
// 256 threads = 256 / LPN rows.
template <int LPN>
__device__ __forceinline__ void lev_rows_body(Blk bk, const double *__restrict__ A, i64 n, int R,
    const Decomp *__restrict__ dc, double *__restrict__ lev, u64 *__restrict__ w,
    u64 *__restrict__ blocksum, const int *skip) {
  extern __shared__ double sL[];          // R*R (L, or V)
  __shared__ u64 wsum[4];
  if (skip && *skip) return;
  const int pinv = dc->pinv;
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) sL[e] = pinv ? dc->V[e] : dc->L[e];
  __syncthreads();
  const int tid = threadIdx.x, wid = tid >> 6;
  const int c = (tid & 63) % LPN;
  const i64 row = (i64)bk.x * (256 / LPN) + tid / LPN;
  const double etol = dc->etol;
  u64 wacc = 0;
  {
    const bool live = row < n;
    double v = (live && c < R) ? A[row * R + c] : 0.0;
    double acc = 0.0;
    if (!pinv) {
      for (int j = 0; j < R; ++j) {
        const double yj = group_value<LPN>(v, j) / sL[j * R + j];
        if (c == j) v = yj;
        else if (c > j && c < R) v = v - sL[c * R + j] * yj;
        acc = acc + yj * yj;
      }
    } else {
      // lane j: t_j = sum_p V(p,j) a_p in ascending p
      double t = 0.0;
      for (int p = 0; p < R; ++p) t = t + sL[p * R + min(c, R - 1)] * group_value<LPN>(v, p);
      for (int j = 0; j < R; ++j) {
        const double lam = dc->lam[j];
        const double tj = group_value<LPN>(t, j);
        if (lam > etol) acc = acc + (tj * tj) / lam;
      }
    }
    if (live && c == 0) {
      const double l = acc > 0.0 ? acc : 0.0;
      lev[row] = l;
      double q = l / (double)R;
      if (!(q > 0.0)) q = 0.0;
      if (q > 1.0) q = 1.0;
      const u64 wi = (u64)(q * 0x1p52);
      w[row] = wi;
      wacc = wi;
    }
  }
  wacc = wave_sum(wacc);
  if ((tid & 63) == 0) wsum[wid] = wacc;
  __syncthreads();
  if (tid == 0) blocksum[bk.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}
template <int LPN>
__global__ void __launch_bounds__(256) k_lev_rows(const double *__restrict__ A, i64 n, int R,
                                                  const Decomp *__restrict__ dc,
                                                  double *__restrict__ lev,
                                                  u64 *__restrict__ w,
                                                  u64 *__restrict__ blocksum,
                                                  const int *skip) {
  lev_rows_body<LPN>(CPAL_BLK, A, n, R, dc, lev, w, blocksum, skip);
}
template <int LPN>
struct B_lev_rows {
  static constexpr int NT = 256, MW = 1;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    lev_rows_body<LPN>(b, a...);
  }
};

// C = inclusive prefix of w, q = w / W.  Blocks of CDF_ROWS rows; blocksum
// holds the sums of w over consecutive groups of rb rows (rb divides
// CDF_ROWS), nbs of them.
#define CDF_ROWS 64
__device__ __forceinline__ void lev_cdf_body(Blk bk, const u64 *__restrict__ w, i64 n,
    const u64 *__restrict__ blocksum, int nbs, int rb, u64 *__restrict__ C, double *__restrict__ q,
    int *flag_or, const DevState *st, int k, int D, cpal_mode_stats *stats) {
  // the update's statistics, when asked for (this is the update's last kernel;
  // every count and flag is final by now)
  if (stats && bk.x == 0 && threadIdx.x == 0) {
    int fl = st->flags;
    for (int m = 0; m < D; ++m)
      if (m != k && st->lev_pinv[m]) fl |= CPAL_FLAG_PINV;
    stats->s_det = st->s_det;
    stats->s_rnd = st->s_rnd_used;
    stats->s_bar = st->s_bar;
    stats->draws = st->draws;
    stats->gathered_nnz = st->gathered;
    stats->p_det = st->p_det;
    stats->flags = fl;
    stats->pad = 0;
  }
  const int lim = (int)(bk.x * (CDF_ROWS / rb));
  u64 before = 0, all = 0;
  for (int b = threadIdx.x; b < nbs; b += blockDim.x) {
    const u64 v = blocksum[b];
    all += v;
    if (b < lim) before += v;
  }
  before = wave_sum(before);
  all = wave_sum(all);
  const i64 i = (i64)bk.x * CDF_ROWS + threadIdx.x;
  const u64 wi = i < n ? w[i] : 0;
  u64 tot;
  const u64 ex = block_excl_scan<u64>(wi, &tot);
  if (i < n) {
    C[i] = before + ex + wi;
    q[i] = all ? (double)wi / (double)all : 0.0;
  }
  if (i == 0 && all == 0 && flag_or) atomicOr(flag_or, CPAL_FLAG_STATE);
}
__global__ void __launch_bounds__(CDF_ROWS) k_lev_cdf(const u64 *__restrict__ w, i64 n,
                                                     const u64 *__restrict__ blocksum, int nbs,
                                                     int rb, u64 *__restrict__ C,
                                                     double *__restrict__ q, int *flag_or,
                                                     const DevState *st, int k, int D,
                                                     cpal_mode_stats *stats) {
  lev_cdf_body(CPAL_BLK, w, n, blocksum, nbs, rb, C, q, flag_or, st, k, D, stats);
}
CPAL_BODY(B_lev_cdf, CDF_ROWS, 1, lev_cdf_body);

int lev_rows_per_block(int R) { return 256 / (R <= 16 ? 16 : (R <= 32 ? 32 : 64)); }

// Row scores of the other sampling distributions compared in App. B (the
// probability of a KRP row is again the product of per-mode probabilities):
// kind 1 uniform (score 1, total n), kind 2 length squared (score
// ||A(i,:)||^2 summed over columns in ascending order, total = the trace of
// the Gram matrix summed in the canonical blocked order: block partials in
// ascending blocks, then the diagonal in ascending column order).
__device__ __forceinline__ void score_norm_body(Blk bk, const double *__restrict__ part, int nblk,
    int R, i64 n, int kind, double *norm, int *pinv_store) {
  if (threadIdx.x != 0) return;
  double S = (double)n;
  if (kind == 2) {
    const int np = R * (R + 1) / 2;
    S = 0.0;
    int p = 0;
    for (int j = 0; j < R; ++j) {   // pair index of (j, j) in the upper triangle
      double g = 0.0;
      for (int b = 0; b < nblk; ++b) g = g + part[(i64)b * np + p];
      S = S + g;
      p += R - j;
    }
  }
  *norm = S;
  if (pinv_store) *pinv_store = 0;
}
__global__ void __launch_bounds__(64) k_score_norm(const double *__restrict__ part, int nblk,
                                                  int R, i64 n, int kind, double *norm,
                                                  int *pinv_store) {
  score_norm_body(CPAL_BLK, part, nblk, R, n, kind, norm, pinv_store);
}
CPAL_BODY(B_score_norm, 64, 1, score_norm_body);

__device__ __forceinline__ void score_rows_body(Blk bk, const double *__restrict__ A, i64 n, int R,
    int kind, const double *__restrict__ norm, int rb, double *__restrict__ lev,
    u64 *__restrict__ w, u64 *__restrict__ blocksum) {
  const i64 i = (i64)bk.x * 256 + threadIdx.x;
  u64 wi = 0;
  if (i < n) {
    double sc = 1.0;
    if (kind == 2) {
      sc = 0.0;
      for (int c = 0; c < R; ++c) {
        const double a = A[i * R + c];
        sc = sc + a * a;
      }
    }
    lev[i] = sc;
    const double S = *norm;
    double v = S > 0.0 ? sc / S : 0.0;
    if (!(v > 0.0)) v = 0.0;
    if (v > 1.0) v = 1.0;
    wi = (u64)(v * 0x1p52);
    w[i] = wi;
  }
  // sums over groups of rb consecutive rows (rb divides 64)
  u64 g = wi;
  for (int off = 1; off < rb; off <<= 1) g += __shfl_xor(g, off, 64);
  if (i < n && (i % rb) == 0) blocksum[i / rb] = g;
}
__global__ void __launch_bounds__(256) k_score_rows(const double *__restrict__ A, i64 n, int R,
                                                  int kind, const double *__restrict__ norm,
                                                  int rb, double *__restrict__ lev,
                                                  u64 *__restrict__ w,
                                                  u64 *__restrict__ blocksum) {
  score_rows_body(CPAL_BLK, A, n, R, kind, norm, rb, lev, w, blocksum);
}
CPAL_BODY(B_score_rows, 256, 1, score_rows_body);

void launch_scores(const double *A, i64 n, int R, int kind, double *part, double *norm,
                   int *pinv_store, double *lev, u64 *w, u64 *blocksum, hipStream_t s) {
  const int nblk = (int)((n + CPAL_GRAM_ROWS - 1) / CPAL_GRAM_ROWS);
  if (kind == 2) launch_lev_gram_partial(A, n, R, part, nullptr, s);
  launch_b<B_score_norm>(k_score_norm, dim3(1), dim3(64), 0, s, part, nblk, R, n, kind, norm,
                         pinv_store);
  const int rb = lev_rows_per_block(R);
  launch_b<B_score_rows>(k_score_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, n,
                         R, kind, norm, rb, lev, w, blocksum);
}

void launch_lev_gram_partial(const double *A, i64 n, int R, double *part, const int *skip,
                             hipStream_t s) {
  const int nblk = (int)((n + CPAL_GRAM_ROWS - 1) / CPAL_GRAM_ROWS);
  const size_t sh = sizeof(double) * CPAL_GRAM_ROWS * R;
  launch_b<B_lev_gram_partial>(k_lev_gram_partial, dim3(nblk), dim3(GRAM_THREADS), sh, s, A, n, R,
                               part, skip);
}

void launch_lev_rowspace(const double *A, int n, int R, double *lev, u64 *w, u64 *blocksum,
                         int *skip, int *pinv_store, hipStream_t s) {
  launch_b<B_lev_rowspace>(k_lev_rowspace, dim3(1), dim3(64), 0, s, A, n, R, lev, w, blocksum,
                           lev_rows_per_block(R), skip, pinv_store);
}

void launch_decomp(const double *part, int nblk, int R, Decomp *out, int *flag_store,
                   const int *skip, hipStream_t s) {
  launch_b<B_decomp>(k_decomp, dim3(1), dim3(64), 0, s, part, nblk, (const i64 *)nullptr, 1, R,
                     out, (int *)nullptr, flag_store, skip);
}

// The Gram matrix of a factor from its block partials in the canonical order
// (the partials of the 256-row blocks added one after another, ascending,
// starting from zero), one thread per packed entry: the same sums k_decomp
// forms in one wave, for factors with many blocks.
__device__ __forceinline__ void gram_seq_body(Blk bk, const double *__restrict__ part, int nblk,
    int np, double *__restrict__ out) {
  const int p = bk.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  double acc = 0.0;
  int b = 0;
  for (; b + 4 <= nblk; b += 4) {
    const double v0 = part[(i64)b * np + p], v1 = part[(i64)(b + 1) * np + p];
    const double v2 = part[(i64)(b + 2) * np + p], v3 = part[(i64)(b + 3) * np + p];
    acc = acc + v0;
    acc = acc + v1;
    acc = acc + v2;
    acc = acc + v3;
  }
  for (; b < nblk; ++b) acc = acc + part[(i64)b * np + p];
  out[p] = acc;
}
__global__ void __launch_bounds__(256) k_gram_seq(const double *__restrict__ part, int nblk, int np,
                                                  double *__restrict__ out) {
  gram_seq_body(CPAL_BLK, part, nblk, np, out);
}
CPAL_BODY(B_gram_seq, 256, 1, gram_seq_body);

// Decomposition of a factor's Gram matrix from nblk block partials; with many
// blocks the partials are first summed by k_gram_seq into gram (np doubles).
void launch_decomp_blocks(const double *part, int nblk, int R, double *gram, Decomp *out,
                          int *flag_store, const int *skip, hipStream_t s) {
  const int np = R * (R + 1) / 2;
  if (nblk > 64 && gram) {
    launch_b<B_gram_seq>(k_gram_seq, dim3((np + 255) / 256), dim3(256), 0, s, part, nblk, np,
                         gram);
    part = gram;
    nblk = 1;
  }
  launch_b<B_decomp>(k_decomp, dim3(1), dim3(64), 0, s, part, nblk, (const i64 *)nullptr, 1, R,
                     out, (int *)nullptr, flag_store, skip);
}

void launch_decomp_dev(const double *part, const i64 *nrows_dev, int rows_per_blk, int R,
                       Decomp *out, int *flag_or, double *gram_tmp, hipStream_t s) {
  const int np = R * (R + 1) / 2;
  launch_b<B_gram_reduce>(k_gram_reduce, dim3(np), dim3(256), 0, s, part, nrows_dev, rows_per_blk,
                          np, gram_tmp);
  launch_b<B_decomp>(k_decomp, dim3(1), dim3(64), 0, s, (const double *)gram_tmp, 1,
                     (const i64 *)nullptr, 1, R, out, flag_or, (int *)nullptr, (const int *)nullptr);
}

void launch_lev_rows(const double *A, i64 n, int R, const Decomp *dc, double *lev, u64 *w,
                     u64 *blocksum, const int *skip, hipStream_t s) {
  const int rb = lev_rows_per_block(R);
  const int nblk = (int)((n + rb - 1) / rb);
  const size_t sh = sizeof(double) * (size_t)R * R;
  if (R <= 16)
    launch_b<B_lev_rows<16>>(k_lev_rows<16>, dim3(nblk), dim3(256), sh, s, A, n, R, dc, lev, w,
                             blocksum, skip);
  else if (R <= 32)
    launch_b<B_lev_rows<32>>(k_lev_rows<32>, dim3(nblk), dim3(256), sh, s, A, n, R, dc, lev, w,
                             blocksum, skip);
  else
    launch_b<B_lev_rows<64>>(k_lev_rows<64>, dim3(nblk), dim3(256), sh, s, A, n, R, dc, lev, w,
                             blocksum, skip);
}

void launch_lev_cdf(const u64 *w, i64 n, int R, const u64 *blocksum, u64 *C, double *q,
                    int *flag_or, const DevState *st, int k, int D, cpal_mode_stats *stats,
                    hipStream_t s) {
  const int rb = lev_rows_per_block(R);
  const int nbs = (int)((n + rb - 1) / rb);
  const int nblk = (int)((n + CDF_ROWS - 1) / CDF_ROWS);
  launch_b<B_lev_cdf>(k_lev_cdf, dim3(nblk), dim3(CDF_ROWS), 0, s, w, n, blocksum, nbs, rb, C, q,
                      flag_or, st, k, D, stats);
}

int lev_row_blocks(i64 n) { return (int)((n + 3) / 4); }   // blocksums at 4 rows per block

}  // namespace cpal
