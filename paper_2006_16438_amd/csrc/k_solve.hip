// Solve of the sketched normal equations, A_k = M G_s^{-1} (eq. (1.2)), and
// the FP32 factor mirror.
#include "cpal_common.h"

namespace cpal {

static int grid_for(i64 n, int blk, int maxg = 8192) {
  i64 g = (n + blk - 1) / blk;
  if (g < 1) g = 1;
  if (g > maxg) g = maxg;
  return (int)g;
}

// ------------------------------------------------------------------- solve --
// A_k(i,:) = M(i,:) G_s^{-1}: forward substitution with the Cholesky factor
// (subtractions in ascending order), back substitution (right-looking:
// subtractions in descending order), both multiplying by the reciprocals of
// the pivots; or the pseudo-inverse from the eigendecomposition.  Lanes =
// columns, LPN lanes per row (R <= LPN); FP64 throughout.  The rows of M
// (row stride ldm; the copies summed in copy order) are loaded before the
// factor is staged.
// Skipped when the update hit a state error.  256 threads.
template <typename T, int LPN>
__device__ __forceinline__ void solve_rows_body(Blk bk, const DevState *st, i64 n, int R,
    const T *__restrict__ M, int ldm, int ncopies, const Decomp *__restrict__ dc,
    double *__restrict__ A, float *__restrict__ A32) {
  extern __shared__ double sL[];   // R*R factor (L, or V)
  __shared__ double rdiag[CPAL_MAXR];
  if (st->flags & CPAL_FLAG_STATE) return;
  const int tid = threadIdx.x;
  const int c = (tid & 63) % LPN;
  const i64 row = ((i64)bk.x * blockDim.x + tid) / LPN;
  const bool live = row < n;
  const bool col = c < R;
  const int cl = col ? c : R - 1;
  T mv[CPAL_MCOPIES];
#pragma unroll
  for (int x = 0; x < CPAL_MCOPIES; ++x)
    mv[x] = (live && col && x < ncopies) ? M[(i64)x * n * ldm + row * ldm + c] : T(0);
  const int pinv = dc->pinv;
  for (int e = tid; e < R * R; e += blockDim.x) {
    const double lv = dc->L[e], vv = dc->V[e];
    sL[e] = pinv ? vv : lv;
  }
  __syncthreads();
  if (!pinv)
    for (int jj = tid; jj < R; jj += blockDim.x) rdiag[jj] = 1.0 / sL[jj * R + jj];
  __syncthreads();
  if (!live) return;   // uniform per lane group
  double v = 0.0;
#pragma unroll
  for (int x = 0; x < CPAL_MCOPIES; ++x)
    if (x < ncopies) v = v + (double)mv[x];
  if (!pinv) {
    for (int j = 0; j < R; ++j) {
      const double yj = group_value<LPN>(v, j) * rdiag[j];
      if (c == j) v = yj;
      else if (c > j && col) v = v - sL[c * R + j] * yj;
    }
    for (int j = R - 1; j >= 0; --j) {
      const double xj = group_value<LPN>(v, j) * rdiag[j];
      if (c == j) v = xj;
      else if (c < j) v = v - sL[j * R + c] * xj;
    }
  } else {
    // x = sum over kept j of ((v_j . m) / lambda_j) v_j
    const double etol = dc->etol;
    double t = 0.0;
    for (int p = 0; p < R; ++p) t = t + sL[p * R + cl] * group_value<LPN>(v, p);
    const double lam = dc->lam[cl];
    const double cj = lam > etol ? t / lam : 0.0;
    double x = 0.0;
    for (int j = 0; j < R; ++j) {
      const double cv = group_value<LPN>(cj, j);
      if (dc->lam[j] > etol) x = x + cv * sL[cl * R + j];
    }
    v = x;
  }
  if (col) {
    A[row * R + c] = v;
    A32[row * R + c] = (float)v;
  }
}
template <typename T, int LPN>
__global__ void __launch_bounds__(256) k_solve_rows(const DevState *st, i64 n, int R,
                                                    const T *__restrict__ M, int ldm,
                                                    int ncopies,
                                                    const Decomp *__restrict__ dc,
                                                    double *__restrict__ A,
                                                    float *__restrict__ A32) {
  solve_rows_body<T, LPN>(CPAL_BLK, st, n, R, M, ldm, ncopies, dc, A, A32);
}
template <typename T, int LPN>
struct B_solve_rows {
  static constexpr int NT = 256, MW = 1;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    solve_rows_body<T, LPN>(b, a...);
  }
};

__global__ void k_to_f32(const double *__restrict__ a, float *__restrict__ b, i64 n) {
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

template <typename T>
static void launch_solve_rows_t(int lpn, int nb, size_t sh, const DevState *st, i64 n, int R,
                                const T *M, int ldm, int ncopies, const Decomp *dc, double *A,
                                float *A32, hipStream_t s) {
  if (lpn == 16)
    launch_b<B_solve_rows<T, 16>>(k_solve_rows<T, 16>, dim3(nb), dim3(256), sh, s, st, n, R, M,
                                  ldm, ncopies, dc, A, A32);
  else if (lpn == 32)
    launch_b<B_solve_rows<T, 32>>(k_solve_rows<T, 32>, dim3(nb), dim3(256), sh, s, st, n, R, M,
                                  ldm, ncopies, dc, A, A32);
  else
    launch_b<B_solve_rows<T, 64>>(k_solve_rows<T, 64>, dim3(nb), dim3(256), sh, s, st, n, R, M,
                                  ldm, ncopies, dc, A, A32);
}

void launch_solve_rows(bool f64, const DevState *st, i64 n, int R, const void *M, int ldm,
                       int ncopies,
                       const Decomp *dc, double *A, float *A32, hipStream_t s) {
  const int lpn = R <= 16 ? 16 : (R <= 32 ? 32 : 64);
  const int nb = (int)((n * lpn + 255) / 256);
  const size_t sh = sizeof(double) * (size_t)R * R;
  if (f64)
    launch_solve_rows_t<double>(lpn, nb, sh, st, n, R, (const double *)M, ldm, ncopies, dc, A, A32,
                                s);
  else
    launch_solve_rows_t<float>(lpn, nb, sh, st, n, R, (const float *)M, ldm, ncopies, dc, A, A32,
                               s);
}

void launch_to_f32(const double *a, float *b, i64 n, hipStream_t s) {
  launch_1(k_to_f32, dim3(grid_for(n, 256)), dim3(256), 0, s, a, b, n);
}
}  // namespace cpal
