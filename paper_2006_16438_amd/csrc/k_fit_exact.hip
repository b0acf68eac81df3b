// Exact fit of the CP model (eq. (6.1) of Sec. 6.2):
//   ||X - M||^2 = ||X||^2 - 2 <X, M> + ||M||^2,
//   <X, M>  = sum over stored entries of x * m(i),
//   ||M||^2 = sum_{r, r'} prod_m (A_m^T A_m)(r, r').
// <X, M> walks the per-mode copy of one mode k (the one whose factor is
// smallest, so that its rows stay in cache): every fiber (other-mode
// coordinates fixed) contributes sum_i x(i) <A_k(i,:), z> with z the
// Hadamard product of the other modes' factor rows.  Sparse tensors walk the
// fiber hash table of mode k, dense tensors the fiber-contiguous copy.
// Partial sums are per workgroup and added in workgroup order, so the result
// is the same on every run.
#include "cpal_common.h"

namespace cpal {

#define FX_THREADS 256
#define FX_GRID 2048

struct FitxModes {
  int D;
  int k;                                  // the walked mode
  i64 n[CPAL_MAXORDER];                   // other modes, ascending (first fastest)
  const double *A[CPAL_MAXORDER];
  const double *Ak;
};

// One fiber of linear other-mode index `key`: z (lanes = columns) into zs.
__device__ __forceinline__ void fx_krp_row(const FitxModes &fm, int R, u64 key, double *zs) {
  const int lane = threadIdx.x & 63;
  i64 idx[CPAL_MAXORDER];
  u64 rem = key;
  for (int u = 0; u < fm.D - 1; ++u) {
    idx[u] = (i64)(rem % (u64)fm.n[u]);
    rem /= (u64)fm.n[u];
  }
  if (lane < R) {
    double z = fm.A[0][idx[0] * R + lane];
    for (int u = 1; u < fm.D - 1; ++u) z = z * fm.A[u][idx[u] * R + lane];
    zs[lane] = z;
  }
}

// value of the walked copy: kind 0 FP32 pairs {i_k, x bits}, 1 FP64 (ik, v64)
struct FxVals {
  int kind;
  const uint2 *pairs;
  const int *ik;
  const double *v64;
  __device__ __forceinline__ void get(u64 e, int &i, double &x) const {
    if (kind == 0) {
      const uint2 v = pairs[e];
      i = (int)v.x;
      x = (double)__uint_as_float(v.y);
    } else {
      i = ik[e];
      x = v64[e];
    }
  }
};

__device__ __forceinline__ double fx_row_dot(const double *__restrict__ Ak, int R, int i,
                                             const double *zs) {
  double d = 0.0;
  for (int c = 0; c < R; ++c) d = d + Ak[(i64)i * R + c] * zs[c];
  return d;
}

__device__ __forceinline__ void fx_block_store(double acc, double *part) {
  __shared__ double red[FX_THREADS];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = FX_THREADS / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Sparse: wave w takes 64 consecutive hash slots at a time; every nonempty
// slot (a fiber) is processed by the whole wave, lanes = its entries.
__global__ void __launch_bounds__(FX_THREADS) k_fitx_sparse(FitxModes fm, int R,
                                                          const FiberSlot *__restrict__ slots,
                                                          u64 nslots, FxVals vals,
                                                          double *__restrict__ part) {
  __shared__ double zsh[FX_THREADS / 64][CPAL_MAXR];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double *zs = zsh[wid];
  const u64 gw = ((u64)blockIdx.x * FX_THREADS + threadIdx.x) >> 6;
  const u64 nw = ((u64)gridDim.x * FX_THREADS) >> 6;
  double acc = 0.0;
  for (u64 base = gw * 64; base < nslots; base += nw * 64) {
    FiberSlot sl;
    sl.key = CPAL_EMPTY_KEY;
    sl.off = 0;
    sl.len = 0;
    if (base + lane < nslots) sl = slots[base + lane];
    u64 mask = __ballot(sl.key != CPAL_EMPTY_KEY);
    while (mask) {
      const int l = __builtin_ctzll(mask);
      mask &= mask - 1;
      const u64 key = __shfl(sl.key, l, 64);
      const unsigned off = __shfl(sl.off, l, 64);
      const unsigned len = __shfl(sl.len, l, 64);
      fx_krp_row(fm, R, key, zs);
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      for (unsigned e0 = 0; e0 < len; e0 += 64) {
        if (e0 + lane < len) {
          int i;
          double x;
          vals.get((u64)off + e0 + lane, i, x);
          acc = acc + x * fx_row_dot(fm.Ak, R, i, zs);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
  }
  fx_block_store(acc, part);
}

// Dense: fiber j of the mode-k copy holds n_k values at j * ldx.
template <typename T>
__global__ void __launch_bounds__(FX_THREADS) k_fitx_dense(FitxModes fm, int R, i64 nk, u64 nfib,
                                                         const T *__restrict__ X, i64 ldx,
                                                         double *__restrict__ part) {
  __shared__ double zsh[FX_THREADS / 64][CPAL_MAXR];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double *zs = zsh[wid];
  const u64 gw = ((u64)blockIdx.x * FX_THREADS + threadIdx.x) >> 6;
  const u64 nw = ((u64)gridDim.x * FX_THREADS) >> 6;
  double acc = 0.0;
  for (u64 j = gw; j < nfib; j += nw) {
    fx_krp_row(fm, R, j, zs);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    for (i64 i = lane; i < nk; i += 64) {
      double x;
      if constexpr (sizeof(T) == 2) x = (double)bf16_to_float(X[(i64)j * ldx + i]);
      else x = (double)X[(i64)j * ldx + i];
      acc = acc + x * fx_row_dot(fm.Ak, R, (int)i, zs);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  fx_block_store(acc, part);
}

// H = G_m (first) or H .* G_m from the 256-row block partials of the Gram of
// factor m (upper triangle, pairs a <= c); one workgroup.
__device__ __forceinline__ void fx_pair_of(int p, int R, int &a, int &c) {
  int row = 0;
  while (p >= R - row) { p -= R - row; ++row; }
  a = row;
  c = row + p;
}

__global__ void __launch_bounds__(256) k_fitx_hadamard(const double *__restrict__ gpart, int nblk,
                                                     int R, double *__restrict__ H, int first) {
  const int np = R * (R + 1) / 2;
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    double g = 0.0;
    for (int b = 0; b < nblk; ++b) g = g + gpart[(i64)b * np + p];
    H[p] = first ? g : H[p] * g;
  }
}

__global__ void __launch_bounds__(256) k_fitx_final(const double *__restrict__ part, int nb,
                                                  const double *__restrict__ H, int R,
                                                  const DevState *st, double *fit_out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) acc = acc + part[b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double xm = red[0];
    double mm = 0.0;
    const int np = R * (R + 1) / 2;
    for (int p = 0; p < np; ++p) {
      int a, c;
      fx_pair_of(p, R, a, c);
      mm = mm + (a == c ? H[p] : 2.0 * H[p]);
    }
    const double xx = st->normX2;
    double f2 = xx - 2.0 * xm + mm;
    if (f2 < 0.0) f2 = 0.0;
    *fit_out = 1.0 - sqrt(f2) / sqrt(xx);
  }
}

void launch_lev_gram_partial(const double *A, i64 n, int R, double *part, const int *skip,
                             hipStream_t s);

size_t fit_exact_scratch_doubles(int R, i64 maxn) {
  const int np = R * (R + 1) / 2;
  return (size_t)FX_GRID + (size_t)np + (size_t)((maxn + CPAL_GRAM_ROWS - 1) / CPAL_GRAM_ROWS) * np;
}

// scratch: fit_exact_scratch_doubles(R, max n) doubles.  kind: 0 sparse FP32
// pairs, 1 sparse FP64, 2 dense FP64, 3 dense FP32, 4 dense BF16.
void launch_fit_exact(int D, const i64 *dims, double *const *A, int R, int k, int kind,
                      const FiberSlot *slots, u64 nslots, const uint2 *pairs, const int *ik,
                      const double *v64, const void *dX, i64 ldx, const DevState *st,
                      double *scratch, double *fit_out, hipStream_t s) {
  FitxModes fm;
  fm.D = D;
  fm.k = k;
  int u = 0;
  u64 nfib = 1;
  for (int m = 0; m < D; ++m) {
    if (m == k) continue;
    fm.n[u] = dims[m];
    fm.A[u] = A[m];
    nfib *= (u64)dims[m];
    ++u;
  }
  fm.Ak = A[k];
  const int np = R * (R + 1) / 2;
  double *part = scratch;
  double *H = scratch + FX_GRID;
  double *gpart = H + np;
  if (kind <= 1) {
    FxVals v{kind, pairs, ik, v64};
    launch_1(k_fitx_sparse, dim3(FX_GRID), dim3(FX_THREADS), 0, s, fm, R, slots,
             nslots, v, part);
  } else if (kind == 2) {
    launch_1(k_fitx_dense<double>, dim3(FX_GRID), dim3(FX_THREADS), 0, s, fm, R,
             dims[k], nfib, (const double *)dX, ldx, part);
  } else if (kind == 3) {
    launch_1(k_fitx_dense<float>, dim3(FX_GRID), dim3(FX_THREADS), 0, s, fm, R,
             dims[k], nfib, (const float *)dX, ldx, part);
  } else {
    launch_1(k_fitx_dense<bf16s>, dim3(FX_GRID), dim3(FX_THREADS), 0, s, fm, R,
             dims[k], nfib, (const bf16s *)dX, ldx, part);
  }
  for (int m = 0; m < D; ++m) {
    const int nblk = (int)((dims[m] + CPAL_GRAM_ROWS - 1) / CPAL_GRAM_ROWS);
    launch_lev_gram_partial(A[m], dims[m], R, gpart, nullptr, s);
    launch_1(k_fitx_hadamard, dim3(1), dim3(256), 0, s, gpart, nblk, R, H, m == 0 ? 1 : 0);
  }
  launch_1(k_fitx_final, dim3(1), dim3(256), 0, s, part, FX_GRID, H, R, st, fit_out);
}

}  // namespace cpal
