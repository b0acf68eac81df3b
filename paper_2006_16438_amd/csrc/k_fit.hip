// Estimated fit (Sec. 6.4): a stratified sample of ceil(alpha s_fit) stored
// nonzeros (uniform, with replacement) and floor((1-alpha) s_fit) zero
// entries (uniform coordinates, stored ones rejected, first accepted in draw
// order), drawn once; F^ = sum_i phi_i (m_i - x_i)^2 with phi = nnz/#nonzero
// samples or (prod n - nnz)/#zero samples; fit = 1 - sqrt(F^)/||X||.
// Philox counters: nonzero draw j -> (j, 1<<16, 0, 0); zero draw j, mode m ->
// (j, m | 2<<16, 0, 0); key (seed, stream_id); index = floor(U n / 2^128).
#include "cpal_common.h"

namespace cpal {

#define FIT_BLK 256

struct FullModes {
  int D;
  i64 n[CPAL_MAXORDER];
  u64 stride[CPAL_MAXORDER];
  const double *A[CPAL_MAXORDER];
};

__global__ void k_fullkey_clear(u64 *__restrict__ set, u64 n) {
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
    set[i] = CPAL_EMPTY_KEY;
}

__global__ void k_fullkey_insert(const int *__restrict__ coords, i64 nnz, FullModes fm,
                                 u64 *__restrict__ set, u64 mask, int shift) {
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (i64)gridDim.x * blockDim.x) {
    u64 key = 0;
    for (int m = 0; m < fm.D; ++m) key += (u64)(unsigned)coords[(i64)m * nnz + e] * fm.stride[m];
    u64 h = key_hash(key, shift);
    for (;;) {
      const u64 old = atomicCAS(&set[h], CPAL_EMPTY_KEY, key);
      if (old == CPAL_EMPTY_KEY || old == key) break;
      h = (h + 1) & mask;
    }
  }
}

__device__ __forceinline__ bool fullkey_present(const u64 *__restrict__ set, u64 mask, int shift,
                                                u64 key) {
  u64 h = key_hash(key, shift);
  for (;;) {
    const u64 v = set[h];
    if (v == key) return true;
    if (v == CPAL_EMPTY_KEY) return false;
    h = (h + 1) & mask;
  }
}

__global__ void k_fit_nz(const int *__restrict__ coords, const void *__restrict__ vals, int vdt,
                         i64 nnz, int D, i64 n_nz, u64 seed, u64 stream_id, int *__restrict__ sc,
                         i64 ld, double *__restrict__ sx) {
  for (i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x; j < n_nz; j += (i64)gridDim.x * blockDim.x) {
    u64 c[4] = {(u64)j, 1ull << 16, 0ull, 0ull};
    philox4x64_10(c, seed, stream_id);
    const i64 e = (i64)scale128(c[0], c[1], (u64)nnz);
    for (int m = 0; m < D; ++m) sc[(i64)m * ld + j] = coords[(i64)m * nnz + e];
    sx[j] = vdt == CPAL_F64 ? ((const double *)vals)[e] : (double)((const float *)vals)[e];
  }
}

// Persistent zero-entry draws, same chunk protocol as the KRP draws.
__global__ void __launch_bounds__(256) k_fit_zero_draw(FullModes fm, i64 n_z, u64 seed,
                                                       u64 stream_id, const u64 *__restrict__ set,
                                                       u64 mask, int shift, u64 *ctl,
                                                       u64 *__restrict__ buf,
                                                       unsigned *__restrict__ chunk_cnt) {
  __shared__ u64 sh_c;
  __shared__ int stop;
  const int tid = threadIdx.x;
  const i64 max_draws = 64 * n_z + (1ll << 20);
  const u64 max_chunks = (u64)((max_draws + CPAL_DRAW_CHUNK - 1) / CPAL_DRAW_CHUNK);
  for (;;) {
    if (tid == 0) {
      const u64 acc = __hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      stop = 0;
      if ((i64)acc >= n_z) {
        stop = 1;
      } else {
        const u64 c = atomicAdd(&ctl[0], 1ull);
        if (c >= max_chunks) stop = 1; else sh_c = c;
      }
    }
    __syncthreads();
    if (stop) break;
    const u64 c = sh_c;
    const i64 j = (i64)c * CPAL_DRAW_CHUNK + tid;
    unsigned ok = 0;
    u64 key = 0;
    if (j < max_draws) {
      for (int m = 0; m < fm.D; ++m) {
        u64 w[4] = {(u64)j, (u64)m | (2ull << 16), 0ull, 0ull};
        philox4x64_10(w, seed, stream_id);
        key += scale128(w[0], w[1], (u64)fm.n[m]) * fm.stride[m];
      }
      ok = !fullkey_present(set, mask, shift, key);
    }
    unsigned tot;
    const unsigned ex = block_excl_scan<unsigned>(ok, &tot);
    if (ok) buf[c * CPAL_DRAW_CHUNK + ex] = key;
    if (tid == 0) {
      chunk_cnt[c] = tot;
      atomicAdd(&ctl[1], (u64)tot);
    }
    __syncthreads();
  }
}

// ctl[0] = chunks handed out, ctl[1] = accepted; writes the accepted zero
// coordinates in draw order after the nonzero part; ctl[2] = zeros kept.
__global__ void __launch_bounds__(1024) k_fit_zero_finish(FullModes fm, i64 n_z, i64 n_nz, u64 *ctl,
                                                          const u64 *__restrict__ buf,
                                                          const unsigned *__restrict__ chunk_cnt,
                                                          int *__restrict__ sc, i64 ld,
                                                          double *__restrict__ sx) {
  const i64 max_draws = 64 * n_z + (1ll << 20);
  const u64 max_chunks = (u64)((max_draws + CPAL_DRAW_CHUNK - 1) / CPAL_DRAW_CHUNK);
  const u64 Q = min(ctl[0], max_chunks);
  u64 carry = 0;
  for (u64 q = 0; q < Q && carry < (u64)n_z; ++q) {
    const unsigned cnt = chunk_cnt[q];
    if (threadIdx.x < cnt && carry + threadIdx.x < (u64)n_z) {
      const i64 j = n_nz + (i64)(carry + threadIdx.x);
      u64 key = buf[q * CPAL_DRAW_CHUNK + threadIdx.x];
      for (int m = 0; m < fm.D; ++m) {
        sc[(i64)m * ld + j] = (int)(key % (u64)fm.n[m]);
        key /= (u64)fm.n[m];
      }
      sx[j] = 0.0;
    }
    carry += cnt;
  }
  if (threadIdx.x == 0) ctl[2] = min(carry, (u64)n_z);
}

// Per-sample squared residual, weighted; one partial per block of FIT_BLK
// samples.  Lanes = columns: a group of LPS lanes (R <= LPS) evaluates one
// sample, lane r forming the product over the DD modes of the factor rows'
// entries r (rows read contiguously), the model value being the group's
// tree sum; each group takes FIT_BLK / (256 / LPS) consecutive samples,
// FIT_UNR in flight, and sums its terms in sample order; the block partial is
// the sum of its groups in order.  DD = 0: any order (runtime loop).
#define FIT_UNR 4
template <int LPS, int DD>
__global__ void __launch_bounds__(256) k_fit_eval(FullModes fm, int R, i64 n_nz, i64 n_fit,
                                                  double phi_nz, double phi_z,
                                                  const int *__restrict__ sc, i64 ld,
                                                  const double *__restrict__ sx,
                                                  double *__restrict__ part) {
  constexpr int G = 256 / LPS;
  constexpr int PER = FIT_BLK / G;
  __shared__ double gsum[G];
  const int tid = threadIdx.x, g = tid / LPS, r = tid % LPS;
  const int D = DD > 0 ? DD : fm.D;
  const int rc = r < R ? r : R - 1;   // lanes past R read column R-1, weight 0
  const i64 j0 = (i64)blockIdx.x * FIT_BLK + (i64)g * PER;
  double acc = 0.0;
  for (int s0 = 0; s0 < PER; s0 += FIT_UNR) {
    double v[FIT_UNR];
#pragma unroll
    for (int q = 0; q < FIT_UNR; ++q) {
      const i64 j = min(j0 + s0 + q, n_fit - 1);
      if (DD > 0) {
        int idx[DD > 0 ? DD : 1];
#pragma unroll
        for (int u = 0; u < (DD > 0 ? DD : 1); ++u) idx[u] = sc[(i64)u * ld + j];
        double f[DD > 0 ? DD : 1];
#pragma unroll
        for (int u = 0; u < (DD > 0 ? DD : 1); ++u) f[u] = fm.A[u][(i64)idx[u] * R + rc];
        double p = f[0];
#pragma unroll
        for (int u = 1; u < (DD > 0 ? DD : 1); ++u) p = p * f[u];
        v[q] = p;
      } else {
        double p = fm.A[0][(i64)sc[j] * R + rc];
        for (int u = 1; u < D; ++u) p = p * fm.A[u][(i64)sc[(i64)u * ld + j] * R + rc];
        v[q] = p;
      }
      if (r >= R) v[q] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < FIT_UNR; ++q) {
      double m = v[q];
#pragma unroll
      for (int off = LPS / 2; off > 0; off >>= 1) m = m + __shfl_xor(m, off, LPS);
      const i64 j = j0 + s0 + q;
      if (r == 0 && j < n_fit) {
        const double d = m - sx[j];
        acc = acc + (j < n_nz ? phi_nz : phi_z) * (d * d);
      }
    }
  }
  if (r == 0) gsum[g] = acc;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int q = 0; q < G; ++q) t = t + gsum[q];
    part[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(256) k_fit_final(const double *__restrict__ part, int nb,
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
  if (threadIdx.x == 0) *fit_out = 1.0 - sqrt(red[0]) / sqrt(st->normX2);
}

// ||X||^2 in FIT_BLK blocks, partials summed in order by k_norm_final.
__global__ void __launch_bounds__(FIT_BLK) k_norm_part(const void *__restrict__ vals, int vdt, i64 nnz,
                                                      double *__restrict__ part) {
  __shared__ double red[FIT_BLK];
  const i64 e = (i64)blockIdx.x * FIT_BLK + threadIdx.x;
  double x = 0.0;
  if (e < nnz) x = vdt == CPAL_F64 ? ((const double *)vals)[e] : (double)((const float *)vals)[e];
  red[threadIdx.x] = x * x;
  __syncthreads();
  for (int off = FIT_BLK / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(1024) k_norm_final(const double *__restrict__ part, i64 nb,
                                                     DevState *st) {
  // sequential over the block partials in 1024 strided chains, then in order
  __shared__ double red[1024];
  double acc = 0.0;
  for (i64 b = threadIdx.x; b < nb; b += 1024) acc = acc + part[b];
  red[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < 1024; ++i) t = t + red[i];
    st->normX2 = t;
  }
}

static int gridc(i64 n, int blk) {
  i64 g = (n + blk - 1) / blk;
  return (int)std::max<i64>(1, std::min<i64>(g, 8192));
}

void fit_build_set(const int *coords, i64 nnz, const FullModes &fm, u64 *set, u64 nslots,
                   int shift, hipStream_t s) {
  launch_1(k_fullkey_clear, dim3(gridc((i64)nslots, 256)), dim3(256), 0, s, set, nslots);
  launch_1(k_fullkey_insert, dim3(gridc(nnz, 256)), dim3(256), 0, s, coords, nnz, fm, set,
           nslots - 1, shift);
}

void fit_draw(const int *coords, const void *vals, int vdt, i64 nnz, const FullModes &fm, i64 n_nz,
              i64 n_z, u64 seed, u64 stream_id, const u64 *set, u64 nslots, int shift, u64 *ctl,
              u64 *buf, unsigned *chunk_cnt, int *sc, i64 ld, double *sx, hipStream_t s) {
  launch_1(k_fit_nz, dim3(gridc(n_nz, 256)), dim3(256), 0, s, coords, vals, vdt, nnz,
           fm.D, n_nz, seed, stream_id, sc, ld, sx);
  if (n_z > 0) {
    launch_1(k_fit_zero_draw, dim3(1024), dim3(256), 0, s, fm, n_z, seed, stream_id, set,
             nslots - 1, shift, ctl, buf, chunk_cnt);
    launch_1(k_fit_zero_finish, dim3(1), dim3(CPAL_DRAW_CHUNK), 0, s, fm, n_z, n_nz, ctl,
             buf, chunk_cnt, sc, ld, sx);
  }
}

void fit_norm(const void *vals, int vdt, i64 nnz, double *part, DevState *st, hipStream_t s) {
  const i64 nb = (nnz + FIT_BLK - 1) / FIT_BLK;
  launch_1(k_norm_part, dim3((unsigned)nb), dim3(FIT_BLK), 0, s, vals, vdt, nnz, part);
  launch_1(k_norm_final, dim3(1), dim3(1024), 0, s, part, nb, st);
}

void fit_eval(const FullModes &fm, int R, i64 n_nz, i64 n_fit, double phi_nz, double phi_z,
              const int *sc, i64 ld, const double *sx, double *part, const DevState *st,
              double *fit_out, hipStream_t s) {
  const int nb = (int)((n_fit + FIT_BLK - 1) / FIT_BLK);
  const int dd = (fm.D >= 2 && fm.D <= 5) ? fm.D : 0;
  auto pick = [dd](auto k2, auto k3, auto k4, auto k5, auto k0) {
    return dd == 2 ? k2 : dd == 3 ? k3 : dd == 4 ? k4 : dd == 5 ? k5 : k0;
  };
  decltype(&k_fit_eval<16, 0>) k;
  if (R <= 16)
    k = pick(k_fit_eval<16, 2>, k_fit_eval<16, 3>, k_fit_eval<16, 4>, k_fit_eval<16, 5>,
             k_fit_eval<16, 0>);
  else if (R <= 32)
    k = pick(k_fit_eval<32, 2>, k_fit_eval<32, 3>, k_fit_eval<32, 4>, k_fit_eval<32, 5>,
             k_fit_eval<32, 0>);
  else
    k = pick(k_fit_eval<64, 2>, k_fit_eval<64, 3>, k_fit_eval<64, 4>, k_fit_eval<64, 5>,
             k_fit_eval<64, 0>);
  launch_1(k, dim3(nb), dim3(256), 0, s, fm, R, n_nz, n_fit, phi_nz, phi_z, sc, ld, sx,
           part);
  launch_1(k_fit_final, dim3(1), dim3(256), 0, s, part, nb, st, fit_out);
}

}  // namespace cpal
