// Randomized range finder initialisation (App. F): every column of the
// initial A_k is a random linear combination of mode-k fibers.  s_init
// fibers are drawn uniformly, with replacement, from the fibers that hold a
// nonzero (fiber u = the u-th nonempty fiber in ascending other-mode linear
// index; u = floor(U nfib / 2^128) from the Philox block at counter
// (j, k << 8 | 3 << 16, 0, 0)), and A_k = sum_j x_{f_j} Omega(j,:) with the
// caller's Gaussian Omega.  The sum runs through the update's gather: the
// draws fill the slots of the sampled system (fiber offset and length, and
// Omega's row as the weighted KRP row), the gather forms M = sum_j x_{f_j}
// Omega(j,:), and A_k is M (no Gram matrix, no solve).
#include "cpal_common.h"

namespace cpal {

// Nonempty fibers of a mode from its hash table: (offset in the mode-sorted
// nonzeros, length) in any order; sorting by offset gives ascending fiber key.
__global__ void k_fiber_list(const FiberSlot *__restrict__ slots, u64 nslots, u64 *__restrict__ off,
                             unsigned *__restrict__ len, unsigned long long *__restrict__ count) {
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < nslots;
       i += (u64)gridDim.x * blockDim.x) {
    const FiberSlot sl = slots[i];
    if (sl.key == CPAL_EMPTY_KEY) continue;
    const u64 p = atomicAdd(count, 1ull);
    off[p] = sl.off;
    len[p] = sl.len;
  }
}

void launch_fiber_list(const FiberSlot *slots, u64 nslots, u64 *off, unsigned *len,
                       unsigned long long *count, hipStream_t s) {
  const u64 g = std::min<u64>((nslots + 255) / 256, 8192);
  launch_1(k_fiber_list, dim3((unsigned)std::max<u64>(g, 1)), dim3(256), 0, s, slots,
           nslots, off, len, count);
}

// One thread per draw j < s_init (blocks of rpb slots, as the row kernel):
// the fiber of the draw, Omega's row j as the slot's weighted row (padded to
// ldz with zeros), and the block totals the gather preparation sums.
// Sparse: fib_off / fib_len are the nonempty fibers in ascending key order;
// dense (fib_off == nullptr): fiber u is the u-th mode-k column, of length
// dense_len, and samp_idx[j] = u locates it.
template <typename TZ>
__global__ void __launch_bounds__(256) k_rrf_rows(
    DevState *st, i64 s_init, int k, u64 seed, u64 stream_id, u64 nfib,
    const u64 *__restrict__ fib_off, const unsigned *__restrict__ fib_len, unsigned dense_len,
    const double *__restrict__ omega, int R, int ldz, TZ *__restrict__ zhat,
    unsigned *__restrict__ foff, unsigned *__restrict__ flen, u64 *__restrict__ samp_idx,
    u64 *__restrict__ part_len, unsigned *__restrict__ part_cnt, unsigned *__restrict__ part_act) {
  const i64 j = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->n_slots = s_init;
    st->s_det = s_init;   // no draw-table entries to release
  }
  unsigned len = 0;
  if (j < s_init) {
    u64 c[4] = {(u64)j, ((u64)k << 8) | (3ull << 16), 0ull, 0ull};
    philox4x64_10(c, seed, stream_id);
    const u64 u = scale128(c[0], c[1], nfib);
    unsigned off = 0;
    if (fib_off) {
      off = (unsigned)fib_off[u];
      len = fib_len[u];
    } else {
      len = dense_len;
    }
    foff[j] = off;
    flen[j] = len;
    samp_idx[j] = u;
    for (int col = 0; col < ldz; ++col)
      zhat[j * ldz + col] = cvt_from<TZ>(col < R ? omega[j * R + col] : 0.0);
  }
  const u64 ln = wave_sum((u64)len);
  const unsigned na = (unsigned)__popcll(__ballot(j < s_init));
  const unsigned nf = (unsigned)__popcll(__ballot(len > 0u));
  __shared__ u64 wln[4];
  __shared__ unsigned wna[4], wnf[4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { wln[w] = ln; wna[w] = na; wnf[w] = nf; }
  __syncthreads();
  if (threadIdx.x == 0) {
    u64 l = 0;
    unsigned a = 0, f = 0;
    for (int q = 0; q < 4; ++q) { l += wln[q]; a += wna[q]; f += wnf[q]; }
    part_len[blockIdx.x] = l;
    part_act[blockIdx.x] = a;
    part_cnt[blockIdx.x] = f;
  }
}

void launch_rrf_rows(int zdt, DevState *st, i64 s_init, int k, u64 seed, u64 stream_id, u64 nfib,
                     const u64 *fib_off, const unsigned *fib_len, unsigned dense_len,
                     const double *omega, int R, int ldz, void *zhat, unsigned *foff,
                     unsigned *flen, u64 *samp_idx, u64 *part_len, unsigned *part_cnt,
                     unsigned *part_act, int rows_per_blk, hipStream_t s) {
  const unsigned nb = (unsigned)((s_init + rows_per_blk - 1) / rows_per_blk);
  if (zdt == CPAL_F64)
    launch_1(k_rrf_rows<double>, dim3(nb), dim3(rows_per_blk), 0, s, st, s_init, k, seed,
             stream_id, nfib, fib_off, fib_len, dense_len, omega, R, ldz,
             (double *)zhat, foff, flen, samp_idx, part_len, part_cnt, part_act);
  else if (zdt == CPAL_F32)
    launch_1(k_rrf_rows<float>, dim3(nb), dim3(rows_per_blk), 0, s, st, s_init, k, seed,
             stream_id, nfib, fib_off, fib_len, dense_len, omega, R, ldz, (float *)zhat,
             foff, flen, samp_idx, part_len, part_cnt, part_act);
  else
    launch_1(k_rrf_rows<bf16s>, dim3(nb), dim3(rows_per_blk), 0, s, st, s_init, k, seed,
             stream_id, nfib, fib_off, fib_len, dense_len, omega, R, ldz, (bf16s *)zhat,
             foff, flen, samp_idx, part_len, part_cnt, part_act);
}

// A_k(i, r) = the sum of the gather's copies of M(i, r) in copy order; the
// FP32 mirror with it.
template <typename TM>
__global__ void k_rrf_store(const TM *__restrict__ M, int ncopies, i64 nk, int R, int ldz,
                            double *__restrict__ A, float *__restrict__ A32) {
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < nk * R;
       e += (i64)gridDim.x * blockDim.x) {
    const i64 i = e / R;
    const int r = (int)(e - i * R);
    double v = 0.0;
    for (int c = 0; c < ncopies; ++c) v = v + (double)M[((i64)c * nk + i) * ldz + r];
    A[e] = v;
    A32[e] = (float)v;
  }
}

void launch_rrf_store(bool f64, const void *M, int ncopies, i64 nk, int R, int ldz, double *A,
                      float *A32, hipStream_t s) {
  const i64 g = std::min<i64>((nk * R + 255) / 256, 16384);
  if (f64)
    launch_1(k_rrf_store<double>, dim3((unsigned)std::max<i64>(g, 1)), dim3(256), 0, s,
             (const double *)M, ncopies, nk, R, ldz, A, A32);
  else
    launch_1(k_rrf_store<float>, dim3((unsigned)std::max<i64>(g, 1)), dim3(256), 0, s,
             (const float *)M, ncopies, nk, R, ldz, A, A32);
}

}  // namespace cpal
