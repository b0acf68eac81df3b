// Internal declarations of the gfx950 CP-ARLS-LEV library: device state,
// per-update mode descriptors, device helpers and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cp_arls_lev.h"
#include "cpal_launch.h"

#define CPAL_MAXR 64
#define CPAL_MAXORDER 8
#define CPAL_GRAM_ROWS 256      // rows per block of the canonical Gram summation
#define CPAL_DRAW_CHUNK 256     // draws per chunk of the persistent fit-sample draw kernel
#define CPAL_KRP_CHUNK 256      // draws per chunk of the KRP row draw kernel (one per thread)
#define CPAL_MCOPIES 8          // copies of M for the gather's adds, one per XCD (power of two)
#define CPAL_GATHER_CHUNK 2048  // stream positions per chunk of the segmented gather

typedef unsigned long long u64;
typedef long long i64;

// Scalars of one decomposition that kernels read and write on the device, so
// that a whole mode update runs without reading counts back to the host.
struct DevState {
  u64 det_count;      // rows with p > tau found by the enumeration (atomic)
  u64 combos;         // size of the candidate product set
  i64 s_det;
  i64 s_rnd;          // random rows requested
  i64 s_rnd_used;     // accepted random draws used for the weights
  i64 s_bar;          // rows of the sampled system
  i64 n_slots;        // slots of the sampled system (deterministic rows + accepted draws)
  i64 draws;
  u64 chunk_next;     // next draw chunk (atomic ticket)
  u64 accepted;       // accepted draws of the top-up pass so far (atomic)
  u64 first_chunks;   // chunks of the first draw pass
  i64 nchunks;        // chunks handed out (a prefix of the chunk sequence)
  i64 gathered;       // nnz of the sampled fibers
  i64 n_fib;          // nonempty sampled fibers
  i64 n_rnd_rows;     // distinct random rows (set when the sampled rows are listed)
  u64 t_next;         // step counter of the next update (third Philox counter word)
  u64 t_cur;          // step counter of the update in progress
  double p_det;
  double tau_eff;     // 1.0 when the enumeration was skipped or capped
  int flags;
  int lev_flags;
  i64 fit_nz;         // fit sample: nonzero entries
  i64 fit_z;          // fit sample: zero entries (accepted)
  u64 ncand[CPAL_MAXORDER];   // candidate rows per other mode (Sec. 5.3)
  int lev_pinv[CPAL_MAXORDER];  // pseudo-inverse used for a mode's leverage
  int lev_skip[CPAL_MAXORDER];  // leverage settled by the full-row-rank test
  double fit;
  double normX2;
  double score_norm[CPAL_MAXORDER];   // total row score of a mode (other distributions)
};

// Symmetric R x R factorization: Cholesky, or eigen-decomposition when the
// matrix is numerically singular.
struct Decomp {
  int pinv;
  int R;
  double etol;
  double pad;
  double L[CPAL_MAXR * CPAL_MAXR];
  double V[CPAL_MAXR * CPAL_MAXR];
  double lam[CPAL_MAXR];
};

// The other modes of an update (ascending), with their sampling vectors.
struct OtherModes {
  int d;
  int k;
  int mode[CPAL_MAXORDER];
  i64 n[CPAL_MAXORDER];
  u64 stride[CPAL_MAXORDER];
  const double *q[CPAL_MAXORDER];
  const u64 *C[CPAL_MAXORDER];
  const double *A[CPAL_MAXORDER];
  const float *A32[CPAL_MAXORDER];
  i64 cand_off[CPAL_MAXORDER];
  double rcp[CPAL_MAXORDER];   // 1 / n[u], rounded
};

// One hash slot of a per-mode fiber index: complement key -> [off, off+len)
// of the mode-sorted nonzeros.
struct __attribute__((aligned(16))) FiberSlot {
  u64 key;
  unsigned off;
  unsigned len;
};
#define CPAL_EMPTY_KEY (~0ull)

// One entry of the table of an update's accepted random draws: KRP row ->
// position of the draw that entered it (its slot carries the row) and the
// number of its other draws.  An empty entry is {CPAL_EMPTY_KEY, ~0u, 0}; the
// table is empty between updates.
struct __attribute__((aligned(16))) DrawEntry {
  u64 key;
  unsigned first;
  unsigned cnt;
};

// ------------------------------------------------------------ device helpers
__device__ __forceinline__ void philox4x64_10(u64 c[4], u64 k0, u64 k1) {
  // Salmon et al. SC'11: 10 rounds; S-box multipliers and Weyl key increments.
  const u64 M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const u64 W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const u64 lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
    const u64 lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
    const u64 n0 = hi1 ^ c[1] ^ k0;
    const u64 n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += W0; k1 += W1;
  }
}

// floor(U * W / 2^128), U = u1 * 2^64 + u0.
__device__ __forceinline__ u64 scale128(u64 u0, u64 u1, u64 W) {
  const u64 a_hi = __umul64hi(u0, W);
  const u64 b_lo = u1 * W, b_hi = __umul64hi(u1, W);
  const u64 mid = b_lo + a_hi;
  return b_hi + (mid < b_lo ? 1ull : 0ull);
}

// Smallest i in [0,n) with C[i] > v.
__device__ __forceinline__ i64 upper_bound_u64(const u64 *__restrict__ C, i64 n, u64 v) {
  i64 lo = 0, hi = n;
  while (lo < hi) {
    const i64 mid = (lo + hi) >> 1;
    if (C[mid] > v) hi = mid; else lo = mid + 1;
  }
  return lo;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// p of the KRP row encoded in lin (other modes ascending, first fastest):
// product of the per-mode q in ascending mode order.
// x / n and x % n (n >= 1, rcp = 1/n rounded).  For x < 2^53 a
// floating-point quotient estimate (off by at most a few units) is corrected
// by whole steps; larger x use the integer division.
__device__ __forceinline__ u64 div_rcp(u64 x, u64 n, double rcp, u64 *rem) {
  if (x >= (1ull << 53)) {
    const u64 q = x / n;
    *rem = x - q * n;
    return q;
  }
  i64 q = (i64)((double)x * rcp);
  i64 r = (i64)x - q * (i64)n;
  while (r < 0) { --q; r += (i64)n; }
  while (r >= (i64)n) { ++q; r -= (i64)n; }
  *rem = (u64)r;
  return (u64)q;
}

__device__ __forceinline__ double prob_of(const OtherModes &om, u64 lin) {
  double p = 0.0;
  u64 rem = lin;
  for (int u = 0; u < om.d; ++u) {
    u64 i;
    rem = div_rcp(rem, (u64)om.n[u], om.rcp[u], &i);
    const double qv = om.q[u][i];
    p = (u == 0) ? qv : p * qv;
  }
  return p;
}

// bfloat16 values are kept as their bit patterns.  Conversion from FP64
// rounds to FP32 first, then to the nearest bfloat16 (ties to even; the
// values here are finite).
typedef unsigned short bf16s;
__device__ __forceinline__ bf16s bf16_from_float(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16s)(u >> 16);
}
__device__ __forceinline__ float bf16_to_float(bf16s b) {
  return __uint_as_float((unsigned)b << 16);
}
template <typename T>
__device__ __forceinline__ T cvt_from(double x) { return (T)x; }
template <>
__device__ __forceinline__ bf16s cvt_from<bf16s>(double x) { return bf16_from_float((float)x); }

// Multiplicative hash of a key (fiber or KRP row) into a table of 2^(64-shift)
// slots.
__device__ __forceinline__ u64 key_hash(u64 key, int shift) {
  return (key * 0x9E3779B97F4A7C15ull) >> shift;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = __lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T o = __shfl_up(v, off, 64);
    if (lane >= off) v += o;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide exclusive scan (blockDim.x multiple of 64, <= 1024); returns the
// exclusive prefix of v and writes the block total to *total.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *total) {
  __shared__ T wsum[17];  // 16 wave slots + the block total
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  T inc = wave_incl_scan(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  if (wid == 0) {
    T x = lane < nw ? wsum[lane] : T(0);
    T xi = wave_incl_scan(x);
    if (lane < nw) wsum[lane] = xi - x;
    if (lane == nw - 1) wsum[16] = xi;
  }
  __syncthreads();
  T res = inc - v + wsum[wid];
  *total = wsum[16];
  __syncthreads();
  return res;
}

// Index of the XCD (accelerator complex die) the calling wave runs on.
__device__ __forceinline__ unsigned xcd_id() {
  return (unsigned)__builtin_amdgcn_s_getreg((3 << 11) | 20);   // HW_REG_XCC_ID, bits [3:0]
}

// Value of v in lane l (l wave-uniform) through two scalar lane reads.
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Lanes = columns: a wave holds 64 / LPN rows, lane c of group g holding
// column c of row g.  group_value(v, j) = column j of the caller's row.
template <int LPN>
__device__ __forceinline__ double group_value(double v, int j) {
  const int g = (int)(threadIdx.x & 63) / LPN;
  double r = lane_value(v, j);
#pragma unroll
  for (int q = 1; q < 64 / LPN; ++q) {
    const double t = lane_value(v, q * LPN + j);
    r = g == q ? t : r;
  }
  return r;
}

// ------------------------------------------------------------ launchers
namespace cpal {

struct Sorter;   // radix sort scratch

// leverage pipeline for one factor matrix (n x R) ---------------------------
void launch_lev_gram_partial(const double *A, i64 n, int R, double *part, const int *skip,
                             hipStream_t s);
void launch_lev_rowspace(const double *A, int n, int R, double *lev, u64 *w, u64 *blocksum,
                         int *skip, int *pinv_store, hipStream_t s);
void launch_decomp(const double *part, int nblk, int R, Decomp *out, int *flag_store,
                   const int *skip, hipStream_t s);
void launch_decomp_blocks(const double *part, int nblk, int R, double *gram, Decomp *out,
                          int *flag_store, const int *skip, hipStream_t s);
void launch_lev_rows(const double *A, i64 n, int R, const Decomp *dc, double *lev, u64 *w,
                     u64 *blocksum, const int *skip, hipStream_t s);
void launch_lev_cdf(const u64 *w, i64 n, int R, const u64 *blocksum, u64 *C, double *q,
                    int *flag_or, const DevState *st, int k, int D, cpal_mode_stats *stats,
                    hipStream_t s);
void launch_scores(const double *A, i64 n, int R, int kind, double *part, double *norm,
                   int *pinv_store, double *lev, u64 *w, u64 *blocksum, hipStream_t s);

// radix sort of u64 keys with optional u32 payload, device-resident count --
size_t sort_scratch_bytes(i64 cap, bool with_vals);
void sort_keys(u64 *keys, unsigned *vals, u64 *tmp_keys, unsigned *tmp_vals, void *scratch,
               i64 cap, const i64 *count_dev, i64 count_host, int bits, hipStream_t s);

// generic exclusive scan of u32 -> u64 with total -----------------------------
void scan_u32_to_u64(const unsigned *in, u64 *out, i64 n, u64 *total, void *scratch,
                     hipStream_t s);
size_t scan_scratch_bytes(i64 n);

}  // namespace cpal
