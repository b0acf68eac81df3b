// Device-wide primitives: exclusive scan of u32 counts, and a stable LSD
// radix sort of u64 keys (optional u32 payload) whose element count may live
// in device memory (so that the pass sequence is fixed and capturable).
//
// Radix pass: 8-bit digits, tiles of 1024 keys (256 threads x 4 rounds).
// Within a round each wavefront ranks its keys by digit with ballots (the
// lanes sharing a digit form a mask), the waves of the block are ordered
// through shared counters, and rounds follow each other, so the scatter is
// stable.  Digit offsets of a tile are the digit-major exclusive prefix of
// the per-tile histograms.
#include "cpal_common.h"

namespace cpal {

#define RS_THREADS 256
#define RS_ROUNDS 4
#define RS_TILE (RS_THREADS * RS_ROUNDS)
#define SCAN_TILE 1024

// ------------------------------------------------------------------ scan ---
__device__ __forceinline__ void scan_part_body(Blk bk, const unsigned *__restrict__ in, i64 cap,
    const i64 *n_dev, u64 *__restrict__ part) {
  const i64 n = n_dev ? min(*n_dev, cap) : cap;
  const i64 base = (i64)bk.x * SCAN_TILE;
  u64 s = 0;
  for (int r = 0; r < SCAN_TILE / 256; ++r) {
    const i64 i = base + r * 256 + threadIdx.x;
    if (i < n) s += in[i];
  }
  s = wave_sum(s);
  __shared__ u64 ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[bk.x] = ws[0] + ws[1] + ws[2] + ws[3];
}
__global__ void __launch_bounds__(256) k_scan_part(const unsigned *__restrict__ in, i64 cap,
                                                   const i64 *n_dev, u64 *__restrict__ part) {
  scan_part_body(CPAL_BLK, in, cap, n_dev, part);
}
CPAL_BODY(B_scan_part, 256, 1, scan_part_body);

__device__ __forceinline__ void scan_top_body(Blk bk, u64 *__restrict__ part, int nb, u64 *total) {
  u64 carry = 0;
  for (int b0 = 0; b0 < nb; b0 += 1024) {
    const int b = b0 + threadIdx.x;
    const u64 v = b < nb ? part[b] : 0;
    u64 tot;
    const u64 ex = block_excl_scan<u64>(v, &tot);
    if (b < nb) part[b] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}
__global__ void __launch_bounds__(1024) k_scan_top(u64 *__restrict__ part, int nb,
                                                   u64 *total) {
  scan_top_body(CPAL_BLK, part, nb, total);
}
CPAL_BODY(B_scan_top, 1024, 1, scan_top_body);

__device__ __forceinline__ void scan_apply_body(Blk bk, const unsigned *__restrict__ in, i64 cap,
    const i64 *n_dev, const u64 *__restrict__ part, u64 *__restrict__ out) {
  const i64 n = n_dev ? min(*n_dev, cap) : cap;
  const i64 base = (i64)bk.x * SCAN_TILE;
  if (base >= n) return;
  u64 carry = part[bk.x];
  for (int r = 0; r < SCAN_TILE / 256; ++r) {
    const i64 i = base + r * 256 + threadIdx.x;
    const u64 v = i < n ? in[i] : 0;
    u64 tot;
    const u64 ex = block_excl_scan<u64>(v, &tot);
    if (i < n) out[i] = carry + ex;
    carry += tot;
  }
}
__global__ void __launch_bounds__(256) k_scan_apply(const unsigned *__restrict__ in, i64 cap,
                                                    const i64 *n_dev, const u64 *__restrict__ part,
                                                    u64 *__restrict__ out) {
  scan_apply_body(CPAL_BLK, in, cap, n_dev, part, out);
}
CPAL_BODY(B_scan_apply, 256, 1, scan_apply_body);

size_t scan_scratch_bytes(i64 n) {
  return sizeof(u64) * (size_t)((n + SCAN_TILE - 1) / SCAN_TILE + 1);
}

// Exclusive scan of in[0..n) (n = *n_dev if given, else cap) into out;
// *total (device, nullable) receives the sum.
void scan_u32_dev(const unsigned *in, u64 *out, i64 cap, const i64 *n_dev, u64 *total,
                  void *scratch, hipStream_t s) {
  const int nb = (int)((cap + SCAN_TILE - 1) / SCAN_TILE);
  u64 *part = (u64 *)scratch;
  if (nb == 0) return;
  launch_b<B_scan_part>(k_scan_part, dim3(nb), dim3(256), 0, s, in, cap, n_dev, part);
  launch_b<B_scan_top>(k_scan_top, dim3(1), dim3(1024), 0, s, part, nb, total);
  launch_b<B_scan_apply>(k_scan_apply, dim3(nb), dim3(256), 0, s, in, cap, n_dev, part, out);
}

void scan_u32_to_u64(const unsigned *in, u64 *out, i64 n, u64 *total, void *scratch,
                     hipStream_t s) {
  scan_u32_dev(in, out, n, nullptr, total, scratch, s);
}

// ----------------------------------------------------------------- radix ---
__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const u64 *__restrict__ keys, i64 cap,
                                                        const i64 *n_dev, int shift,
                                                        unsigned *__restrict__ hist, int nb) {
  __shared__ unsigned h[256];
  const i64 n = n_dev ? min(*n_dev, cap) : cap;
  h[threadIdx.x] = 0;
  __syncthreads();
  const i64 base = (i64)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const i64 i = base + r * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&h[(unsigned)(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(i64)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// fused_offsets: when hist_off is null the block derives its digit offsets
// from the raw histograms (small inputs: nb <= 256), otherwise hist_off holds
// the digit-major exclusive scan.
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(
    const u64 *__restrict__ keys, const unsigned *__restrict__ vals, i64 cap, const i64 *n_dev,
    int shift, const unsigned *__restrict__ hist, const u64 *__restrict__ hist_off, int nb,
    u64 *__restrict__ okeys, unsigned *__restrict__ ovals) {
  __shared__ u64 goff[256];
  __shared__ unsigned run[256];
  __shared__ unsigned wcnt[RS_THREADS / 64][256];
  const i64 n = n_dev ? min(*n_dev, cap) : cap;
  const i64 base = (i64)blockIdx.x * RS_TILE;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (base >= n) return;  // uniform per block
  // digit offsets of this tile
  if (hist_off) {
    goff[tid] = hist_off[(i64)tid * nb + blockIdx.x];
  } else {
    u64 tot = 0, before = 0;
    const unsigned *row = hist + (i64)tid * nb;
    const int me = (int)blockIdx.x;
    if ((nb & 3) == 0) {   // rows start 16-byte aligned
      const uint4 *r4 = (const uint4 *)row;
#pragma unroll 8
      for (int b4 = 0; b4 < nb / 4; ++b4) {
        const uint4 v = r4[b4];
        const int b = 4 * b4;
        tot += (u64)v.x + v.y + v.z + v.w;
        before += (u64)(b < me ? v.x : 0u) + (b + 1 < me ? v.y : 0u) + (b + 2 < me ? v.z : 0u) +
                  (b + 3 < me ? v.w : 0u);
      }
    } else {
#pragma unroll 8
      for (int b = 0; b < nb; ++b) {
        const unsigned v = row[b];
        tot += v;
        if (b < me) before += v;
      }
    }
    u64 alltot;
    const u64 ex = block_excl_scan<u64>(tot, &alltot);
    goff[tid] = ex + before;
  }
  run[tid] = 0;
  for (int w = 0; w < RS_THREADS / 64; ++w) wcnt[w][tid] = 0;
  __syncthreads();
  for (int r = 0; r < RS_ROUNDS; ++r) {
    const i64 i = base + r * RS_THREADS + tid;
    const bool valid = i < n;
    const u64 key = valid ? keys[i] : 0ull;
    const unsigned val = (valid && vals) ? vals[i] : 0u;
    const unsigned dig = (unsigned)(key >> shift) & 255u;
    u64 peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dig >> b) & 1u;
      const u64 m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const u64 lt = __lanemask_lt();
    const unsigned rank = (unsigned)__popcll(peers & lt);
    if (valid && rank == 0) wcnt[wid][dig] = (unsigned)__popcll(peers);
    __syncthreads();
    if (valid) {
      unsigned pos = run[dig] + rank;
      for (int w = 0; w < wid; ++w) pos += wcnt[w][dig];
      const u64 dst = goff[dig] + pos;
      okeys[dst] = key;
      if (vals) ovals[dst] = val;
    }
    __syncthreads();
    {
      unsigned add = 0;
      for (int w = 0; w < RS_THREADS / 64; ++w) { add += wcnt[w][tid]; wcnt[w][tid] = 0; }
      run[tid] += add;
    }
    __syncthreads();
    (void)lane;
  }
}

static int rs_blocks(i64 cap) { return (int)((cap + RS_TILE - 1) / RS_TILE); }

size_t sort_scratch_bytes(i64 cap, bool /*with_vals*/) {
  const i64 nb = rs_blocks(cap);
  const i64 nh = 256 * nb;
  size_t b = sizeof(unsigned) * (size_t)nh;          // hist
  b = (b + 255) & ~(size_t)255;
  b += sizeof(u64) * (size_t)nh;                     // hist offsets
  b = (b + 255) & ~(size_t)255;
  b += scan_scratch_bytes(nh);
  return b + 256;
}

// Sort keys[0..n) (n = *count_dev, or count_host if count_dev is null;
// n <= cap) on the low `bits` bits, payload in vals (nullable).  The passes
// alternate between (keys, vals) and (tmp_keys, tmp_vals); the return value
// is the key buffer holding the result (its payload is the matching buffer).
u64 *sort_keys_pp(u64 *keys, unsigned *vals, u64 *tmp_keys, unsigned *tmp_vals, void *scratch,
                  i64 cap, const i64 *count_dev, i64 count_host, int bits, hipStream_t s) {
  if (cap <= 0) return keys;
  const int nb = rs_blocks(cap);
  const i64 nh = 256 * (i64)nb;
  char *p = (char *)scratch;
  unsigned *hist = (unsigned *)p;
  p += ((sizeof(unsigned) * (size_t)nh + 255) & ~(size_t)255);
  u64 *hoff = (u64 *)p;
  p += ((sizeof(u64) * (size_t)nh + 255) & ~(size_t)255);
  void *scan_scratch = p;
  const i64 capn = count_dev ? cap : min(cap, count_host);
  const bool fused = nb <= 256;
  int passes = (bits + 7) / 8;
  if (passes < 1) passes = 1;
  u64 *src_k = keys, *dst_k = tmp_keys;
  unsigned *src_v = vals, *dst_v = vals ? tmp_vals : nullptr;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = 8 * ps;
    launch_1(k_rs_hist, dim3(nb), dim3(RS_THREADS), 0, s, src_k, capn, count_dev,
             shift, hist, nb);
    if (!fused) scan_u32_to_u64(hist, hoff, nh, nullptr, scan_scratch, s);
    launch_1(k_rs_scatter, dim3(nb), dim3(RS_THREADS), 0, s, src_k, src_v, capn,
             count_dev, shift, hist, fused ? (const u64 *)nullptr : hoff, nb, dst_k,
             dst_v);
    u64 *tk = src_k; src_k = dst_k; dst_k = tk;
    unsigned *tv = src_v; src_v = dst_v; dst_v = tv;
  }
  return src_k;
}

// Same, but the result always ends in keys/vals (one copy when the number of
// passes is odd).
void sort_keys(u64 *keys, unsigned *vals, u64 *tmp_keys, unsigned *tmp_vals, void *scratch,
               i64 cap, const i64 *count_dev, i64 count_host, int bits, hipStream_t s) {
  u64 *r = sort_keys_pp(keys, vals, tmp_keys, tmp_vals, scratch, cap, count_dev, count_host, bits,
                        s);
  if (r != keys) {
    const i64 capn = count_dev ? cap : min(cap, count_host);
    hipMemcpyAsync(keys, r, sizeof(u64) * (size_t)capn, hipMemcpyDeviceToDevice, s);
    if (vals) hipMemcpyAsync(vals, tmp_vals, sizeof(unsigned) * (size_t)capn,
                             hipMemcpyDeviceToDevice, s);
  }
}

}  // namespace cpal
