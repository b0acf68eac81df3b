// SkrpLev on the device (Alg. 1): deterministic rows (Sec. 5.3), random rows
// by per-mode draws (Lemma 5.3) with rejection of p > tau (Alg. 2), and the
// bookkeeping of the combined rows (Sec. 4.1, 4.3).
//
// Canonical choices shared with the CPU reference by specification only:
//  * p of a multi-index = product of the per-mode q in ascending mode order;
//  * draw j of mode m at step t uses Philox4x64-10 with counter
//    (j, m | k<<8, t, 0) and key (seed, stream_id); v = floor(U W_m / 2^128)
//    with U = word1*2^64 + word0; the row is the smallest i with C_m(i) > v;
//  * the random rows are the first s_rnd accepted draws in draw order;
//  * the deterministic set is sorted by linear index; if it holds >= s rows
//    the s most probable are kept (ties: smaller linear index);
//  * p_det sums the kept p in linear-index order in blocks of 256.
#include "cpal_common.h"

namespace cpal {

__device__ __forceinline__ double block_max_d(double v) {
  __shared__ double red[16];
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < nw; ++w) r = fmax(r, red[w]);
  __syncthreads();
  return r;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v) {
  __shared__ T red[16];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  T r = 0;
  for (int w = 0; w < nw; ++w) r += red[w];
  __syncthreads();
  return r;
}

#define DET_STAGE 8192
#define DET_ROWS 8   // candidate test: rows per thread per block scan
// Reset of the per-update state, maxima alpha_m, candidate lists (Sec. 5.3):
// row i of mode o_t is a candidate iff the product with every other mode at
// its maximum exceeds tau.  One block of 1024 threads; the other modes' q
// are read once (into shared memory, at the candidate-list offsets, when
// those end within DET_STAGE entries).
__device__ __forceinline__ void det_cand_body(Blk bk, const OtherModes &om, double tau, u64 cap,
    DevState *st, int *__restrict__ cand) {
  __shared__ double sq[DET_STAGE];
  __shared__ double red[16][CPAL_MAXORDER];
  __shared__ double alpha[CPAL_MAXORDER];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) {
    // this update's step counter (device-side, so that a captured update
    // replays with the next value)
    st->t_cur = st->t_next;
    st->t_next = st->t_cur + 1;
    st->det_count = 0; st->combos = 0; st->s_det = 0; st->s_rnd = 0; st->s_rnd_used = 0;
    st->s_bar = 0; st->n_slots = 0; st->draws = 0; st->chunk_next = 0; st->accepted = 0;
    st->nchunks = 0; st->gathered = 0; st->p_det = 0.0; st->tau_eff = 1.0; st->flags = 0;
    for (int u = 0; u < CPAL_MAXORDER; ++u) st->ncand[u] = 0;
  }
  // a probability vector with no mass cannot be sampled: the update is void
  // (checked at the first barrier, so its loads overlap the staging below)
  int bad0 = 0;
  if (tid == 0)
    for (int u = 0; u < om.d; ++u) bad0 |= om.C[u][om.n[u] - 1] == 0;
  i64 lim = 0;   // staged at the candidate-list offsets
  for (int u = 0; u < om.d; ++u) lim = max(lim, om.cand_off[u] + om.n[u]);
  const bool staged = lim <= DET_STAGE;
  // maxima alpha_u (and the staging copy)
  double m[CPAL_MAXORDER];
#pragma unroll
  for (int u = 0; u < CPAL_MAXORDER; ++u) {
    m[u] = 0.0;
    if (u < om.d) {
      for (i64 i = tid; i < om.n[u]; i += blockDim.x) {
        const double v = om.q[u][i];
        if (staged) sq[om.cand_off[u] + i] = v;
        m[u] = fmax(m[u], v);
      }
      for (int off = 32; off > 0; off >>= 1) m[u] = fmax(m[u], __shfl_xor(m[u], off, 64));
      if (lane == 0) red[wid][u] = m[u];
    }
  }
  if (__syncthreads_or(bad0)) {
    if (tid == 0) st->flags |= CPAL_FLAG_STATE;
    return;
  }
  if (!(tau < 1.0)) return;
  if (tid < om.d) {
    double r = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w][tid]);
    alpha[tid] = r;
  }
  __syncthreads();
  double combos = 1.0;
  u64 combos_u = 1;
  for (int t = 0; t < om.d; ++t) {
    const i64 n = om.n[t];
    const double *q = om.q[t];
    const double *qs = sq + om.cand_off[t];
    int *out = cand + om.cand_off[t];
    u64 count = 0;
    // DET_ROWS consecutive rows per thread per pass: one block scan per
    // DET_ROWS * blockDim.x rows keeps the candidates in ascending order
    for (i64 base = 0; base < n; base += (i64)DET_ROWS * blockDim.x) {
      unsigned pred[DET_ROWS], c = 0;
#pragma unroll
      for (int r = 0; r < DET_ROWS; ++r) {
        const i64 i = base + (i64)tid * DET_ROWS + r;
        pred[r] = 0;
        if (i < n) {
          const double qi = staged ? qs[i] : q[i];
          double b = (t == 0) ? qi : alpha[0];
          for (int u = 1; u < om.d; ++u) b = b * ((u == t) ? qi : alpha[u]);
          pred[r] = b > tau;
        }
        c += pred[r];
      }
      unsigned tot;
      unsigned ex = block_excl_scan<unsigned>(c, &tot);
#pragma unroll
      for (int r = 0; r < DET_ROWS; ++r)
        if (pred[r]) out[count + ex++] = (int)(base + (i64)tid * DET_ROWS + r);
      count += tot;
    }
    if (tid == 0) st->ncand[t] = count;
    combos *= (double)count;
    combos_u *= count;
  }
  if (tid == 0) {
    if (combos > (double)cap) {
      st->flags |= CPAL_FLAG_DETCAP;
      st->combos = 0;
      st->tau_eff = 1.0;
    } else {
      st->combos = combos_u;
      st->tau_eff = tau;
    }
  }
}
__global__ void __launch_bounds__(1024) k_det_cand(OtherModes om, double tau, u64 cap,
                                                   DevState *st, int *__restrict__ cand) {
  det_cand_body(CPAL_BLK, om, tau, cap, st, cand);
}
CPAL_BODY(B_det_cand, 1024, 1, det_cand_body);

// Enumeration of the candidate product set in mixed-radix order (first other
// mode fastest).  The candidate lists are ascending, so this order is
// ascending in the linear index, and an order-preserving compaction of the
// rows with p > tau yields the deterministic set already sorted.  Block b
// owns the contiguous range [b*per, (b+1)*per) of combinations; pass 1
// counts, pass 2 writes at the block's prefix offset.
#define DET_BLOCKS 256
__device__ __forceinline__ bool det_row(const OtherModes &om, const int *__restrict__ cand,
                                        const unsigned *nc, u64 e, double tau, u64 &lin) {
  unsigned rem = (unsigned)e;
  double p = 0.0;
  lin = 0;
  for (int u = 0; u < om.d; ++u) {
    const unsigned c = rem % nc[u];
    rem /= nc[u];
    const int i = cand[om.cand_off[u] + c];
    const double qv = om.q[u][i];
    p = (u == 0) ? qv : p * qv;
    lin += (u64)i * om.stride[u];
  }
  return p > tau;
}

__device__ __forceinline__ void det_count_body(Blk bk, const OtherModes &om, double tau,
    DevState *st, const int *__restrict__ cand, unsigned *__restrict__ blk_cnt) {
  const u64 combos = st->combos;
  unsigned nc[CPAL_MAXORDER];
  for (int u = 0; u < om.d; ++u) nc[u] = (unsigned)st->ncand[u];
  const u64 per = (combos + DET_BLOCKS - 1) / DET_BLOCKS;
  const u64 b0 = (u64)bk.x * per, b1 = min(combos, b0 + per);
  unsigned cnt = 0;
  for (u64 e = b0 + threadIdx.x; e < b1; e += blockDim.x) {
    u64 lin;
    cnt += det_row(om, cand, nc, e, tau, lin) ? 1u : 0u;
  }
  cnt = wave_sum(cnt);
  __shared__ unsigned ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) blk_cnt[bk.x] = ws[0] + ws[1] + ws[2] + ws[3];
}
__global__ void __launch_bounds__(256) k_det_count(OtherModes om, double tau, DevState *st,
                                                   const int *__restrict__ cand,
                                                   unsigned *__restrict__ blk_cnt) {
  det_count_body(CPAL_BLK, om, tau, st, cand, blk_cnt);
}
CPAL_BODY(B_det_count, 256, 1, det_count_body);

__device__ __forceinline__ void det_scatter_body(Blk bk, const OtherModes &om, double tau,
    DevState *st, const int *__restrict__ cand, const unsigned *__restrict__ blk_cnt,
    u64 *__restrict__ det_keys, u64 det_cap) {
  const u64 combos = st->combos;
  unsigned nc[CPAL_MAXORDER];
  for (int u = 0; u < om.d; ++u) nc[u] = (unsigned)st->ncand[u];
  const u64 per = (combos + DET_BLOCKS - 1) / DET_BLOCKS;
  const u64 b0 = (u64)bk.x * per, b1 = min(combos, b0 + per);
  __shared__ u64 sh_off;
  if (threadIdx.x < 64) {
    u64 before = 0, all = 0;
    for (int b = threadIdx.x; b < DET_BLOCKS; b += 64) {
      const u64 v = blk_cnt[b];
      all += v;
      if (b < (int)bk.x) before += v;
    }
    before = wave_sum(before);
    all = wave_sum(all);
    if (threadIdx.x == 0) {
      sh_off = before;
      if (bk.x == 0) st->det_count = all;
    }
  }
  __syncthreads();
  u64 off = sh_off;
  for (u64 base = b0; base < b1; base += blockDim.x) {
    const u64 e = base + threadIdx.x;
    u64 lin = 0;
    const unsigned pass = (e < b1 && det_row(om, cand, nc, e, tau, lin)) ? 1u : 0u;
    unsigned tot;
    const unsigned ex = block_excl_scan<unsigned>(pass, &tot);
    if (pass && off + ex < det_cap) det_keys[off + ex] = lin;
    off += tot;
  }
}
__global__ void __launch_bounds__(256) k_det_scatter(OtherModes om, double tau, DevState *st,
                                                     const int *__restrict__ cand,
                                                     const unsigned *__restrict__ blk_cnt,
                                                     u64 *__restrict__ det_keys, u64 det_cap) {
  det_scatter_body(CPAL_BLK, om, tau, st, cand, blk_cnt, det_keys, det_cap);
}
CPAL_BODY(B_det_scatter, 256, 1, det_scatter_body);

// Sizes of the sampled system once p_det (tot) is known.
__device__ __forceinline__ void det_finish_state(DevState *st, i64 n, i64 s, double tot) {
  st->s_det = n;
  st->p_det = tot;
  i64 s_rnd = s - n;
  if (s_rnd > 0 && !(1.0 - tot > 0x1p-40)) {
    s_rnd = 0;
    st->flags |= CPAL_FLAG_PDET_ONE;
  }
  st->s_rnd = s_rnd;
  st->chunk_next = 0;
  st->accepted = 0;
}

// Deterministic rows: truncation to the s most probable when needed, output
// to samp_idx[0..s_det), p_det, s_rnd.  One block of 1024 threads.  Fewer
// than s rows that fit in shared memory (the usual case) stay there: p, the
// partial sums and the total never leave the block.
__device__ __forceinline__ void det_finish_body(Blk bk, const OtherModes &om, DevState *st,
    const u64 *__restrict__ det_keys, double *__restrict__ det_p, double *__restrict__ kept_p,
    double *__restrict__ psum, u64 det_cap, i64 s, u64 *__restrict__ samp_idx,
    unsigned char *__restrict__ keep) {
  const int tid = threadIdx.x;
  if (st->flags & CPAL_FLAG_STATE) {
    if (tid == 0) { st->s_det = 0; st->s_rnd = 0; st->p_det = 0.0; }
    return;
  }
  const u64 cnt = st->det_count;
  i64 n = (i64)min(cnt, det_cap);
  if (tid == 0 && cnt > det_cap) st->flags |= CPAL_FLAG_OVERFLOW;
  __shared__ double sp[DET_STAGE];
  __shared__ double spart[DET_STAGE / 256];
  if (n < s && n <= DET_STAGE) {
    for (i64 i = tid; i < n; i += blockDim.x) {
      const u64 key = det_keys[i];
      samp_idx[i] = key;
      sp[i] = prob_of(om, key);
    }
    __syncthreads();
    const i64 nb = (n + 255) / 256;
    if (tid < nb) {
      double part = 0.0;
      const i64 e = min(n, (i64)(tid + 1) * 256);
#pragma unroll 16
      for (i64 i = (i64)tid * 256; i < e; ++i) part = part + sp[i];
      spart[tid] = part;
    }
    __syncthreads();
    if (tid == 0) {
      double tot = 0.0;
      for (i64 b = 0; b < nb; ++b) tot = tot + spart[b];
      det_finish_state(st, n, s, tot);
    }
    return;
  }
  for (i64 i = tid; i < n; i += blockDim.x) det_p[i] = prob_of(om, det_keys[i]);
  __syncthreads();
  if (n >= s) {
    // threshold theta: the largest bit pattern with #{p >= theta} >= s
    u64 lo = 0, hi = 1ull << 63;
    while (hi - lo > 1) {
      const u64 mid = lo + (hi - lo) / 2;
      u64 c = 0;
      for (i64 i = tid; i < n; i += blockDim.x) c += (u64)(__double_as_longlong(det_p[i]) >= (i64)mid);
      c = block_sum<u64>(c);
      if (c >= (u64)s) lo = mid; else hi = mid;
    }
    const i64 theta = (i64)lo;
    u64 gt = 0;
    for (i64 i = tid; i < n; i += blockDim.x) gt += (u64)(__double_as_longlong(det_p[i]) > theta);
    gt = block_sum<u64>(gt);
    const u64 need = (u64)s - gt;
    // first `need` rows equal to theta in linear-index order
    u64 eq_seen = 0, out_pos = 0;
    for (i64 base = 0; base < n; base += blockDim.x) {
      const i64 i = base + tid;
      i64 bits = 0;
      unsigned is_eq = 0;
      if (i < n) { bits = __double_as_longlong(det_p[i]); is_eq = bits == theta; }
      unsigned eqtot;
      const unsigned eq_ex = block_excl_scan<unsigned>(is_eq, &eqtot);
      unsigned kp = 0;
      if (i < n) kp = (bits > theta) || (is_eq && eq_seen + eq_ex < need);
      unsigned ktot;
      const unsigned k_ex = block_excl_scan<unsigned>(kp, &ktot);
      if (kp) {
        samp_idx[out_pos + k_ex] = det_keys[i];
        kept_p[out_pos + k_ex] = det_p[i];
      }
      eq_seen += eqtot;
      out_pos += ktot;
    }
    n = s;
    if (tid == 0) st->flags |= CPAL_FLAG_DET_TRUNC;
  } else {
    for (i64 i = tid; i < n; i += blockDim.x) { samp_idx[i] = det_keys[i]; kept_p[i] = det_p[i]; }
  }
  __syncthreads();
  // p_det in blocks of 256 (ascending linear index), partials summed in
  // order; the probabilities are staged in shared memory when they fit
  const i64 nb = (n + 255) / 256;
  const bool staged = n <= DET_STAGE;
  if (staged)
    for (i64 i = tid; i < n; i += blockDim.x) sp[i] = kept_p[i];
  __syncthreads();
  for (i64 b = tid; b < nb; b += blockDim.x) {
    double part = 0.0;
    const i64 e = min(n, (b + 1) * 256);
    if (staged) {
      for (i64 i = b * 256; i < e; ++i) part = part + sp[i];
    } else {
#pragma unroll 16
      for (i64 i = b * 256; i < e; ++i) part = part + kept_p[i];
    }
    psum[b] = part;
  }
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (i64 b = 0; b < nb; ++b) tot = tot + psum[b];
    det_finish_state(st, n, s, tot);
  }
  (void)keep;
}
__global__ void __launch_bounds__(1024) k_det_finish(OtherModes om, DevState *st,
                                                     const u64 *__restrict__ det_keys,
                                                     double *__restrict__ det_p,
                                                     double *__restrict__ kept_p,
                                                     double *__restrict__ psum, u64 det_cap,
                                                     i64 s, u64 *__restrict__ samp_idx,
                                                     unsigned char *__restrict__ keep) {
  det_finish_body(CPAL_BLK, om, st, det_keys, det_p, kept_p, psum, det_cap, s, samp_idx, keep);
}
CPAL_BODY(B_det_finish, 1024, 1, det_finish_body);

__device__ __forceinline__ i64 max_draws_of(i64 s_rnd) { return 64 * s_rnd + (1ll << 20); }

// Random rows (Alg. 2) in chunks of CPAL_KRP_CHUNK consecutive draws, one
// draw per thread of a 256-thread block; a chunk's accepted rows (product
// probability <= tau_eff, i.e. outside the deterministic set) are compacted
// in draw order into buf, their positions in the chunk into bpos and their
// number into chunk_cnt.  The chunks processed always form a prefix of the
// draw sequence that holds at least s_rnd accepted draws (or all
// max_draws draws):
//  * first pass: chunk b for block b < the expected need, s_rnd / (1 - p_det)
//    draws plus a margin; no atomics;
//  * top-up pass: when the first pass fell short, blocks take further chunks
//    in increasing order (atomic ticket) until enough were accepted.
// When the other modes' CDFs fit (stage_n > 0 entries) every block first
// copies them to shared memory and the binary searches run there.
__device__ __forceinline__ i64 draw_need_chunks(const DevState *st, i64 s_rnd) {
  const double rate = fmax(1.0 - st->p_det, 1.0 / 1024.0);
  return (i64)ceil((double)s_rnd / rate * 1.02 / CPAL_KRP_CHUNK) + 2;
}

struct DrawModes {
  u64 W[CPAL_MAXORDER];
  const u64 *C[CPAL_MAXORDER];
  bool staged;
};

template <int DD>
__device__ __forceinline__ void draw_setup(const OtherModes &om, int stage_n, unsigned char *dsm,
                                           DrawModes &dm) {
  const int d = DD > 0 ? DD : om.d;
#pragma unroll
  for (int u = 0; u < d; ++u) {
    dm.W[u] = om.C[u][om.n[u] - 1];
    dm.C[u] = om.C[u];
  }
  dm.staged = stage_n > 0;
  if (stage_n > 0) {   // block-uniform: every thread reaches the barrier below
    u64 *sC = (u64 *)dsm;
    int off = 0;
#pragma unroll
    for (int u = 0; u < d; ++u) {
      for (int i = threadIdx.x; i < om.n[u]; i += blockDim.x) sC[off + i] = om.C[u][i];
      dm.C[u] = sC + off;
      off += (int)om.n[u];
    }
    __syncthreads();
  }
}

// Draws of chunk c; returns the chunk's accepted count (block-uniform).
// DD = number of other modes (0: any, runtime loop).
template <int DD>
__device__ __forceinline__ unsigned draw_chunk(const OtherModes &om, const DrawModes &dm, u64 c,
                                               double tau, i64 max_draws, u64 seed, u64 stream_id,
                                               u64 t, u64 *__restrict__ buf,
                                               unsigned short *__restrict__ bpos,
                                               unsigned *__restrict__ chunk_cnt) {
  const int tid = threadIdx.x;
  const i64 j = (i64)c * CPAL_KRP_CHUNK + tid;
  u64 lin = 0;
  double p = 0.0;
  const int d = DD > 0 ? DD : om.d;
#pragma unroll
  for (int u = 0; u < d; ++u) {
    u64 ctr[4] = {(u64)j, (u64)om.mode[u] | ((u64)om.k << 8), t, 0ull};
    philox4x64_10(ctr, seed, stream_id);
    const u64 x = scale128(ctr[0], ctr[1], dm.W[u]);
    const i64 i = upper_bound_u64(dm.C[u], om.n[u], x);
    // q_i = w_i / W, recomputed from the CDF when it is staged in shared
    // memory (the same operations, so the same value)
    const double qv = dm.staged ? (double)(dm.C[u][i] - (i > 0 ? dm.C[u][i - 1] : 0ull)) /
                                      (double)dm.W[u]
                                : om.q[u][i];
    p = (u == 0) ? qv : p * qv;
    lin += (u64)i * om.stride[u];
  }
  const bool ok = (j < max_draws) && p <= tau;
  unsigned tot;
  const unsigned pos = block_excl_scan<unsigned>(ok ? 1u : 0u, &tot);
  if (ok) {
    buf[c * CPAL_KRP_CHUNK + pos] = lin;
    bpos[c * CPAL_KRP_CHUNK + pos] = (unsigned short)tid;
  }
  if (tid == 0) chunk_cnt[c] = tot;
  return tot;
}

template <int DD>
__device__ __forceinline__ void draw_first_body(Blk bk, const OtherModes &om, DevState *st,
    u64 seed, u64 stream_id, u64 *__restrict__ buf, unsigned short *__restrict__ bpos,
    unsigned *__restrict__ chunk_cnt, int stage_n) {
  extern __shared__ __attribute__((aligned(16))) unsigned char dsm[];
  const i64 s_rnd = st->s_rnd;
  const u64 t = st->t_cur;
  const i64 max_draws = max_draws_of(s_rnd);
  const i64 max_chunks = (max_draws + CPAL_KRP_CHUNK - 1) / CPAL_KRP_CHUNK;
  const i64 first = s_rnd == 0 ? 0 : min(min(draw_need_chunks(st, s_rnd), max_chunks),
                                         (i64)bk.n);
  if (bk.x == 0 && threadIdx.x == 0) {
    st->first_chunks = (u64)first;
    st->chunk_next = (u64)first;
  }
  if ((i64)bk.x >= first) return;   // uniform per block
  DrawModes dm;
  draw_setup<DD>(om, stage_n, dsm, dm);
  draw_chunk<DD>(om, dm, bk.x, st->tau_eff, max_draws, seed, stream_id, t, buf, bpos,
             chunk_cnt);
}
template <int DD>
__global__ void __launch_bounds__(256) k_draw_first(OtherModes om, DevState *st, u64 seed,
                                                    u64 stream_id, u64 *__restrict__ buf,
                                                    unsigned short *__restrict__ bpos,
                                                    unsigned *__restrict__ chunk_cnt,
                                                    int stage_n) {
  draw_first_body<DD>(CPAL_BLK, om, st, seed, stream_id, buf, bpos, chunk_cnt, stage_n);
}
template <int DD>
struct B_draw_first {
  static constexpr int NT = 256, MW = 1;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    draw_first_body<DD>(b, a...);
  }
};

template <int DD>
__device__ __forceinline__ void draw_more_body(Blk bk, const OtherModes &om, DevState *st, u64 seed,
    u64 stream_id, u64 *__restrict__ buf, unsigned short *__restrict__ bpos,
    unsigned *__restrict__ chunk_cnt, int stage_n) {
  extern __shared__ __attribute__((aligned(16))) unsigned char dsm[];
  __shared__ u64 sh_c;
  __shared__ int stop;
  const int tid = threadIdx.x;
  const i64 s_rnd = st->s_rnd;
  const u64 t = st->t_cur;
  if (s_rnd == 0) return;
  const i64 max_draws = max_draws_of(s_rnd);
  const u64 max_chunks = (u64)((max_draws + CPAL_KRP_CHUNK - 1) / CPAL_KRP_CHUNK);
  const u64 first = st->first_chunks;
  u64 acc0 = 0;
  for (u64 c = tid; c < first; c += blockDim.x) acc0 += chunk_cnt[c];
  acc0 = wave_sum(acc0);
  __shared__ u64 ws[4];
  if ((tid & 63) == 0) ws[tid >> 6] = acc0;
  __syncthreads();
  acc0 = ws[0] + ws[1] + ws[2] + ws[3];
  if ((i64)acc0 >= s_rnd || first >= max_chunks) return;   // uniform per block
  DrawModes dm;
  draw_setup<DD>(om, stage_n, dsm, dm);
  for (;;) {
    if (tid == 0) {
      const u64 acc = __hip_atomic_load(&st->accepted, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      stop = 0;
      if ((i64)(acc0 + acc) >= s_rnd) {
        stop = 1;
      } else {
        const u64 c = atomicAdd(&st->chunk_next, 1ull);
        if (c >= max_chunks) stop = 1; else sh_c = c;
      }
    }
    __syncthreads();
    if (stop) break;
    const unsigned tot = draw_chunk<DD>(om, dm, sh_c, st->tau_eff, max_draws, seed, stream_id, t, buf,
                                    bpos, chunk_cnt);
    if (tid == 0) atomicAdd(&st->accepted, (u64)tot);
    __syncthreads();
  }
}
template <int DD>
__global__ void __launch_bounds__(256) k_draw_more(OtherModes om, DevState *st, u64 seed,
                                                   u64 stream_id, u64 *__restrict__ buf,
                                                   unsigned short *__restrict__ bpos,
                                                   unsigned *__restrict__ chunk_cnt,
                                                   int stage_n) {
  draw_more_body<DD>(CPAL_BLK, om, st, seed, stream_id, buf, bpos, chunk_cnt, stage_n);
}
template <int DD>
struct B_draw_more {
  static constexpr int NT = 256, MW = 1;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    draw_more_body<DD>(b, a...);
  }
};

// Finishes the entry of accepted draw `pos` of row `key` in the draw table
// (linear probing from slot h, whose compare-and-swap returned old).  The
// draw that enters a row stores its position (its slot carries the row); a
// later draw of the same row only counts itself as a repeat.  The table has
// at least twice as many entries as draws, so a free entry exists.
// With det_rep the row is carried by its earliest draw (an atomic minimum
// over the draws of the row, the entry's first starting at ~0), so which slot
// carries a repeated row, and with it the order of the sums over the rows,
// does not depend on timing.
__device__ __forceinline__ void draw_insert_from(DrawEntry *tab, u64 mask, u64 key, u64 h,
                                                 u64 old, unsigned pos, bool det_rep) {
  for (u64 probe = 0; old != CPAL_EMPTY_KEY && old != key && probe < mask; ++probe) {
    h = (h + 1) & mask;
    old = atomicCAS(&tab[h].key, CPAL_EMPTY_KEY, key);
  }
  if (old == CPAL_EMPTY_KEY) {
    if (det_rep) atomicMin(&tab[h].first, pos);
    else tab[h].first = pos;
  } else if (old == key) {
    atomicAdd(&tab[h].cnt, 1u);
    if (det_rep) atomicMin(&tab[h].first, pos);
  }
}

#define CMP_WINS 64   // windows of 256 chunks whose owned chunk is kept at once

// The first s_rnd accepted draws in draw order: every block scans the chunk
// counts (a prefix of the chunk sequence) itself, window by window of 256
// chunks, and keeps where the one chunk of each window that it owns (chunk
// blockIdx.x of the window; launched with 256 blocks of 256 threads) goes;
// then it copies the accepted rows of its chunks to their place and enters
// them into the draw table, four chunks at a time with their first
// compare-and-swaps in flight together.  The table so holds, per row, the
// position of one of its draws and its number of further draws: the repeats
// of Sec. 4.1 without sorting the draws (which draw represents the row
// depends on timing; the row, its count and weight do not).  Block 0 also records the number of rows used and the
// draw count (index of the s_rnd-th accepted draw + 1).
__device__ __forceinline__ void compact_body(Blk bk, DevState *st, const u64 *__restrict__ buf,
    const unsigned *__restrict__ chunk_cnt, const unsigned short *__restrict__ bpos,
    u64 *__restrict__ keys, DrawEntry *tab, u64 tmask, int tshift, int det_rep) {
  __shared__ i64 sh_draws;
  __shared__ u64 own_off[CMP_WINS];
  __shared__ unsigned own_cnt[CMP_WINS];
  const int tid = threadIdx.x;
  const i64 s_rnd = st->s_rnd;
    const i64 max_draws = max_draws_of(s_rnd);
  const u64 max_chunks = (u64)((max_draws + CPAL_KRP_CHUNK - 1) / CPAL_KRP_CHUNK);
  const u64 Q = min(st->chunk_next, max_chunks);
  const u64 nwin = (Q + 255) / 256;
  if (tid == 0) sh_draws = -1;
  u64 carry = 0;
  for (u64 wb = 0; wb < nwin; wb += CMP_WINS) {
    const int nw = (int)min((u64)CMP_WINS, nwin - wb);
    for (int wi = 0; wi < nw; ++wi) {
      const u64 b0 = (wb + wi) * 256;
      const u64 q = b0 + tid;
      const unsigned v = q < Q ? chunk_cnt[q] : 0u;
      u64 tot;
      const u64 off = carry + block_excl_scan<u64>((u64)v, &tot);
      if (q < Q && s_rnd > 0 && off <= (u64)(s_rnd - 1) && (u64)(s_rnd - 1) < off + v)
        sh_draws = (i64)q * CPAL_KRP_CHUNK + bpos[q * CPAL_KRP_CHUNK + (s_rnd - 1 - off)] + 1;
      if (tid == (int)bk.x) {
        // rows of the owned chunk that fall among the first s_rnd
        own_off[wi] = off;
        own_cnt[wi] = off < (u64)s_rnd ? (unsigned)min((u64)v, (u64)s_rnd - off) : 0u;
      }
      carry += tot;
    }
    __syncthreads();
    for (int w0 = 0; w0 < nw; w0 += 4) {
      u64 key[4], h[4], old[4];
      unsigned pos[4];
      bool has[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int wi = w0 + r;
        has[r] = wi < nw && (unsigned)tid < own_cnt[wi];
        if (has[r]) {
          const u64 q = (wb + wi) * 256 + bk.x;
          key[r] = buf[q * CPAL_KRP_CHUNK + tid];
          pos[r] = (unsigned)(own_off[wi] + tid);
          keys[pos[r]] = key[r];
          h[r] = key_hash(key[r], tshift);
          old[r] = atomicCAS(&tab[h[r]].key, CPAL_EMPTY_KEY, key[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (has[r]) draw_insert_from(tab, tmask, key[r], h[r], old[r], pos[r], det_rep != 0);
    }
    __syncthreads();   // own_off / own_cnt are refilled by the next batch
  }
  __syncthreads();
  if (bk.x == 0 && tid == 0) {
    st->nchunks = (i64)Q;
    if (s_rnd == 0) {
      st->s_rnd_used = 0;
      st->draws = 0;
    } else if ((i64)carry < s_rnd) {
      st->s_rnd_used = (i64)carry;
      st->draws = max_draws;
      st->flags |= CPAL_FLAG_DRAWCAP;
    } else {
      st->s_rnd_used = s_rnd;
      st->draws = sh_draws;
    }
  }
}
__global__ void __launch_bounds__(256) k_compact(DevState *st, const u64 *__restrict__ buf,
                                                 const unsigned *__restrict__ chunk_cnt,
                                                 const unsigned short *__restrict__ bpos,
                                                 u64 *__restrict__ keys, DrawEntry *tab,
                                                 u64 tmask, int tshift, int det_rep) {
  compact_body(CPAL_BLK, st, buf, chunk_cnt, bpos, keys, tab, tmask, tshift, det_rep);
}
CPAL_BODY(B_compact, 256, 1, compact_body);

__global__ void k_set_step(DevState *st, u64 t) { st->t_next = t; }

void launch_set_step(DevState *st, u64 t, hipStream_t s) {
  launch_1(k_set_step, dim3(1), dim3(1), 0, s, st, t);
}

void launch_det_cand(const OtherModes &om, double tau, u64 cap, DevState *st, int *cand,
                     hipStream_t s) {
  launch_b<B_det_cand>(k_det_cand, dim3(1), dim3(1024), 0, s, om, tau, cap, st, cand);
}
void launch_det_enum(const OtherModes &om, double tau, DevState *st, const int *cand,
                     unsigned *blk_cnt, u64 *det_keys, u64 det_cap, hipStream_t s) {
  launch_b<B_det_count>(k_det_count, dim3(DET_BLOCKS), dim3(256), 0, s, om, tau, st, cand,
                        blk_cnt);
  launch_b<B_det_scatter>(k_det_scatter, dim3(DET_BLOCKS), dim3(256), 0, s, om, tau, st, cand,
                          blk_cnt, det_keys, det_cap);
}
void launch_det_finish(const OtherModes &om, DevState *st, const u64 *det_keys, double *det_p,
                       double *kept_p, double *psum, u64 det_cap, i64 s, u64 *samp_idx,
                       hipStream_t st_) {
  launch_b<B_det_finish>(k_det_finish, dim3(1), dim3(1024), 0, st_, om, st, det_keys, det_p,
                         kept_p, psum, det_cap, s, samp_idx, (unsigned char *)nullptr);
}
template <int DD>
static void launch_draw_t(const OtherModes &om, DevState *st, u64 seed, u64 stream_id, u64 *buf,
                          unsigned short *bpos, unsigned *chunk_cnt, int grid_first,
                          int grid_more, int stage_n, size_t sh, hipStream_t s) {
  launch_b<B_draw_first<DD>>(k_draw_first<DD>, dim3(grid_first), dim3(256), sh, s, om, st, seed,
                             stream_id, buf, bpos, chunk_cnt, stage_n);
  launch_b<B_draw_more<DD>>(k_draw_more<DD>, dim3(grid_more), dim3(256), sh, s, om, st, seed,
                            stream_id, buf, bpos, chunk_cnt, stage_n);
}
void launch_draw(const OtherModes &om, DevState *st, u64 seed, u64 stream_id, u64 *buf,
                 unsigned short *bpos, unsigned *chunk_cnt, int grid_first, int grid_more,
                 hipStream_t s) {
  i64 tot = 0;
  for (int u = 0; u < om.d; ++u) tot += om.n[u];
  const int stage_n = tot <= 8192 ? (int)tot : 0;   // <= 64 KB of shared memory
  const size_t sh = (size_t)stage_n * sizeof(u64);
  const int dd = om.d <= 4 ? om.d : 0;
  if (dd == 1)
    launch_draw_t<1>(om, st, seed, stream_id, buf, bpos, chunk_cnt, grid_first, grid_more, stage_n,
                     sh, s);
  else if (dd == 2)
    launch_draw_t<2>(om, st, seed, stream_id, buf, bpos, chunk_cnt, grid_first, grid_more, stage_n,
                     sh, s);
  else if (dd == 3)
    launch_draw_t<3>(om, st, seed, stream_id, buf, bpos, chunk_cnt, grid_first, grid_more, stage_n,
                     sh, s);
  else if (dd == 4)
    launch_draw_t<4>(om, st, seed, stream_id, buf, bpos, chunk_cnt, grid_first, grid_more, stage_n,
                     sh, s);
  else
    launch_draw_t<0>(om, st, seed, stream_id, buf, bpos, chunk_cnt, grid_first, grid_more, stage_n,
                     sh, s);
}
void launch_compact(DevState *st, const u64 *buf, const unsigned *chunk_cnt,
                    const unsigned short *bpos, u64 *keys, DrawEntry *tab, u64 tmask, int tshift,
                    bool det_rep, hipStream_t s) {
  launch_b<B_compact>(k_compact, dim3(256), dim3(256), 0, s, st, buf, chunk_cnt, bpos, keys, tab,
                      tmask, tshift, det_rep ? 1 : 0);
}

__global__ void k_draw_table_clear(DrawEntry *__restrict__ tab, u64 n) {
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x)
    tab[i] = DrawEntry{CPAL_EMPTY_KEY, ~0u, 0u};
}

void launch_draw_table_clear(DrawEntry *tab, u64 n, hipStream_t s) {
  const u64 g = std::min<u64>((n + 255) / 256, 4096);
  launch_1(k_draw_table_clear, dim3((unsigned)std::max<u64>(g, 1)), dim3(256), 0, s, tab, n);
}

}  // namespace cpal
