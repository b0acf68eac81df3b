// TnsrSamp and the sampled MTTKRP (Sec. 6.3, eq. (1.2)): every nonzero (i_k, x)
// of sampled fiber j adds omega_j x z_j to M(i_k,:) (gather precision T).
// M's rows have the padded stride ldz of the weighted KRP rows, so that a
// row's adds touch whole aligned lines (one 128-byte line for R <= 32 in
// FP32): atomic adds write through to memory line by line.
#include "cpal_common.h"

namespace cpal {

void scan_u32_dev(const unsigned *in, u64 *out, i64 cap, const i64 *n_dev, u64 *total,
                  void *scratch, hipStream_t s);
int gather_row_width(int R);

// ------------------------------------------------------------------ gather --
// The sampled fibers form one stream of nnz(X~) = sum_j len_j nonzeros; wave
// w takes stream positions [64c, 64c+64) for c = w, w + #waves, ...  A lane
// finds its row j in a 64-entry window of the fiber prefix sums (shuffles),
// loads its (i_k, x) pair and the wave then adds x * omega_j z_j into
// M(i_k,:), two nonzeros per instruction when R <= 32 (lanes = columns).
template <typename T>
struct NzLoad;
template <>
struct NzLoad<float> {
  const uint2 *pairs;
  __device__ __forceinline__ void get(u64 e, int &ik, float &x) const {
    const uint2 v = pairs[e];
    ik = (int)v.x;
    x = __uint_as_float(v.y);
  }
};
template <>
struct NzLoad<double> {
  const int *ik;
  const double *val;
  __device__ __forceinline__ void get(u64 e, int &i, double &x) const {
    i = ik[e];
    x = val[e];
  }
};

template <typename T>
__global__ void __launch_bounds__(256) k_gather(const DevState *st, int R,
                                                const u64 *__restrict__ cpos,
                                                const unsigned *__restrict__ coff,
                                                const unsigned *__restrict__ cidx, NzLoad<T> nz,
                                                const T *__restrict__ zhat, T *__restrict__ M,
                                                int ldz) {
  const i64 total = st->gathered;
  const i64 nf = st->n_fib;
  const int lane = threadIdx.x & 63;
  const i64 gw = ((i64)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const i64 nw = ((i64)gridDim.x * blockDim.x) >> 6;
  const bool half = R <= 32;
  const int col = half ? (lane & 31) : lane;
  const int sub = half ? (lane >> 5) : 0;
  for (i64 start = gw * 64; start < total; start += nw * 64) {
    // last nonempty fiber j0 with cpos[j0] <= start; 64 positions span <= 64 fibers
    i64 lo = 0, hi = nf;
    while (lo < hi) {
      const i64 mid = (lo + hi) >> 1;
      if (cpos[mid] > (u64)start) hi = mid; else lo = mid + 1;
    }
    const i64 j0 = lo - 1;
    const u64 winv = (j0 + lane < nf) ? cpos[j0 + lane] : ~0ull;
    const i64 p = start + lane;
    const bool valid = p < total;
    int wl = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
      const int cand = wl + step;
      const u64 v = __shfl(winv, cand < 64 ? cand : 63, 64);
      if (cand < 64 && v <= (u64)p) wl = cand;
    }
    const i64 j = j0 + wl;
    const u64 fp = __shfl(winv, wl, 64);
    int ik = 0;
    T x = T(0);
    i64 zr = 0;
    if (valid) {
      nz.get((u64)coff[j] + (u64)(p - (i64)fp), ik, x);
      zr = cidx[j];
    }
    for (int src = 0; src < 64; src += half ? 2 : 1) {
      const int sl = src + sub;
      const int ik_s = __shfl(ik, sl, 64);
      const T x_s = __shfl(x, sl, 64);
      const i64 z_s = __shfl(zr, sl, 64);
      const bool v_s = __shfl((int)valid, sl, 64) != 0;
      if (v_s && col < R) unsafeAtomicAdd(&M[(i64)ik_s * ldz + col], x_s * zhat[z_s * ldz + col]);
    }
  }
}

// The stream of gathered nonzeros (the sampled fibers one after the other)
// is cut into chunks of GT_CHUNK positions; the chunk's first and last
// nonempty fibers come from chunk_first, their stream positions are staged in
// shared memory (GT_WIN >= GT_CHUNK + 1 entries) and every position finds its
// fiber there.
#define GT_THREADS 512
#define GT_PER_THREAD 4
#define GT_CHUNK (GT_THREADS * GT_PER_THREAD)
static_assert(GT_CHUNK == CPAL_GATHER_CHUNK, "gather chunk must match the preparation's");
// A chunk's window holds the fibers starting inside it (at most GT_CHUNK)
// and the one overlapping its first position.
#define GT_WIN (GT_CHUNK + 8)   // the chunk's fiber starts and the end of its last fiber

// Segmented gather: workgroup g takes the chunks g, g + G, ... of GT_CHUNK
// stream positions; for a chunk
//  1. per thread, GT_PER_THREAD positions: the nonempty fiber holding the
//     position (binary search in the chunk's window of fiber starts), the
//     nonzero (i_k, x) and the fiber's sampled row, with every load
//     unconditional (positions past the chunk are clamped and masked);
//  2. the chunk's nonzeros are sorted by i_k in shared memory (stable LSD
//     radix sort, 6-bit digits ranked with wave ballots, keys i_k << 12 |
//     position in the chunk), unless the chunk spans at most sort_min
//     fibers (then they stay in stream order: long fibers have distinct
//     rows, and a sort would only delay the adds);
//  3. lane groups of LPN lanes (LPN = padded row width ldz) take equal
//     slices of the sorted list, lane c summing x * zhat(row, c) in a
//     register while i_k stays the same; a run that ends inside the slice is
//     added to M(i_k, c) at once, the first and last runs of every slice are
//     merged across slices in shared memory first, so every row of the chunk
//     costs one global atomic add per column (rows need i_k < 2^20).
#define GS_DIG 6
#define GS_BATCH 16   // sorted entries a lane group loads ahead (fits 128 VGPRs)

// Stable LSD radix sort of the chunk's GT_CHUNK keys ka (row << 12 |
// position) on key bits [12, 12 + bits), 6-bit digits ranked with wave
// ballots; returns the buffer holding the result (ka or kb).
__device__ __forceinline__ unsigned *chunk_radix(unsigned *ka, unsigned *kb, unsigned *tab,
                                                 int bits) {
  constexpr int NW = GT_THREADS / 64;
  constexpr int NT = 64 * GT_PER_THREAD * NW;   // digit x round x wave counters
  const int tid = threadIdx.x, w = tid >> 6;
  const u64 lt = __lanemask_lt();
  unsigned *src = ka, *dst = kb;
  for (int shift = 12; shift < 12 + bits; shift += GS_DIG) {
    for (int e = tid; e < NT; e += GT_THREADS) tab[e] = 0u;
    __syncthreads();
    unsigned key[GT_PER_THREAD], dg[GT_PER_THREAD], rk[GT_PER_THREAD];
#pragma unroll
    for (int r = 0; r < GT_PER_THREAD; ++r) {
      key[r] = src[r * GT_THREADS + tid];
      dg[r] = (key[r] >> shift) & 63u;
      u64 peers = ~0ull;
#pragma unroll
      for (int b = 0; b < GS_DIG; ++b) {
        const bool bit = (dg[r] >> b) & 1u;
        const u64 m = __ballot(bit);
        peers &= bit ? m : ~m;
      }
      rk[r] = (unsigned)__popcll(peers & lt);
      if (rk[r] == 0) tab[(dg[r] * GT_PER_THREAD + r) * NW + w] = (unsigned)__popcll(peers);
    }
    __syncthreads();
    {   // exclusive scan of tab in (digit, round, wave) order
      unsigned v[NT / GT_THREADS], sum = 0;
#pragma unroll
      for (int q = 0; q < NT / GT_THREADS; ++q) { v[q] = tab[tid * (NT / GT_THREADS) + q]; sum += v[q]; }
      unsigned tot;
      unsigned run = block_excl_scan<unsigned>(sum, &tot);
#pragma unroll
      for (int q = 0; q < NT / GT_THREADS; ++q) {
        tab[tid * (NT / GT_THREADS) + q] = run;
        run += v[q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < GT_PER_THREAD; ++r)
      dst[tab[(dg[r] * GT_PER_THREAD + r) * NW + w] + rk[r]] = key[r];
    __syncthreads();
    unsigned *t = src; src = dst; dst = t;
  }
  return src;
}

// Steps 1 and 2 for chunk ch; returns the sorted keys (ka or kb).
template <typename T>
__device__ __forceinline__ unsigned *seg_load_sort(
    i64 ch, i64 nch, i64 total, i64 nf, const u64 *__restrict__ cpos,
    const unsigned *__restrict__ coff, const unsigned *__restrict__ cidx,
    const unsigned *__restrict__ chunk_first, const NzLoad<T> &nz, int ikbits, int sort_min,
    u64 *win, unsigned *ka, unsigned *kb, T *lx, unsigned *lz, unsigned *tab) {
  const int tid = threadIdx.x;
  const i64 base = ch * GT_CHUNK;
  const i64 last = min(total, base + GT_CHUNK) - 1;
  const i64 jlo = chunk_first[ch];
  const i64 jhi = (ch + 1 < nch) ? (i64)chunk_first[ch + 1] : nf - 1;
  const int nwin = (int)(jhi - jlo + 1);   // <= GT_CHUNK + 1 <= GT_WIN
  __syncthreads();   // the previous chunk is finished with every shared array
  for (int e = tid; e < nwin; e += GT_THREADS) win[e] = cpos[jlo + e];
  __syncthreads();
  int jw[GT_PER_THREAD];
  u64 ee[GT_PER_THREAD];
#pragma unroll
  for (int u = 0; u < GT_PER_THREAD; ++u) {
    const u64 p = (u64)min(base + (i64)u * GT_THREADS + tid, last);
    int lo = 0, hi = nwin;   // last index with win[idx] <= p
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (win[mid] <= p) lo = mid; else hi = mid;
    }
    jw[u] = lo;
    ee[u] = p - win[lo];
  }
  unsigned zrow[GT_PER_THREAD];
#pragma unroll
  for (int u = 0; u < GT_PER_THREAD; ++u) {
    ee[u] += coff[jlo + jw[u]];
    zrow[u] = cidx[jlo + jw[u]];
  }
#pragma unroll
  for (int u = 0; u < GT_PER_THREAD; ++u) {
    int ik;
    T x;
    nz.get(ee[u], ik, x);
    const int li = u * GT_THREADS + tid;   // = position - base
    ka[li] = (base + li <= last) ? (((unsigned)ik << 12) | (unsigned)li) : 0xFFFFFFFFu;
    lx[li] = x;
    lz[li] = zrow[u];
  }
  __syncthreads();   // every entry is written before any group reads it
  // a chunk spanning at most sort_min fibers stays in stream order (rows are
  // distinct within a fiber, so sorting would merge little); the branch is
  // uniform over the workgroup
  return chunk_radix(ka, kb, tab, nwin > sort_min ? ikbits : 0);
}

// Step 3 over n row-sorted entries; entry q -> (row, x, KRP row) by get(q).
// A lane group of LPN lanes takes one entry at a time, lane c holding the
// columns c, c + LPN, ..., c + (CPL-1) LPN of the row (LPN * CPL = the
// padded row width): with CPL = 2 a wave instruction serves four entries,
// halving the per-entry bookkeeping.
template <typename T, int LPN, int CPL, typename Get, typename Add>
__device__ __forceinline__ void seg_reduce(const Get &get, int n, int R,
                                           const T *__restrict__ zhat, int ldz,
                                           const Add &add, int *srow,
                                           T (*svec)[LPN * CPL]) {
  constexpr int NG = GT_THREADS / LPN;
  constexpr int PER = GT_CHUNK / NG;
  constexpr int B = GS_BATCH / CPL;
  const int tid = threadIdx.x, gi = tid / LPN, c = tid % LPN;
  const int q0 = gi * PER, q1 = min(n, q0 + PER);
  int cur = -1, first = -1;
  T acc[CPL], facc[CPL];
#pragma unroll
  for (int j = 0; j < CPL; ++j) { acc[j] = T(0); facc[j] = T(0); }
  if (q0 < q1) {
    {
      unsigned r0;
      T x0;
      unsigned z0;
      get(q0, r0, x0, z0);
      cur = (int)r0;
    }
    for (int q = q0; q < q1; q += B) {
      unsigned rr[B];
      T xv[B], zv[B][CPL];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        unsigned zr;
        get(min(q + b, q1 - 1), rr[b], xv[b], zr);
#pragma unroll
        for (int j = 0; j < CPL; ++j) zv[b][j] = zhat[(i64)zr * ldz + c + j * LPN];
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        if (q + b < q1) {
          const int r = (int)rr[b];
          if (r != cur) {
            if (first < 0) {
              first = cur;
#pragma unroll
              for (int j = 0; j < CPL; ++j) facc[j] = acc[j];
            } else {
#pragma unroll
              for (int j = 0; j < CPL; ++j)
                if (c + j * LPN < R) add(cur, c + j * LPN, acc[j]);
            }
            cur = r;
#pragma unroll
            for (int j = 0; j < CPL; ++j) acc[j] = T(0);
          }
#pragma unroll
          for (int j = 0; j < CPL; ++j) acc[j] += xv[b] * zv[b][j];
        }
      }
    }
  }
  // slice ends: slot 2gi = first run, 2gi+1 = last run (-1: none)
  if (first < 0) {
    first = cur;
#pragma unroll
    for (int j = 0; j < CPL; ++j) facc[j] = acc[j];
    cur = -1;
  }
  if (c == 0) { srow[2 * gi] = first; srow[2 * gi + 1] = cur; }
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    svec[2 * gi][c + j * LPN] = facc[j];
    svec[2 * gi + 1][c + j * LPN] = acc[j];
  }
  __syncthreads();
  if (gi == 0 && n > 0) {
    int mr = -1;
    T ma[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) ma[j] = T(0);
    for (int sl = 0; sl < 2 * NG; ++sl) {
      const int r = srow[sl];
      if (r < 0) continue;
      if (r != mr) {
        if (mr >= 0) {
#pragma unroll
          for (int j = 0; j < CPL; ++j)
            if (c + j * LPN < R) add(mr, c + j * LPN, ma[j]);
        }
        mr = r;
#pragma unroll
        for (int j = 0; j < CPL; ++j) ma[j] = T(0);
      }
#pragma unroll
      for (int j = 0; j < CPL; ++j) ma[j] += svec[sl][c + j * LPN];
    }
    if (mr >= 0) {
#pragma unroll
      for (int j = 0; j < CPL; ++j)
        if (c + j * LPN < R) add(mr, c + j * LPN, ma[j]);
    }
  }
}

// Where a reduced run of row r goes: an atomic add into a copy of M in
// global memory, or a plain add into a row block in shared memory that only
// this workgroup touches (rows relative to the block; each row is added once
// per batch, so the adds of one batch never collide).
template <typename T>
struct GlobalAdd {
  T *M;
  int ldz;
  __device__ __forceinline__ void operator()(int r, int c, T v) const {
    unsafeAtomicAdd(&M[(i64)r * ldz + c], v);
  }
};
template <typename T>
struct LdsAdd {
  T *blk;
  int ld;
  __device__ __forceinline__ void operator()(int r, int c, T v) const { blk[r * ld + c] += v; }
};

template <typename T>
struct LdsEntries {
  const unsigned *keys;
  const T *lx;
  const unsigned *lz;
  __device__ __forceinline__ void operator()(int q, unsigned &r, T &x, unsigned &z) const {
    const unsigned k = keys[q];
    r = k >> 12;
    x = lx[k & 4095u];
    z = lz[k & 4095u];
  }
};

// Two workgroups per CU (4 waves per SIMD: at most 128 VGPRs; the FP32
// kernel's shared memory fits twice).  Lane groups of LPN lanes, CPL columns
// per lane (LPN * CPL = the padded row width ldz).
template <typename T, int LPN, int CPL>
__device__ __forceinline__ void gather_seg_body(Blk bk, const DevState *st, int R,
    const u64 *__restrict__ cpos, const unsigned *__restrict__ coff,
    const unsigned *__restrict__ cidx, const unsigned *__restrict__ chunk_first,
    const NzLoad<T> &nz, int ikbits, int sort_min, const T *__restrict__ zhat, int ldz,
    T *__restrict__ M, i64 nk) {
  constexpr int NG = GT_THREADS / LPN;
  __shared__ u64 win[GT_WIN];
  __shared__ unsigned ka[GT_CHUNK], kb[GT_CHUNK];
  __shared__ T lx[GT_CHUNK];
  __shared__ unsigned lz[GT_CHUNK];
  __shared__ unsigned tab[64 * GT_PER_THREAD * (GT_THREADS / 64)];
  __shared__ int srow[2 * NG];
  __shared__ T svec[2 * NG][LPN * CPL];
  const i64 total = st->gathered;
  const i64 nf = st->n_fib;
  const i64 nch = (total + GT_CHUNK - 1) / GT_CHUNK;
  // this XCD's copy of M: the adds of workgroups on one XCD stay in its L2
  T *Mx = M + (i64)(xcd_id() & (CPAL_MCOPIES - 1)) * nk * ldz;
  for (i64 ch = bk.x; ch < nch; ch += bk.n) {
    const unsigned *keys = seg_load_sort<T>(ch, nch, total, nf, cpos, coff, cidx, chunk_first, nz,
                                            ikbits, sort_min, win, ka, kb, lx, lz, tab);
    const int nvalid = (int)(min(total, (ch + 1) * GT_CHUNK) - ch * GT_CHUNK);
    seg_reduce<T, LPN, CPL>(LdsEntries<T>{keys, lx, lz}, nvalid, R, zhat, ldz,
                            GlobalAdd<T>{Mx, ldz}, srow, svec);
  }
}
template <typename T, int LPN, int CPL>
__global__ void __launch_bounds__(GT_THREADS, 4) k_gather_seg(
    const DevState *st, int R, const u64 *__restrict__ cpos, const unsigned *__restrict__ coff,
    const unsigned *__restrict__ cidx, const unsigned *__restrict__ chunk_first, NzLoad<T> nz,
    int ikbits, int sort_min, const T *__restrict__ zhat, int ldz, T *__restrict__ M, i64 nk) {
  gather_seg_body<T, LPN, CPL>(CPAL_BLK, st, R, cpos, coff, cidx, chunk_first, nz, ikbits, sort_min,
    zhat, ldz, M, nk);
}
template <typename T, int LPN, int CPL>
struct B_gather_seg {
  static constexpr int NT = GT_THREADS, MW = 4;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    gather_seg_body<T, LPN, CPL>(b, a...);
  }
};

// ----------------------------------------------------------- bucketed gather --
// For modes whose sampled fibers are long, a stream chunk spans one or two
// fibers, its rows are all distinct and every nonzero costs a global row add
// (two 64-byte atomic requests for a 25-column FP32 row, and the gather runs
// at the chip's atomic request rate).  Here the gathered nonzeros are first
// moved into BK_BUCKETS buckets of 2^bshift consecutive output rows (count,
// scan, scatter), then reduced chunk by chunk like the stream: a chunk of a
// bucket holds many nonzeros of each of its rows, which are summed in
// registers before their one add.  A bucketed nonzero is one 16-byte record
// {row, value bits, KRP row, 0}.  FP32 gather; the order inside a bucket
// depends on timing (rounding order only).
#define BK_BUCKETS 4096   // at most
#define BK_THREADS 256
#define BK_PER (GT_CHUNK / BK_THREADS)
#define BK_GRID 1024      // at most

// A bucketed nonzero: one 16-byte record {row, KRP row, value} written by a
// single store (FP32: {row, value bits, KRP row, 0}; FP64: {row, KRP row,
// value bits low, high}).
template <typename T>
struct BktRec;
template <>
struct BktRec<float> {
  static __device__ __forceinline__ uint4 make(int ik, float x, unsigned zr) {
    return make_uint4((unsigned)ik, __float_as_uint(x), zr, 0u);
  }
  static __device__ __forceinline__ void get(const uint4 &v, unsigned &ik, float &x,
                                             unsigned &zr) {
    ik = v.x;
    x = __uint_as_float(v.y);
    zr = v.z;
  }
};
template <>
struct BktRec<double> {
  static __device__ __forceinline__ uint4 make(int ik, double x, unsigned zr) {
    const u64 b = (u64)__double_as_longlong(x);
    return make_uint4((unsigned)ik, zr, (unsigned)b, (unsigned)(b >> 32));
  }
  static __device__ __forceinline__ void get(const uint4 &v, unsigned &ik, double &x,
                                             unsigned &zr) {
    ik = v.x;
    zr = v.y;
    x = __longlong_as_double((long long)(((u64)v.w << 32) | v.z));
  }
};

// A compact record of the shared-block bucketed gather: the row within its
// bucket (bucket width at most 2^9 rows) and the KRP row in one word
// ((zr << 9) | local row; zr < 2^23), then the value: 12 bytes in FP64,
// 8 in FP32.
#define BK_CROWBITS 9
template <typename T>
struct BktC;
template <>
struct BktC<double> {
  typedef uint3 V;
  static __device__ __forceinline__ V make(unsigned local, double x, unsigned zr) {
    const u64 b = (u64)__double_as_longlong(x);
    return make_uint3((zr << BK_CROWBITS) | local, (unsigned)b, (unsigned)(b >> 32));
  }
  static __device__ __forceinline__ void get(const V &v, unsigned &local, double &x,
                                             unsigned &zr) {
    local = v.x & ((1u << BK_CROWBITS) - 1u);
    zr = v.x >> BK_CROWBITS;
    x = __longlong_as_double((long long)(((u64)v.z << 32) | v.y));
  }
};
template <>
struct BktC<float> {
  typedef uint2 V;
  static __device__ __forceinline__ V make(unsigned local, float x, unsigned zr) {
    return make_uint2((zr << BK_CROWBITS) | local, __float_as_uint(x));
  }
  static __device__ __forceinline__ void get(const V &v, unsigned &local, float &x,
                                             unsigned &zr) {
    local = v.x & ((1u << BK_CROWBITS) - 1u);
    zr = v.x >> BK_CROWBITS;
    x = __uint_as_float(v.y);
  }
};

// Calls f(ik, x, KRP row) for every position of stream chunk ch (the chunk's
// fiber starts are staged in win; positions find their fiber there) whose
// fiber is shorter than lmin nonzeros (lmin = 0: every position); the other
// positions load nothing from the nonzeros (they re-read the chunk's first
// one, a cached line).
template <typename T, typename F>
__device__ __forceinline__ void bk_chunk(i64 ch, i64 nch, i64 total, i64 nf,
                                         const u64 *__restrict__ cpos,
                                         const unsigned *__restrict__ coff,
                                         const unsigned *__restrict__ cidx,
                                         const unsigned *__restrict__ chunk_first,
                                         const NzLoad<T> &nz, u64 *win, unsigned lmin, F &&f) {
  const int tid = threadIdx.x;
  const i64 base = ch * GT_CHUNK;
  const i64 last = min(total, base + GT_CHUNK) - 1;
  const i64 jlo = chunk_first[ch];
  const i64 jhi = (ch + 1 < nch) ? (i64)chunk_first[ch + 1] : nf - 1;
  const int nwin = (int)(jhi - jlo + 1);   // <= GT_CHUNK + 1, plus the end below
  __syncthreads();   // the previous chunk is finished with win
  for (int e = tid; e <= nwin; e += BK_THREADS)
    win[e] = jlo + e < nf ? cpos[jlo + e] : (u64)total;
  __syncthreads();
  // all BK_PER positions of the thread are located first, then every load
  // is issued before any is used (positions past the chunk are clamped to
  // its last one and skipped at the end)
  int jw[BK_PER];
  u64 pp[BK_PER];
  bool keep[BK_PER];
#pragma unroll
  for (int u = 0; u < BK_PER; ++u) {
    const u64 p = (u64)min(base + (i64)u * BK_THREADS + tid, last);
    int lo = 0, hi = nwin;   // last index with win[idx] <= p
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (win[mid] <= p) lo = mid; else hi = mid;
    }
    jw[u] = lo;
    pp[u] = p - win[lo];
    keep[u] = base + (i64)u * BK_THREADS + tid <= last &&
              (lmin == 0u || win[lo + 1] - win[lo] < (u64)lmin);
  }
  unsigned zr[BK_PER];
#pragma unroll
  for (int u = 0; u < BK_PER; ++u) {
    pp[u] = keep[u] ? pp[u] + coff[jlo + jw[u]] : (u64)coff[jlo];
    zr[u] = cidx[jlo + jw[u]];
  }
  int ik[BK_PER];
  T x[BK_PER];
#pragma unroll
  for (int u = 0; u < BK_PER; ++u) nz.get(pp[u], ik[u], x[u]);
#pragma unroll
  for (int u = 0; u < BK_PER; ++u) f(keep[u], ik[u], x[u], zr[u]);   // every lane
}

// Runs of equal buckets among a wave's lanes (lanes in stream order): run
// heads, the run's length at its head, and each lane's head.
struct BucketRuns {
  int bkt;       // this lane's bucket, -1 without a position
  bool head;
  int len;       // at a head: lanes in its run
  int headlane;
};
__device__ __forceinline__ BucketRuns bucket_runs(bool kp, int bkt) {
  const int lane = threadIdx.x & 63;
  bkt = kp ? bkt : -1;
  const int prev = __shfl_up(bkt, 1, 64);
  const bool bnd = lane == 0 || prev != bkt;
  const u64 bm = __ballot(bnd);
  const u64 rest = (bm >> lane) >> 1;
  BucketRuns r;
  r.bkt = bkt;
  r.head = kp && bnd;
  r.len = rest ? __ffsll((long long)rest) : 64 - lane;
  r.headlane = 63 - __clzll(bm & ((2ull << lane) - 1ull));
  return r;
}

// Workgroup w takes the consecutive chunks [w cpw, (w + 1) cpw) of the stream
// in both passes, so its counts and its scatter see the same nonzeros.
// (The count pass reads the rows only: an NzLoad whose value is never used.)
template <typename T>
__device__ __forceinline__ void bkt_count_body(Blk bk, const DevState *st,
    const u64 *__restrict__ cpos, const unsigned *__restrict__ coff,
    const unsigned *__restrict__ cidx, const unsigned *__restrict__ chunk_first,
    const NzLoad<T> &nz, int bshift, int nb, unsigned lmin, unsigned *__restrict__ cnt) {
  __shared__ u64 win[GT_WIN];
  __shared__ unsigned h[BK_BUCKETS];
  const i64 total = st->gathered, nf = st->n_fib;
  const i64 nch = (total + GT_CHUNK - 1) / GT_CHUNK;
  const i64 cpw = (nch + bk.n - 1) / bk.n;
  const i64 c0 = (i64)bk.x * cpw, c1 = min(nch, c0 + cpw);
  for (int b = threadIdx.x; b < nb; b += BK_THREADS) h[b] = 0u;
  for (i64 ch = c0; ch < c1; ++ch)
    bk_chunk<T>(ch, nch, total, nf, cpos, coff, cidx, chunk_first, nz, win, lmin,
                [&](bool kp, int ik, T, unsigned) {
                  const BucketRuns r = bucket_runs(kp, (int)((unsigned)ik >> bshift));
                  if (r.head) atomicAdd(&h[r.bkt], (unsigned)r.len);
                });
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += BK_THREADS)
    cnt[(i64)b * bk.n + bk.x] = h[b];
}
template <typename T>
__global__ void __launch_bounds__(BK_THREADS) k_bkt_count(
    const DevState *st, const u64 *__restrict__ cpos, const unsigned *__restrict__ coff,
    const unsigned *__restrict__ cidx, const unsigned *__restrict__ chunk_first, NzLoad<T> nz,
    int bshift, int nb, unsigned lmin, unsigned *__restrict__ cnt) {
  bkt_count_body<T>(CPAL_BLK, st, cpos, coff, cidx, chunk_first, nz, bshift, nb, lmin, cnt);
}
template <typename T>
struct B_bkt_count {
  static constexpr int NT = BK_THREADS, MW = 1;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    bkt_count_body<T>(b, a...);
  }
};

// off = exclusive scan of cnt in (bucket, workgroup) order.
template <typename T>
__device__ __forceinline__ void bkt_scatter_body(Blk bk, const DevState *st,
    const u64 *__restrict__ cpos, const unsigned *__restrict__ coff,
    const unsigned *__restrict__ cidx, const unsigned *__restrict__ chunk_first,
    const NzLoad<T> &nz, int bshift, int nb, unsigned lmin, const u64 *__restrict__ off,
    uint4 *__restrict__ bent, int compact) {
  __shared__ u64 win[GT_WIN];
  __shared__ unsigned cur[BK_BUCKETS];
  const i64 total = st->gathered, nf = st->n_fib;
  const i64 nch = (total + GT_CHUNK - 1) / GT_CHUNK;
  const i64 cpw = (nch + bk.n - 1) / bk.n;
  const i64 c0 = (i64)bk.x * cpw, c1 = min(nch, c0 + cpw);
  for (int b = threadIdx.x; b < nb; b += BK_THREADS)
    cur[b] = (unsigned)off[(i64)b * bk.n + bk.x];
  for (i64 ch = c0; ch < c1; ++ch)
    bk_chunk<T>(ch, nch, total, nf, cpos, coff, cidx, chunk_first, nz, win, lmin,
                [&](bool kp, int ik, T x, unsigned zr) {
                  // one cursor add per run of equal buckets; the run's records
                  // take consecutive slots in stream order
                  const BucketRuns r = bucket_runs(kp, (int)((unsigned)ik >> bshift));
                  unsigned base = 0;
                  if (r.head) base = atomicAdd(&cur[r.bkt], (unsigned)r.len);
                  const unsigned hb = (unsigned)__shfl((int)base, r.headlane, 64);
                  const unsigned slot = hb + (unsigned)((threadIdx.x & 63) - r.headlane);
                  if (kp) {
                    if (compact)
                      ((typename BktC<T>::V *)bent)[slot] =
                          BktC<T>::make((unsigned)ik & ((1u << bshift) - 1u), x, zr);
                    else
                      bent[slot] = BktRec<T>::make(ik, x, zr);   // one 16-byte store
                  }
                });
}
template <typename T>
__global__ void __launch_bounds__(BK_THREADS) k_bkt_scatter(
    const DevState *st, const u64 *__restrict__ cpos, const unsigned *__restrict__ coff,
    const unsigned *__restrict__ cidx, const unsigned *__restrict__ chunk_first, NzLoad<T> nz,
    int bshift, int nb, unsigned lmin, const u64 *__restrict__ off, uint4 *__restrict__ bent,
    int compact) {
  bkt_scatter_body<T>(CPAL_BLK, st, cpos, coff, cidx, chunk_first, nz, bshift, nb, lmin, off, bent,
                      compact);
}
template <typename T>
struct B_bkt_scatter {
  static constexpr int NT = BK_THREADS, MW = 1;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    bkt_scatter_body<T>(b, a...);
  }
};

// The bucketed nonzeros in chunks of GT_CHUNK: loaded directly, sorted on
// the low `sortbits` bits of the row (rows of one bucket differ only there;
// a chunk crossing a bucket boundary merges a little less, nothing else),
// then reduced as in the segmented gather.
template <typename T, int LPN, int CPL>
__device__ __forceinline__ void gather_bkt_body(Blk bk, const DevState *st, int R,
    const uint4 *__restrict__ bent, int sortbits, const T *__restrict__ zhat, int ldz,
    T *__restrict__ M, i64 nk) {
  constexpr int NG = GT_THREADS / LPN;
  __shared__ unsigned ka[GT_CHUNK], kb[GT_CHUNK];
  __shared__ T lx[GT_CHUNK];
  __shared__ unsigned lz[GT_CHUNK];
  __shared__ unsigned tab[64 * GT_PER_THREAD * (GT_THREADS / 64)];
  __shared__ int srow[2 * NG];
  __shared__ T svec[2 * NG][LPN * CPL];
  const i64 total = st->gathered;
  const i64 nch = (total + GT_CHUNK - 1) / GT_CHUNK;
  T *Mx = M + (i64)(xcd_id() & (CPAL_MCOPIES - 1)) * nk * ldz;
  const int tid = threadIdx.x;
  for (i64 ch = bk.x; ch < nch; ch += bk.n) {
    const i64 base = ch * GT_CHUNK;
    const i64 last = min(total, base + GT_CHUNK) - 1;
    __syncthreads();   // the previous chunk is finished with every shared array
#pragma unroll
    for (int u = 0; u < GT_PER_THREAD; ++u) {
      const int li = u * GT_THREADS + tid;
      const bool valid = base + li <= last;
      unsigned ik = 0, zr = 0;
      T x = T(0);
      if (valid) BktRec<T>::get(bent[base + li], ik, x, zr);
      ka[li] = valid ? ((ik << 12) | (unsigned)li) : 0xFFFFFFFFu;
      lx[li] = x;
      lz[li] = zr;
    }
    __syncthreads();
    const unsigned *keys = chunk_radix(ka, kb, tab, sortbits);
    const int nvalid = (int)(last - base + 1);
    seg_reduce<T, LPN, CPL>(LdsEntries<T>{keys, lx, lz}, nvalid, R, zhat, ldz,
                            GlobalAdd<T>{Mx, ldz}, srow, svec);
  }
}
template <typename T, int LPN, int CPL>
__global__ void __launch_bounds__(GT_THREADS, 4) k_gather_bkt(
    const DevState *st, int R, const uint4 *__restrict__ bent, int sortbits,
    const T *__restrict__ zhat, int ldz, T *__restrict__ M, i64 nk) {
  gather_bkt_body<T, LPN, CPL>(CPAL_BLK, st, R, bent, sortbits, zhat, ldz, M, nk);
}
template <typename T, int LPN, int CPL>
struct B_gather_bkt {
  static constexpr int NT = GT_THREADS, MW = 4;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    gather_bkt_body<T, LPN, CPL>(b, a...);
  }
};

size_t gather_bkt_count_words() { return (size_t)BK_BUCKETS * BK_GRID; }

// max_total bounds the stream length (the context's nonzeros): the count and
// scatter grids are sized from it (about 8 chunks per workgroup, 64 to
// BK_GRID workgroups) and the buckets from n_k, so that small gathers do not
// pay for a scan of BK_BUCKETS x BK_GRID counts.
template <typename T>
static void launch_gather_bkt_t(const DevState *st, int R, const u64 *cpos, const unsigned *coff,
                                const unsigned *cidx, const unsigned *chunk_first, NzLoad<T> nz,
                                i64 nk, i64 max_total, const T *zhat, int ldz, T *M, int grid,
                                unsigned *cnt, u64 *off, void *scan_scratch, uint4 *bent,
                                hipStream_t s) {
  int ikbits = 1;
  while ((1ll << ikbits) < nk) ++ikbits;
  const int bshift = ikbits > 12 ? ikbits - 12 : 0;   // row >> bshift < BK_BUCKETS
  const int nb = (int)((nk + (1ll << bshift) - 1) >> bshift);
  const i64 chunks = (max_total + GT_CHUNK - 1) / GT_CHUNK;
  const int gb = (int)std::min<i64>(BK_GRID, std::max<i64>(64, (chunks + 7) / 8));
  launch_b<B_bkt_count<T>>(k_bkt_count<T>, dim3(gb), dim3(BK_THREADS), 0, s, st, cpos, coff, cidx,
                           chunk_first, nz, bshift, nb, 0u, cnt);
  scan_u32_dev(cnt, off, (i64)nb * gb, nullptr, nullptr, scan_scratch, s);
  launch_b<B_bkt_scatter<T>>(k_bkt_scatter<T>, dim3(gb), dim3(BK_THREADS), 0, s, st, cpos, coff,
                             cidx, chunk_first, nz, bshift, nb, 0u, off, bent, 0);
  const int rm = gather_row_width(R);
#define CPAL_BKT_LAUNCH(LPN, CPL)                                                                 \
  launch_b<B_gather_bkt<T, LPN, CPL>>(k_gather_bkt<T, LPN, CPL>, dim3(grid), dim3(GT_THREADS), 0, \
                                      s, st, R, bent, bshift, zhat, ldz, M, nk)
  if (rm == 16) CPAL_BKT_LAUNCH(16, 1);
  else if (rm == 32) CPAL_BKT_LAUNCH(16, 2);
  else CPAL_BKT_LAUNCH(32, 2);
#undef CPAL_BKT_LAUNCH
}

void launch_gather_bkt(bool f64, const DevState *st, int R, const u64 *cpos,
                       const unsigned *coff, const unsigned *cidx, const unsigned *chunk_first,
                       const uint2 *pairs, const int *ik, const double *v64, i64 nk,
                       i64 max_total, const void *zhat, int ldz, void *M, int grid, unsigned *cnt,
                       u64 *off, void *scan_scratch, uint4 *bent, hipStream_t s) {
  if (f64)
    launch_gather_bkt_t<double>(st, R, cpos, coff, cidx, chunk_first, NzLoad<double>{ik, v64},
                                nk, max_total, (const double *)zhat, ldz, (double *)M, grid, cnt,
                                off, scan_scratch, bent, s);
  else
    launch_gather_bkt_t<float>(st, R, cpos, coff, cidx, chunk_first, NzLoad<float>{pairs}, nk,
                               max_total, (const float *)zhat, ldz, (float *)M, grid, cnt, off,
                               scan_scratch, bent, s);
}

// brow[c] += x zp[c] for c < R (a shared FP64 row; atomic adds, since lanes
// of one wave can meet on a row).  The column guard is uniform over the
// wave; lanes without a nonzero pass x = 0 and a row of their own.
// Adds of a wave's 64 records into a shared FP64 block of rows (stride LDB):
// lane l holds record rec_lane(l) of the 64 (local row rl, value x, KRP row
// zr), and pass k gives each row of 16 lanes the record of its lane k (a DPP
// row broadcast), so that one add instruction covers 4 records x 16
// consecutive columns: four row windows of the block instead of 64 random
// rows at one column, which the shared memory takes at the rate of
// consecutive words (8.9 cycles per 64-lane FP64 add on gfx950, 26.7 for 64
// random rows).  Records 4k .. 4k+3 meet in pass k.
__device__ __forceinline__ unsigned rec_lane(int lane) {
  return 4u * (unsigned)(lane & 15) + (unsigned)(lane >> 4);
}

template <int K>
__device__ __forceinline__ int row_bcast(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x150 + K, 0xF, 0xF, false);   // row_newbcast:K
}

// Passes K... (eight of them): their records first (row, value, KRP row),
// then per column group every load before the adds.
template <typename T, int... K>
__device__ __forceinline__ void tile_add_passes(double *blk, int LDB, int rl, long long xb,
                                                unsigned zr, const T *__restrict__ zhat, int ldz,
                                                int R, int j, std::integer_sequence<int, K...>) {
  constexpr int NP = sizeof...(K);
  const int rr[NP] = {row_bcast<K>(rl)...};
  const unsigned zz[NP] = {(unsigned)row_bcast<K>((int)zr)...};
  const unsigned xlo[NP] = {(unsigned)row_bcast<K>((int)(unsigned)xb)...};
  const unsigned xhi[NP] = {(unsigned)row_bcast<K>((int)(unsigned)(xb >> 32))...};
  for (int c0 = 0; c0 < R; c0 += 16) {
    if (c0 + j < R) {
      T zv[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) zv[k] = zhat[(u64)zz[k] * (u64)ldz + c0 + j];
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        const double xv = __longlong_as_double((long long)(((u64)xhi[k] << 32) | xlo[k]));
        __hip_atomic_fetch_add(blk + rr[k] * LDB + c0 + j, xv * (double)zv[k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
}

template <int O, int... K>
constexpr std::integer_sequence<int, (O + K)...> shifted(std::integer_sequence<int, K...>) {
  return {};
}

// Called by all 64 lanes of a wave (rl a valid row of the block for every
// lane; x = 0 for lanes without a record).
template <typename T>
__device__ __forceinline__ void tile_add_rows(double *blk, int LDB, int rl, double x,
                                              unsigned zr, const T *__restrict__ zhat, int ldz,
                                              int R) {
  const int j = threadIdx.x & 15;
  const long long xb = __double_as_longlong(x);
  tile_add_passes<T>(blk, LDB, rl, xb, zr, zhat, ldz, R, j,
                     shifted<0>(std::make_integer_sequence<int, 8>{}));
  tile_add_passes<T>(blk, LDB, rl, xb, zr, zhat, ldz, R, j,
                     shifted<8>(std::make_integer_sequence<int, 8>{}));
}

// ------------------------------------------- bucketed gather, shared blocks --
// The same count and scatter passes with buckets of 2^bshift = up to 512
// output rows, so that a bucket's rows fit one FP64 block of shared memory;
// the buckets' records are cut into slices (at least BL_SLICE records, about
// BL_SLICES slices in all) and workgroup g takes
// the slices g, g + G, ...: it adds every record of the slice into the
// bucket's shared block (tile_add_rows: 4 records x 16 columns per atomic
// FP64 add, as in the tile gather), then adds the block into its XCD's copy
// of M (one global add per nonzero entry of the block and slice).  Records
// of a bucket follow the stream order of the scatter, i.e. fiber after fiber,
// so the records of a pass mostly share one weighted KRP row.  The records
// are compact (BktC) while the KRP row fits 23 bits, else 16-byte BktRec.
#define BL_THREADS 1024
#define BL_MAXNB 2048
#define BL_SLICE 65536
#define BL_SLICES 4096
#define BL_K 4
#define BL_MAXBLK (112 * 1024)

template <typename T>
__device__ __forceinline__ void gather_bktl_body(Blk bk, const DevState *st, int R,
    const uint4 *__restrict__ bent, const u64 *__restrict__ off, int gb, int nb, int bshift,
    const T *__restrict__ zhat, int ldz, T *__restrict__ M, i64 nk, int compact) {
  extern __shared__ double bl_blk[];    // (1 << bshift) rows, odd stride LDB
  __shared__ unsigned bst[BL_MAXNB + 1];   // first record of each bucket
  __shared__ unsigned sst[BL_MAXNB + 1];   // first slice of each bucket
  constexpr int NW = BL_THREADS / 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // the records: off[nb gb] of them (the scan's total)
  const unsigned total = (unsigned)off[(u64)nb * (u64)gb];
  // slice length: at least BL_SLICE records, and about BL_SLICES slices in
  // all, so that the per-slice block flush stays small against the adds
  const unsigned slen = max((unsigned)BL_SLICE, (total + BL_SLICES - 1) / BL_SLICES);
  for (int b = tid; b <= nb; b += BL_THREADS) bst[b] = (unsigned)off[(u64)b * (u64)gb];
  __syncthreads();
  {   // slices per bucket, two buckets per thread (nb <= 2 BL_THREADS)
    const int b0 = 2 * tid, b1 = b0 + 1;
    const unsigned c0 = b0 < nb ? (bst[b0 + 1] - bst[b0] + slen - 1) / slen : 0u;
    const unsigned c1 = b1 < nb ? (bst[b1 + 1] - bst[b1] + slen - 1) / slen : 0u;
    unsigned tot;
    const unsigned ex = block_excl_scan<unsigned>(c0 + c1, &tot);
    if (b0 < nb) sst[b0] = ex;
    if (b1 < nb) sst[b1] = ex + c0;
    if (tid == 0) sst[nb] = tot;
  }
  __syncthreads();
  const unsigned nsl = sst[nb];
  const int LDB = R | 1, RB = 1 << bshift;
  T *Mx = M + (i64)(xcd_id() & (CPAL_MCOPIES - 1)) * nk * ldz;
  for (unsigned sl = bk.x; sl < nsl; sl += bk.n) {
    int b = 0, hb = nb;   // last bucket with sst[b] <= sl
    while (hb - b > 1) {
      const int mid = (b + hb) >> 1;
      if (sst[mid] <= sl) b = mid; else hb = mid;
    }
    const unsigned a0 = bst[b] + (sl - sst[b]) * slen;
    const unsigned a1 = min(bst[b + 1], a0 + slen);
    const i64 r0 = (i64)b << bshift;
    const int nrows = (int)min((i64)RB, nk - r0);
    for (int e = tid; e < nrows * LDB; e += BL_THREADS) bl_blk[e] = 0.0;
    __syncthreads();
    for (unsigned q0 = a0 + (unsigned)w * (64u * BL_K); q0 < a1; q0 += NW * 64u * BL_K) {
      // every lane loads and adds (no divergent branch): a lane past the
      // slice re-reads its last record and adds zeros to a row of its own
      unsigned rk[BL_K], rz[BL_K];
      T rx[BL_K];
      const unsigned pl = rec_lane(lane);
      if (compact) {
        typename BktC<T>::V rec[BL_K];
        const typename BktC<T>::V *cb = (const typename BktC<T>::V *)bent;
#pragma unroll
        for (int u = 0; u < BL_K; ++u) rec[u] = cb[min(q0 + (unsigned)(u * 64) + pl, a1 - 1)];
#pragma unroll
        for (int u = 0; u < BL_K; ++u) BktC<T>::get(rec[u], rk[u], rx[u], rz[u]);
      } else {
        uint4 rec[BL_K];
#pragma unroll
        for (int u = 0; u < BL_K; ++u) rec[u] = bent[min(q0 + (unsigned)(u * 64) + pl, a1 - 1)];
#pragma unroll
        for (int u = 0; u < BL_K; ++u) {
          BktRec<T>::get(rec[u], rk[u], rx[u], rz[u]);
          rk[u] -= (unsigned)r0;
        }
      }
#pragma unroll
      for (int u = 0; u < BL_K; ++u) {
        if (q0 + (unsigned)(u * 64) >= a1) break;   // wave-uniform
        const unsigned zr = rz[u];
        const T x = rx[u];
        const int rl = (int)rk[u];
        const bool ok = q0 + (unsigned)(u * 64) + pl < a1 && (unsigned)rl < (unsigned)nrows;
        tile_add_rows<T>(bl_blk, LDB, ok ? rl : lane % nrows, ok ? (double)x : 0.0,
                         ok ? zr : 0u, zhat, ldz, R);
      }
    }
    __syncthreads();
    for (int e = tid; e < nrows * R; e += BL_THREADS) {
      const int r = e / R, c = e - r * R;
      const double v = bl_blk[r * LDB + c];
      if (v != 0.0) unsafeAtomicAdd(&Mx[(r0 + r) * ldz + c], (T)v);
    }
    __syncthreads();   // the block is read before the next slice clears it
  }
}
template <typename T>
__global__ void __launch_bounds__(BL_THREADS) k_gather_bktl(
    const DevState *st, int R, const uint4 *__restrict__ bent, const u64 *__restrict__ off,
    int gb, int nb, int bshift, const T *__restrict__ zhat, int ldz, T *__restrict__ M, i64 nk,
    int compact) {
  gather_bktl_body<T>(CPAL_BLK, st, R, bent, off, gb, nb, bshift, zhat, ldz, M, nk, compact);
}
template <typename T>
struct B_gather_bktl {
  static constexpr int NT = BL_THREADS, MW = 1;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    gather_bktl_body<T>(b, a...);
  }
};

// Bucket width of the shared-block bucketed gather: the largest power of two
// <= 512 rows whose FP64 block fits BL_MAXBLK; -1 when the mode needs more
// than BL_MAXNB buckets.
int gather_bktl_shift(int R, i64 nk) {
  const size_t row = (size_t)(R | 1) * 8;
  int sh = 9;
  while (sh > 0 && ((size_t)1 << sh) * row > BL_MAXBLK) --sh;
  while (sh > 0 && ((i64)1 << (sh - 1)) >= nk) --sh;
  if (((nk + (1ll << sh) - 1) >> sh) > BL_MAXNB) return -1;
  return sh;
}

template <typename T>
static void launch_gather_bktl_t(const DevState *st, int R, const u64 *cpos, const unsigned *coff,
                                 const unsigned *cidx, const unsigned *chunk_first, NzLoad<T> nz,
                                 i64 nk, i64 max_total, const T *zhat, int ldz, T *M,
                                 unsigned *cnt, u64 *off, void *scan_scratch, uint4 *bent,
                                 unsigned lmin, int compact, hipStream_t s) {
  const int bshift = gather_bktl_shift(R, nk);
  const int nb = (int)((nk + (1ll << bshift) - 1) >> bshift);
  const i64 chunks = (max_total + GT_CHUNK - 1) / GT_CHUNK;
  const int gb = (int)std::min<i64>(BK_GRID, std::max<i64>(64, (chunks + 7) / 8));
  launch_b<B_bkt_count<T>>(k_bkt_count<T>, dim3(gb), dim3(BK_THREADS), 0, s, st, cpos, coff, cidx,
                           chunk_first, nz, bshift, nb, lmin, cnt);
  // the scan also writes the number of records after the last bucket's
  // counts (off[nb gb]): with lmin > 0 it is below the stream length
  scan_u32_dev(cnt, off, (i64)nb * gb, nullptr, off + (i64)nb * gb, scan_scratch, s);
  launch_b<B_bkt_scatter<T>>(k_bkt_scatter<T>, dim3(gb), dim3(BK_THREADS), 0, s, st, cpos, coff,
                             cidx, chunk_first, nz, bshift, nb, lmin, off, bent, compact);
  const size_t smem = ((size_t)1 << bshift) * (size_t)(R | 1) * 8;
  const i64 slices = max_total / BL_SLICE + nb + 1;
  const int grid = (int)std::min<i64>(512, std::max<i64>(1, slices));
  launch_b<B_gather_bktl<T>>(k_gather_bktl<T>, dim3(grid), dim3(BL_THREADS), smem, s, st, R, bent,
                             off, gb, nb, bshift, zhat, ldz, M, nk, compact);
}

void launch_gather_bktl(bool f64, const DevState *st, int R, const u64 *cpos,
                        const unsigned *coff, const unsigned *cidx, const unsigned *chunk_first,
                        const uint2 *pairs, const int *ik, const double *v64, i64 nk,
                        i64 max_total, const void *zhat, int ldz, void *M, unsigned *cnt,
                        u64 *off, void *scan_scratch, uint4 *bent, unsigned lmin, int compact,
                        hipStream_t s) {
  if (f64)
    launch_gather_bktl_t<double>(st, R, cpos, coff, cidx, chunk_first, NzLoad<double>{ik, v64},
                                 nk, max_total, (const double *)zhat, ldz, (double *)M, cnt, off,
                                 scan_scratch, bent, lmin, compact, s);
  else
    launch_gather_bktl_t<float>(st, R, cpos, coff, cidx, chunk_first, NzLoad<float>{pairs}, nk,
                                max_total, (const float *)zhat, ldz, (float *)M, cnt, off,
                                scan_scratch, bent, lmin, compact, s);
}

// ------------------------------------------------------------ owner gather --
// Owner-computes form of the same sum, with no atomic operation anywhere:
// the rows of M are cut into blocks of 2^rshift rows and the nonempty
// sampled fibers into OWN_PARTS parts; workgroup (b, p) alone forms rows
// [b 2^rshift, (b+1) 2^rshift) of copy p of M from the fibers of part p,
// accumulating them in shared memory and storing each row once (plain
// stores, every row of every copy, so M needs no clearing).  The solve adds
// the copies in a fixed order.  A fiber's nonzeros are sorted by row, so
// its nonzeros in row block b are one contiguous segment; k_own_bounds
// records the segment boundaries of every fiber, bnd[f (nb + 1) + b] =
// number of nonzeros of fiber f with row < b 2^rshift.  Within a workgroup
// the segments of its fibers are taken in fiber order in batches of
// GT_CHUNK nonzeros, each batch is sorted by row (stable) and reduced in
// registers, and each row of the batch is added to the shared block once.
// The order of every sum therefore depends only on the sample and the
// launch shape, not on timing: an update in FP64 is bit-reproducible.
#define OWN_PARTS CPAL_MCOPIES

template <typename T>
struct RowLoad;
template <>
struct RowLoad<float> {
  const uint2 *pairs;
  __device__ __forceinline__ unsigned operator()(u64 e) const { return pairs[e].x; }
};
template <>
struct RowLoad<double> {
  const int *ik;
  __device__ __forceinline__ unsigned operator()(u64 e) const { return (unsigned)ik[e]; }
};

// One wave per nonempty fiber f: lane e of a 64-entry step writes
// bnd[f][b] = e for every block b after its predecessor's block up to its
// own; the blocks after the last nonzero get the fiber length.  Each entry
// of the fiber's row is written exactly once.
template <typename T>
__device__ __forceinline__ void own_bounds_body(Blk bk, const DevState *st,
    const u64 *__restrict__ cpos, const unsigned *__restrict__ coff, RowLoad<T> rows, int rshift,
    int nb, unsigned *__restrict__ bnd) {
  const i64 nf = st->n_fib;
  const u64 total = (u64)st->gathered;
  const int lane = threadIdx.x & 63;
  const i64 nw = ((i64)bk.n * blockDim.x) >> 6;
  for (i64 f = ((i64)bk.x * blockDim.x + threadIdx.x) >> 6; f < nf; f += nw) {
    const u64 p0 = cpos[f];
    const unsigned len = (unsigned)((f + 1 < nf ? cpos[f + 1] : total) - p0);
    const u64 base = coff[f];
    unsigned *tb = bnd + (u64)f * (u64)(nb + 1);
    int carry = -1;   // block of the previous nonzero of the fiber
    for (unsigned e0 = 0; e0 < len; e0 += 64) {
      const unsigned e = e0 + (unsigned)lane;
      const bool valid = e < len;
      const int bu = valid ? (int)(rows(base + e) >> rshift) : nb;
      int bp = __shfl_up(bu, 1, 64);
      if (lane == 0) bp = carry;
      if (valid)
        for (int bb = bp + 1; bb <= bu; ++bb) tb[bb] = e;
      carry = __shfl(bu, (int)min(63u, len - 1 - e0), 64);
    }
    for (int bb = carry + 1 + lane; bb <= nb; bb += 64) tb[bb] = len;
  }
}
template <typename T>
__global__ void __launch_bounds__(256) k_own_bounds(const DevState *st,
                                                    const u64 *__restrict__ cpos,
                                                    const unsigned *__restrict__ coff,
                                                    RowLoad<T> rows, int rshift, int nb,
                                                    unsigned *__restrict__ bnd) {
  own_bounds_body<T>(CPAL_BLK, st, cpos, coff, rows, rshift, nb, bnd);
}
template <typename T>
struct B_own_bounds {
  static constexpr int NT = 256, MW = 1;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    own_bounds_body<T>(b, a...);
  }
};

template <typename T, int LPN, int CPL>
__device__ __forceinline__ void gather_own_body(Blk bk, const DevState *st, int R,
    const unsigned *__restrict__ coff, const unsigned *__restrict__ cidx,
    const unsigned *__restrict__ bnd, int nb, int rshift, const NzLoad<T> &nz,
    const T *__restrict__ zhat, int ldz, T *__restrict__ M, i64 nk) {
  constexpr int NG = GT_THREADS / LPN;
  constexpr int LDB = LPN * CPL + 1;   // shared row stride (odd: rows spread over banks)
  extern __shared__ char own_smem[];
  T *blk = (T *)own_smem;              // (1 << rshift) x LDB
  __shared__ unsigned ka[GT_CHUNK], kb[GT_CHUNK];
  __shared__ T lx[GT_CHUNK];
  __shared__ unsigned lz[GT_CHUNK];
  __shared__ unsigned tab[64 * GT_PER_THREAD * (GT_THREADS / 64)];
  __shared__ int srow[2 * NG];
  __shared__ T svec[2 * NG][LPN * CPL];
  __shared__ unsigned gst[GT_THREADS], gend[GT_THREADS], gz[GT_THREADS];
  __shared__ u64 gbase[GT_THREADS];
  const int tid = threadIdx.x;
  const int p = (int)(bk.x % OWN_PARTS), b = (int)(bk.x / OWN_PARTS);
  const int rb = 1 << rshift;
  const i64 r0 = (i64)b << rshift;
  const i64 nf = st->n_fib;
  const i64 f0 = nf * p / OWN_PARTS, f1 = nf * (p + 1) / OWN_PARTS;
  for (int e = tid; e < rb * LDB; e += GT_THREADS) blk[e] = T(0);
  for (i64 g0 = f0; g0 < f1; g0 += GT_THREADS) {
    const i64 f = g0 + tid;
    unsigned lo = 0, len = 0;
    if (f < f1) {
      const unsigned *tb = bnd + (u64)f * (u64)(nb + 1) + b;
      lo = tb[0];
      len = tb[1] - lo;
    }
    unsigned tot;
    const unsigned ex = block_excl_scan<unsigned>(len, &tot);
    __syncthreads();   // the previous group's batches are finished with g*
    gst[tid] = ex;
    gend[tid] = ex + len;
    gbase[tid] = f < f1 ? (u64)coff[f] + lo : 0;
    gz[tid] = f < f1 ? cidx[f] : 0u;
    __syncthreads();
    for (unsigned q0 = 0; q0 < tot; q0 += GT_CHUNK) {
#pragma unroll
      for (int u = 0; u < GT_PER_THREAD; ++u) {
        const int li = u * GT_THREADS + tid;
        const unsigned q = q0 + (unsigned)li;
        if (q < tot) {
          int lo2 = 0, hi2 = GT_THREADS - 1;   // first fiber of the group ending after q
          while (lo2 < hi2) {
            const int mid = (lo2 + hi2) >> 1;
            if (gend[mid] > q) hi2 = mid; else lo2 = mid + 1;
          }
          int ik;
          T x;
          nz.get(gbase[lo2] + (q - gst[lo2]), ik, x);
          ka[li] = ((unsigned)((i64)ik - r0) << 12) | (unsigned)li;
          lx[li] = x;
          lz[li] = gz[lo2];
        } else {
          ka[li] = 0xFFFFFFFFu;
          lx[li] = T(0);
          lz[li] = 0u;
        }
      }
      __syncthreads();
      const unsigned *keys = chunk_radix(ka, kb, tab, rshift);
      const int nvalid = (int)min((unsigned)GT_CHUNK, tot - q0);
      seg_reduce<T, LPN, CPL>(LdsEntries<T>{keys, lx, lz}, nvalid, R, zhat, ldz,
                              LdsAdd<T>{blk, LDB}, srow, svec);
      __syncthreads();   // the merged adds are in the block before the next batch
    }
  }
  __syncthreads();
  T *Mp = M + (i64)p * nk * ldz;
  const i64 nrows = min((i64)rb, nk - r0);
  for (i64 e = tid; e < nrows * ldz; e += GT_THREADS) {
    const i64 r = e / ldz;
    const int c = (int)(e - r * ldz);
    Mp[(r0 + r) * ldz + c] = blk[r * LDB + c];
  }
}
template <typename T, int LPN, int CPL>
__global__ void __launch_bounds__(GT_THREADS, 2) k_gather_own(
    const DevState *st, int R, const unsigned *__restrict__ coff,
    const unsigned *__restrict__ cidx, const unsigned *__restrict__ bnd, int nb, int rshift,
    NzLoad<T> nz, const T *__restrict__ zhat, int ldz, T *__restrict__ M, i64 nk) {
  gather_own_body<T, LPN, CPL>(CPAL_BLK, st, R, coff, cidx, bnd, nb, rshift, nz, zhat, ldz, M, nk);
}
template <typename T, int LPN, int CPL>
struct B_gather_own {
  static constexpr int NT = GT_THREADS, MW = 2;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    gather_own_body<T, LPN, CPL>(b, a...);
  }
};

// Row block of the owner gather: the largest power of two <= 512 rows whose
// shared block (row stride ldz + 1 of the gather precision) fits OWN_BLK_BYTES,
// and not above the mode's row count rounded up to a power of two.
#define OWN_BLK_BYTES (68 * 1024)
int gather_own_shift(bool f64, int ldz, i64 nk) {
  const size_t row = (size_t)(ldz + 1) * (f64 ? 8 : 4);
  int sh = 9;
  while (sh > 4 && ((size_t)1 << sh) * row > OWN_BLK_BYTES) --sh;
  while (sh > 4 && ((i64)1 << (sh - 1)) >= nk) --sh;
  return sh;
}

int gather_own_blocks(bool f64, int ldz, i64 nk) {
  const int sh = gather_own_shift(f64, ldz, nk);
  return (int)((nk + (1ll << sh) - 1) >> sh);
}

template <typename T>
static void launch_gather_own_t(int rm, dim3 grid, size_t smem, hipStream_t s, const DevState *st,
                                int R, const u64 *cpos, const unsigned *coff, const unsigned *cidx,
                                RowLoad<T> rows, const NzLoad<T> &nz, unsigned *bnd, int nb, int sh,
                                const T *zhat, int ldz, T *M, i64 nk) {
  launch_b<B_own_bounds<T>>(k_own_bounds<T>, dim3(1024), dim3(256), 0, s, st, cpos, coff, rows, sh,
                            nb, bnd);
#define CPAL_OWN_LAUNCH(LPN, CPL)                                                              \
  launch_b<B_gather_own<T, LPN, CPL>>(k_gather_own<T, LPN, CPL>, grid, dim3(GT_THREADS), smem, \
                                      s, st, R, coff, cidx, bnd, nb, sh, nz, zhat, ldz, M, nk)
  if (rm == 16) CPAL_OWN_LAUNCH(16, 1);
  else if (rm == 32) CPAL_OWN_LAUNCH(16, 2);
  else CPAL_OWN_LAUNCH(32, 2);
#undef CPAL_OWN_LAUNCH
}

void launch_gather_own(bool f64, const DevState *st, int R, const u64 *cpos,
                       const unsigned *coff, const unsigned *cidx, const uint2 *pairs,
                       const int *ik, const double *v64, i64 nk, const void *zhat, int ldz,
                       void *M, unsigned *bnd, hipStream_t s) {
  const int sh = gather_own_shift(f64, ldz, nk);
  const int nb = (int)((nk + (1ll << sh) - 1) >> sh);
  const int rm = gather_row_width(R);
  const size_t smem = ((size_t)1 << sh) * (size_t)(ldz + 1) * (f64 ? 8 : 4);
  const dim3 grid((unsigned)nb * OWN_PARTS);
  if (f64) {
    launch_gather_own_t<double>(rm, grid, smem, s, st, R, cpos, coff, cidx, RowLoad<double>{ik},
                                NzLoad<double>{ik, v64}, bnd, nb, sh, (const double *)zhat, ldz,
                                (double *)M, nk);
  } else {
    launch_gather_own_t<float>(rm, grid, smem, s, st, R, cpos, coff, cidx, RowLoad<float>{pairs},
                               NzLoad<float>{pairs}, bnd, nb, sh, (const float *)zhat, ldz,
                               (float *)M, nk);
  }
}

// ------------------------------------------------------------- tile gather --
// Row blocks of M held in shared memory, fed by every sampled fiber's segment
// in the block: the rows of M are cut into blocks of 2^rshift rows and the
// nonempty sampled fibers into CPAL_MCOPIES parts of about equal nonzero
// count; workgroup (b, p) forms rows of block b of copy p of M from the
// fibers of part p (every row of every copy is stored, so M needs no
// clearing; the solve sums the copies in a fixed order).  Part p runs on XCD
// p (workgroups are dealt to the XCDs in turn), so a die reads only its own
// part's weighted KRP rows and nonzeros.
//  1. k_tile_bounds: for groups of TB_FIB fibers, bnd[b ldb + f] = number of
//     nonzeros of fiber f with row < b 2^rshift (a fiber's rows ascend, so
//     its nonzeros in block b are [bnd[b], bnd[b+1])), staged in shared
//     memory and stored block-major, TB_FIB entries (64 bytes) per block;
//  2. k_gather_tile: windows of TL_THREADS fibers, their nonempty segments
//     in block b listed in shared memory (start in the window's stream,
//     nonzero offset, KRP row); each wave takes 64 consecutive positions of
//     the stream at a time, one nonzero per lane, and adds x * zhat(j, c)
//     into the shared block column by column.  The shared block is FP64 in
//     both precisions (shared-memory FP64 adds run at full rate on this
//     chip, FP32 ones about ten times slower); lanes of one wave can meet on
//     a row (nonzeros of different fibers), so the adds are atomic, and the
//     order of a row's adds depends on timing (rounding order only).
#define TB_FIB 16
#define TB_THREADS 1024
#define TB_MAXNB 1023         // (TB_MAXNB + 1) * TB_FIB entries of shared memory
#define TL_THREADS 1024
#define TL_K 4               // chunks of 64 positions a wave has in flight
#define TL_MAXBLK (128 * 1024)   // bytes of the shared row block
#define TL_CHUNKS 8192            // 64-position chunks of a window with a segment table

// First fiber of part p: the least f with cpos[f] >= ceil(p total / parts).
__device__ __forceinline__ i64 tile_part_start(const u64 *__restrict__ cpos, i64 nf, u64 total,
                                               int p, int parts) {
  if (p <= 0) return 0;
  if (p >= parts) return nf;
  const u64 t = (total * (u64)p + (u64)parts - 1) / (u64)parts;
  i64 lo = 0, hi = nf;
  while (lo < hi) {
    const i64 mid = (lo + hi) >> 1;
    if (cpos[mid] >= t) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// Workgroup g takes the fibers [TB_FIB g, TB_FIB (g + 1)) as one stream of their
// nonzeros, TB_PER positions per thread and step: the first nonzero of a
// fiber in each block it reaches marks tb[block][fiber] with its index in the
// fiber (one writer per entry: a fiber's rows ascend); tb[nb][fiber] = the
// fiber's length; a suffix minimum along the blocks then gives every entry
// the index of the fiber's first nonzero in that block or a later one.
#define TB_PER 4
template <typename T>
__device__ __forceinline__ void tile_bounds_body(Blk bk, const DevState *st,
    const u64 *__restrict__ cpos, const unsigned *__restrict__ coff, RowLoad<T> rows, int rshift,
    int nb, u64 ldb, unsigned lmin, unsigned *__restrict__ bnd) {
  __shared__ unsigned tb[(TB_MAXNB + 1) * TB_FIB];   // tb[bb TB_FIB + i]
  __shared__ u64 gs[TB_FIB + 1];
  __shared__ unsigned ge[TB_FIB + 1];   // starts in the stream of the fibers taken
  __shared__ unsigned gb[TB_FIB];
  __shared__ unsigned smin[TB_FIB * (TB_THREADS / TB_FIB)];
  const i64 nf = st->n_fib;
  const u64 total = (u64)st->gathered;
  const i64 f0 = (i64)bk.x * TB_FIB;
  if (f0 >= nf) return;
  const int nfg = (int)min((i64)TB_FIB, nf - f0);
  const int tid = threadIdx.x;
  if (tid <= nfg) gs[tid] = f0 + tid < nf ? cpos[f0 + tid] : total;
  if (tid < nfg) gb[tid] = coff[f0 + tid];
  const int nent = (nb + 1) * TB_FIB;
  for (int t = tid; t < nent; t += TB_THREADS) tb[t] = 0xFFFFFFFFu;
  __syncthreads();
  if (tid == 0) {   // fibers shorter than lmin count as empty (lmin = 0: none)
    unsigned acc = 0;
    for (int i = 0; i < nfg; ++i) {
      ge[i] = acc;
      const unsigned len = (unsigned)(gs[i + 1] - gs[i]);
      acc += (lmin == 0u || len >= lmin) ? len : 0u;
    }
    ge[nfg] = acc;
  }
  __syncthreads();
  if (tid < TB_FIB) tb[nb * TB_FIB + tid] = tid < nfg ? ge[tid + 1] - ge[tid] : 0u;
  const unsigned G = ge[nfg];
  for (unsigned q0 = 0; q0 < G; q0 += TB_THREADS * TB_PER) {
    int fi[TB_PER];
    unsigned ee[TB_PER];
#pragma unroll
    for (int u = 0; u < TB_PER; ++u) {
      const unsigned q = min(q0 + (unsigned)(u * TB_THREADS + tid), G - 1);
      int lo = 0, hi = nfg;   // last fiber taken starting at or before q
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (ge[mid] <= q) lo = mid; else hi = mid;
      }
      fi[u] = lo;
      ee[u] = q - ge[lo];
    }
    unsigned rc[TB_PER], rp[TB_PER];
#pragma unroll
    for (int u = 0; u < TB_PER; ++u) {
      const u64 pos = (u64)gb[fi[u]] + ee[u];
      rc[u] = rows(pos);
      rp[u] = ee[u] ? rows(pos - 1) : 0u;
    }
#pragma unroll
    for (int u = 0; u < TB_PER; ++u) {
      if (q0 + (unsigned)(u * TB_THREADS + tid) >= G) continue;
      const int bu = min((int)(rc[u] >> rshift), nb - 1);
      const int bp = ee[u] ? min((int)(rp[u] >> rshift), nb - 1) : -1;
      if (bp != bu) tb[bu * TB_FIB + fi[u]] = ee[u];
    }
  }
  __syncthreads();
  // suffix minimum along bb per fiber column: thread (i, sg) takes the
  // entries [sg seg, (sg + 1) seg) of column i
  constexpr int NSEG = TB_THREADS / TB_FIB;
  const int i = tid % TB_FIB, sg = tid / TB_FIB;
  const int seg = (nb + 1 + NSEG - 1) / NSEG;
  const int b0 = sg * seg, b1 = min(nb + 1, b0 + seg);
  unsigned m = 0xFFFFFFFFu;
  for (int bb = b1 - 1; bb >= b0; --bb) {
    m = min(m, tb[bb * TB_FIB + i]);
    tb[bb * TB_FIB + i] = m;
  }
  smin[sg * TB_FIB + i] = m;
  __syncthreads();
  unsigned after = 0xFFFFFFFFu;
  for (int s2 = sg + 1; s2 < NSEG; ++s2) after = min(after, smin[s2 * TB_FIB + i]);
  for (int bb = b0; bb < b1; ++bb) tb[bb * TB_FIB + i] = min(tb[bb * TB_FIB + i], after);
  __syncthreads();
  for (int t = tid; t < nent; t += TB_THREADS) {
    const int bb = t / TB_FIB, i2 = t - bb * TB_FIB;
    bnd[(u64)bb * ldb + (u64)f0 + i2] = tb[t];
  }
}
template <typename T>
__global__ void __launch_bounds__(TB_THREADS) k_tile_bounds(
    const DevState *st, const u64 *__restrict__ cpos, const unsigned *__restrict__ coff,
    RowLoad<T> rows, int rshift, int nb, u64 ldb, unsigned lmin, unsigned *__restrict__ bnd) {
  tile_bounds_body<T>(CPAL_BLK, st, cpos, coff, rows, rshift, nb, ldb, lmin, bnd);
}
template <typename T>
struct B_tile_bounds {
  static constexpr int NT = TB_THREADS, MW = 1;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    tile_bounds_body<T>(b, a...);
  }
};

template <typename T>
__device__ __forceinline__ void gather_tile_body(Blk bk, const DevState *st, int R,
    const u64 *__restrict__ cpos, const unsigned *__restrict__ coff,
    const unsigned *__restrict__ cidx, const unsigned *__restrict__ bnd, u64 ldb, int rshift,
    const NzLoad<T> &nz, const T *__restrict__ zhat, int ldz, T *__restrict__ M, i64 nk) {
  extern __shared__ double tl_blk[];   // (1 << rshift) rows, odd stride LDB
  __shared__ unsigned cs[TL_THREADS + 1], cb[TL_THREADS], cz[TL_THREADS];
  __shared__ unsigned short csa[TL_CHUNKS];   // segment holding position 64 c of the window
  constexpr int NW = TL_THREADS / 64;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int p = (int)(bk.x & (CPAL_MCOPIES - 1)), b = (int)(bk.x / CPAL_MCOPIES);
  const int LDB = R | 1;
  const i64 r0 = (i64)b << rshift;
  const int nrows = (int)min((i64)1 << rshift, nk - r0);
  const i64 nf = st->n_fib;
  const u64 total = (u64)st->gathered;
  const i64 fa = tile_part_start(cpos, nf, total, p, CPAL_MCOPIES);
  const i64 fb = tile_part_start(cpos, nf, total, p + 1, CPAL_MCOPIES);
  for (int e = tid; e < nrows * LDB; e += TL_THREADS) tl_blk[e] = 0.0;
  const unsigned *blo = bnd + (u64)b * ldb, *bhi = blo + ldb;
  // the window's per-fiber inputs, loaded one window ahead
  unsigned nlo = 0, nlen = 0, noff = 0, nz_ = 0;
  auto fetch = [&](i64 f) {
    nlo = 0; nlen = 0; noff = 0; nz_ = 0;
    if (f < fb) {
      nlo = blo[f];
      nlen = min(bhi[f] - nlo, 1u << rshift);
      noff = coff[f];
      nz_ = cidx[f];
    }
  };
  fetch(fa + tid);
  for (i64 w0 = fa; w0 < fb; w0 += TL_THREADS) {
    const unsigned lo = nlo, len = nlen, off = noff, zrow = nz_;
    fetch(w0 + TL_THREADS + tid);
    // one scan of (nonempty << 20 | length): a segment holds at most
    // 2^rshift <= 512 nonzeros (rows are distinct within a fiber), so the
    // window's stream length stays below 2^20
    unsigned tot;
    const unsigned ex = block_excl_scan<unsigned>((len ? 1u << 20 : 0u) | len, &tot);
    const int nne = (int)(tot >> 20);
    const unsigned nw = tot & 0xFFFFFu;
    if (len) {
      const int ci = (int)(ex >> 20);
      cs[ci] = ex & 0xFFFFFu;
      cb[ci] = off + lo;
      cz[ci] = zrow;
    }
    if (tid == 0) cs[nne] = nw;
    __syncthreads();
    // the segment of every 64-position chunk's first position (segments
    // partition the window: one writer per chunk); windows of more chunks
    // search all segments
    const unsigned nck = (nw + 63) >> 6;
    const bool tab = nck <= TL_CHUNKS;
    if (tab)
      for (int sg = tid; sg < nne; sg += TL_THREADS)
        for (unsigned c = (cs[sg] + 63) >> 6; (c << 6) < cs[sg + 1]; ++c) csa[c] = (unsigned short)sg;
    __syncthreads();
    // TL_K chunks of 64 positions per wave and step: their searches and
    // nonzero loads are all issued before the first chunk's adds
    for (unsigned qb = (unsigned)w * (64u * TL_K); qb < nw; qb += NW * 64u * TL_K) {
      int ik[TL_K];
      T x[TL_K];
      unsigned zr[TL_K];
      u64 pos[TL_K];
      const unsigned pl = rec_lane(lane);
#pragma unroll
      for (int u = 0; u < TL_K; ++u) {
        const unsigned q = min(qb + (unsigned)(u * 64) + pl, nw - 1);
        int lo2 = 0, hi2 = nne;   // last segment with cs[seg] <= q
        if (tab) {   // between the segments of q's chunk start and the next chunk's
          const unsigned cq = q >> 6;
          lo2 = csa[cq];
          hi2 = cq + 1 < nck ? (int)csa[cq + 1] + 1 : nne;
        }
        while (hi2 - lo2 > 1) {
          const int mid = (lo2 + hi2) >> 1;
          if (cs[mid] <= q) lo2 = mid; else hi2 = mid;
        }
        pos[u] = (u64)cb[lo2] + (q - cs[lo2]);
        zr[u] = cz[lo2];
      }
#pragma unroll
      for (int u = 0; u < TL_K; ++u) nz.get(pos[u], ik[u], x[u]);
#pragma unroll
      for (int u = 0; u < TL_K; ++u) {
        if (qb + (unsigned)(u * 64) >= nw) break;   // wave-uniform
        const int rl = ik[u] - (int)r0;
        const bool ok = qb + (unsigned)(u * 64) + pl < nw && (unsigned)rl < (unsigned)nrows;
        tile_add_rows<T>(tl_blk, LDB, ok ? rl : lane % nrows, ok ? (double)x[u] : 0.0,
                         ok ? zr[u] : 0u, zhat, ldz, R);
      }
    }
    __syncthreads();   // the window's segment lists are finished with
  }
  __syncthreads();
  T *Mp = M + (i64)p * nk * ldz;
  for (int e = tid; e < nrows * ldz; e += TL_THREADS) {
    const int r = e / ldz, c = e - r * ldz;
    Mp[(r0 + r) * ldz + c] = c < R ? (T)tl_blk[r * LDB + c] : T(0);
  }
}
template <typename T>
__global__ void __launch_bounds__(TL_THREADS) k_gather_tile(
    const DevState *st, int R, const u64 *__restrict__ cpos, const unsigned *__restrict__ coff,
    const unsigned *__restrict__ cidx, const unsigned *__restrict__ bnd, u64 ldb, int rshift,
    NzLoad<T> nz, const T *__restrict__ zhat, int ldz, T *__restrict__ M, i64 nk) {
  gather_tile_body<T>(CPAL_BLK, st, R, cpos, coff, cidx, bnd, ldb, rshift, nz, zhat, ldz, M, nk);
}
template <typename T>
struct B_gather_tile {
  static constexpr int NT = TL_THREADS, MW = 1;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    gather_tile_body<T>(b, a...);
  }
};

// Row block of the tile gather for a mode of nk rows: the largest power of two
// <= 512 whose FP64 block (odd row stride) fits TL_MAXBLK, made smaller while
// the launch has fewer than 512 workgroups; -1 when the mode needs more than
// TB_MAXNB blocks.
int gather_tile_shift(int R, i64 nk) {
  const size_t row = (size_t)(R | 1) * 8;
  int sh = 9;
  while (sh > 4 && ((size_t)1 << sh) * row > TL_MAXBLK) --sh;
  while (sh > 5 && ((nk + (1ll << sh) - 1) >> sh) * CPAL_MCOPIES < 512) --sh;
  if (((nk + (1ll << sh) - 1) >> sh) > TB_MAXNB) return -1;
  return sh;
}

int gather_tile_blocks(int R, i64 nk) {
  const int sh = gather_tile_shift(R, nk);
  return sh < 0 ? -1 : (int)((nk + (1ll << sh) - 1) >> sh);
}

// Bounds stride (fibers, padded to TB_FIB) for up to max_fib nonempty fibers.
u64 gather_tile_ldb(i64 max_fib) { return (u64)((max_fib + TB_FIB - 1) / TB_FIB) * TB_FIB; }

// lmin > 0: fibers shorter than lmin nonzeros are left out (their segments
// are empty), for the hybrid gather below.
void launch_gather_tile(bool f64, const DevState *st, int R, const u64 *cpos,
                        const unsigned *coff, const unsigned *cidx, const uint2 *pairs,
                        const int *ik, const double *v64, i64 nk, i64 max_fib, const void *zhat,
                        int ldz, void *M, unsigned *bnd, unsigned lmin, hipStream_t s) {
  const int sh = gather_tile_shift(R, nk);
  const int nb = (int)((nk + (1ll << sh) - 1) >> sh);
  const u64 ldb = gather_tile_ldb(max_fib);
  const dim3 gb((unsigned)(ldb / TB_FIB));
  const dim3 gt((unsigned)nb * CPAL_MCOPIES);
  const size_t smem = ((size_t)1 << sh) * (size_t)(R | 1) * 8;
  if (f64) {
    launch_b<B_tile_bounds<double>>(k_tile_bounds<double>, gb, dim3(TB_THREADS), 0, s, st, cpos,
                                    coff, RowLoad<double>{ik}, sh, nb, ldb, lmin, bnd);
    launch_b<B_gather_tile<double>>(k_gather_tile<double>, gt, dim3(TL_THREADS), smem, s, st, R,
                                    cpos, coff, cidx, bnd, ldb, sh, NzLoad<double>{ik, v64},
                                    (const double *)zhat, ldz, (double *)M, nk);
  } else {
    launch_b<B_tile_bounds<float>>(k_tile_bounds<float>, gb, dim3(TB_THREADS), 0, s, st, cpos,
                                   coff, RowLoad<float>{pairs}, sh, nb, ldb, lmin, bnd);
    launch_b<B_gather_tile<float>>(k_gather_tile<float>, gt, dim3(TL_THREADS), smem, s, st, R,
                                   cpos, coff, cidx, bnd, ldb, sh, NzLoad<float>{pairs},
                                   (const float *)zhat, ldz, (float *)M, nk);
  }
}

// Hybrid gather: the tile gather takes the fibers of at least lmin nonzeros
// (their per-block segments are long: lmin / blocks nonzeros on average) and
// stores every row of the 8 copies of M; the shared-block bucketed gather
// then adds the nonzeros of the shorter fibers (bucketed, so that their short
// segments cost no per-segment work).  lmin = lfac times the tile gather's
// row blocks.
unsigned gather_hyb_lmin(int R, i64 nk, int lfac) {
  return (unsigned)std::max(1, lfac) * (unsigned)std::max(1, gather_tile_blocks(R, nk));
}

void launch_gather_bktl(bool f64, const DevState *st, int R, const u64 *cpos,
                        const unsigned *coff, const unsigned *cidx, const unsigned *chunk_first,
                        const uint2 *pairs, const int *ik, const double *v64, i64 nk,
                        i64 max_total, const void *zhat, int ldz, void *M, unsigned *cnt,
                        u64 *off, void *scan_scratch, uint4 *bent, unsigned lmin, int compact,
                        hipStream_t s);

void launch_gather_hyb(bool f64, const DevState *st, int R, const u64 *cpos,
                       const unsigned *coff, const unsigned *cidx, const unsigned *chunk_first,
                       const uint2 *pairs, const int *ik, const double *v64, i64 nk,
                       i64 max_total, i64 max_fib, const void *zhat, int ldz, void *M,
                       unsigned *bnd, unsigned *cnt, u64 *off, void *scan_scratch, uint4 *bent,
                       int lfac, int compact, hipStream_t s) {
  const unsigned lmin = gather_hyb_lmin(R, nk, lfac);
  launch_gather_tile(f64, st, R, cpos, coff, cidx, pairs, ik, v64, nk, max_fib, zhat, ldz, M, bnd,
                     lmin, s);
  launch_gather_bktl(f64, st, R, cpos, coff, cidx, chunk_first, pairs, ik, v64, nk, max_total,
                     zhat, ldz, M, cnt, off, scan_scratch, bent, lmin, compact, s);
}

int gather_row_width(int R);

template <typename T>
static void launch_gather_seg_t(int rm, int grid, hipStream_t s, const DevState *st, int R,
                                const u64 *cpos, const unsigned *coff, const unsigned *cidx,
                                const unsigned *chunk_first, const NzLoad<T> &nz, int ikbits,
                                int sort_min, const T *zhat, int ldz, T *M, i64 nk) {
#define CPAL_SEG_LAUNCH(LPN, CPL)                                                                 \
  launch_b<B_gather_seg<T, LPN, CPL>>(k_gather_seg<T, LPN, CPL>, dim3(grid), dim3(GT_THREADS), 0, \
                                      s, st, R, cpos, coff, cidx, chunk_first, nz, ikbits,         \
                                      sort_min, zhat, ldz, M, nk)
  if (rm == 16) CPAL_SEG_LAUNCH(16, 1);
  else if (rm == 32) CPAL_SEG_LAUNCH(16, 2);
  else CPAL_SEG_LAUNCH(32, 2);
#undef CPAL_SEG_LAUNCH
}

void launch_gather_seg(bool f64, const DevState *st, int R, const u64 *cpos, const unsigned *coff,
                       const unsigned *cidx, const unsigned *chunk_first, const uint2 *pairs,
                       const int *ik, const double *v64, i64 nk, const void *zhat, int ldz, void *M,
                       int grid, int sort_min, hipStream_t s) {
  int ikbits = 1;
  while ((1ll << ikbits) < nk) ++ikbits;
  const int rm = gather_row_width(R);
  if (f64) {
    NzLoad<double> nz{ik, v64};
    launch_gather_seg_t<double>(rm, grid, s, st, R, cpos, coff, cidx, chunk_first, nz, ikbits,
                                sort_min, (const double *)zhat, ldz, (double *)M, nk);
  } else {
    NzLoad<float> nz{pairs};
    launch_gather_seg_t<float>(rm, grid, s, st, R, cpos, coff, cidx, chunk_first, nz, ikbits,
                               sort_min, (const float *)zhat, ldz, (float *)M, nk);
  }
}

__device__ __forceinline__ void zero_words_body(Blk bk, unsigned *__restrict__ p, i64 n) {
  for (i64 i = (i64)bk.x * blockDim.x + threadIdx.x; i < n; i += (i64)bk.n * blockDim.x)
    p[i] = 0u;
}
__global__ void k_zero_words(unsigned *__restrict__ p, i64 n) {
  zero_words_body(CPAL_BLK, p, n);
}
CPAL_BODY(B_zero_words, 256, 1, zero_words_body);

void launch_zero_words(void *p, i64 nwords, hipStream_t s) {
  if (nwords <= 0) return;
  i64 g = (nwords + 255) / 256;
  if (g > 8192) g = 8192;
  launch_b<B_zero_words>(k_zero_words, dim3((int)g), dim3(256), 0, s, (unsigned *)p, nwords);
}

i64 gather_chunks_cap(i64 nnz) { return nnz / GT_CHUNK + 2; }

int gather_row_width(int R) { return R <= 16 ? 16 : (R <= 32 ? 32 : 64); }

void launch_gather(bool f64, const DevState *st, int R, const u64 *cpos, const unsigned *coff,
                   const unsigned *cidx, const uint2 *pairs, const int *ik, const double *v64,
                   const void *zhat, void *M, int ldz, int grid, hipStream_t s) {
  if (f64) {
    NzLoad<double> nz{ik, v64};
    launch_1(k_gather<double>, dim3(grid), dim3(256), 0, s, st, R, cpos, coff, cidx, nz,
             (const double *)zhat, (double *)M, ldz);
  } else {
    NzLoad<float> nz{pairs};
    launch_1(k_gather<float>, dim3(grid), dim3(256), 0, s, st, R, cpos, coff, cidx, nz,
             (const float *)zhat, (float *)M, ldz);
  }
}
}  // namespace cpal
