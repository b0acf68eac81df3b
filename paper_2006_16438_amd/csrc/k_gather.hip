// Sampled system of one mode update: KrpSamp (rows of the KRP as Hadamard
// products of factor rows, eq. (2.1)), TnsrSamp (fibers of the sampled rows,
// Sec. 6.3) and the weighted normal equations of the sketched problem
// (eq. (1.2)):  G_s = sum_j omega_j z_j z_j^T (FP64),
//               M(i_k,:) += omega_j x z_j  over every nonzero (i_k, x) of
//               fiber j (gather precision T),
//               A_k = M G_s^{-1}.
// Also the per-mode fiber index built once at init: nonzeros sorted by
// (complement key, i_k) and an open-addressing hash table key -> fiber.
#include "cpal_common.h"

namespace cpal {

// ------------------------------------------------------------- sample rows --
// Slots j of the sampled system, ROWS_BLK per block: the deterministic rows
// first, then one slot per accepted random draw in sorted order, of which
// the first of every run of equal rows is the combined row (Sec. 4.1) and
// the others stay empty (omega = 0, no fiber); three phases:
//  1. thread per slot: omega_j, w_j, the other-mode indices of row j and the
//     fiber hash probe;
//  2. lanes = columns: z_j (FP64, Hadamard product of the other factors' rows
//     in ascending mode order) into shared memory and the weighted row
//     omega_j z_j in T (zero-padded to ldz) to zhat, rows read and written
//     contiguously, ROWS_UNR rows per lane group in flight;
//  3. the block's part of G_s (pairs a <= c, packed row by row) on the
//     matrix cores.
// Blocks past the slots only clear their share of M.  DD = number of other modes
// (0: any, runtime loops).
#define ROWS_BLK 256
#define ROWS_UNR 4
typedef double d4 __attribute__((ext_vector_type(4)));

// Phase 3 for NT = ceil(R/16) column blocks.  Wave w multiplies the rows
// [64w, 64w+64) of the block: tiles (ta <= tc) of 16 x 16, D += A B with
// A(i,k) = omega_k z_k(16 ta + i), B(k,j) = z_k(16 tc + j); lane l holds
// A(l%16, l/16), B(l/16, l%16) and D(l/16 + 4v, l%16).  The four waves'
// tiles are then summed in wave order through shared memory (red aliases z).
template <int NT>
__device__ __forceinline__ void gs_tiles(const double *sz, const double *som, int ld, int R,
                                         int rows, double *red, double *__restrict__ gp) {
  constexpr int NTL = NT * (NT + 1) / 2;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int i16 = lane & 15, k4 = lane >> 4;
  d4 acc[NTL];
#pragma unroll
  for (int t = 0; t < NTL; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  const int kb = wid * (ROWS_BLK / 4), ke = min(rows, kb + ROWS_BLK / 4);
  for (int k0 = kb; k0 < ke; k0 += 4) {
    const int k = k0 + k4;
    const bool ok = k < ke;
    const double w = ok ? som[k] : 0.0;
    double z[NT];
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      const int col = 16 * b + i16;
      z[b] = (ok && col < R) ? sz[k * ld + col] : 0.0;
    }
    int t = 0;
#pragma unroll
    for (int ta = 0; ta < NT; ++ta) {
      const double av = w * z[ta];
#pragma unroll
      for (int tc = ta; tc < NT; ++tc) {
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, z[tc], acc[t], 0, 0, 0);
        ++t;
      }
    }
  }
  __syncthreads();   // every wave is done with sz before red overwrites it
#pragma unroll
  for (int t = 0; t < NTL; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[((wid * NTL + t) * 64 + lane) * 4 + v] = acc[t][v];
  __syncthreads();
  const int np = R * (R + 1) / 2;
  for (int p = tid; p < np; p += ROWS_BLK) {
    int a = 0, c = p;
    while (c >= R - a) { c -= R - a; ++a; }
    c += a;
    const int ta = a >> 4, tc = c >> 4, i = a & 15, j = c & 15;
    const int t = ta * NT - (ta * (ta - 1)) / 2 + (tc - ta);
    const int l = j + 16 * (i & 3), v = i >> 2;
    double sum = 0.0;
    for (int w = 0; w < 4; ++w) sum = sum + red[((w * NTL + t) * 64 + l) * 4 + v];
    gp[p] = sum;
  }
}

template <typename T, int DD>
__global__ void __launch_bounds__(ROWS_BLK) k_rows(
    OtherModes om, DevState *st, int R, u64 *__restrict__ samp_idx, double *__restrict__ samp_om,
    double *__restrict__ samp_w, const u64 *__restrict__ skeys,
    const FiberSlot *__restrict__ slots, u64 hmask, int hshift, T *__restrict__ zhat,
    unsigned *__restrict__ foff, unsigned *__restrict__ flen, double *__restrict__ gpart,
    u64 *__restrict__ part_len, unsigned *__restrict__ part_cnt, unsigned *__restrict__ part_act,
    T *__restrict__ M, i64 mlen, int ldz) {
  extern __shared__ double sz[];           // ROWS_BLK x (R+1); phase 3 reuses it
  __shared__ double som[ROWS_BLK];
  __shared__ unsigned sim[CPAL_MAXORDER][ROWS_BLK];
  const int tid = threadIdx.x;
  const int ld = R + 1;
  const int d = DD > 0 ? DD : om.d;
  const i64 s_det = st->s_det, s_used = st->s_rnd_used;
  const i64 n_slots = s_det + s_used;
  const double p_det = st->p_det;
  if (blockIdx.x == 0 && tid == 0) st->n_slots = n_slots;
  for (i64 e = (i64)blockIdx.x * blockDim.x + tid; e < mlen; e += (i64)gridDim.x * blockDim.x)
    M[e] = T(0);
  const i64 base = (i64)blockIdx.x * ROWS_BLK;
  if (base >= n_slots) return;   // uniform per block
  const int rows = (int)min((i64)ROWS_BLK, n_slots - base);
  // phase 1
  double omj = 0.0;
  bool active = false;
  if (tid < rows) {
    const i64 j = base + tid;
    u64 lin;
    double wj = 0.0;
    bool rnd = false;
    u64 cnt = 0;
    active = true;
    if (j < s_det) {
      lin = samp_idx[j];
    } else {
      // slot s_det + i of the sorted accepted draws: the first of a run of
      // equal rows carries the run (its length by galloping then bisection)
      const i64 i = j - s_det;
      lin = skeys[i];
      rnd = true;
      active = i == 0 || skeys[i - 1] != lin;
      if (active) {
        i64 lo = i, hi = s_used, step = 1;
        for (;;) {
          const i64 t = i + step;
          if (t >= s_used) break;
          if (skeys[t] != lin) { hi = t; break; }
          lo = t;
          step <<= 1;
        }
        while (hi - lo > 1) {
          const i64 mid = (lo + hi) >> 1;
          if (skeys[mid] == lin) lo = mid; else hi = mid;
        }
        cnt = (u64)(hi - i);
      }
    }
    u64 rem = lin;
    double p = 0.0;
    for (int u = 0; u < d; ++u) {
      u64 i;
      rem = div_rcp(rem, (u64)om.n[u], om.rcp[u], &i);
      sim[u][tid] = (unsigned)i;
      if (rnd) {
        const double qv = om.q[u][i];
        p = (u == 0) ? qv : p * qv;
      }
    }
    if (!rnd) {
      omj = 1.0;
      wj = 1.0;
    } else if (active) {
      omj = ((double)cnt * (1.0 - p_det)) / ((double)s_used * p);
      wj = sqrt(omj);
    }
    samp_idx[j] = lin;
    samp_om[j] = omj;
    samp_w[j] = wj;
    unsigned off = 0, len = 0;
    if (active) {
      u64 h = fiber_hash(lin, hshift);
      for (;;) {
        const FiberSlot sl = slots[h];
        if (sl.key == lin) { off = sl.off; len = sl.len; break; }
        if (sl.key == CPAL_EMPTY_KEY) break;
        h = (h + 1) & hmask;
      }
    }
    foff[j] = off;
    flen[j] = len;
  }
  {   // the workgroup's rows of the sampled system (active slots), gathered
      // length and nonempty-fiber count, totalled by the gather preparation
    const unsigned na = (unsigned)__popcll(__ballot(active));
    const u64 ln = wave_sum((u64)(tid < rows ? flen[base + tid] : 0u));
    const unsigned nf = (unsigned)__popcll(__ballot(tid < rows && flen[base + tid] > 0u));
    __shared__ unsigned wact[ROWS_BLK / 64], wnf[ROWS_BLK / 64];
    __shared__ u64 wln[ROWS_BLK / 64];
    if ((tid & 63) == 0) { wact[tid >> 6] = na; wnf[tid >> 6] = nf; wln[tid >> 6] = ln; }
    __syncthreads();
    if (tid == 0) {
      unsigned t = 0, f = 0;
      u64 l = 0;
      for (int q = 0; q < ROWS_BLK / 64; ++q) { t += wact[q]; f += wnf[q]; l += wln[q]; }
      part_act[blockIdx.x] = t;
      part_len[blockIdx.x] = l;
      part_cnt[blockIdx.x] = f;
    }
  }
  som[tid] = omj;
  __syncthreads();
  // phase 2
  const int lane = tid & 63, wid = tid >> 6;
  const int nwav = ROWS_BLK / 64;
  const int half = ldz <= 32 ? 1 : 0;          // two rows per wave when a row fits 32 lanes
  const int rpw = 1 + half;
  const int c = half ? (lane & 31) : lane;     // c < ldz covers the padded row
  const int sub = half ? (lane >> 5) : 0;
  const int cl = min(c, R - 1);                // column read (lanes past R discard it)
  for (int r0 = wid * rpw * ROWS_UNR; r0 < rows; r0 += nwav * rpw * ROWS_UNR) {
    double v[ROWS_UNR];
    if (DD > 0) {
      constexpr int DM = DD > 0 ? DD : 1;
      unsigned idx[ROWS_UNR][DM];
#pragma unroll
      for (int q = 0; q < ROWS_UNR; ++q) {
        const int rr = min(r0 + q * rpw + sub, rows - 1);
#pragma unroll
        for (int u = 0; u < DM; ++u) idx[q][u] = sim[u][rr];
      }
      double f[ROWS_UNR][DM];
#pragma unroll
      for (int q = 0; q < ROWS_UNR; ++q)
#pragma unroll
        for (int u = 0; u < DM; ++u) f[q][u] = om.A[u][(i64)idx[q][u] * R + cl];
#pragma unroll
      for (int q = 0; q < ROWS_UNR; ++q) {
        double x = f[q][0];
#pragma unroll
        for (int u = 1; u < DM; ++u) x = x * f[q][u];
        v[q] = x;
      }
    } else {
#pragma unroll
      for (int q = 0; q < ROWS_UNR; ++q) {
        const int rr = min(r0 + q * rpw + sub, rows - 1);
        double x = om.A[0][(i64)sim[0][rr] * R + cl];
        for (int u = 1; u < d; ++u) x = x * om.A[u][(i64)sim[u][rr] * R + cl];
        v[q] = x;
      }
    }
#pragma unroll
    for (int q = 0; q < ROWS_UNR; ++q) {
      const int rr = r0 + q * rpw + sub;
      if (rr < rows && c < ldz) {
        T out = T(0);
        if (c < R) {
          sz[rr * ld + c] = v[q];
          out = (T)(som[rr] * v[q]);
        }
        zhat[(base + rr) * ldz + c] = out;
      }
    }
  }
  __syncthreads();
  // phase 3
  double *gp = gpart + (i64)blockIdx.x * (R * (R + 1) / 2);
  const int nt = (R + 15) / 16;
  if (nt == 1) gs_tiles<1>(sz, som, ld, R, rows, sz, gp);
  else if (nt == 2) gs_tiles<2>(sz, som, ld, R, rows, sz, gp);
  else if (nt == 3) gs_tiles<3>(sz, som, ld, R, rows, sz, gp);
  else gs_tiles<4>(sz, som, ld, R, rows, sz, gp);
}

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
      if (v_s && col < R) unsafeAtomicAdd(&M[(i64)ik_s * R + col], x_s * zhat[z_s * ldz + col]);
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
#define GT_WIN 4096

// Gather preparation: the stream position of every fiber (exclusive prefix
// of the lengths over the slots) and the compacted nonempty fibers: for the
// c-th nonempty fiber, cpos = first stream position, coff = offset in the
// mode-sorted nonzeros, cidx = its slot (for the weighted KRP row); also
// chunk_first[ch] = the nonempty fiber holding stream position ch*GT_CHUNK.
// Empty fibers add nothing to M (they still enter G_s), and with only
// nonempty fibers a chunk of GT_CHUNK positions spans at most GT_CHUNK + 1 of
// them.  Workgroup b covers the ROWS_BLK slots of the row kernel's
// workgroup b, whose totals it takes from part_len / part_cnt; every
// workgroup sums the totals before its own, workgroup 0 also stores the
// grand totals.
__global__ void __launch_bounds__(ROWS_BLK) k_gather_prep(DevState *st,
                                                          const unsigned *__restrict__ flen,
                                                          const unsigned *__restrict__ foff,
                                                          const u64 *__restrict__ part_len,
                                                          const unsigned *__restrict__ part_cnt,
                                                          const unsigned *__restrict__ part_act,
                                                          u64 *__restrict__ cpos,
                                                          unsigned *__restrict__ coff,
                                                          unsigned *__restrict__ cidx,
                                                          unsigned *__restrict__ chunk_first) {
  const i64 n = st->n_slots;
  const int nb = (int)((n + ROWS_BLK - 1) / ROWS_BLK);
  const int b = blockIdx.x, tid = threadIdx.x;
  if (b >= nb && !(b == 0 && nb == 0)) return;   // uniform per block
  u64 bl = 0, al = 0, bc = 0, ac = 0, aa = 0;
  for (int q = tid; q < nb; q += ROWS_BLK) {
    const u64 l = part_len[q], c = part_cnt[q];
    al += l;
    ac += c;
    aa += part_act[q];
    if (q < b) { bl += l; bc += c; }
  }
  bl = wave_sum(bl); al = wave_sum(al); bc = wave_sum(bc); ac = wave_sum(ac); aa = wave_sum(aa);
  __shared__ u64 red[5][ROWS_BLK / 64];
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = bl; red[1][tid >> 6] = al; red[2][tid >> 6] = bc; red[3][tid >> 6] = ac;
    red[4][tid >> 6] = aa;
  }
  __syncthreads();
  bl = al = bc = ac = aa = 0;
  for (int q = 0; q < ROWS_BLK / 64; ++q) {
    bl += red[0][q]; al += red[1][q]; bc += red[2][q]; ac += red[3][q]; aa += red[4][q];
  }
  if (b == 0 && tid == 0) {
    st->gathered = (i64)al;
    st->n_fib = (i64)ac;
    st->s_bar = (i64)aa;
  }
  if (b >= nb) return;
  const i64 i = (i64)b * ROWS_BLK + tid;
  const unsigned l = i < n ? flen[i] : 0u;
  u64 tl, tc;
  const u64 el = block_excl_scan<u64>((u64)l, &tl);
  const u64 ec = block_excl_scan<u64>((u64)(l > 0), &tc);
  if (l > 0) {
    const u64 c = bc + ec, p0 = bl + el;
    cpos[c] = p0;
    coff[c] = foff[i];
    cidx[c] = (unsigned)i;
    const u64 c0 = (p0 + GT_CHUNK - 1) / GT_CHUNK, c1 = (p0 + l - 1) / GT_CHUNK;
    for (u64 ch = c0; ch <= c1; ++ch) chunk_first[ch] = (unsigned)c;
  }
}

// Segmented gather: workgroup g takes the chunks g, g + G, ... of GT_CHUNK
// stream positions; for a chunk
//  1. per thread, GT_PER_THREAD positions: the nonempty fiber holding the
//     position (binary search in the chunk's window of fiber starts), the
//     nonzero (i_k, x) and the fiber's sampled row, with every load
//     unconditional (positions past the chunk are clamped and masked);
//  2. the chunk's nonzeros are sorted by i_k in shared memory (stable LSD
//     radix sort, 6-bit digits ranked with wave ballots, keys i_k << 12 |
//     position in the chunk);
//  3. lane groups of LPN lanes (LPN = padded row width ldz) take equal
//     slices of the sorted list, lane c summing x * zhat(row, c) in a
//     register while i_k stays the same; a run that ends inside the slice is
//     added to M(i_k, c) at once, the first and last runs of every slice are
//     merged across slices in shared memory first, so every row of the chunk
//     costs one global atomic add per column (rows need i_k < 2^20).
#define GS_DIG 6
#define GS_BATCH 32

// Steps 1 and 2 for chunk ch; returns the sorted keys (ka or kb).
template <typename T>
__device__ __forceinline__ unsigned *seg_load_sort(
    i64 ch, i64 nch, i64 total, i64 nf, const u64 *__restrict__ cpos,
    const unsigned *__restrict__ coff, const unsigned *__restrict__ cidx,
    const unsigned *__restrict__ chunk_first, const NzLoad<T> &nz, int ikbits, u64 *win,
    unsigned *ka, unsigned *kb, T *lx, unsigned *lz, unsigned *tab) {
  constexpr int NW = GT_THREADS / 64;
  constexpr int NT = 64 * GT_PER_THREAD * NW;   // digit x round x wave counters
  const int tid = threadIdx.x, w = tid >> 6;
  const u64 lt = __lanemask_lt();
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
  unsigned *src = ka, *dst = kb;
  for (int shift = 12; shift < 12 + ikbits; shift += GS_DIG) {
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

// Step 3 over n row-sorted entries; entry q -> (row, x, KRP row) by get(q).
template <typename T, int LPN, typename Get>
__device__ __forceinline__ void seg_reduce(const Get &get, int n, int R,
                                           const T *__restrict__ zhat, int ldz,
                                           T *__restrict__ M, int *srow, T (*svec)[LPN]) {
  constexpr int NG = GT_THREADS / LPN;
  constexpr int PER = GT_CHUNK / NG;
  const int tid = threadIdx.x, gi = tid / LPN, c = tid % LPN;
  const int q0 = gi * PER, q1 = min(n, q0 + PER);
  int cur = -1, first = -1;
  T acc = T(0), facc = T(0);
  if (q0 < q1) {
    {
      unsigned r0;
      T x0;
      unsigned z0;
      get(q0, r0, x0, z0);
      cur = (int)r0;
    }
    for (int q = q0; q < q1; q += GS_BATCH) {
      unsigned rr[GS_BATCH];
      T xv[GS_BATCH], zv[GS_BATCH];
#pragma unroll
      for (int b = 0; b < GS_BATCH; ++b) {
        unsigned zr;
        get(min(q + b, q1 - 1), rr[b], xv[b], zr);
        zv[b] = zhat[(i64)zr * ldz + c];
      }
#pragma unroll
      for (int b = 0; b < GS_BATCH; ++b) {
        if (q + b < q1) {
          const int r = (int)rr[b];
          if (r != cur) {
            if (first < 0) { first = cur; facc = acc; }
            else if (c < R) unsafeAtomicAdd(&M[(i64)cur * R + c], acc);
            cur = r;
            acc = T(0);
          }
          acc += xv[b] * zv[b];
        }
      }
    }
  }
  // slice ends: slot 2gi = first run, 2gi+1 = last run (-1: none)
  if (first < 0) { first = cur; facc = acc; cur = -1; }
  if (c == 0) { srow[2 * gi] = first; srow[2 * gi + 1] = cur; }
  svec[2 * gi][c] = facc;
  svec[2 * gi + 1][c] = acc;
  __syncthreads();
  if (gi == 0 && n > 0) {
    int mr = -1;
    T ma = T(0);
    for (int sl = 0; sl < 2 * NG; ++sl) {
      const int r = srow[sl];
      if (r < 0) continue;
      if (r != mr) {
        if (mr >= 0 && c < R) unsafeAtomicAdd(&M[(i64)mr * R + c], ma);
        mr = r;
        ma = T(0);
      }
      ma += svec[sl][c];
    }
    if (mr >= 0 && c < R) unsafeAtomicAdd(&M[(i64)mr * R + c], ma);
  }
}

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

template <typename T, int LPN>
__global__ void __launch_bounds__(GT_THREADS) k_gather_seg(
    const DevState *st, int R, const u64 *__restrict__ cpos, const unsigned *__restrict__ coff,
    const unsigned *__restrict__ cidx, const unsigned *__restrict__ chunk_first, NzLoad<T> nz,
    int ikbits, const T *__restrict__ zhat, int ldz, T *__restrict__ M, i64 nk) {
  constexpr int NG = GT_THREADS / LPN;
  __shared__ u64 win[GT_WIN];
  __shared__ unsigned ka[GT_CHUNK], kb[GT_CHUNK];
  __shared__ T lx[GT_CHUNK];
  __shared__ unsigned lz[GT_CHUNK];
  __shared__ unsigned tab[64 * GT_PER_THREAD * (GT_THREADS / 64)];
  __shared__ int srow[2 * NG];
  __shared__ T svec[2 * NG][LPN];
  const i64 total = st->gathered;
  const i64 nf = st->n_fib;
  const i64 nch = (total + GT_CHUNK - 1) / GT_CHUNK;
  // this XCD's copy of M: the adds of workgroups on one XCD stay in its L2
  T *Mx = M + (i64)(xcd_id() & (CPAL_MCOPIES - 1)) * nk * R;
  for (i64 ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    const unsigned *keys = seg_load_sort<T>(ch, nch, total, nf, cpos, coff, cidx, chunk_first, nz,
                                            ikbits, win, ka, kb, lx, lz, tab);
    const int nvalid = (int)(min(total, (ch + 1) * GT_CHUNK) - ch * GT_CHUNK);
    seg_reduce<T, LPN>(LdsEntries<T>{keys, lx, lz}, nvalid, R, zhat, ldz, Mx, srow, svec);
  }
}

int gather_row_width(int R);

void launch_gather_seg(bool f64, const DevState *st, int R, const u64 *cpos, const unsigned *coff,
                       const unsigned *cidx, const unsigned *chunk_first, const uint2 *pairs,
                       const int *ik, const double *v64, i64 nk, const void *zhat, int ldz, void *M,
                       int grid, hipStream_t s) {
  int ikbits = 1;
  while ((1ll << ikbits) < nk) ++ikbits;
  const int rm = gather_row_width(R);
  if (f64) {
    NzLoad<double> nz{ik, v64};
    auto k = rm == 16 ? k_gather_seg<double, 16> : rm == 32 ? k_gather_seg<double, 32>
                                                            : k_gather_seg<double, 64>;
    hipLaunchKernelGGL(k, dim3(grid), dim3(GT_THREADS), 0, s, st, R, cpos, coff, cidx,
                       chunk_first, nz, ikbits, (const double *)zhat, ldz, (double *)M, nk);
  } else {
    NzLoad<float> nz{pairs};
    auto k = rm == 16 ? k_gather_seg<float, 16> : rm == 32 ? k_gather_seg<float, 32>
                                                           : k_gather_seg<float, 64>;
    hipLaunchKernelGGL(k, dim3(grid), dim3(GT_THREADS), 0, s, st, R, cpos, coff, cidx,
                       chunk_first, nz, ikbits, (const float *)zhat, ldz, (float *)M, nk);
  }
}

// ------------------------------------------------------------------- solve --
// A_k(i,:) = M(i,:) G_s^{-1}: forward substitution with the Cholesky factor
// (subtractions in ascending order), back substitution (right-looking:
// subtractions in descending order), or the pseudo-inverse from the
// eigendecomposition.  Lanes = columns, LPN lanes per row (R <= LPN); FP64
// throughout.  Skipped when the update hit a state error.  256 threads.
template <typename T, int LPN>
__global__ void __launch_bounds__(256) k_solve_rows(const DevState *st, i64 n, int R,
                                                    const T *__restrict__ M, int ncopies,
                                                    const Decomp *__restrict__ dc,
                                                    double *__restrict__ A,
                                                    float *__restrict__ A32) {
  extern __shared__ double sL[];   // R*R factor (L, or V)
  if (st->flags & CPAL_FLAG_STATE) return;
  const int pinv = dc->pinv;
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) sL[e] = pinv ? dc->V[e] : dc->L[e];
  __syncthreads();
  const int tid = threadIdx.x;
  const int c = (tid & 63) % LPN;
  const i64 row = ((i64)blockIdx.x * blockDim.x + tid) / LPN;
  if (row >= n) return;   // uniform per lane group
  const bool col = c < R;
  const int cl = col ? c : R - 1;
  double v = 0.0;
  if (col)
    for (int x = 0; x < ncopies; ++x) v = v + (double)M[(i64)x * n * R + row * R + c];
  if (!pinv) {
    for (int j = 0; j < R; ++j) {
      const double yj = group_value<LPN>(v, j) / sL[j * R + j];
      if (c == j) v = yj;
      else if (c > j && col) v = v - sL[c * R + j] * yj;
    }
    for (int j = R - 1; j >= 0; --j) {
      const double xj = group_value<LPN>(v, j) / sL[j * R + j];
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

__global__ void k_stats(const DevState *st, int k, int D, cpal_mode_stats *out) {
  int fl = st->flags;
  for (int m = 0; m < D; ++m)
    if (m != k && st->lev_pinv[m]) fl |= CPAL_FLAG_PINV;
  out->s_det = st->s_det;
  out->s_rnd = st->s_rnd_used;
  out->s_bar = st->s_bar;
  out->draws = st->draws;
  out->gathered_nnz = st->gathered;
  out->p_det = st->p_det;
  out->flags = fl;
  out->pad = 0;
}

__global__ void k_to_f32(const double *__restrict__ a, float *__restrict__ b, i64 n) {
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
    b[i] = (float)a[i];
}

// ------------------------------------------------------------- fiber index --
// comp = lin(other coords) * n_k + i_k; err bit 1 = coordinate out of range.
__global__ void k_mode_keys(const int *__restrict__ coords, i64 nnz, int D, OtherModes om,
                            i64 nk, u64 *__restrict__ comp, unsigned *__restrict__ ids,
                            int *err) {
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (i64)gridDim.x * blockDim.x) {
    u64 key = 0;
    bool bad = false;
    for (int u = 0; u < om.d; ++u) {
      const int c = coords[(i64)om.mode[u] * nnz + e];
      bad |= c < 0 || c >= om.n[u];
      key += (u64)(unsigned)c * om.stride[u];
    }
    const int ck = coords[(i64)om.k * nnz + e];
    bad |= ck < 0 || ck >= nk;
    if (bad) atomicOr(err, 1);
    comp[e] = key * (u64)nk + (u64)(unsigned)ck;
    ids[e] = (unsigned)e;
  }
}

// fiber starts; err bit 2 = duplicate coordinate
__global__ void k_fiber_mark(const u64 *__restrict__ comp, i64 nnz, i64 nk,
                             unsigned *__restrict__ flag, int *err) {
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (i64)gridDim.x * blockDim.x) {
    unsigned f = 1;
    if (e > 0) {
      const u64 a = comp[e - 1], b = comp[e];
      if (a == b) atomicOr(err, 2);
      f = (a / (u64)nk) != (b / (u64)nk);
    }
    flag[e] = f;
  }
}

__global__ void k_fiber_starts(const unsigned *__restrict__ flag, const u64 *__restrict__ fid,
                               i64 nnz, unsigned *__restrict__ fstart) {
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (i64)gridDim.x * blockDim.x)
    if (flag[e]) fstart[fid[e]] = (unsigned)e;
}

__global__ void k_hash_insert(const u64 *__restrict__ comp, i64 nnz, i64 nk,
                              const unsigned *__restrict__ fstart, u64 nfib,
                              FiberSlot *__restrict__ slots, u64 hmask, int hshift) {
  for (u64 f = (u64)blockIdx.x * blockDim.x + threadIdx.x; f < nfib; f += (u64)gridDim.x * blockDim.x) {
    const unsigned off = fstart[f];
    const unsigned end = (f + 1 < nfib) ? fstart[f + 1] : (unsigned)nnz;
    const u64 key = comp[off] / (u64)nk;
    u64 h = fiber_hash(key, hshift);
    for (;;) {
      const u64 old = atomicCAS(&slots[h].key, CPAL_EMPTY_KEY, key);
      if (old == CPAL_EMPTY_KEY) {
        slots[h].off = off;
        slots[h].len = end - off;
        break;
      }
      h = (h + 1) & hmask;
    }
  }
}

__global__ void k_slots_clear(FiberSlot *__restrict__ slots, u64 n) {
  for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
    slots[i].key = CPAL_EMPTY_KEY;
    slots[i].off = 0;
    slots[i].len = 0;
  }
}

// mode-sorted nonzeros in the gather layout
__global__ void k_mode_pairs(const u64 *__restrict__ comp, const unsigned *__restrict__ ids, i64 nnz,
                             i64 nk, const void *__restrict__ vals, int vdt,
                             uint2 *__restrict__ pairs, int *__restrict__ ik32,
                             double *__restrict__ v64) {
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (i64)gridDim.x * blockDim.x) {
    const unsigned id = ids[e];
    const int ik = (int)(comp[e] % (u64)nk);
    const double v = vdt == CPAL_F64 ? ((const double *)vals)[id] : (double)((const float *)vals)[id];
    if (pairs) pairs[e] = make_uint2((unsigned)ik, __float_as_uint((float)v));
    if (ik32) { ik32[e] = ik; v64[e] = v; }
  }
}

// ------------------------------------------------------------- launchers ---
static int grid_for(i64 n, int blk, int maxg = 8192) {
  i64 g = (n + blk - 1) / blk;
  if (g < 1) g = 1;
  if (g > maxg) g = maxg;
  return (int)g;
}

void launch_rows(bool f64, const OtherModes &om, DevState *st, int R, i64 cap, u64 *samp_idx,
                 double *samp_om, double *samp_w, const u64 *skeys,
                 const FiberSlot *slots, u64 hmask, int hshift, void *zhat, unsigned *foff,
                 unsigned *flen, double *gpart, u64 *part_len, unsigned *part_cnt,
                 unsigned *part_act, void *M, i64 mlen, int ldz, hipStream_t s) {
  const int nb = (int)((cap + ROWS_BLK - 1) / ROWS_BLK);
  // z rows, then the four waves' G_s tiles (4 x NTL x 256 doubles)
  const int nt = (R + 15) / 16;
  const size_t sh = sizeof(double) * std::max<size_t>((size_t)ROWS_BLK * (R + 1),
                                                      (size_t)1024 * (nt * (nt + 1) / 2));
  const int dd = (om.d >= 2 && om.d <= 4) ? om.d : 0;
  if (f64) {
    auto k = dd == 2 ? k_rows<double, 2> : dd == 3 ? k_rows<double, 3>
           : dd == 4 ? k_rows<double, 4> : k_rows<double, 0>;
    hipLaunchKernelGGL(k, dim3(nb), dim3(ROWS_BLK), sh, s, om, st, R, samp_idx, samp_om, samp_w,
                       skeys, slots, hmask, hshift, (double *)zhat, foff, flen, gpart,
                       part_len, part_cnt, part_act, (double *)M, mlen, ldz);
  } else {
    auto k = dd == 2 ? k_rows<float, 2> : dd == 3 ? k_rows<float, 3>
           : dd == 4 ? k_rows<float, 4> : k_rows<float, 0>;
    hipLaunchKernelGGL(k, dim3(nb), dim3(ROWS_BLK), sh, s, om, st, R, samp_idx, samp_om, samp_w,
                       skeys, slots, hmask, hshift, (float *)zhat, foff, flen, gpart,
                       part_len, part_cnt, part_act, (float *)M, mlen, ldz);
  }
}

int rows_blocks(i64 cap) { return (int)((cap + ROWS_BLK - 1) / ROWS_BLK); }
int rows_per_block() { return ROWS_BLK; }

void launch_gather_prep(DevState *st, const unsigned *flen, const unsigned *foff, i64 cap,
                        const u64 *part_len, const unsigned *part_cnt, const unsigned *part_act,
                        u64 *cpos, unsigned *coff, unsigned *cidx, unsigned *chunk_first,
                        hipStream_t s) {
  const int nb = std::max(1, (int)((cap + ROWS_BLK - 1) / ROWS_BLK));
  hipLaunchKernelGGL(k_gather_prep, dim3(nb), dim3(ROWS_BLK), 0, s, st, flen, foff, part_len,
                     part_cnt, part_act, cpos, coff, cidx, chunk_first);
}


i64 gather_chunks_cap(i64 nnz) { return nnz / GT_CHUNK + 2; }

int gather_row_width(int R) { return R <= 16 ? 16 : (R <= 32 ? 32 : 64); }

void launch_gather(bool f64, const DevState *st, int R, const u64 *cpos, const unsigned *coff,
                   const unsigned *cidx, const uint2 *pairs, const int *ik, const double *v64,
                   const void *zhat, void *M, int ldz, int grid, hipStream_t s) {
  if (f64) {
    NzLoad<double> nz{ik, v64};
    hipLaunchKernelGGL(k_gather<double>, dim3(grid), dim3(256), 0, s, st, R, cpos, coff, cidx, nz,
                       (const double *)zhat, (double *)M, ldz);
  } else {
    NzLoad<float> nz{pairs};
    hipLaunchKernelGGL(k_gather<float>, dim3(grid), dim3(256), 0, s, st, R, cpos, coff, cidx, nz,
                       (const float *)zhat, (float *)M, ldz);
  }
}

// Sampled rows in order (active slots only, s_bar of them) into the caller's
// buffers, at most cap; *count = s_bar.  One workgroup (audit path).
__global__ void __launch_bounds__(1024) k_samples_out(const DevState *st,
                                                      const u64 *__restrict__ samp_idx,
                                                      const double *__restrict__ samp_om,
                                                      const double *__restrict__ samp_w, i64 cap,
                                                      u64 *idx, double *om, double *w,
                                                      i64 *count) {
  const i64 n = st->n_slots, s_det = st->s_det;
  i64 carry = 0;
  for (i64 b0 = 0; b0 < n; b0 += 1024) {
    const i64 j = b0 + threadIdx.x;
    const unsigned a = (j < n && (j < s_det || samp_om[j] > 0.0)) ? 1u : 0u;
    unsigned tot;
    const unsigned ex = block_excl_scan<unsigned>(a, &tot);
    const i64 o = carry + ex;
    if (a && o < cap) {
      if (idx) idx[o] = samp_idx[j];
      if (om) om[o] = samp_om[j];
      if (w) w[o] = samp_w[j];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && count) *count = st->s_bar;
}

void launch_samples_out(const DevState *st, const u64 *samp_idx, const double *samp_om,
                        const double *samp_w, i64 cap, u64 *idx, double *om, double *w,
                        i64 *count, hipStream_t s) {
  hipLaunchKernelGGL(k_samples_out, dim3(1), dim3(1024), 0, s, st, samp_idx, samp_om, samp_w, cap,
                     idx, om, w, count);
}

void launch_solve_rows(bool f64, const DevState *st, i64 n, int R, const void *M, int ncopies,
                       const Decomp *dc, double *A, float *A32, hipStream_t s) {
  const int lpn = R <= 16 ? 16 : (R <= 32 ? 32 : 64);
  const int nb = (int)((n * lpn + 255) / 256);
  const size_t sh = sizeof(double) * (size_t)R * R;
  if (f64) {
    auto k = lpn == 16 ? k_solve_rows<double, 16> : lpn == 32 ? k_solve_rows<double, 32>
                                                              : k_solve_rows<double, 64>;
    hipLaunchKernelGGL(k, dim3(nb), dim3(256), sh, s, st, n, R, (const double *)M, ncopies, dc, A,
                       A32);
  } else {
    auto k = lpn == 16 ? k_solve_rows<float, 16> : lpn == 32 ? k_solve_rows<float, 32>
                                                             : k_solve_rows<float, 64>;
    hipLaunchKernelGGL(k, dim3(nb), dim3(256), sh, s, st, n, R, (const float *)M, ncopies, dc, A,
                       A32);
  }
}

void launch_stats(const DevState *st, int k, int D, cpal_mode_stats *out, hipStream_t s) {
  hipLaunchKernelGGL(k_stats, dim3(1), dim3(1), 0, s, st, k, D, out);
}

void launch_to_f32(const double *a, float *b, i64 n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n, 256)), dim3(256), 0, s, a, b, n);
}

void launch_mode_keys(const int *coords, i64 nnz, int D, const OtherModes &om, i64 nk, u64 *comp,
                      unsigned *ids, int *err, hipStream_t s) {
  hipLaunchKernelGGL(k_mode_keys, dim3(grid_for(nnz, 256)), dim3(256), 0, s, coords, nnz, D, om,
                     nk, comp, ids, err);
}

void launch_fiber_mark(const u64 *comp, i64 nnz, i64 nk, unsigned *flag, int *err,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_fiber_mark, dim3(grid_for(nnz, 256)), dim3(256), 0, s, comp, nnz, nk, flag,
                     err);
}

void launch_fiber_starts(const unsigned *flag, const u64 *fid, i64 nnz, unsigned *fstart,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_fiber_starts, dim3(grid_for(nnz, 256)), dim3(256), 0, s, flag, fid, nnz,
                     fstart);
}

void launch_hash_build(const u64 *comp, i64 nnz, i64 nk, const unsigned *fstart, u64 nfib,
                       FiberSlot *slots, u64 nslots, int hshift, hipStream_t s) {
  hipLaunchKernelGGL(k_slots_clear, dim3(grid_for((i64)nslots, 256)), dim3(256), 0, s, slots,
                     nslots);
  hipLaunchKernelGGL(k_hash_insert, dim3(grid_for((i64)nfib, 256)), dim3(256), 0, s, comp, nnz,
                     nk, fstart, nfib, slots, nslots - 1, hshift);
}

void launch_mode_pairs(const u64 *comp, const unsigned *ids, i64 nnz, i64 nk, const void *vals,
                       int vdt, uint2 *pairs, int *ik32, double *v64, hipStream_t s) {
  hipLaunchKernelGGL(k_mode_pairs, dim3(grid_for(nnz, 256)), dim3(256), 0, s, comp, ids, nnz, nk,
                     vals, vdt, pairs, ik32, v64);
}

}  // namespace cpal
