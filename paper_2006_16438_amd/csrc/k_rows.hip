// Sampled system of one mode update, per slot: KrpSamp (rows of the KRP as
// Hadamard products of factor rows, eq. (2.1)) with the combined repeats of
// Sec. 4.1, the fiber probe of TnsrSamp (Sec. 6.3), the slots' part of
//   G_s = sum_j omega_j z_j z_j^T (FP64, the normal equations of the sketched
//   problem, eq. (1.2)),
// the stream layout of the sampled fibers for the gather, and the sampled
// rows handed to callers.
#include "cpal_common.h"

namespace cpal {

// ------------------------------------------------------------- sample rows --
// Slots j of the sampled system, ROWS_BLK per block: the deterministic rows
// first, then one slot per accepted random draw in draw order; the draw
// table gives every row the draw that entered it and its number of draws, so
// that draw's slot is the combined row (Sec. 4.1) and the slots of its other
// draws stay empty (omega = 0, no fiber); three phases:
//  1. thread per slot: omega_j, w_j, the other-mode indices of row j and the
//     fiber hash probe; the slot of a combined row records its table entry
//     (tpos) so that the gather preparation can empty the table again;
//  2. lanes = columns: z_j (FP64, Hadamard product of the other factors' rows
//     in ascending mode order) into shared memory and the weighted row
//     omega_j z_j in T (zero-padded to ldz) to zhat, rows read and written
//     contiguously, ROWS_UNR rows per lane group in flight;
//  3. the block's part of G_s (pairs a <= c, packed row by row) on the
//     matrix cores.
// Blocks past the slots only clear their share of M.  DD = number of other modes
// (0: any, runtime loops).
#define ROWS_BLK 256
#define ROWS_UNR 8
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
#pragma unroll 4
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

template <typename TZ, typename TM, int DD>
__device__ __forceinline__ void rows_body(Blk bk, const OtherModes &om, DevState *st, int R,
    u64 *__restrict__ samp_idx, double *__restrict__ samp_om, double *__restrict__ samp_w,
    const u64 *__restrict__ dkeys, const DrawEntry *__restrict__ tab, u64 tmask, int tshift,
    unsigned *__restrict__ tpos, const FiberSlot *__restrict__ slots, u64 hmask, int hshift,
    unsigned dense_len, TZ *__restrict__ zhat, unsigned *__restrict__ foff,
    unsigned *__restrict__ flen, double *__restrict__ gpart, u64 *__restrict__ part_len,
    unsigned *__restrict__ part_cnt, unsigned *__restrict__ part_act, TM *__restrict__ M, i64 mlen,
    int ldz) {
  extern __shared__ double sz[];           // ROWS_BLK x (R+1); phase 3 reuses it
  __shared__ double som[ROWS_BLK];
  __shared__ unsigned sim[CPAL_MAXORDER][ROWS_BLK];
  const int tid = threadIdx.x;
  const int ld = R + 1;
  const int d = DD > 0 ? DD : om.d;
  const i64 s_det = st->s_det, s_used = st->s_rnd_used;
  const i64 n_slots = s_det + s_used;
  const double p_det = st->p_det;
  if (bk.x == 0 && tid == 0) st->n_slots = n_slots;
  for (i64 e = (i64)bk.x * blockDim.x + tid; e < mlen; e += (i64)bk.n * blockDim.x)
    M[e] = TM(0);
  const i64 base = (i64)bk.x * ROWS_BLK;
  if (base >= n_slots) return;   // uniform per block
  const int rows = (int)min((i64)ROWS_BLK, n_slots - base);
  // phase 1: the first draw-table probe, the first fiber probe and the q
  // loads are all issued before any of them is used
  double omj = 0.0;
  bool active = false;
  unsigned len = 0;
  if (tid < rows) {
    const i64 j = base + tid;
    const bool rnd = j >= s_det;
    const i64 i = j - s_det;   // accepted draw of a random slot
    const u64 lin = rnd ? dkeys[i] : samp_idx[j];
    u64 hd = key_hash(lin, tshift), hf = key_hash(lin, hshift);
    DrawEntry e{lin, 0u, 0u};
    if (rnd) e = tab[hd];
    const bool dense = slots == nullptr;   // every fiber: the whole mode-k column
    FiberSlot sl{dense ? lin : CPAL_EMPTY_KEY, 0u, dense_len};
    if (!dense) sl = slots[hf];
    constexpr int MO = CPAL_MAXORDER - 1;
    unsigned ix[MO];
    double qv[MO];
    u64 rem = lin;
#pragma unroll
    for (int u = 0; u < MO; ++u) {
      ix[u] = 0;
      if (u < d) {
        u64 iu;
        rem = div_rcp(rem, (u64)om.n[u], om.rcp[u], &iu);
        ix[u] = (unsigned)iu;
        sim[u][tid] = ix[u];
      }
    }
#pragma unroll
    for (int u = 0; u < MO; ++u) qv[u] = (rnd && u < d) ? om.q[u][ix[u]] : 1.0;
    // the row's table entry says whether this draw carries the row and how
    // many draws it has
    u64 cnt = 1;
    active = true;
    if (rnd) {
      for (u64 probe = 0; e.key != lin && e.key != CPAL_EMPTY_KEY && probe < tmask; ++probe) {
        hd = (hd + 1) & tmask;
        e = tab[hd];
      }
      active = e.key == lin && e.first == (unsigned)i;
      cnt = 1 + (u64)e.cnt;
      tpos[i] = active ? (unsigned)hd : ~0u;
    }
    unsigned off = 0;
    for (;;) {
      if (sl.key == lin) { off = sl.off; len = sl.len; break; }
      if (sl.key == CPAL_EMPTY_KEY) break;
      hf = (hf + 1) & hmask;
      sl = slots[hf];
    }
    if (!active) { off = 0; len = 0; }
    double wj = 0.0;
    if (!rnd) {
      omj = 1.0;
      wj = 1.0;
    } else if (active) {
      double p = qv[0];
#pragma unroll
      for (int u = 1; u < MO; ++u)
        if (u < d) p = p * qv[u];
      omj = ((double)cnt * (1.0 - p_det)) / ((double)s_used * p);
      wj = sqrt(omj);
    }
    samp_idx[j] = lin;
    samp_om[j] = omj;
    samp_w[j] = wj;
    foff[j] = off;
    flen[j] = len;
  }
  {   // the workgroup's rows of the sampled system (active slots), gathered
      // length and nonempty-fiber count, totalled by the gather preparation
    const unsigned na = (unsigned)__popcll(__ballot(active));
    const u64 ln = wave_sum((u64)len);
    const unsigned nf = (unsigned)__popcll(__ballot(len > 0u));
    __shared__ unsigned wact[ROWS_BLK / 64], wnf[ROWS_BLK / 64];
    __shared__ u64 wln[ROWS_BLK / 64];
    if ((tid & 63) == 0) { wact[tid >> 6] = na; wnf[tid >> 6] = nf; wln[tid >> 6] = ln; }
    __syncthreads();
    if (tid == 0) {
      unsigned t = 0, f = 0;
      u64 l = 0;
      for (int q = 0; q < ROWS_BLK / 64; ++q) { t += wact[q]; f += wnf[q]; l += wln[q]; }
      part_act[bk.x] = t;
      part_len[bk.x] = l;
      part_cnt[bk.x] = f;
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
        TZ out = TZ(0);
        if (c < R) {
          sz[rr * ld + c] = v[q];
          out = cvt_from<TZ>(som[rr] * v[q]);
        }
        zhat[(base + rr) * ldz + c] = out;
      }
    }
  }
  __syncthreads();
  // phase 3
  double *gp = gpart + (i64)bk.x * (R * (R + 1) / 2);
  const int nt = (R + 15) / 16;
  if (nt == 1) gs_tiles<1>(sz, som, ld, R, rows, sz, gp);
  else if (nt == 2) gs_tiles<2>(sz, som, ld, R, rows, sz, gp);
  else if (nt == 3) gs_tiles<3>(sz, som, ld, R, rows, sz, gp);
  else gs_tiles<4>(sz, som, ld, R, rows, sz, gp);
}
template <typename TZ, typename TM, int DD>
__global__ void __launch_bounds__(ROWS_BLK) k_rows(
    OtherModes om, DevState *st, int R, u64 *__restrict__ samp_idx, double *__restrict__ samp_om,
    double *__restrict__ samp_w, const u64 *__restrict__ dkeys, const DrawEntry *__restrict__ tab,
    u64 tmask, int tshift, unsigned *__restrict__ tpos,
    const FiberSlot *__restrict__ slots, u64 hmask, int hshift, unsigned dense_len,
    TZ *__restrict__ zhat, unsigned *__restrict__ foff, unsigned *__restrict__ flen,
    double *__restrict__ gpart, u64 *__restrict__ part_len, unsigned *__restrict__ part_cnt,
    unsigned *__restrict__ part_act, TM *__restrict__ M, i64 mlen, int ldz) {
  rows_body<TZ, TM, DD>(CPAL_BLK, om, st, R, samp_idx, samp_om, samp_w, dkeys, tab, tmask, tshift,
    tpos, slots, hmask, hshift, dense_len, zhat, foff, flen, gpart, part_len, part_cnt, part_act, M,
    mlen, ldz);
}
template <typename TZ, typename TM, int DD>
struct B_rows {
  static constexpr int NT = ROWS_BLK, MW = 1;
  template <class... A>
  __device__ __forceinline__ static void run(Blk b, const A &...a) {
    rows_body<TZ, TM, DD>(b, a...);
  }
};


// Gather preparation: the stream position of every fiber (exclusive prefix
// of the lengths over the slots) and the compacted nonempty fibers: for the
// c-th nonempty fiber, cpos = first stream position, coff = offset in the
// mode-sorted nonzeros, cidx = its slot (for the weighted KRP row); also
// chunk_first[ch] = the nonempty fiber holding stream position
// ch * CPAL_GATHER_CHUNK.  Empty fibers add nothing to M (they still enter
// G_s), and with only nonempty fibers a chunk of CPAL_GATHER_CHUNK positions
// spans at most CPAL_GATHER_CHUNK + 1 of them.  Workgroup b covers the ROWS_BLK slots of the row kernel's
// workgroup b, whose totals it takes from part_len / part_cnt; every
// workgroup sums the totals before its own, workgroup 0 also stores the
// grand totals.  It also empties the draw-table entries of its slots (every
// entry the update filled belongs to exactly one combined row).
__device__ __forceinline__ void gather_prep_body(Blk bk, DevState *st,
    const unsigned *__restrict__ flen, const unsigned *__restrict__ foff,
    const u64 *__restrict__ part_len, const unsigned *__restrict__ part_cnt,
    const unsigned *__restrict__ part_act, u64 *__restrict__ cpos, unsigned *__restrict__ coff,
    unsigned *__restrict__ cidx, unsigned *__restrict__ chunk_first,
    const unsigned *__restrict__ tpos, DrawEntry *__restrict__ tab) {
  const i64 n = st->n_slots;
  const int nb = (int)((n + ROWS_BLK - 1) / ROWS_BLK);
  const int b = bk.x, tid = threadIdx.x;
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
  const i64 s_det = st->s_det;
  if (i >= s_det && i < n) {
    const unsigned tp = tpos[i - s_det];
    if (tp != ~0u) tab[tp] = DrawEntry{CPAL_EMPTY_KEY, ~0u, 0u};
  }
  const unsigned l = i < n ? flen[i] : 0u;
  u64 tl, tc;
  const u64 el = block_excl_scan<u64>((u64)l, &tl);
  const u64 ec = block_excl_scan<u64>((u64)(l > 0), &tc);
  if (l > 0) {
    const u64 c = bc + ec, p0 = bl + el;
    cpos[c] = p0;
    coff[c] = foff[i];
    cidx[c] = (unsigned)i;
    const u64 c0 = (p0 + CPAL_GATHER_CHUNK - 1) / CPAL_GATHER_CHUNK;
    const u64 c1 = (p0 + l - 1) / CPAL_GATHER_CHUNK;
    for (u64 ch = c0; ch <= c1; ++ch) chunk_first[ch] = (unsigned)c;
  }
}
__global__ void __launch_bounds__(ROWS_BLK) k_gather_prep(DevState *st,
                                                          const unsigned *__restrict__ flen,
                                                          const unsigned *__restrict__ foff,
                                                          const u64 *__restrict__ part_len,
                                                          const unsigned *__restrict__ part_cnt,
                                                          const unsigned *__restrict__ part_act,
                                                          u64 *__restrict__ cpos,
                                                          unsigned *__restrict__ coff,
                                                          unsigned *__restrict__ cidx,
                                                          unsigned *__restrict__ chunk_first,
                                                          const unsigned *__restrict__ tpos,
                                                          DrawEntry *__restrict__ tab) {
  gather_prep_body(CPAL_BLK, st, flen, foff, part_len, part_cnt, part_act, cpos, coff, cidx,
    chunk_first, tpos, tab);
}
CPAL_BODY(B_gather_prep, ROWS_BLK, 1, gather_prep_body);

// ------------------------------------------------------------- launchers ---
template <typename TZ, typename TM>
static void launch_rows_t(const OtherModes &om, DevState *st, int R, int nb, size_t sh, u64 *samp_idx,
                          double *samp_om, double *samp_w, const u64 *dkeys, const DrawEntry *tab,
                          u64 tmask, int tshift, unsigned *tpos, const FiberSlot *slots, u64 hmask,
                          int hshift, unsigned dense_len, void *zhat, unsigned *foff,
                          unsigned *flen, double *gpart, u64 *part_len, unsigned *part_cnt,
                          unsigned *part_act, void *M, i64 mlen, int ldz, hipStream_t s) {
  const int dd = (om.d >= 2 && om.d <= 4) ? om.d : 0;
#define CPAL_ROWS_LAUNCH(DD)                                                                    \
  launch_b<B_rows<TZ, TM, DD>>(k_rows<TZ, TM, DD>, dim3(nb), dim3(ROWS_BLK), sh, s, om, st, R,   \
                               samp_idx, samp_om, samp_w, dkeys, tab, tmask, tshift, tpos, slots, \
                               hmask, hshift, dense_len, (TZ *)zhat, foff, flen, gpart, part_len, \
                               part_cnt, part_act, (TM *)M, mlen, ldz)
  if (dd == 2) CPAL_ROWS_LAUNCH(2);
  else if (dd == 3) CPAL_ROWS_LAUNCH(3);
  else if (dd == 4) CPAL_ROWS_LAUNCH(4);
  else CPAL_ROWS_LAUNCH(0);
#undef CPAL_ROWS_LAUNCH
}

// zdt: precision of the weighted KRP rows (CPAL_F64, CPAL_F32 or CPAL_BF16);
// M is FP64 for CPAL_F64, else FP32.  slots == nullptr: dense tensor, every
// fiber has dense_len entries and no index is probed.
void launch_rows(int zdt, const OtherModes &om, DevState *st, int R, i64 cap, u64 *samp_idx,
                 double *samp_om, double *samp_w, const u64 *dkeys, const DrawEntry *tab,
                 u64 tmask, int tshift, unsigned *tpos,
                 const FiberSlot *slots, u64 hmask, int hshift, unsigned dense_len, void *zhat,
                 unsigned *foff, unsigned *flen, double *gpart, u64 *part_len, unsigned *part_cnt,
                 unsigned *part_act, void *M, i64 mlen, int ldz, hipStream_t s) {
  const int nb = (int)((cap + ROWS_BLK - 1) / ROWS_BLK);
  // z rows, then the four waves' G_s tiles (4 x NTL x 256 doubles)
  const int nt = (R + 15) / 16;
  const size_t sh = sizeof(double) * std::max<size_t>((size_t)ROWS_BLK * (R + 1),
                                                      (size_t)1024 * (nt * (nt + 1) / 2));
  if (zdt == CPAL_F64)
    launch_rows_t<double, double>(om, st, R, nb, sh, samp_idx, samp_om, samp_w, dkeys, tab, tmask,
                                  tshift, tpos, slots, hmask, hshift, dense_len, zhat, foff, flen,
                                  gpart, part_len, part_cnt, part_act, M, mlen, ldz, s);
  else if (zdt == CPAL_F32)
    launch_rows_t<float, float>(om, st, R, nb, sh, samp_idx, samp_om, samp_w, dkeys, tab, tmask,
                                tshift, tpos, slots, hmask, hshift, dense_len, zhat, foff, flen,
                                gpart, part_len, part_cnt, part_act, M, mlen, ldz, s);
  else
    launch_rows_t<bf16s, float>(om, st, R, nb, sh, samp_idx, samp_om, samp_w, dkeys, tab, tmask,
                                tshift, tpos, slots, hmask, hshift, dense_len, zhat, foff, flen,
                                gpart, part_len, part_cnt, part_act, M, mlen, ldz, s);
}

int rows_blocks(i64 cap) { return (int)((cap + ROWS_BLK - 1) / ROWS_BLK); }
int rows_per_block() { return ROWS_BLK; }

void launch_gather_prep(DevState *st, const unsigned *flen, const unsigned *foff, i64 cap,
                        const u64 *part_len, const unsigned *part_cnt, const unsigned *part_act,
                        u64 *cpos, unsigned *coff, unsigned *cidx, unsigned *chunk_first,
                        const unsigned *tpos, DrawEntry *tab, hipStream_t s) {
  const int nb = std::max(1, (int)((cap + ROWS_BLK - 1) / ROWS_BLK));
  launch_b<B_gather_prep>(k_gather_prep, dim3(nb), dim3(ROWS_BLK), 0, s, st, flen, foff, part_len,
                          part_cnt, part_act, cpos, coff, cidx, chunk_first, tpos, tab);
}

// Sampled rows for callers (audit path): the deterministic rows in their
// order, then the distinct random rows in ascending order, at most cap of
// them; *count = s_bar.
//  1. k_samples_list (one workgroup): deterministic slots straight to the
//     output, the slots of combined random rows as (row, slot) pairs;
//  2. radix sort of the pairs by row;
//  3. k_samples_write: the sorted rows after the deterministic ones.
__global__ void __launch_bounds__(1024) k_samples_list(DevState *st,
                                                       const u64 *__restrict__ samp_idx,
                                                       const double *__restrict__ samp_om,
                                                       const double *__restrict__ samp_w, i64 cap,
                                                       u64 *idx, double *om, double *w,
                                                       u64 *__restrict__ rkeys,
                                                       unsigned *__restrict__ rslot) {
  const i64 n = st->n_slots, s_det = st->s_det;
  for (i64 j = threadIdx.x; j < min(s_det, cap); j += 1024) {
    if (idx) idx[j] = samp_idx[j];
    if (om) om[j] = samp_om[j];
    if (w) w[j] = samp_w[j];
  }
  i64 carry = 0;
  for (i64 b0 = s_det; b0 < n; b0 += 1024) {
    const i64 j = b0 + threadIdx.x;
    const unsigned a = (j < n && samp_om[j] > 0.0) ? 1u : 0u;
    unsigned tot;
    const unsigned ex = block_excl_scan<unsigned>(a, &tot);
    if (a) {
      rkeys[carry + ex] = samp_idx[j];
      rslot[carry + ex] = (unsigned)j;
    }
    carry += tot;
  }
  if (threadIdx.x == 0) st->n_rnd_rows = carry;
}

__global__ void __launch_bounds__(256) k_samples_write(const DevState *st,
                                                       const u64 *__restrict__ rkeys,
                                                       const unsigned *__restrict__ rslot,
                                                       const double *__restrict__ samp_om,
                                                       const double *__restrict__ samp_w, i64 cap,
                                                       u64 *idx, double *om, double *w,
                                                       i64 *count) {
  const i64 nr = st->n_rnd_rows, s_det = st->s_det;
  for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < nr; r += (i64)gridDim.x * blockDim.x) {
    const i64 o = s_det + r;
    if (o >= cap) break;
    const unsigned j = rslot[r];
    if (idx) idx[o] = rkeys[r];
    if (om) om[o] = samp_om[j];
    if (w) w[o] = samp_w[j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && count) *count = st->s_bar;
}

u64 *sort_keys_pp(u64 *keys, unsigned *vals, u64 *tmp_keys, unsigned *tmp_vals, void *scratch,
                  i64 cap, const i64 *count_dev, i64 count_host, int bits, hipStream_t s);

void launch_samples_out(DevState *st, const u64 *samp_idx, const double *samp_om,
                        const double *samp_w, i64 slots_cap, int key_bits, u64 *rkeys,
                        u64 *rkeys_tmp, unsigned *rslot, unsigned *rslot_tmp, void *sort_scratch,
                        i64 cap, u64 *idx, double *om, double *w, i64 *count, hipStream_t s) {
  launch_1(k_samples_list, dim3(1), dim3(1024), 0, s, st, samp_idx, samp_om, samp_w,
           cap, idx, om, w, rkeys, rslot);
  const u64 *sk = sort_keys_pp(rkeys, rslot, rkeys_tmp, rslot_tmp, sort_scratch, slots_cap,
                               &st->n_rnd_rows, 0, key_bits, s);
  const unsigned *sv = sk == rkeys ? rslot : rslot_tmp;
  const int nb = (int)std::min<i64>(std::max<i64>((slots_cap + 255) / 256, 1), 1024);
  launch_1(k_samples_write, dim3(nb), dim3(256), 0, s, st, sk, sv, samp_om, samp_w, cap,
           idx, om, w, count);
}
}  // namespace cpal
