// Dense tensors (every entry stored, mode 0 fastest).  Per mode k the
// library keeps a copy in the gather precision in which every mode-k fiber
// is contiguous, and the sampled contraction of eq. (1.2) becomes a dense
// product: the rows of the sampled system are whole mode-k fibers, so
//   M = X~^T diag(omega) Z   (n_k x R, inner dimension = the sampled rows)
// runs on the matrix cores with BF16 inputs and FP32 accumulation
// (v_mfma_f32_16x16x32_bf16, 32 sampled fibers per instruction), in FP32
// (v_mfma_f32_16x16x4_f32) or in FP64 (v_mfma_f64_16x16x4_f64).
#include "cpal_common.h"

namespace cpal {

// ------------------------------------------------------------ per-mode copies
// Input [B][n_k][A] (A = product of the sizes of the modes before k, index
// fastest) -> output [B][A][ldx], ldx >= n_k: the fiber with other-mode
// linear index a + A b starts at (a + A b) * ldx.  32 x 32 tiles through
// shared memory, one 256-thread workgroup per tile.
template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_dense_copy_t(const TI *__restrict__ in,
                                                      TO *__restrict__ out, i64 A, i64 nk,
                                                      i64 ldx, i64 ta, i64 tk) {
  __shared__ double tile[32][33];
  const i64 t = blockIdx.x;
  const i64 tpb = ta * tk;
  const i64 b = t / tpb, r = t - b * tpb;
  const i64 k0 = (r / ta) * 32, a0 = (r % ta) * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int y = ty; y < 32; y += 8) {
    const i64 ik = k0 + y, a = a0 + tx;
    tile[y][tx] = (ik < nk && a < A) ? (double)in[(b * nk + ik) * A + a] : 0.0;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    const i64 a = a0 + y, ik = k0 + tx;
    if (a < A && ik < nk) out[(b * A + a) * ldx + ik] = cvt_from<TO>(tile[tx][y]);
  }
}

// Mode 0 (A = 1): [B][n_k] -> [B][ldx] with the precision conversion.
template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_dense_copy_0(const TI *__restrict__ in,
                                                      TO *__restrict__ out, i64 nk, i64 ldx,
                                                      i64 total) {
  for (i64 e = (i64)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (i64)gridDim.x * blockDim.x) {
    const i64 b = e / nk, ik = e - b * nk;
    out[b * ldx + ik] = cvt_from<TO>((double)in[e]);
  }
}

template <typename TI, typename TO>
static void dense_copy(const TI *in, TO *out, i64 A, i64 nk, i64 B, i64 ldx, hipStream_t s) {
  if (A == 1) {
    const i64 total = B * nk;
    const i64 g = std::min<i64>((total + 255) / 256, 1 << 20);
    launch_1((k_dense_copy_0<TI, TO>), dim3((unsigned)g), dim3(256), 0, s, in, out, nk,
             ldx, total);
  } else {
    const i64 ta = (A + 31) / 32, tk = (nk + 31) / 32;
    launch_1((k_dense_copy_t<TI, TO>), dim3((unsigned)(B * ta * tk)), dim3(256), 0, s,
             in, out, A, nk, ldx, ta, tk);
  }
}

// Copy of mode k of a dense tensor (values of dtype vdt, dims[0..D)) in the
// gather precision xdt; out must be zeroed (padding past n_k stays zero).
void launch_dense_copy(const void *vals, int vdt, const i64 *dims, int D, int k, int xdt,
                       void *out, i64 ldx, hipStream_t s) {
  i64 A = 1, B = 1;
  for (int m = 0; m < k; ++m) A *= dims[m];
  for (int m = k + 1; m < D; ++m) B *= dims[m];
  const i64 nk = dims[k];
  if (vdt == CPAL_F64) {
    const double *in = (const double *)vals;
    if (xdt == CPAL_F64) dense_copy(in, (double *)out, A, nk, B, ldx, s);
    else if (xdt == CPAL_F32) dense_copy(in, (float *)out, A, nk, B, ldx, s);
    else dense_copy(in, (bf16s *)out, A, nk, B, ldx, s);
  } else {
    const float *in = (const float *)vals;
    if (xdt == CPAL_F64) dense_copy(in, (double *)out, A, nk, B, ldx, s);
    else if (xdt == CPAL_F32) dense_copy(in, (float *)out, A, nk, B, ldx, s);
    else dense_copy(in, (bf16s *)out, A, nk, B, ldx, s);
  }
}

// ------------------------------------------------------ sampled contraction
// Workgroup (c, y) takes the sampled fibers [c kc, (c+1) kc) of the compacted
// list (slot cidx, fiber samp_idx[slot]) and the rows [y RB, (y+1) RB) of
// M.  Groups of KG fibers (128 in BF16, 16 otherwise) are staged in shared
// memory (16-byte loads; the next group's loads are in flight during the
// current group's products) with the group's weighted KRP rows (zhat, omega
// z in the gather precision).  Wave w owns TW row tiles of 16; every tile
// meets NR column tiles of 16 (R <= 16 NR).  Operand layouts (lane l,
// g = l / 16); A and B take the fibers of one instruction in the same
// lane/element order, so the product sums each fiber once:
//   A(i, k) = fiber k at row i: lane l has row l % 16 and fibers
//             8g..8g+7 of each step of 32 (BF16) or fiber g of each step
//             of 4 (FP32, FP64);
//   B(k, j) = zhat(fiber k, column j), the same k assignment, j = l % 16;
//   D(i, j): lane 16 (i / 4) + j, element i % 4 (BF16, FP32);
//            lane 16 (i % 4) + j, element i / 4 (FP64).
// The workgroup's partial M goes to part[c] (n_k x ldz); k_dense_reduce sums
// the partials in workgroup order.
typedef short s8v __attribute__((ext_vector_type(8)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

struct DenseBF16 {
  typedef bf16s TX;
  typedef float TA;
  typedef f4v AV;
};
struct DenseF32 {
  typedef float TX;
  typedef float TA;
  typedef f4v AV;
};
struct DenseF64 {
  typedef double TX;
  typedef double TA;
  typedef d4v AV;
};

#define DN_THREADS 256
#define DN_KCMAX 1024

template <typename P, int NR, int TW>
__global__ void __launch_bounds__(DN_THREADS) k_dense_mttkrp(
    const DevState *st, i64 nk, int ldz, i64 ldx, const unsigned *__restrict__ cidx,
    const u64 *__restrict__ samp_idx, const typename P::TX *__restrict__ X,
    const typename P::TX *__restrict__ zhat, typename P::TA *__restrict__ part, int kc) {
  typedef typename P::TX TX;
  typedef typename P::AV AV;
  constexpr int KG = sizeof(TX) == 2 ? 128 : 16;        // fibers per group
  constexpr int RB = 4 * TW * 16;                     // rows per workgroup
  constexpr int NC = 16 * NR;                         // columns covered
  constexpr int E = 16 / (int)sizeof(TX);             // elements per 16-byte load
  constexpr int NV = KG * RB / E / DN_THREADS;        // loads per thread and group
  static_assert(NV * E * DN_THREADS == KG * RB, "staging must tile the group");
  __shared__ __attribute__((aligned(16))) TX sX[KG][RB];
  __shared__ TX sZ[KG][NC];
  __shared__ u64 slin[DN_KCMAX];
  __shared__ unsigned sslot[DN_KCMAX];
  const i64 nf = st->n_fib;
  const i64 f0 = (i64)blockIdx.x * kc;
  if (f0 >= nf) return;   // uniform per workgroup
  const int nfc = (int)min((i64)kc, nf - f0);
  const i64 r0 = (i64)blockIdx.y * RB;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, g = lane >> 4;
  for (int q = tid; q < nfc; q += DN_THREADS) {
    const unsigned slot = cidx[f0 + q];
    sslot[q] = slot;
    slin[q] = samp_idx[slot];
  }
  __syncthreads();
  AV acc[TW][NR];
#pragma unroll
  for (int t = 0; t < TW; ++t)
#pragma unroll
    for (int n = 0; n < NR; ++n) acc[t][n] = AV{0, 0, 0, 0};
  uint4 pre[NV];
  auto load_group = [&](int q0) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int v = u * DN_THREADS + tid;
      const int q = v / (RB / E), e0 = (v % (RB / E)) * E;
      const i64 row = r0 + e0;
      uint4 val = {0u, 0u, 0u, 0u};
      if (q0 + q < nfc && row < nk)   // rows past n_k up to ldx are zero padding
        val = *(const uint4 *)(X + slin[q0 + q] * (u64)ldx + row);
      pre[u] = val;
    }
  };
  load_group(0);
  for (int q0 = 0; q0 < nfc; q0 += KG) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int v = u * DN_THREADS + tid;
      const int q = v / (RB / E), e0 = (v % (RB / E)) * E;
      *(uint4 *)(&sX[q][e0]) = pre[u];
    }
    for (int e = tid; e < KG * NC; e += DN_THREADS) {
      const int q = e / NC, c = e - q * NC;
      sZ[q][c] = (q0 + q < nfc && c < ldz) ? zhat[(i64)sslot[q0 + q] * ldz + c] : TX(0);
    }
    __syncthreads();
    if (q0 + KG < nfc) load_group(q0 + KG);
#pragma unroll
    for (int t = 0; t < TW; ++t) {
      const int row = (wid * TW + t) * 16 + (lane & 15);
#pragma unroll
      for (int n = 0; n < NR; ++n) {
        const int col = n * 16 + (lane & 15);
        if constexpr (sizeof(TX) == 2) {
#pragma unroll
          for (int kk = 0; kk < KG / 32; ++kk) {   // 32 fibers per instruction
            s8v a, b;
#pragma unroll
            for (int p = 0; p < 8; ++p) {
              a[p] = (short)sX[32 * kk + 8 * g + p][row];
              b[p] = (short)sZ[32 * kk + 8 * g + p][col];
            }
            acc[t][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a),
                                                                __builtin_bit_cast(bf8v, b),
                                                                acc[t][n], 0, 0, 0);
          }
        } else if constexpr (sizeof(TX) == 4) {
#pragma unroll
          for (int s = 0; s < 4; ++s)
            acc[t][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(sX[4 * s + g][row],
                                                             sZ[4 * s + g][col], acc[t][n], 0,
                                                             0, 0);
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s)
            acc[t][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(sX[4 * s + g][row],
                                                             sZ[4 * s + g][col], acc[t][n], 0,
                                                             0, 0);
        }
      }
    }
    __syncthreads();
  }
  typename P::TA *pc = part + (i64)blockIdx.x * nk * ldz;
#pragma unroll
  for (int t = 0; t < TW; ++t)
#pragma unroll
    for (int n = 0; n < NR; ++n)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = (sizeof(TX) == 8) ? (g + 4 * v) : (4 * g + v);
        const i64 row = r0 + (wid * TW + t) * 16 + i;
        const int col = n * 16 + (lane & 15);
        if (row < nk && col < ldz) pc[row * ldz + col] = acc[t][n][v];
      }
}

// M(row, col) = the sum of the workgroup partials (col < R; the padding
// columns are cleared).  A workgroup takes 16 entries; its 16 thread groups
// sum 16 consecutive slices of the partials each, and the slice sums are
// added in slice order, so the result does not depend on timing.
template <typename TA>
__global__ void __launch_bounds__(256) k_dense_reduce(const DevState *st, i64 nk, int R, int ldz,
                                                     const TA *__restrict__ part, int kc,
                                                     TA *__restrict__ M) {
  __shared__ TA red[16][17];
  const i64 nch = (st->n_fib + kc - 1) / kc;
  const i64 stride = nk * ldz;
  const int el = threadIdx.x & 15, sl = threadIdx.x >> 4;
  const i64 e = (i64)blockIdx.x * 16 + el;
  const i64 per = (nch + 15) / 16;
  const i64 c0 = sl * per, c1 = min(nch, c0 + per);
  TA sum = TA(0);
  if (e < stride) {
#pragma unroll 4
    for (i64 c = c0; c < c1; ++c) sum = sum + part[c * stride + e];
  }
  red[sl][el] = sum;
  __syncthreads();
  if (sl == 0 && e < stride) {
    TA tot = TA(0);
    for (int q = 0; q < 16; ++q) tot = tot + red[q][el];
    M[e] = (int)(e % ldz) < R ? tot : TA(0);
  }
}

// Tile shape per precision: rows per workgroup = 64 TW (TW row tiles per
// wave, a power of two): short row blocks give several workgroups per CU
// (memory parallelism for the fiber stream) at no cost in partials, which
// are kept per row.
static int dense_tw(int xdt, int nr) {
  if (xdt == CPAL_BF16) return 1;   // 128 fibers x 64 rows: four 16-byte loads per thread
  int tw = (xdt == CPAL_F64 ? 2 : 4) / nr;
  while (tw & (tw - 1)) tw &= tw - 1;
  return std::max(1, tw);
}

int dense_rows_per_block(int xdt, int R) { return 64 * dense_tw(xdt, (R + 15) / 16); }

template <typename P>
static void launch_dense_p(const DevState *st, i64 nk, int R, int ldz, i64 ldx,
                           const unsigned *cidx, const u64 *samp_idx, const void *X,
                           const void *zhat, void *part, int kc, int nchunks, int xdt,
                           hipStream_t s) {
  typedef typename P::TX TX;
  typedef typename P::TA TA;
  const int nr = (R + 15) / 16;
  const int tw = dense_tw(xdt, nr);
  const int rb = 64 * tw;
  const dim3 grid((unsigned)nchunks, (unsigned)((nk + rb - 1) / rb));
  const TX *x = (const TX *)X;
  const TX *z = (const TX *)zhat;
  TA *p = (TA *)part;
  // TW follows dense_tw()
  if constexpr (sizeof(TX) == 8) {
    if (nr == 1) launch_1((k_dense_mttkrp<P, 1, 2>), grid, dim3(DN_THREADS), 0, s, st, nk, ldz, ldx, cidx, samp_idx, x, z, p, kc);
    else if (nr == 2) launch_1((k_dense_mttkrp<P, 2, 1>), grid, dim3(DN_THREADS), 0, s, st, nk, ldz, ldx, cidx, samp_idx, x, z, p, kc);
    else if (nr == 3) launch_1((k_dense_mttkrp<P, 3, 1>), grid, dim3(DN_THREADS), 0, s, st, nk, ldz, ldx, cidx, samp_idx, x, z, p, kc);
    else launch_1((k_dense_mttkrp<P, 4, 1>), grid, dim3(DN_THREADS), 0, s, st, nk, ldz, ldx, cidx, samp_idx, x, z, p, kc);
  } else if constexpr (sizeof(TX) == 4) {
    if (nr == 1) launch_1((k_dense_mttkrp<P, 1, 4>), grid, dim3(DN_THREADS), 0, s, st, nk, ldz, ldx, cidx, samp_idx, x, z, p, kc);
    else if (nr == 2) launch_1((k_dense_mttkrp<P, 2, 2>), grid, dim3(DN_THREADS), 0, s, st, nk, ldz, ldx, cidx, samp_idx, x, z, p, kc);
    else if (nr == 3) launch_1((k_dense_mttkrp<P, 3, 1>), grid, dim3(DN_THREADS), 0, s, st, nk, ldz, ldx, cidx, samp_idx, x, z, p, kc);
    else launch_1((k_dense_mttkrp<P, 4, 1>), grid, dim3(DN_THREADS), 0, s, st, nk, ldz, ldx, cidx, samp_idx, x, z, p, kc);
  } else {   // BF16: one row tile per wave (dense_tw)
    if (nr == 1) launch_1((k_dense_mttkrp<P, 1, 1>), grid, dim3(DN_THREADS), 0, s, st, nk, ldz, ldx, cidx, samp_idx, x, z, p, kc);
    else if (nr == 2) launch_1((k_dense_mttkrp<P, 2, 1>), grid, dim3(DN_THREADS), 0, s, st, nk, ldz, ldx, cidx, samp_idx, x, z, p, kc);
    else if (nr == 3) launch_1((k_dense_mttkrp<P, 3, 1>), grid, dim3(DN_THREADS), 0, s, st, nk, ldz, ldx, cidx, samp_idx, x, z, p, kc);
    else launch_1((k_dense_mttkrp<P, 4, 1>), grid, dim3(DN_THREADS), 0, s, st, nk, ldz, ldx, cidx, samp_idx, x, z, p, kc);
  }
}

// Sampled contraction of a dense mode-k copy into M (n_k x ldz, FP64 when
// xdt is CPAL_F64, else FP32).  kc: fibers per workgroup (multiple of 16,
// <= 1024); nchunks: workgroups along the fiber list (>= ceil(s_bar / kc)).
void launch_dense_mttkrp(int xdt, const DevState *st, i64 nk, int R, int ldz, i64 ldx,
                         const unsigned *cidx, const u64 *samp_idx, const void *X,
                         const void *zhat, void *part, int kc, int nchunks, void *M,
                         hipStream_t s) {
  if (xdt == CPAL_BF16)
    launch_dense_p<DenseBF16>(st, nk, R, ldz, ldx, cidx, samp_idx, X, zhat, part, kc, nchunks,
                              xdt, s);
  else if (xdt == CPAL_F32)
    launch_dense_p<DenseF32>(st, nk, R, ldz, ldx, cidx, samp_idx, X, zhat, part, kc, nchunks,
                             xdt, s);
  else
    launch_dense_p<DenseF64>(st, nk, R, ldz, ldx, cidx, samp_idx, X, zhat, part, kc, nchunks,
                             xdt, s);
  const i64 total = nk * ldz;
  const unsigned g = (unsigned)((total + 15) / 16);
  if (xdt == CPAL_F64)
    launch_1(k_dense_reduce<double>, dim3(g), dim3(256), 0, s, st, nk, R, ldz,
             (const double *)part, kc, (double *)M);
  else
    launch_1(k_dense_reduce<float>, dim3(g), dim3(256), 0, s, st, nk, R, ldz,
             (const float *)part, kc, (float *)M);
}

}  // namespace cpal
