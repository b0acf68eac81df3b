// Per-mode fiber index built once at init (Sec. 6.3): nonzeros sorted by
// (complement key, i_k) and an open-addressing hash table key -> fiber.
#include "cpal_common.h"

namespace cpal {

static int grid_for(i64 n, int blk, int maxg = 8192) {
  i64 g = (n + blk - 1) / blk;
  if (g < 1) g = 1;
  if (g > maxg) g = maxg;
  return (int)g;
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
    u64 h = key_hash(key, hshift);
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

void launch_mode_keys(const int *coords, i64 nnz, int D, const OtherModes &om, i64 nk, u64 *comp,
                      unsigned *ids, int *err, hipStream_t s) {
  launch_1(k_mode_keys, dim3(grid_for(nnz, 256)), dim3(256), 0, s, coords, nnz, D, om,
           nk, comp, ids, err);
}

void launch_fiber_mark(const u64 *comp, i64 nnz, i64 nk, unsigned *flag, int *err,
                       hipStream_t s) {
  launch_1(k_fiber_mark, dim3(grid_for(nnz, 256)), dim3(256), 0, s, comp, nnz, nk, flag,
           err);
}

void launch_fiber_starts(const unsigned *flag, const u64 *fid, i64 nnz, unsigned *fstart,
                         hipStream_t s) {
  launch_1(k_fiber_starts, dim3(grid_for(nnz, 256)), dim3(256), 0, s, flag, fid, nnz,
           fstart);
}

void launch_hash_build(const u64 *comp, i64 nnz, i64 nk, const unsigned *fstart, u64 nfib,
                       FiberSlot *slots, u64 nslots, int hshift, hipStream_t s) {
  launch_1(k_slots_clear, dim3(grid_for((i64)nslots, 256)), dim3(256), 0, s, slots,
           nslots);
  launch_1(k_hash_insert, dim3(grid_for((i64)nfib, 256)), dim3(256), 0, s, comp, nnz,
           nk, fstart, nfib, slots, nslots - 1, hshift);
}

void launch_mode_pairs(const u64 *comp, const unsigned *ids, i64 nnz, i64 nk, const void *vals,
                       int vdt, uint2 *pairs, int *ik32, double *v64, hipStream_t s) {
  launch_1(k_mode_pairs, dim3(grid_for(nnz, 256)), dim3(256), 0, s, comp, ids, nnz, nk,
           vals, vdt, pairs, ik32, v64);
}

}  // namespace cpal
