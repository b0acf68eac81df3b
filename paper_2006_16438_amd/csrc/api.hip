// Host runtime behind the C ABI of include/cp_arls_lev.h: validation, device
// memory, the per-mode fiber indexes built at init and the kernel sequence of
// one mode update.  Every stage runs on the context's stream; no count is
// read back to the host during an update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "cpal_common.h"

namespace cpal {
void launch_decomp_dev(const double *part, const i64 *nrows_dev, int rows_per_blk, int R,
                       Decomp *out, int *flag_or, double *gram_tmp, hipStream_t s);
void launch_gather_prep(DevState *st, const unsigned *flen, const unsigned *foff, i64 cap,
                        const u64 *part_len, const unsigned *part_cnt, const unsigned *part_act,
                        u64 *cpos, unsigned *coff, unsigned *cidx, unsigned *chunk_first,
                        const unsigned *tpos, DrawEntry *tab, hipStream_t s);
int gather_row_width(int R);
i64 gather_chunks_cap(i64 nnz);
void launch_gather_seg(bool f64, const DevState *st, int R, const u64 *cpos, const unsigned *coff,
                       const unsigned *cidx, const unsigned *chunk_first, const uint2 *pairs,
                       const int *ik, const double *v64, i64 nk, const void *zhat, int ldz, void *M,
                       int grid, int sort_min, hipStream_t s);
void launch_zero_words(void *p, i64 nwords, hipStream_t s);
int gather_own_blocks(bool f64, int ldz, i64 nk);
void launch_fiber_list(const FiberSlot *slots, u64 nslots, u64 *off, unsigned *len,
                       unsigned long long *count, hipStream_t s);
void launch_rrf_rows(int zdt, DevState *st, i64 s_init, int k, u64 seed, u64 stream_id, u64 nfib,
                     const u64 *fib_off, const unsigned *fib_len, unsigned dense_len,
                     const double *omega, int R, int ldz, void *zhat, unsigned *foff,
                     unsigned *flen, u64 *samp_idx, u64 *part_len, unsigned *part_cnt,
                     unsigned *part_act, int rows_per_blk, hipStream_t s);
void launch_rrf_store(bool f64, const void *M, int ncopies, i64 nk, int R, int ldz, double *A,
                      float *A32, hipStream_t s);
void launch_gather_own(bool f64, const DevState *st, int R, const u64 *cpos,
                       const unsigned *coff, const unsigned *cidx, const uint2 *pairs,
                       const int *ik, const double *v64, i64 nk, const void *zhat, int ldz,
                       void *M, unsigned *bnd, hipStream_t s);
int gather_tile_blocks(int R, i64 nk);
u64 gather_tile_ldb(i64 max_fib);
void launch_gather_tile(bool f64, const DevState *st, int R, const u64 *cpos,
                        const unsigned *coff, const unsigned *cidx, const uint2 *pairs,
                        const int *ik, const double *v64, i64 nk, i64 max_fib, const void *zhat,
                        int ldz, void *M, unsigned *bnd, unsigned lmin, hipStream_t s);
void launch_gather_hyb(bool f64, const DevState *st, int R, const u64 *cpos,
                       const unsigned *coff, const unsigned *cidx, const unsigned *chunk_first,
                       const uint2 *pairs, const int *ik, const double *v64, i64 nk,
                       i64 max_total, i64 max_fib, const void *zhat, int ldz, void *M,
                       unsigned *bnd, unsigned *cnt, u64 *off, void *scan_scratch, uint4 *bent,
                       int lfac, int compact, hipStream_t s);
size_t gather_bkt_count_words();
int gather_bktl_shift(int R, i64 nk);
void launch_gather_bktl(bool f64, const DevState *st, int R, const u64 *cpos,
                        const unsigned *coff, const unsigned *cidx, const unsigned *chunk_first,
                        const uint2 *pairs, const int *ik, const double *v64, i64 nk,
                        i64 max_total, const void *zhat, int ldz, void *M, unsigned *cnt,
                        u64 *off, void *scan_scratch, uint4 *bent, unsigned lmin, int compact,
                        hipStream_t s);
void launch_gather_bkt(bool f64, const DevState *st, int R, const u64 *cpos,
                       const unsigned *coff, const unsigned *cidx, const unsigned *chunk_first,
                       const uint2 *pairs, const int *ik, const double *v64, i64 nk,
                       i64 max_total, const void *zhat, int ldz, void *M, int grid, unsigned *cnt,
                       u64 *off, void *scan_scratch, uint4 *bent, hipStream_t s);
int lev_row_blocks(i64 n);
void scan_u32_dev(const unsigned *in, u64 *out, i64 cap, const i64 *n_dev, u64 *total,
                  void *scratch, hipStream_t s);
void launch_det_cand(const OtherModes &om, double tau, u64 cap, DevState *st, int *cand,
                     hipStream_t s);
void launch_det_enum(const OtherModes &om, double tau, DevState *st, const int *cand,
                     unsigned *blk_cnt, u64 *det_keys, u64 det_cap, hipStream_t s);
void launch_det_finish(const OtherModes &om, DevState *st, const u64 *det_keys, double *det_p,
                       double *kept_p, double *psum, u64 det_cap, i64 s, u64 *samp_idx,
                       hipStream_t st_);
void launch_set_step(DevState *st, u64 t, hipStream_t s);
void launch_draw(const OtherModes &om, DevState *st, u64 seed, u64 stream_id, u64 *buf,
                 unsigned short *bpos, unsigned *chunk_cnt, int grid_first, int grid_more,
                 hipStream_t s);
void launch_compact(DevState *st, const u64 *buf, const unsigned *chunk_cnt,
                    const unsigned short *bpos, u64 *keys, DrawEntry *tab, u64 tmask, int tshift,
                    bool det_rep,
                    hipStream_t s);
void launch_draw_table_clear(DrawEntry *tab, u64 n, hipStream_t s);
void launch_samples_out(DevState *st, const u64 *samp_idx, const double *samp_om,
                        const double *samp_w, i64 slots_cap, int key_bits, u64 *rkeys,
                        u64 *rkeys_tmp, unsigned *rslot, unsigned *rslot_tmp, void *sort_scratch,
                        i64 cap, u64 *idx, double *om, double *w, i64 *count, hipStream_t s);
void launch_dense_copy(const void *vals, int vdt, const i64 *dims, int D, int k, int xdt,
                       void *out, i64 ldx, hipStream_t s);
void launch_dense_mttkrp(int xdt, const DevState *st, i64 nk, int R, int ldz, i64 ldx,
                         const unsigned *cidx, const u64 *samp_idx, const void *X,
                         const void *zhat, void *part, int kc, int nchunks, void *M,
                         hipStream_t s);
void launch_rows(int zdt, const OtherModes &om, DevState *st, int R, i64 cap, u64 *samp_idx,
                 double *samp_om, double *samp_w, const u64 *dkeys, const DrawEntry *tab,
                 u64 tmask, int tshift, unsigned *tpos,
                 const FiberSlot *slots, u64 hmask, int hshift, unsigned dense_len, void *zhat,
                 unsigned *foff,
                 unsigned *flen, double *gpart, u64 *part_len, unsigned *part_cnt,
                 unsigned *part_act, void *M, i64 mlen, int ldz, hipStream_t s);
int rows_blocks(i64 cap);
int rows_per_block();
void launch_gather(bool f64, const DevState *st, int R, const u64 *cpos, const unsigned *coff,
                   const unsigned *cidx, const uint2 *pairs, const int *ik, const double *v64,
                   const void *zhat, void *M, int ldz, int grid, hipStream_t s);
void launch_solve_rows(bool f64, const DevState *st, i64 n, int R, const void *M, int ldm,
                       int ncopies,
                       const Decomp *dc, double *A, float *A32, hipStream_t s);
void launch_to_f32(const double *a, float *b, i64 n, hipStream_t s);
void launch_mode_keys(const int *coords, i64 nnz, int D, const OtherModes &om, i64 nk, u64 *comp,
                      unsigned *ids, int *err, hipStream_t s);
void launch_fiber_mark(const u64 *comp, i64 nnz, i64 nk, unsigned *flag, int *err,
                       hipStream_t s);
void launch_fiber_starts(const unsigned *flag, const u64 *fid, i64 nnz, unsigned *fstart,
                         hipStream_t s);
void launch_hash_build(const u64 *comp, i64 nnz, i64 nk, const unsigned *fstart, u64 nfib,
                       FiberSlot *slots, u64 nslots, int hshift, hipStream_t s);
void launch_mode_pairs(const u64 *comp, const unsigned *ids, i64 nnz, i64 nk, const void *vals,
                       int vdt, uint2 *pairs, int *ik32, double *v64, hipStream_t s);
struct FullModes {
  int D;
  i64 n[CPAL_MAXORDER];
  u64 stride[CPAL_MAXORDER];
  const double *A[CPAL_MAXORDER];
};
void fit_build_set(const int *coords, i64 nnz, const FullModes &fm, u64 *set, u64 nslots,
                   int shift, hipStream_t s);
void fit_draw(const int *coords, const void *vals, int vdt, i64 nnz, const FullModes &fm, i64 n_nz,
              i64 n_z, u64 seed, u64 stream_id, const u64 *set, u64 nslots, int shift, u64 *ctl,
              u64 *buf, unsigned *chunk_cnt, int *sc, i64 ld, double *sx, hipStream_t s);
void fit_norm(const void *vals, int vdt, i64 nnz, double *part, DevState *st, hipStream_t s);
void fit_eval(const FullModes &fm, int R, i64 n_nz, i64 n_fit, double phi_nz, double phi_z,
              const int *sc, i64 ld, const double *sx, double *part, const DevState *st,
              double *fit_out, hipStream_t s);
size_t fit_exact_scratch_doubles(int R, i64 maxn);
void launch_fit_exact(int D, const i64 *dims, double *const *A, int R, int k, int kind,
                      const FiberSlot *slots, u64 nslots, const uint2 *pairs, const int *ik,
                      const double *v64, const void *dX, i64 ldx, const DevState *st,
                      double *scratch, double *fit_out, hipStream_t s);

// The calling thread's launch sink (cpal_launch.h).
LaunchSink *&launch_sink() {
  static thread_local LaunchSink *sink = nullptr;
  return sink;
}
}  // namespace cpal

using namespace cpal;

namespace {

int bits_for(u64 n) {  // bits needed to hold values in [0, n)
  int b = 0;
  while (b < 64 && (n - 1) >> b) ++b;
  return std::max(b, 1);
}

struct Mode {
  i64 n = 0;
  u64 Nk = 1;
  int key_bits = 1;
  double *A = nullptr;
  float *A32 = nullptr;
  double *lev = nullptr;
  u64 *w = nullptr;
  u64 *C = nullptr;
  double *q = nullptr;
  FiberSlot *slots = nullptr;
  u64 nslots = 0;
  int hshift = 0;
  u64 nfib = 0;
  uint2 *pairs = nullptr;
  int *ik = nullptr;
  double *v64 = nullptr;
  void *dX = nullptr;   // dense tensor: copy with every mode-m fiber contiguous
  i64 dld = 0;          //   fiber stride (n_m rounded up to 8)
  int g_grid = 0;       // gather launch: workgroups (0: the default)
  int g_sort_min = 0;   //   segmented gather: chunks of <= this many fibers skip the sort
};

}  // namespace

struct cpal_ctx {
  int D = 0;
  i64 dims[CPAL_MAXORDER] = {0};
  int R = 0;
  i64 s = 0;
  double tau = 1.0;
  int sampling = CPAL_SAMPLE_LEVERAGE;   // probability of a factor row (App. B)
  u64 seed = 0, stream_id = 0;
  bool f64 = true;
  int zdt = CPAL_F64;    // gather precision (CPAL_F64, CPAL_F32, CPAL_BF16 for dense)
  bool dense = false;    // every entry stored (mode 0 fastest)
  void *dpart = nullptr; // dense: partial M per workgroup of sampled fibers
  int dkc = 64;          // dense: sampled fibers per workgroup
  int dnch = 1;          // dense: workgroups along the sampled fibers
  i64 nnz = 0;
  u64 enum_cap = 1ull << 26;
  hipStream_t stream = nullptr;
  u64 t = 0;
  bool failed = false;
  bool samples_valid = false;   // samp_* hold the output of a mode update
  std::string err;
  cpal_allocator al{};          // alloc == nullptr: hipMalloc / hipFree
  std::vector<void *> allocs;
  Mode mode[CPAL_MAXORDER];
  // scratch
  DevState *st = nullptr;
  Decomp *dc = nullptr;
  double *lev_part = nullptr;
  u64 *lev_bsum = nullptr;
  int *cand = nullptr;
  i64 cand_off[CPAL_MAXORDER] = {0};
  u64 det_cap = 0;
  u64 *det_keys = nullptr, *det_tmp = nullptr;
  unsigned *det_blk = nullptr;
  double *det_p = nullptr, *kept_p = nullptr, *psum = nullptr;
  u64 *dbuf = nullptr;
  unsigned short *dpos = nullptr;
  unsigned *chunk_cnt = nullptr;
  i64 max_chunks = 0;
  u64 *keys = nullptr, *keys_tmp = nullptr;   // accepted draws in draw order (+ sort buffer)
  DrawEntry *dtab = nullptr;                  // draw table: row -> first draw, count
  u64 dtab_n = 0;
  int dtab_shift = 0;
  unsigned *tpos = nullptr;                   // per draw: its table entry if it is a row's first
  unsigned *ord = nullptr, *ord_tmp = nullptr;  // slots of the listed random rows (sort payload)
  int last_key_bits = 0;                      // key width of the last updated mode
  u64 *samp_idx = nullptr;
  double *samp_om = nullptr, *samp_w = nullptr;
  void *zhat = nullptr;
  unsigned *foff = nullptr, *flen = nullptr;
  u64 *fpos = nullptr;
  double *gpart = nullptr;
  void *M = nullptr;
  void *sort_scratch = nullptr;
  void *scan_scratch = nullptr;
  int draw_grid = 0;        // first draw pass: blocks for 1.5 s draws (the unneeded exit)
  int draw_more_grid = 256; // top-up draw pass
  int gather_grid = 2048;
  int ldz = 0;                  // row stride of the weighted KRP rows (16-byte multiple)
  int gs_grid = 512;            // workgroups of the segmented gather
  unsigned *chunk_first = nullptr;  // first nonempty fiber of each gather chunk
  // bucketed gather (allocated when a mode first uses it): counts and offsets
  // per (bucket, workgroup), scan scratch, nonzeros moved into buckets
  unsigned *bk_cnt = nullptr;
  u64 *bk_off = nullptr;
  void *bk_scan = nullptr;
  uint4 *bk_ent = nullptr;
  // owner gather (allocated at init for FP64 contexts, else when a mode
  // first uses it): per nonempty sampled fiber, its segment bounds per row block
  unsigned *own_bnd = nullptr;
  // tile gather (allocated when a mode first uses it): block-major segment
  // bounds of the nonempty sampled fibers
  unsigned *tile_bnd = nullptr;
  u64 *cpos = nullptr;              // nonempty fibers: stream position,
  unsigned *coff = nullptr;         //   offset in the mode-sorted nonzeros,
  unsigned *cidx = nullptr;         //   sampled row
  u64 *gp_len = nullptr;
  unsigned *gp_cnt = nullptr, *gp_act = nullptr;
  double *gram_tmp = nullptr;
  // fit sample (Sec. 6.4)
  i64 fit_nz = 0, fit_n = 0, fit_ld = 0;
  double phi_nz = 0.0, phi_z = 0.0;
  int *fit_sc = nullptr;
  double *fit_x = nullptr;
  double *fit_part = nullptr;
  int fit_flags = 0;
  double *fitx_scratch = nullptr;   // exact fit: block partials, Hadamard of Grams
  double *fit_host_buf = nullptr;   // one device double the driver reads back
  // stage timing
  unsigned timing = 0;          // mask of timed stages
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_rec;

  hipEvent_t take_event() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e;
    hipEventCreate(&e);
    return e;
  }
  hipEvent_t stage_begin(int stage) {
    if (!(timing >> stage & 1u)) return nullptr;
    hipEvent_t e = take_event();
    hipEventRecord(e, stream);
    return e;
  }
  void stage_end(int stage, hipEvent_t b) {
    if (!b) return;
    hipEvent_t e = take_event();
    hipEventRecord(e, stream);
    ev_rec.push_back({stage, {b, e}});
  }

  // every device allocation goes through the caller's provider (or hipMalloc)
  void *raw_alloc(size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    void *p = nullptr;
    if (al.alloc) {
      p = al.alloc(bytes, al.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
    }
    return p;
  }
  void raw_free(void *p) {
    if (!p) return;
    if (al.alloc) al.free(p, al.user);
    else hipFree(p);
  }
  template <typename T>
  T *alloc(size_t count) {
    void *p = raw_alloc(count * sizeof(T));
    if (!p) throw cpal_status(CPAL_E_NOMEM);
    allocs.push_back(p);
    return (T *)p;
  }
  void release() {
    for (void *p : allocs) raw_free(p);
    allocs.clear();
    for (auto &r : ev_rec) { hipEventDestroy(r.second.first); hipEventDestroy(r.second.second); }
    ev_rec.clear();
    for (hipEvent_t e : ev_pool) hipEventDestroy(e);
    ev_pool.clear();
  }
};

namespace {

cpal_status fail(cpal_ctx *c, cpal_status code, const char *msg) {
  if (c) c->err = msg;
  return code;
}

cpal_status owner_defaults(cpal_ctx *c);
bool uses_owner(const cpal_ctx *c, int k, int sort_min);
bool uses_tile(const cpal_ctx *c, int k, int sort_min);

FullModes full_modes(const cpal_ctx *c) {
  FullModes fm;
  std::memset(&fm, 0, sizeof(fm));
  fm.D = c->D;
  u64 stride = 1;
  for (int m = 0; m < c->D; ++m) {
    fm.n[m] = c->dims[m];
    fm.stride[m] = stride;
    stride *= (u64)c->dims[m];
    fm.A[m] = c->mode[m].A;
  }
  return fm;
}

// Copies of M a mode's gather adds into: one per XCD for the segmented
// gather, a single one for the atomic gather of very tall modes.
i64 m_copies(i64 n) { return n <= (1 << 20) ? CPAL_MCOPIES : 1; }

OtherModes others_of(const cpal_ctx *c, int k) {
  OtherModes om;
  std::memset(&om, 0, sizeof(om));
  om.k = k;
  u64 stride = 1;
  for (int m = 0; m < c->D; ++m) {
    if (m == k) continue;
    const int u = om.d++;
    om.mode[u] = m;
    om.n[u] = c->dims[m];
    om.stride[u] = stride;
    stride *= (u64)c->dims[m];
    om.q[u] = c->mode[m].q;
    om.C[u] = c->mode[m].C;
    om.A[u] = c->mode[m].A;
    om.A32[u] = c->mode[m].A32;
    om.cand_off[u] = c->cand_off[m];
    om.rcp[u] = 1.0 / (double)c->dims[m];
  }
  return om;
}

// Leverage of mode m from the current factor (Def. 3.4), cached.
// Leverage scores, weights and CDF of factor m (Def. 3.4); stats (nullable)
// receives the statistics of the update of mode m that produced the factor.
void refresh_leverage(cpal_ctx *c, int m, cpal_mode_stats *stats = nullptr) {
  Mode &md = c->mode[m];
  if (c->sampling != CPAL_SAMPLE_LEVERAGE) {
    launch_scores(md.A, md.n, c->R, c->sampling, c->lev_part, &c->st->score_norm[m],
                  &c->st->lev_pinv[m], md.lev, md.w, c->lev_bsum, c->stream);
    launch_lev_cdf(md.w, md.n, c->R, c->lev_bsum, md.C, md.q, nullptr, c->st, m, c->D, stats,
                   c->stream);
    return;
  }
  const int *skip = nullptr;
  if (md.n < c->R) {
    // fewer rows than columns: all scores are 1 when A has full row rank
    launch_lev_rowspace(md.A, (int)md.n, c->R, md.lev, md.w, c->lev_bsum, &c->st->lev_skip[m],
                        &c->st->lev_pinv[m], c->stream);
    skip = &c->st->lev_skip[m];
  }
  launch_lev_gram_partial(md.A, md.n, c->R, c->lev_part, skip, c->stream);
  const int nblk = (int)((md.n + CPAL_GRAM_ROWS - 1) / CPAL_GRAM_ROWS);
  launch_decomp_blocks(c->lev_part, nblk, c->R, c->gram_tmp, c->dc, &c->st->lev_pinv[m], skip,
                       c->stream);
  launch_lev_rows(md.A, md.n, c->R, c->dc, md.lev, md.w, c->lev_bsum, skip, c->stream);
  launch_lev_cdf(md.w, md.n, c->R, c->lev_bsum, md.C, md.q, nullptr, c->st, m, c->D, stats,
                 c->stream);
}

cpal_status check_hip(cpal_ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return CPAL_OK;
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
  c->err = buf;
  c->failed = true;
  return CPAL_E_DEVICE;
}

void build_index(cpal_ctx *c, int k, const cpal_tensor *X, u64 *comp, unsigned *ids, u64 *comp_t,
                 unsigned *ids_t, unsigned *flag, u64 *fid, unsigned *fstart, void *sscratch,
                 void *cscratch, int *err_dev, u64 *nfib_dev) {
  const i64 nnz = c->nnz;
  Mode &md = c->mode[k];
  OtherModes om = others_of(c, k);
  launch_mode_keys(X->coords, nnz, c->D, om, md.n, comp, ids, err_dev, c->stream);
  u64 full = 1;
  for (int m = 0; m < c->D; ++m) full *= (u64)c->dims[m];
  sort_keys(comp, ids, comp_t, ids_t, sscratch, nnz, nullptr, nnz, bits_for(full), c->stream);
  launch_fiber_mark(comp, nnz, md.n, flag, err_dev, c->stream);
  scan_u32_to_u64(flag, fid, nnz, nfib_dev, cscratch, c->stream);
  launch_fiber_starts(flag, fid, nnz, fstart, c->stream);
  u64 nfib = 0;
  hipMemcpyAsync(&nfib, nfib_dev, sizeof(u64), hipMemcpyDeviceToHost, c->stream);
  hipStreamSynchronize(c->stream);
  md.nfib = nfib;
  u64 ns = 64;
  while (ns < 2 * nfib) ns <<= 1;
  int lg = 0;
  while ((1ull << lg) < ns) ++lg;
  md.nslots = ns;
  md.hshift = 64 - lg;
  md.slots = c->alloc<FiberSlot>(ns);
  launch_hash_build(comp, nnz, md.n, fstart, nfib, md.slots, ns, md.hshift, c->stream);
  if (c->f64) {
    md.ik = c->alloc<int>(nnz);
    md.v64 = c->alloc<double>(nnz);
  } else {
    md.pairs = c->alloc<uint2>(nnz);
  }
  launch_mode_pairs(comp, ids, nnz, md.n, X->values, X->value_dtype, md.pairs, md.ik, md.v64,
                    c->stream);
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// Context creation; `share`, when given and built from a tensor of the same
// shape, storage and gather precision, lends its per-mode index (or dense
// copies) and ||X||^2 instead of building them again (restarts of one tensor
// in a batch).  The lender must outlive the borrower.
cpal_status init_impl(const cpal_tensor *X, const cpal_options *opt, double *const *factors,
                      void *hip_stream, const cpal_allocator *alloc, const cpal_ctx *share,
                      cpal_ctx **out) {
  if (!out) return CPAL_E_ARG;
  *out = nullptr;
  if (!X || !opt || !factors) return CPAL_E_ARG;
  const bool dense = X->dense != 0;
  if (X->order < 2 || X->order > CPAL_MAXORDER || !X->dims || !X->values) return CPAL_E_ARG;
  if (!dense && (!X->coords || X->nnz < 1 || X->nnz >= (1ll << 32))) return CPAL_E_ARG;
  if (X->value_dtype != CPAL_F32 && X->value_dtype != CPAL_F64) return CPAL_E_ARG;
  if (opt->rank < 1 || opt->rank > CPAL_MAXR || opt->samples < 1) return CPAL_E_ARG;
  if (opt->samples > (1ll << 28)) return CPAL_E_ARG;
  if (!(opt->tau >= 0.0 && opt->tau <= 1.0)) return CPAL_E_ARG;
  if (opt->gather_dtype != CPAL_F64 && opt->gather_dtype != CPAL_F32 &&
      !(dense && opt->gather_dtype == CPAL_BF16))
    return CPAL_E_ARG;
  if (dense && opt->fit_samples != 0) return CPAL_E_ARG;   // the Sec. 6.4 sample is over nonzeros
  if (opt->det_enum_cap < 0 || opt->det_enum_cap > (1ll << 31)) return CPAL_E_ARG;
  if (opt->fit_samples < 0) return CPAL_E_ARG;
  if (opt->sampling < CPAL_SAMPLE_LEVERAGE || opt->sampling > CPAL_SAMPLE_LENGTH_SQUARED)
    return CPAL_E_ARG;
  if (alloc && (!alloc->alloc || !alloc->free)) return CPAL_E_ARG;
  long double fulld = 1;
  for (int m = 0; m < X->order; ++m) {
    if (X->dims[m] < 1 || X->dims[m] > (1ll << 31) - 1) return CPAL_E_ARG;
    if (!factors[m]) return CPAL_E_ARG;
    fulld *= (long double)X->dims[m];
  }
  if (fulld >= 4611686018427387904.0L) return CPAL_E_ARG;  // 2^62
  u64 full = 1;
  for (int m = 0; m < X->order; ++m) full *= (u64)X->dims[m];

  cpal_ctx *c = new cpal_ctx();
  if (alloc) c->al = *alloc;
  c->D = X->order;
  for (int m = 0; m < c->D; ++m) c->dims[m] = X->dims[m];
  c->R = opt->rank;
  c->s = opt->samples;
  c->tau = opt->tau;
  c->sampling = opt->sampling;
  c->seed = opt->seed;
  c->stream_id = opt->stream_id;
  c->f64 = opt->gather_dtype == CPAL_F64;
  c->zdt = opt->gather_dtype;
  c->dense = dense;
  c->nnz = dense ? 0 : X->nnz;
  if (share) {
    bool same = share->D == c->D && share->dense == dense && share->zdt == c->zdt &&
                share->nnz == c->nnz;
    for (int m = 0; same && m < c->D; ++m) same = share->dims[m] == c->dims[m];
    if (!same) share = nullptr;
  }
  c->enum_cap = opt->det_enum_cap ? (u64)opt->det_enum_cap : (1ull << 26);
  c->stream = (hipStream_t)hip_stream;
  try {
    const int R = c->R;
    const i64 s = c->s;
    i64 maxn = 0, sumn = 0;
    for (int m = 0; m < c->D; ++m) {
      Mode &md = c->mode[m];
      md.n = c->dims[m];
      md.A = factors[m];
      u64 Nk = 1;
      for (int o = 0; o < c->D; ++o) if (o != m) Nk *= (u64)c->dims[o];
      md.Nk = Nk;
      md.key_bits = bits_for(Nk);
      md.A32 = c->alloc<float>((size_t)md.n * R);
      md.lev = c->alloc<double>(md.n);
      md.w = c->alloc<u64>(md.n);
      md.C = c->alloc<u64>(md.n);
      md.q = c->alloc<double>(md.n);
      c->cand_off[m] = sumn;
      sumn += md.n;
      maxn = std::max(maxn, md.n);
    }
    c->st = c->alloc<DevState>(1);
    hipMemsetAsync(c->st, 0, sizeof(DevState), c->stream);
    c->dc = c->alloc<Decomp>(1);
    const int np = R * (R + 1) / 2;
    c->lev_part = c->alloc<double>((size_t)((maxn + CPAL_GRAM_ROWS - 1) / CPAL_GRAM_ROWS) * np);
    c->lev_bsum = c->alloc<u64>(lev_row_blocks(maxn) + 1);
    c->cand = c->alloc<int>(sumn);
    // |D| < 1/tau (every p > tau and the p sum to at most 1, Sec. 5.3), |D| is at
    // most the other modes' KRP row count and, when enumerated, at most
    // det_enum_cap: the deterministic set always fits
    {
      u64 cap = c->enum_cap;
      u64 maxNk = 0;
      for (int m = 0; m < c->D; ++m) maxNk = std::max(maxNk, c->mode[m].Nk);
      cap = std::min(cap, maxNk);
      if (c->tau > 0.0) {
        const double b = std::floor((1.0 + 0x1p-30) / c->tau) + 1.0;
        if (b < (double)cap) cap = (u64)b;
      }
      c->det_cap = std::max<u64>(cap, 1);
    }
    c->det_keys = c->alloc<u64>(c->det_cap);
    c->det_tmp = c->alloc<u64>(c->det_cap);
    c->det_blk = c->alloc<unsigned>(256);
    c->det_p = c->alloc<double>(c->det_cap);
    c->kept_p = c->alloc<double>(s);
    c->psum = c->alloc<double>(c->det_cap / 256 + 2);
    const i64 max_draws = 64 * s + (1ll << 20);
    c->max_chunks = (max_draws + CPAL_KRP_CHUNK - 1) / CPAL_KRP_CHUNK;
    c->dbuf = c->alloc<u64>((size_t)c->max_chunks * CPAL_KRP_CHUNK);
    c->dpos = c->alloc<unsigned short>((size_t)c->max_chunks * CPAL_KRP_CHUNK);
    c->chunk_cnt = c->alloc<unsigned>(c->max_chunks);
    c->draw_grid = (int)std::min<i64>(c->max_chunks,
                                      (i64)std::ceil(1.5 * (double)s / CPAL_KRP_CHUNK) + 2);
    c->keys = c->alloc<u64>(s);
    c->keys_tmp = c->alloc<u64>(s);
    c->dtab_n = 64;
    while (c->dtab_n < 2 * (u64)s) c->dtab_n <<= 1;
    c->dtab_shift = 64;
    for (u64 v = c->dtab_n; v > 1; v >>= 1) --c->dtab_shift;
    c->dtab = c->alloc<DrawEntry>(c->dtab_n);
    launch_draw_table_clear(c->dtab, c->dtab_n, c->stream);
    c->tpos = c->alloc<unsigned>(s);
    c->ord = c->alloc<unsigned>(s);
    c->ord_tmp = c->alloc<unsigned>(s);
    c->samp_idx = c->alloc<u64>(s);
    c->samp_om = c->alloc<double>(s);
    c->samp_w = c->alloc<double>(s);
    const size_t tsz = c->f64 ? sizeof(double) : sizeof(float);
    c->ldz = gather_row_width(R);   // rows padded to the gather's unrolled width
    c->zhat = c->alloc<char>((size_t)s * c->ldz * tsz);
    c->foff = c->alloc<unsigned>(s);
    c->flen = c->alloc<unsigned>(s);
    c->fpos = c->alloc<u64>(s + 1);
    c->gpart = c->alloc<double>((size_t)rows_blocks(s) * np);
    {
      i64 mcap = 0;
      for (int m = 0; m < c->D; ++m)
        mcap = std::max<i64>(mcap, (dense ? 1 : m_copies(c->dims[m])) * c->dims[m]);
      c->M = c->alloc<char>((size_t)mcap * c->ldz * tsz);   // rows padded to ldz
    }
    c->gram_tmp = c->alloc<double>(np);
    c->fitx_scratch = c->alloc<double>(fit_exact_scratch_doubles(R, maxn));
    c->fit_host_buf = c->alloc<double>(1);
    // gather stream length: at most nnz (sparse), s * max n_m (dense)
    c->chunk_first = c->alloc<unsigned>(gather_chunks_cap(dense ? s * maxn : c->nnz));
    if (dense) {   // sampled fibers per workgroup of the dense contraction: <= 256
      // partials (BF16, whose row blocks are 4x shorter: <= 64 partials)
      const i64 parts = c->zdt == CPAL_BF16 ? 64 : 256;
      i64 kc = ((s + parts - 1) / parts + 31) / 32 * 32;
      kc = std::min<i64>(std::max<i64>(kc, 64), 1024);
      c->dkc = (int)kc;
      c->dnch = (int)((s + kc - 1) / kc);
      c->dpart = c->alloc<char>((size_t)c->dnch * maxn * c->ldz * tsz);
    }
    c->cpos = c->alloc<u64>(s);
    c->coff = c->alloc<unsigned>(s);
    c->cidx = c->alloc<unsigned>(s);
    c->gp_len = c->alloc<u64>(rows_blocks(s) + 1);
    c->gp_cnt = c->alloc<unsigned>(rows_blocks(s) + 1);
    c->gp_act = c->alloc<unsigned>(rows_blocks(s) + 1);
    const i64 sort_cap = std::max<i64>((i64)c->det_cap, c->nnz);
    c->sort_scratch = c->alloc<char>(sort_scratch_bytes(sort_cap, true));
    c->scan_scratch = c->alloc<char>(scan_scratch_bytes(std::max<i64>(sort_cap, s)));

    // per-mode fiber indexes (Sec. 6.3), or per-mode copies of a dense tensor
    const i64 nnz = c->nnz;
    u64 *comp = nullptr, *comp_t = nullptr, *fid = nullptr, *nfib_dev = nullptr;
    unsigned *ids = nullptr, *ids_t = nullptr, *flag = nullptr, *fstart = nullptr;
    int *err_dev = nullptr;
    std::vector<void *> tmp;
    auto talloc = [&](size_t bytes) {
      void *p = c->raw_alloc(bytes);
      if (!p) {
        for (void *q : tmp) c->raw_free(q);
        throw cpal_status(CPAL_E_NOMEM);
      }
      tmp.push_back(p);
      return p;
    };
    auto tfree_all = [&]() {
      for (void *q : tmp) c->raw_free(q);
      tmp.clear();
    };
    int err_host = 0;
    hipError_t e = hipSuccess;
    if (share) {   // borrow the index (or dense copies) and ||X||^2
      for (int k = 0; k < c->D; ++k) {
        Mode &md = c->mode[k];
        const Mode &sm = share->mode[k];
        md.slots = sm.slots; md.nslots = sm.nslots; md.hshift = sm.hshift; md.nfib = sm.nfib;
        md.pairs = sm.pairs; md.ik = sm.ik; md.v64 = sm.v64; md.dX = sm.dX; md.dld = sm.dld;
      }
      hipMemcpyAsync(&c->st->normX2, &share->st->normX2, sizeof(double),
                     hipMemcpyDeviceToDevice, c->stream);
      e = hipStreamSynchronize(c->stream);
    }
    if (share) {
      // nothing to build
    } else if (dense) {
      const size_t xsz = c->zdt == CPAL_F64 ? 8 : c->zdt == CPAL_F32 ? 4 : 2;
      const i64 N = (i64)full;
      for (int k = 0; k < c->D; ++k) {
        Mode &md = c->mode[k];
        md.dld = (md.n + 7) / 8 * 8;
        const size_t bytes = (size_t)(N / md.n) * (size_t)md.dld * xsz;
        md.dX = c->alloc<char>(bytes);
        hipMemsetAsync(md.dX, 0, bytes, c->stream);
        launch_dense_copy(X->values, X->value_dtype, c->dims, c->D, k, c->zdt, md.dX, md.dld,
                          c->stream);
      }
      // ||X||^2
      double *part = (double *)talloc(sizeof(double) * (size_t)(N / 256 + 2));
      fit_norm(X->values, X->value_dtype, N, part, c->st, c->stream);
      e = hipStreamSynchronize(c->stream);
      tfree_all();
    } else {
      comp = (u64 *)talloc(sizeof(u64) * nnz);
      comp_t = (u64 *)talloc(sizeof(u64) * nnz);
      fid = (u64 *)talloc(sizeof(u64) * nnz);
      ids = (unsigned *)talloc(sizeof(unsigned) * nnz);
      ids_t = (unsigned *)talloc(sizeof(unsigned) * nnz);
      flag = (unsigned *)talloc(sizeof(unsigned) * nnz);
      fstart = (unsigned *)talloc(sizeof(unsigned) * nnz);
      nfib_dev = (u64 *)talloc(sizeof(u64));
      err_dev = (int *)talloc(sizeof(int));
      hipMemsetAsync(err_dev, 0, sizeof(int), c->stream);
      for (int k = 0; k < c->D; ++k)
        build_index(c, k, X, comp, ids, comp_t, ids_t, flag, fid, fstart, c->sort_scratch,
                    c->scan_scratch, err_dev, nfib_dev);
      hipMemcpyAsync(&err_host, err_dev, sizeof(int), hipMemcpyDeviceToHost, c->stream);
      // ||X||^2 (uses fid as scratch for the block partials)
      fit_norm(X->values, X->value_dtype, nnz, (double *)fid, c->st, c->stream);
      e = hipStreamSynchronize(c->stream);
      tfree_all();
    }
    if (!dense && e == hipSuccess && !err_host && opt->fit_samples > 0) {
      // stratified fit sample, drawn once (Sec. 6.4)
      const double alpha = opt->fit_nnz_fraction;
      if (!(alpha >= 0.0 && alpha <= 1.0)) throw cpal_status(CPAL_E_ARG);
      const i64 n_nz = (i64)std::ceil(alpha * (double)opt->fit_samples);
      i64 n_z = (i64)std::floor((1.0 - alpha) * (double)opt->fit_samples);
      const u64 zeros = (u64)full - (u64)nnz;
      if (zeros == 0) n_z = 0;
      c->fit_ld = n_nz + n_z;
      c->fit_nz = n_nz;
      c->phi_nz = n_nz ? (double)nnz / (double)n_nz : 0.0;
      c->fit_sc = c->alloc<int>((size_t)c->D * std::max<i64>(c->fit_ld, 1));
      c->fit_x = c->alloc<double>(std::max<i64>(c->fit_ld, 1));
      c->fit_part = c->alloc<double>(c->fit_ld / 256 + 2);
      u64 ns = 64;
      while (ns < 2 * (u64)nnz) ns <<= 1;
      int lg = 0;
      while ((1ull << lg) < ns) ++lg;
      const i64 zd = 64 * n_z + (1ll << 20);
      const i64 zchunks = (zd + CPAL_DRAW_CHUNK - 1) / CPAL_DRAW_CHUNK;
      u64 *set = (u64 *)talloc(sizeof(u64) * ns);
      u64 *ctl = (u64 *)talloc(sizeof(u64) * 4);
      u64 *zbuf = (u64 *)talloc(sizeof(u64) * (size_t)zchunks * CPAL_DRAW_CHUNK);
      unsigned *zcnt = (unsigned *)talloc(sizeof(unsigned) * zchunks);
      hipMemsetAsync(ctl, 0, sizeof(u64) * 4, c->stream);
      const FullModes fm = full_modes(c);
      fit_build_set(X->coords, nnz, fm, set, ns, 64 - lg, c->stream);
      fit_draw(X->coords, X->values, X->value_dtype, nnz, fm, n_nz, n_z, c->seed, c->stream_id,
               set, ns, 64 - lg, ctl, zbuf, zcnt, c->fit_sc, c->fit_ld, c->fit_x, c->stream);
      u64 got = 0;
      if (n_z > 0) hipMemcpyAsync(&got, ctl + 2, sizeof(u64), hipMemcpyDeviceToHost, c->stream);
      e = hipStreamSynchronize(c->stream);
      tfree_all();
      c->fit_n = n_nz + (i64)got;
      // the zero stratum's weight uses the zeros actually drawn (fewer than
      // n_z when the draw guard stopped the rejection sampling)
      c->phi_z = got ? (double)zeros / (double)got : 0.0;
      if ((i64)got < n_z) c->fit_flags |= CPAL_FLAG_DRAWCAP;
    }
    if (e != hipSuccess) {
      cpal_status st = check_hip(c, e, "init (fiber index)");
      c->release();
      delete c;
      return st;
    }
    if (err_host) {
      c->release();
      delete c;
      return CPAL_E_ARG;  // coordinate out of range (1) or duplicate coordinate (2)
    }
    // mirrors and leverage of every initial factor (Alg. 3 setup)
    for (int m = 0; m < c->D; ++m) {
      launch_to_f32(c->mode[m].A, c->mode[m].A32, c->mode[m].n * R, c->stream);
      refresh_leverage(c, m);
    }
    std::vector<u64> W(c->D, 0);
    for (int m = 0; m < c->D; ++m)
      hipMemcpyAsync(&W[m], c->mode[m].C + (c->mode[m].n - 1), sizeof(u64), hipMemcpyDeviceToHost,
                     c->stream);
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      cpal_status st = check_hip(c, e, "init (leverage)");
      c->release();
      delete c;
      return st;
    }
    for (int m = 0; m < c->D; ++m) {
      if (W[m] == 0) {
        c->release();
        delete c;
        return CPAL_E_STATE;
      }
    }
    if (c->f64 && !dense) {   // FP64 gathers default to the owner gather
      const cpal_status st = owner_defaults(c);
      if (st != CPAL_OK) {
        c->release();
        delete c;
        return st;
      }
    }
  } catch (cpal_status st) {
    c->release();
    delete c;
    return st;
  }
  *out = c;
  return CPAL_OK;
}

}  // namespace

namespace {

int default_gather_grid(const cpal_ctx *c, int k) {
  if (c->dense) return c->dnch;
  return c->mode[k].n <= (1 << 20) ? c->gs_grid : c->gather_grid;
}

// Dense contraction with `nch` workgroups along the sampled fibers (at most
// the c->dnch the partials are sized for): sampled fibers per workgroup, a
// multiple of 32.
int dense_kc(const cpal_ctx *c, int nch) {
  if (nch <= 0 || nch > c->dnch) nch = c->dnch;
  i64 kc = ((c->s + nch - 1) / nch + 31) / 32 * 32;
  return (int)std::min<i64>(std::max<i64>(kc, c->dkc), 1024);
}

// Steps of one mode update before the gather: SkrpLev's deterministic and
// random rows with repeats combined (Alg. 1, 2; Sec. 4.1, 4.3), the sampled
// KRP rows, fiber probes and G_s partials, and the gather stream layout.
void update_front(cpal_ctx *c, int k) {
  hipStream_t s = c->stream;
  Mode &md = c->mode[k];
  const OtherModes om = others_of(c, k);
  const int R = c->R;
  hipEvent_t tb = c->stage_begin(CPAL_STAGE_SAMPLE);
  launch_det_cand(om, c->tau, c->enum_cap, c->st, c->cand, s);
  if (c->tau < 1.0)
    launch_det_enum(om, c->tau, c->st, c->cand, c->det_blk, c->det_keys, c->det_cap, s);
  launch_det_finish(om, c->st, c->det_keys, c->det_p, c->kept_p, c->psum, c->det_cap, c->s,
                    c->samp_idx, s);
  launch_draw(om, c->st, c->seed, c->stream_id, c->dbuf, c->dpos, c->chunk_cnt,
              c->draw_grid, c->draw_more_grid, s);
  launch_compact(c->st, c->dbuf, c->chunk_cnt, c->dpos, c->keys, c->dtab, c->dtab_n - 1,
                 c->dtab_shift, c->f64, s);
  c->last_key_bits = md.key_bits;
  c->stage_end(CPAL_STAGE_SAMPLE, tb);
  tb = c->stage_begin(CPAL_STAGE_ROWS);
  const int ncopies = c->dense ? 1 : (int)m_copies(md.n);
  launch_rows(c->zdt, om, c->st, R, c->s, c->samp_idx, c->samp_om, c->samp_w, c->keys, c->dtab,
              c->dtab_n - 1, c->dtab_shift, c->tpos, c->dense ? nullptr : md.slots,
              md.nslots - 1, md.hshift, (unsigned)md.n, c->zhat, c->foff, c->flen, c->gpart,
              c->gp_len, c->gp_cnt, c->gp_act, c->M,
              (c->dense || uses_owner(c, k, md.g_sort_min) || uses_tile(c, k, md.g_sort_min))
                  ? 0 : ncopies * md.n * c->ldz,
              c->ldz, s);
  launch_gather_prep(c->st, c->flen, c->foff, c->s, c->gp_len, c->gp_cnt, c->gp_act, c->cpos,
                     c->coff, c->cidx, c->chunk_first, c->tpos, c->dtab, s);
  c->stage_end(CPAL_STAGE_ROWS, tb);
}

// The bucketed gather's buffers (sparse contexts; nonzeros up to nnz).
cpal_status ensure_bucket_buffers(cpal_ctx *c) {
  if (c->bk_ent) return CPAL_OK;
  try {
    const size_t nw = gather_bkt_count_words();
    c->bk_cnt = c->alloc<unsigned>(nw);
    c->bk_off = c->alloc<u64>(nw);
    c->bk_scan = c->alloc<char>(scan_scratch_bytes((i64)nw));
    c->bk_ent = c->alloc<uint4>((size_t)c->nnz);
  } catch (cpal_status st) {
    return st;
  }
  return CPAL_OK;
}

bool bucket_capable(const cpal_ctx *c, int k) {
  return !c->dense && c->mode[k].n <= (1 << 20);
}

// The bucketed gather with shared-memory bucket blocks (buckets of up to 512
// rows, at most BL_MAXNB of them; modes of at least 1024 rows, where the
// slices of the buckets keep the chip busy).
bool bucket_lds_capable(const cpal_ctx *c, int k) {
  return bucket_capable(c, k) && c->mode[k].n >= 1024 &&
         gather_bktl_shift(c->R, c->mode[k].n) >= 0;
}

// The owner gather writes every row of the CPAL_MCOPIES copies of M (sparse
// modes of at most 2^20 rows).
bool owner_capable(const cpal_ctx *c, int k) {
  return !c->dense && c->mode[k].n <= (1 << 20);
}

cpal_status ensure_owner_buffers(cpal_ctx *c) {
  if (c->own_bnd) return CPAL_OK;
  i64 nbmax = 0;
  for (int m = 0; m < c->D; ++m)
    if (owner_capable(c, m))
      nbmax = std::max<i64>(nbmax, gather_own_blocks(c->f64, c->ldz, c->mode[m].n));
  try {
    c->own_bnd = c->alloc<unsigned>((size_t)c->s * (size_t)(nbmax + 1));
  } catch (cpal_status st) {
    return st;
  }
  return CPAL_OK;
}

// Every sparse mode of at most 2^20 rows runs the owner gather.
cpal_status owner_defaults(cpal_ctx *c) {
  const cpal_status st = ensure_owner_buffers(c);
  if (st != CPAL_OK) return st;
  for (int m = 0; m < c->D; ++m)
    if (owner_capable(c, m)) c->mode[m].g_sort_min = -2;
  return CPAL_OK;
}

// The gather a mode update of mode k runs with sort threshold sort_min.
bool uses_owner(const cpal_ctx *c, int k, int sort_min) {
  return sort_min == -2 && c->own_bnd && owner_capable(c, k);
}

// The tile gather writes every row of the CPAL_MCOPIES copies of M (sparse
// modes of at most TB_MAXNB row blocks).  Its workgroups are (row block,
// fiber part) pairs: modes of fewer than 32 blocks (1024 rows) would leave
// most of the chip idle, and are left to the other gathers.
bool tile_capable(const cpal_ctx *c, int k) {
  const int nb = c->dense || c->mode[k].n > (1 << 20) ? -1 : gather_tile_blocks(c->R, c->mode[k].n);
  return nb >= 32;
}

cpal_status ensure_tile_buffers(cpal_ctx *c) {
  if (c->tile_bnd) return CPAL_OK;
  i64 nbmax = 0;
  for (int m = 0; m < c->D; ++m)
    if (tile_capable(c, m)) nbmax = std::max<i64>(nbmax, gather_tile_blocks(c->R, c->mode[m].n));
  try {
    c->tile_bnd = c->alloc<unsigned>((size_t)gather_tile_ldb(c->s) * (size_t)(nbmax + 1));
  } catch (cpal_status st) {
    return st;
  }
  return CPAL_OK;
}

bool uses_tile(const cpal_ctx *c, int k, int sort_min) {
  return (sort_min == -3 && c->tile_bnd && tile_capable(c, k)) ||
         (sort_min == -5 && c->tile_bnd && c->bk_ent && tile_capable(c, k) &&
          bucket_lds_capable(c, k));
}

// The shared-block bucketed gather's records pack the KRP row (slot index,
// below the sample count) into 23 bits: compact records while it fits.
int bktl_compact(const cpal_ctx *c) { return c->s < ((i64)1 << 23) ? 1 : 0; }

// TnsrSamp + sampled MTTKRP (Sec. 6.3, eq. (1.2)) into M.  sort_min < 0
// selects the bucketed gather (bucket_capable modes).
void update_gather(cpal_ctx *c, int k, int grid, int sort_min) {
  hipStream_t s = c->stream;
  Mode &md = c->mode[k];
  const int R = c->R;
  if (grid <= 0) grid = default_gather_grid(c, k);
  if (c->dense) {   // M = X~^T diag(omega) Z on the matrix cores
    const int kc = dense_kc(c, grid);
    launch_dense_mttkrp(c->zdt, c->st, md.n, R, c->ldz, md.dld, c->cidx, c->samp_idx, md.dX,
                        c->zhat, c->dpart, kc, (int)((c->s + kc - 1) / kc), c->M, s);
  }
  else if (sort_min == -5 && uses_tile(c, k, sort_min))
    launch_gather_hyb(c->f64, c->st, R, c->cpos, c->coff, c->cidx, c->chunk_first, md.pairs,
                      md.ik, md.v64, md.n, c->nnz, c->s, c->zhat, c->ldz, c->M, c->tile_bnd,
                      c->bk_cnt, c->bk_off, c->bk_scan, c->bk_ent, grid > 0 && grid <= 256 ? grid : 16,
                      bktl_compact(c), s);
  else if (uses_tile(c, k, sort_min))
    launch_gather_tile(c->f64, c->st, R, c->cpos, c->coff, c->cidx, md.pairs, md.ik, md.v64, md.n,
                       c->s, c->zhat, c->ldz, c->M, c->tile_bnd, 0u, s);
  else if (uses_owner(c, k, sort_min))
    launch_gather_own(c->f64, c->st, R, c->cpos, c->coff, c->cidx, md.pairs, md.ik, md.v64, md.n,
                      c->zhat, c->ldz, c->M, c->own_bnd, s);
  else if (sort_min == -4 && c->bk_ent && bucket_lds_capable(c, k))
    launch_gather_bktl(c->f64, c->st, R, c->cpos, c->coff, c->cidx, c->chunk_first, md.pairs,
                       md.ik, md.v64, md.n, c->nnz, c->zhat, c->ldz, c->M, c->bk_cnt, c->bk_off,
                       c->bk_scan, c->bk_ent, 0u, bktl_compact(c), s);
  else if (sort_min == -1 && c->bk_ent && bucket_capable(c, k))
    launch_gather_bkt(c->f64, c->st, R, c->cpos, c->coff, c->cidx, c->chunk_first, md.pairs,
                      md.ik, md.v64, md.n, c->nnz, c->zhat, c->ldz, c->M, grid, c->bk_cnt,
                      c->bk_off, c->bk_scan, c->bk_ent, s);
  else if (md.n <= (1 << 20))
    launch_gather_seg(c->f64, c->st, R, c->cpos, c->coff, c->cidx, c->chunk_first, md.pairs,
                      md.ik, md.v64, md.n, c->zhat, c->ldz, c->M, grid, std::max(sort_min, 0), s);
  else
    launch_gather(c->f64, c->st, R, c->cpos, c->coff, c->cidx, md.pairs, md.ik, md.v64, c->zhat,
                  c->M, c->ldz, grid, s);
}

// Solve A_k = M G_s^{-1}, the leverage of the new A_k, statistics.
void update_back(cpal_ctx *c, int k, cpal_mode_stats *stats_dev) {
  hipStream_t s = c->stream;
  Mode &md = c->mode[k];
  const int R = c->R;
  const int ncopies = c->dense ? 1 : (int)m_copies(md.n);
  hipEvent_t tb = c->stage_begin(CPAL_STAGE_SOLVE);
  launch_decomp_dev(c->gpart, &c->st->n_slots, rows_per_block(), R, c->dc, &c->st->flags,
                    c->gram_tmp, s);
  launch_solve_rows(c->f64, c->st, md.n, R, c->M, c->ldz, ncopies, c->dc, md.A, md.A32, s);
  c->stage_end(CPAL_STAGE_SOLVE, tb);
  tb = c->stage_begin(CPAL_STAGE_LEVERAGE);
  refresh_leverage(c, k, stats_dev);   // its last kernel also writes the statistics
  c->stage_end(CPAL_STAGE_LEVERAGE, tb);
}

}  // namespace

// ------------------------------------------------------------------------
// Scratch of the allocation-free entry point (cp_arls_lev_leverage_noalloc):
// a file-scope device array, one per GPU, held until the process ends.  In
// host code `scratch` only names the symbol; its device address on each GPU
// comes from hipGetSymbolAddress with that GPU current and is used
// everywhere host code needs the array.
#define CPAL_NOALLOC_BYTES (16u << 20)
#define CPAL_NOALLOC_DEVICES 64
static __device__ __align__(256) unsigned char scratch[CPAL_NOALLOC_BYTES];

namespace {

std::mutex g_noalloc_mu;
void *g_noalloc_ptr[CPAL_NOALLOC_DEVICES] = {};

std::string &noalloc_error() {
  static thread_local std::string e = "null context";
  return e;
}

cpal_status noalloc_fail(cpal_status st, const char *msg) {
  noalloc_error() = msg;
  return st;
}

// The device address of `scratch` on the current GPU, looked up once per GPU.
cpal_status noalloc_scratch(unsigned char **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= CPAL_NOALLOC_DEVICES)
    return noalloc_fail(CPAL_E_DEVICE, "leverage_noalloc: no current device");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return noalloc_fail(CPAL_E_DEVICE, "leverage_noalloc: hipGetSymbolAddress failed");
    g_noalloc_ptr[dev] = p;
  }
  *out = (unsigned char *)g_noalloc_ptr[dev];
  return CPAL_OK;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of scratch the leverage kernels need for an n x R matrix: Gram
// partials per 256-row block, the decomposition, per-row sampling weights
// and their block sums, the summed Gram matrix, two flags.
size_t noalloc_bytes(i64 n, int R) {
  const size_t np = (size_t)R * (R + 1) / 2;
  const size_t nblk = (size_t)((n + CPAL_GRAM_ROWS - 1) / CPAL_GRAM_ROWS);
  return align256(nblk * np * sizeof(double)) + align256(sizeof(Decomp)) +
         align256((size_t)n * sizeof(u64)) + align256((size_t)(lev_row_blocks(n) + 1) * sizeof(u64)) +
         align256(np * sizeof(double)) + align256(2 * sizeof(int));
}

// The leverage computation of a context's factor (Gram, Cholesky or
// row-space test / pseudo-inverse, per-row scores) on the caller's matrix
// with every intermediate in the static scratch.  Nothing needs clearing:
// every scratch word a kernel reads was written earlier in the sequence.
cpal_status leverage_noalloc(const double *A, i64 n, int R, double *lev, hipStream_t s) {
  if (!A || !lev || n < 1 || R < 1 || R > CPAL_MAXR)
    return noalloc_fail(CPAL_E_ARG, "leverage_noalloc: invalid arguments");
  if (noalloc_bytes(n, R) > CPAL_NOALLOC_BYTES)
    return noalloc_fail(CPAL_E_ARG, "leverage_noalloc: the matrix needs more scratch than the "
                                    "16 MiB static array (too many rows for this rank)");
  unsigned char *base = nullptr;
  const cpal_status st = noalloc_scratch(&base);
  if (st != CPAL_OK) return st;
  const size_t np = (size_t)R * (R + 1) / 2;
  const int nblk = (int)((n + CPAL_GRAM_ROWS - 1) / CPAL_GRAM_ROWS);
  size_t off = 0;
  double *part = (double *)(base + off);
  off += align256((size_t)nblk * np * sizeof(double));
  Decomp *dc = (Decomp *)(base + off);
  off += align256(sizeof(Decomp));
  u64 *w = (u64 *)(base + off);
  off += align256((size_t)n * sizeof(u64));
  u64 *bsum = (u64 *)(base + off);
  off += align256((size_t)(lev_row_blocks(n) + 1) * sizeof(u64));
  double *gram = (double *)(base + off);
  off += align256(np * sizeof(double));
  int *flags = (int *)(base + off);   // [0] full-row-rank skip, [1] pseudo-inverse used
  const int *skip = nullptr;
  if (n < R) {
    launch_lev_rowspace(A, (int)n, R, lev, w, bsum, &flags[0], &flags[1], s);
    skip = &flags[0];
  }
  launch_lev_gram_partial(A, n, R, part, skip, s);
  launch_decomp_blocks(part, nblk, R, gram, dc, &flags[1], skip, s);
  launch_lev_rows(A, n, R, dc, lev, w, bsum, skip, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return noalloc_fail(CPAL_E_DEVICE, hipGetErrorString(e));
  return CPAL_OK;
}

}  // namespace

extern "C" {

cpal_status cp_arls_lev_init(const cpal_tensor *X, const cpal_options *opt,
                             double *const *factors, void *hip_stream,
                             const cpal_allocator *alloc, cpal_ctx **out) {
  return init_impl(X, opt, factors, hip_stream, alloc, nullptr, out);
}

cpal_status cp_arls_lev_mode_update(cpal_ctx *c, int32_t k, cpal_mode_stats *stats_dev) {
  if (!c) return CPAL_E_ARG;
  if (k < 0 || k >= c->D) return fail(c, CPAL_E_ARG, "mode out of range");
  if (c->failed) return fail(c, CPAL_E_STATE, "context failed earlier");
  update_front(c, k);
  hipEvent_t tb = c->stage_begin(CPAL_STAGE_GATHER);
  update_gather(c, k, c->mode[k].g_grid, c->mode[k].g_sort_min);
  c->stage_end(CPAL_STAGE_GATHER, tb);
  update_back(c, k, stats_dev);
  c->t += 1;
  c->samples_valid = true;
  return check_hip(c, hipGetLastError(), "mode_update launch");
}

cpal_status cp_arls_lev_set_gather_config(cpal_ctx *c, int32_t k, int32_t grid, int32_t sort_min) {
  if (!c || k < 0 || k >= c->D || grid < 0 || grid > (1 << 20) || sort_min < -5)
    return CPAL_E_ARG;
  if (c->dense && grid > c->dnch) return CPAL_E_ARG;
  if (sort_min == -1) {   // the bucketed gather
    if (!bucket_capable(c, k)) return CPAL_E_ARG;
    const cpal_status st = ensure_bucket_buffers(c);
    if (st != CPAL_OK) return fail(c, st, "bucketed gather: buffers");
  }
  if (sort_min == -2) {   // the owner gather
    if (!owner_capable(c, k)) return CPAL_E_ARG;
    const cpal_status st = ensure_owner_buffers(c);
    if (st != CPAL_OK) return fail(c, st, "owner gather: buffers");
  }
  if (sort_min == -4) {   // the bucketed gather with shared-memory blocks
    if (!bucket_lds_capable(c, k)) return CPAL_E_ARG;
    const cpal_status st = ensure_bucket_buffers(c);
    if (st != CPAL_OK) return fail(c, st, "bucketed gather: buffers");
  }
  if (sort_min == -5) {   // the hybrid gather: tile (long fibers) + shared-block bucketed
    if (!tile_capable(c, k) || !bucket_lds_capable(c, k) || grid > 256) return CPAL_E_ARG;
    cpal_status st = ensure_tile_buffers(c);
    if (st == CPAL_OK) st = ensure_bucket_buffers(c);
    if (st != CPAL_OK) return fail(c, st, "hybrid gather: buffers");
  }
  if (sort_min == -3) {   // the tile gather
    if (!tile_capable(c, k)) return CPAL_E_ARG;
    const cpal_status st = ensure_tile_buffers(c);
    if (st != CPAL_OK) return fail(c, st, "tile gather: buffers");
  }
  c->mode[k].g_grid = grid;
  c->mode[k].g_sort_min = sort_min;
  return CPAL_OK;
}

cpal_status cp_arls_lev_get_gather_config(const cpal_ctx *c, int32_t k, int32_t *grid,
                                          int32_t *sort_min) {
  if (!c || k < 0 || k >= c->D || !grid || !sort_min) return CPAL_E_ARG;
  *grid = c->mode[k].g_grid ? c->mode[k].g_grid : default_gather_grid(c, k);
  if (c->dense) {   // the effective workgroups along the sampled fibers
    const int kc = dense_kc(c, *grid);
    *grid = (int)((c->s + kc - 1) / kc);
  }
  *sort_min = c->mode[k].g_sort_min;
  return CPAL_OK;
}

cpal_status cp_arls_lev_autotune(cpal_ctx *c, int32_t reps) {
  if (!c || reps < 0 || reps > 16) return CPAL_E_ARG;
  if (c->failed) return fail(c, CPAL_E_STATE, "context failed earlier");
  if (reps == 0) reps = 2;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return fail(c, CPAL_E_DEVICE, "autotune: event creation");
  }
  const unsigned timing = c->timing;
  c->timing = 0;
  cpal_status res = CPAL_OK;
  for (int k = 0; k < c->D && res == CPAL_OK; ++k) {
    Mode &md = c->mode[k];
    // the sampled system of an update of mode k at the current step, as
    // mode_update would build it; the factors are not touched
    launch_set_step(c->st, c->t, c->stream);
    update_front(c, k);
    const bool seg = !c->dense && md.n <= (1 << 20);
    static const int seg_grids[] = {256, 512, 1024, 2048};
    static const int seg_sort[] = {0, 4, 32, 1 << 30};
    static const int flat_grids[] = {1024, 2048, 4096, 8192};
    // dense: workgroups along the sampled fibers (fewer, longer ones write
    // fewer partials of M); the contraction writes M itself (nothing to clear)
    const int dense_grids[] = {c->dnch, std::max(1, c->dnch / 2), std::max(1, c->dnch / 4),
                               std::max(1, c->dnch / 8)};
    const i64 mwords = c->dense ? 0 : (i64)m_copies(md.n) * md.n * c->ldz * (c->f64 ? 2 : 1);
    float best = 1e30f;
    int best_grid = 0, best_sort = 0;
    // the bucketed gather (sort threshold -1) when its buffers can be had,
    // and the owner gather (-2, one launch shape: its grid follows n_k)
    const bool bkt = bucket_capable(c, k) && ensure_bucket_buffers(c) == CPAL_OK;
    const bool own = owner_capable(c, k) && ensure_owner_buffers(c) == CPAL_OK;
    const bool tile = tile_capable(c, k) && ensure_tile_buffers(c) == CPAL_OK;
    // candidates: ng grids x ns sort thresholds, then the owner (-2), tile
    // (-3), shared-block bucketed (-4) and hybrid (-5, three long-fiber
    // thresholds) gathers
    std::vector<std::pair<int, int>> extra;   // (grid, sort_min)
    if (own) extra.push_back({0, -2});
    if (tile) extra.push_back({0, -3});
    if (bkt && bucket_lds_capable(c, k)) extra.push_back({0, -4});
    if (tile && bkt && bucket_lds_capable(c, k))
      for (int lf : {8, 16, 32}) extra.push_back({lf, -5});
    const int ng = 4, ns = seg ? (bkt ? 5 : 4) : 1;
    std::vector<std::pair<int, int>> cand;   // (grid, sort_min), in order of preference
    for (int gi = 0; gi < ng; ++gi)
      for (int si = 0; si < ns; ++si)
        cand.push_back({c->dense ? dense_grids[gi] : seg ? seg_grids[gi] : flat_grids[gi],
                        !seg ? 0 : si < 4 ? seg_sort[si] : -1});
    cand.insert(cand.end(), extra.begin(), extra.end());
    // every candidate once per round, `reps` rounds, best time of each: a
    // drift of the clocks during the trials (a cold GPU speeding up) then
    // affects all candidates alike
    std::vector<float> tmin(cand.size(), 1e30f);
    for (int r = 0; r < reps && res == CPAL_OK; ++r)
      for (size_t ci = 0; ci < cand.size() && res == CPAL_OK; ++ci) {
        launch_zero_words(c->M, mwords, c->stream);
        hipEventRecord(e0, c->stream);
        update_gather(c, k, cand[ci].first, cand[ci].second);
        hipEventRecord(e1, c->stream);
        if (hipEventSynchronize(e1) != hipSuccess) {
          res = check_hip(c, hipGetLastError(), "autotune trial");
          break;
        }
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        tmin[ci] = std::min(tmin[ci], ms);
      }
    // a later candidate replaces the best one only when it is at least 3%
    // faster, so that near ties resolve the same way from run to run
    for (size_t ci = 0; ci < cand.size(); ++ci)
      if (tmin[ci] < 0.97f * best) {
        best = tmin[ci];
        best_grid = cand[ci].first;
        best_sort = cand[ci].second;
      }
    md.g_grid = best_grid;
    md.g_sort_min = best_sort;
  }
  c->timing = timing;
  // the trials consumed no step: the next update samples with the same t
  launch_set_step(c->st, c->t, c->stream);
  c->samples_valid = false;   // the sample buffers hold a trial's rows
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (res != CPAL_OK) return res;
  return check_hip(c, hipStreamSynchronize(c->stream), "autotune");
}

cpal_status cp_arls_lev_fit_estimate(cpal_ctx *c, double *fit_dev) {
  if (!c || !fit_dev) return CPAL_E_ARG;
  if (c->failed) return fail(c, CPAL_E_STATE, "context failed earlier");
  if (c->fit_n <= 0) return fail(c, CPAL_E_STATE, "no fit sample (fit_samples = 0)");
  fit_eval(full_modes(c), c->R, c->fit_nz, c->fit_n, c->phi_nz, c->phi_z, c->fit_sc, c->fit_ld,
           c->fit_x, c->fit_part, c->st, fit_dev, c->stream);
  return check_hip(c, hipGetLastError(), "fit_estimate launch");
}

// The exact fit (eq. (6.1)) from the copy of the mode with the fewest rows.
static void launch_exact_fit(cpal_ctx *c, double *fit_dev) {
  int k = 0;
  for (int m = 1; m < c->D; ++m)
    if (c->dims[m] < c->dims[k]) k = m;
  const Mode &md = c->mode[k];
  double *A[CPAL_MAXORDER];
  for (int m = 0; m < c->D; ++m) A[m] = c->mode[m].A;
  const int kind = c->dense ? (c->zdt == CPAL_F64 ? 2 : c->zdt == CPAL_F32 ? 3 : 4)
                            : (c->f64 ? 1 : 0);
  launch_fit_exact(c->D, c->dims, A, c->R, k, kind, md.slots, md.nslots, md.pairs, md.ik, md.v64,
                   md.dX, md.dld, c->st, c->fitx_scratch, fit_dev, c->stream);
}

cpal_status cp_arls_lev_fit_exact(cpal_ctx *c, double *fit_dev) {
  if (!c || !fit_dev) return CPAL_E_ARG;
  if (c->failed) return fail(c, CPAL_E_STATE, "context failed earlier");
  launch_exact_fit(c, fit_dev);
  return check_hip(c, hipGetLastError(), "fit_exact launch");
}

cpal_status cp_arls_lev_run(cpal_ctx *c, const cpal_run_options *ro, double *trace,
                            cpal_run_result *res) {
  if (!c || !ro || !trace || !res) return CPAL_E_ARG;
  if (ro->eta < 1 || ro->pi < 1 || ro->max_epochs < 1 || !(ro->tol >= 0.0) ||
      (ro->exact_fit != 0 && ro->exact_fit != 1))
    return fail(c, CPAL_E_ARG, "run: invalid options");
  if (c->failed) return fail(c, CPAL_E_STATE, "context failed earlier");
  if (!ro->exact_fit && c->fit_n <= 0)
    return fail(c, CPAL_E_STATE, "run: the estimated fit needs fit_samples > 0");
  std::memset(res, 0, sizeof(*res));
  double best = -INFINITY;
  int fails = 0, e = 0;
  for (; e < ro->max_epochs;) {
    for (int it = 0; it < ro->eta; ++it)
      for (int k = 0; k < c->D; ++k) {
        const cpal_status st = cp_arls_lev_mode_update(c, k, nullptr);
        if (st != CPAL_OK) return st;
      }
    if (ro->exact_fit) {
      launch_exact_fit(c, c->fit_host_buf);
    } else {
      const cpal_status st = cp_arls_lev_fit_estimate(c, c->fit_host_buf);
      if (st != CPAL_OK) return st;
    }
    double fit = 0.0;
    hipMemcpyAsync(&fit, c->fit_host_buf, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    const cpal_status st = check_hip(c, hipStreamSynchronize(c->stream), "run: epoch fit");
    if (st != CPAL_OK) return st;
    trace[e++] = fit;
    // an epoch improves when its fit beats the best earlier one by more than tol
    if (fit > best + ro->tol) {
      fails = 0;
    } else {
      ++fails;
    }
    if (fit > best) best = fit;
    if (fails >= ro->pi) {
      res->stopped = 1;
      break;
    }
  }
  res->epochs = e;
  res->best_fit = best;
  launch_exact_fit(c, c->fit_host_buf);
  double fx = 0.0;
  hipMemcpyAsync(&fx, c->fit_host_buf, sizeof(double), hipMemcpyDeviceToHost, c->stream);
  const cpal_status st = check_hip(c, hipStreamSynchronize(c->stream), "run: final fit");
  res->final_exact_fit = fx;
  return st;
}

cpal_status cp_arls_lev_rrf_init(cpal_ctx *c, int64_t s_init, const double *const *omega_dev) {
  if (!c || !omega_dev || s_init < 1 || s_init > c->s) return CPAL_E_ARG;
  for (int k = 0; k < c->D; ++k)
    if (!omega_dev[k]) return CPAL_E_ARG;
  if (c->failed) return fail(c, CPAL_E_STATE, "context failed earlier");
  hipStream_t s = c->stream;
  u64 *off = nullptr, *off_t = nullptr;
  unsigned *len = nullptr, *len_t = nullptr;
  unsigned long long *cnt = nullptr;
  u64 maxfib = 0;
  for (int k = 0; k < c->D; ++k) maxfib = std::max<u64>(maxfib, c->mode[k].nfib);
  if (!c->dense) {   // the nonempty fibers of each mode in ascending key order
    off = (u64 *)c->raw_alloc(sizeof(u64) * maxfib);
    off_t = (u64 *)c->raw_alloc(sizeof(u64) * maxfib);
    len = (unsigned *)c->raw_alloc(sizeof(unsigned) * maxfib);
    len_t = (unsigned *)c->raw_alloc(sizeof(unsigned) * maxfib);
    cnt = (unsigned long long *)c->raw_alloc(sizeof(unsigned long long));
    if (!off || !off_t || !len || !len_t || !cnt) {
      c->raw_free(off); c->raw_free(off_t); c->raw_free(len); c->raw_free(len_t); c->raw_free(cnt);
      return fail(c, CPAL_E_NOMEM, "rrf_init: fiber lists");
    }
  }
  for (int k = 0; k < c->D; ++k) {
    Mode &md = c->mode[k];
    u64 nfib = 0;
    if (c->dense) {
      nfib = 1;
      for (int m = 0; m < c->D; ++m)
        if (m != k) nfib *= (u64)c->dims[m];
    } else {
      nfib = md.nfib;
      hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s);
      launch_fiber_list(md.slots, md.nslots, off, len, cnt, s);
      sort_keys(off, len, off_t, len_t, c->sort_scratch, (i64)nfib, nullptr, (i64)nfib,
                bits_for((u64)c->nnz + 1), s);
    }
    launch_rrf_rows(c->zdt, c->st, s_init, k, c->seed, c->stream_id, nfib, c->dense ? nullptr : off,
                    c->dense ? nullptr : len, (unsigned)md.n, omega_dev[k], c->R, c->ldz, c->zhat,
                    c->foff, c->flen, c->samp_idx, c->gp_len, c->gp_cnt, c->gp_act,
                    rows_per_block(), s);
    launch_gather_prep(c->st, c->flen, c->foff, s_init, c->gp_len, c->gp_cnt, c->gp_act, c->cpos,
                       c->coff, c->cidx, c->chunk_first, c->tpos, c->dtab, s);
    const int ncopies = c->dense ? 1 : (int)m_copies(md.n);
    if (!c->dense && !uses_owner(c, k, md.g_sort_min) && !uses_tile(c, k, md.g_sort_min))
      launch_zero_words(c->M, (i64)ncopies * md.n * c->ldz * (c->f64 ? 2 : 1), s);
    update_gather(c, k, md.g_grid, md.g_sort_min);
    launch_rrf_store(c->f64, c->M, ncopies, md.n, c->R, c->ldz, md.A, md.A32, s);
    refresh_leverage(c, k);
  }
  const cpal_status st = check_hip(c, hipStreamSynchronize(s), "rrf_init");
  c->raw_free(off); c->raw_free(off_t); c->raw_free(len); c->raw_free(len_t); c->raw_free(cnt);
  c->samples_valid = false;   // the sampled-system buffers hold the last mode's draws
  return st;
}

cpal_status cp_arls_lev_samples(const cpal_ctx *c, uint64_t *idx_dev, double *omega_dev,
                                double *w_dev, int64_t cap, int64_t *count_dev) {
  if (!c || cap < 0) return CPAL_E_ARG;
  if (!c->samples_valid) return CPAL_E_STATE;
  launch_samples_out(c->st, c->samp_idx, c->samp_om, c->samp_w, c->s, c->last_key_bits, c->keys,
                     c->keys_tmp, c->ord, c->ord_tmp, c->sort_scratch, cap, (u64 *)idx_dev,
                     omega_dev, w_dev, (i64 *)count_dev, c->stream);
  return CPAL_OK;
}

cpal_status cp_arls_lev_leverage(const cpal_ctx *c, int32_t m, double *lev_dev) {
  if (!c || !lev_dev || m < 0 || m >= c->D) return CPAL_E_ARG;
  hipMemcpyAsync(lev_dev, c->mode[m].lev, sizeof(double) * c->mode[m].n, hipMemcpyDeviceToDevice,
                 c->stream);
  return CPAL_OK;
}

cpal_status cp_arls_lev_refresh(cpal_ctx *c, int32_t m) {
  if (!c || m < 0 || m >= c->D) return CPAL_E_ARG;
  launch_to_f32(c->mode[m].A, c->mode[m].A32, c->mode[m].n * c->R, c->stream);
  refresh_leverage(c, m);
  return check_hip(c, hipGetLastError(), "refresh");
}

cpal_status cp_arls_lev_get_step(const cpal_ctx *c, uint64_t *t) {
  if (!c || !t) return CPAL_E_ARG;
  *t = c->t;
  return CPAL_OK;
}

cpal_status cp_arls_lev_set_step(cpal_ctx *c, uint64_t t) {
  if (!c) return CPAL_E_ARG;
  c->t = t;
  launch_set_step(c->st, t, c->stream);   // the kernels read the counter on the device
  return check_hip(c, hipGetLastError(), "set_step");
}

cpal_status cp_arls_lev_set_timing(cpal_ctx *c, int32_t enable) {
  if (!c) return CPAL_E_ARG;
  c->timing = (unsigned)enable & ((1u << CPAL_NSTAGES) - 1u);
  return CPAL_OK;
}

cpal_status cp_arls_lev_stage_times(cpal_ctx *c, double *ms, int64_t *count, int32_t reset) {
  if (!c || !ms || !count) return CPAL_E_ARG;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return check_hip(c, e, "stage_times");
  for (int i = 0; i < CPAL_NSTAGES; ++i) { ms[i] = 0.0; count[i] = 0; }
  for (auto &r : c->ev_rec) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.second.first, r.second.second) == hipSuccess) {
      ms[r.first] += (double)t;
      count[r.first] += 1;
    }
  }
  if (reset) {
    for (auto &r : c->ev_rec) {
      c->ev_pool.push_back(r.second.first);
      c->ev_pool.push_back(r.second.second);
    }
    c->ev_rec.clear();
  }
  return CPAL_OK;
}

const char *cp_arls_lev_last_error(const cpal_ctx *c) {
  if (!c) return noalloc_error().c_str();
  return c->err.c_str();
}

cpal_status cp_arls_lev_leverage_noalloc(const double *A_dev, int64_t n, int32_t R,
                                         double *lev_dev, void *hip_stream) {
  return leverage_noalloc(A_dev, n, R, lev_dev, (hipStream_t)hip_stream);
}

void cp_arls_lev_destroy(cpal_ctx *c) {
  if (!c) return;
  hipStreamSynchronize(c->stream);
  c->release();
  delete c;
}

// ------------------------------------------------------------------ batches
}  // extern "C"

struct cpal_batch {
  std::vector<cpal_ctx *> ctx;
  hipStream_t user = nullptr;
  std::vector<hipStream_t> streams;
  hipEvent_t start = nullptr;
  std::vector<hipEvent_t> done;
  int graphs = 0;   // 0: launch each step; 1 / 2: replay the step's graph of branches / stages
  hipGraphExec_t exec[CPAL_MAXORDER] = {nullptr};    // graph of branches per mode
  hipGraphExec_t exec2[CPAL_MAXORDER] = {nullptr};   // stage-major graph per mode
  void *plan_mem[CPAL_MAXORDER] = {nullptr};         // its launch tables (device)
  int64_t kernels[2][CPAL_MAXORDER] = {};            // kernel launches per captured graph
  cpal_mode_stats *stats = nullptr;                 // statistics written by the graphs
  std::vector<int> tensor_of;                       // tensor of each decomposition
  cpal_allocator al{};                              // alloc == nullptr: hipMalloc / hipFree
};

namespace {

// streams a batch spreads its decompositions over: measured on batch256,
// kernel-by-kernel steps ran 7.3k / 9.1k / 10.3k mode updates/s with 4 / 8 /
// 16 streams (graph replay 11.7k-11.9k either way)
constexpr int kBatchStreams = 16;

// Kernel nodes of a captured graph.
int64_t kernel_nodes(hipGraph_t g) {
  size_t n = 0;
  if (hipGraphGetNodes(g, nullptr, &n) != hipSuccess || n == 0) return 0;
  std::vector<hipGraphNode_t> nodes(n);
  if (hipGraphGetNodes(g, nodes.data(), &n) != hipSuccess) return 0;
  int64_t k = 0;
  for (size_t i = 0; i < n; ++i) {
    hipGraphNodeType t;
    if (hipGraphNodeGetType(nodes[i], &t) == hipSuccess && t == hipGraphNodeTypeKernel) ++k;
  }
  return k;
}

void drop_stage_graph(cpal_batch *b, int mode);

void batch_free(cpal_batch *b) {
  for (hipGraphExec_t g : b->exec)
    if (g) hipGraphExecDestroy(g);
  for (int m = 0; m < CPAL_MAXORDER; ++m) drop_stage_graph(b, m);
  if (b->stats) {
    if (b->al.alloc) b->al.free(b->stats, b->al.user);
    else hipFree(b->stats);
  }
  for (cpal_ctx *c : b->ctx)
    if (c) cp_arls_lev_destroy(c);
  for (hipStream_t s : b->streams) hipStreamDestroy(s);
  for (hipEvent_t e : b->done) hipEventDestroy(e);
  if (b->start) hipEventDestroy(b->start);
  delete b;
}

// The batch's streams wait for the caller's stream; afterwards the caller's
// stream waits for every batch stream.
void batch_fork(cpal_batch *b) {
  hipEventRecord(b->start, b->user);
  for (hipStream_t s : b->streams) hipStreamWaitEvent(s, b->start, 0);
}
void batch_join(cpal_batch *b) {
  for (size_t j = 0; j < b->streams.size(); ++j) {
    hipEventRecord(b->done[j], b->streams[j]);
    hipStreamWaitEvent(b->user, b->done[j], 0);
  }
}

// Capture mode step `mode` of every decomposition into one graph: the
// decompositions' kernels are recorded on the batch's streams (forked from
// and joined back into streams[0]); each writes its statistics to b->stats.
// Stage timing is off while capturing; the host step counters are restored
// (a capture runs no kernel).
cpal_status batch_capture(cpal_batch *b, int mode) {
  hipStream_t s0 = b->streams[0];
  if (hipStreamBeginCapture(s0, hipStreamCaptureModeRelaxed) != hipSuccess) return CPAL_E_DEVICE;
  hipEventRecord(b->start, s0);
  for (size_t j = 1; j < b->streams.size(); ++j) hipStreamWaitEvent(b->streams[j], b->start, 0);
  cpal_status res = CPAL_OK;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    cpal_ctx *c = b->ctx[i];
    if (mode >= c->D) continue;
    const u64 t = c->t;
    const unsigned timing = c->timing;
    c->timing = 0;
    const cpal_status st = cp_arls_lev_mode_update(c, mode, b->stats + i);
    c->timing = timing;
    c->t = t;
    if (st != CPAL_OK && res == CPAL_OK) res = st;
  }
  for (size_t j = 1; j < b->streams.size(); ++j) {
    hipEventRecord(b->done[j], b->streams[j]);
    hipStreamWaitEvent(s0, b->done[j], 0);
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s0, &g);
  if (e != hipSuccess || !g) return CPAL_E_DEVICE;
  b->kernels[0][mode] = kernel_nodes(g);
  if (res == CPAL_OK && hipGraphInstantiate(&b->exec[mode], g, nullptr, nullptr, 0) != hipSuccess)
    res = CPAL_E_DEVICE;
  hipGraphDestroy(g);
  return res;
}

// ------------------------------------------------------- stage-major steps
// A batch's mode step as a few launches per stage instead of one launch per
// stage per decomposition: every decomposition's update is described (not
// launched) through the launch sink, giving it a sequence of launches; the
// launches are then issued in rounds, each taking the next launch of some
// decompositions.  Launches of one body and block size in a round become one
// k_multi launch over all of them (argument packs and block prefix in device
// memory); launches without a batched form run on the batch's other streams
// beside it.  A round starts after the previous one has finished, so each
// decomposition's launches keep their order.

// One described launch of an update.
struct DescLaunch {
  MultiLaunch ml = nullptr;   // batched form; nullptr: solo
  std::vector<unsigned char> pack;
  size_t align = 1;
  unsigned grid = 0, block = 0;
  size_t shmem = 0;
  int occ = 0;                // earlier launches of the same form in the sequence
  std::function<void(hipStream_t)> solo;
};

struct SeqSink : LaunchSink {
  std::vector<DescLaunch> seq;
  void batchable(MultiLaunch ml, const void *pack, size_t bytes, size_t align, unsigned grid,
                 unsigned block, size_t shmem) override {
    DescLaunch l;
    l.ml = ml;
    l.pack.assign((const unsigned char *)pack, (const unsigned char *)pack + bytes);
    l.align = align;
    l.grid = grid;
    l.block = block;
    l.shmem = shmem;
    for (const DescLaunch &e : seq) l.occ += e.ml == ml && e.block == block;
    seq.push_back(std::move(l));
  }
  void solo(std::function<void(hipStream_t)> f) override {
    DescLaunch l;
    l.solo = std::move(f);
    seq.push_back(std::move(l));
  }
};

// A batched launch of a round: launches `members` (decomposition, position)
// of one form; its packs and prefix sit at the given offsets of the tables.
struct MultiGroup {
  MultiLaunch ml;
  unsigned block;
  size_t shmem = 0;
  unsigned blocks = 0;
  std::vector<std::pair<int, size_t>> members;
  size_t packs_off = 0, pre_off = 0;
};
struct StageRound {
  std::vector<MultiGroup> groups;
  std::vector<std::pair<int, size_t>> solos;
};

// Rounds for the sequences: every solo launch at the head of a sequence runs
// in the next round; a batched head runs once no other sequence still has
// the same launch (form and occurrence) ahead of its head, so that launches
// of one stage meet in one round (when every head waits, all run).
std::vector<StageRound> plan_rounds(const std::vector<std::vector<DescLaunch>> &seqs) {
  const size_t n = seqs.size();
  std::vector<size_t> pos(n, 0);
  std::vector<StageRound> rounds;
  typedef std::tuple<MultiLaunch, unsigned, int> Form;
  for (;;) {
    StageRound r;
    std::map<Form, std::vector<std::pair<int, size_t>>> heads;
    for (size_t i = 0; i < n; ++i) {
      if (pos[i] >= seqs[i].size()) continue;
      const DescLaunch &h = seqs[i][pos[i]];
      if (!h.ml) r.solos.push_back({(int)i, pos[i]});
      else heads[Form(h.ml, h.block, h.occ)].push_back({(int)i, pos[i]});
    }
    if (r.solos.empty() && heads.empty()) break;
    std::vector<const std::vector<std::pair<int, size_t>> *> ready;
    for (const auto &kv : heads) {
      bool wait = false;
      for (size_t j = 0; j < n && !wait; ++j)
        for (size_t q = pos[j] + 1; q < seqs[j].size() && !wait; ++q) {
          const DescLaunch &e = seqs[j][q];
          wait = Form(e.ml, e.block, e.occ) == kv.first;
        }
      if (!wait) ready.push_back(&kv.second);
    }
    if (ready.empty() && r.solos.empty())
      for (const auto &kv : heads) ready.push_back(&kv.second);
    for (const auto *m : ready) {
      MultiGroup g;
      const DescLaunch &h = seqs[(*m)[0].first][(*m)[0].second];
      g.ml = h.ml;
      g.block = h.block;
      g.members = *m;
      r.groups.push_back(std::move(g));
    }
    for (const auto &p : r.solos) ++pos[p.first];
    for (const MultiGroup &g : r.groups)
      for (const auto &p : g.members) ++pos[p.first];
    rounds.push_back(std::move(r));
  }
  return rounds;
}

void drop_stage_graph(cpal_batch *b, int mode) {
  if (b->exec2[mode]) hipGraphExecDestroy(b->exec2[mode]);
  b->exec2[mode] = nullptr;
  if (b->plan_mem[mode]) {
    if (b->al.alloc) b->al.free(b->plan_mem[mode], b->al.user);
    else hipFree(b->plan_mem[mode]);
  }
  b->plan_mem[mode] = nullptr;
  b->kernels[1][mode] = 0;
}

// Launch rounds of described sequences and their tables in device memory.
struct StagePlan {
  std::vector<std::vector<DescLaunch>> seqs;
  std::vector<StageRound> rounds;
  void *mem = nullptr;   // packs and prefixes (batch allocator)
};

void plan_free(cpal_batch *b, StagePlan &p) {
  if (p.mem) {
    if (b->al.alloc) b->al.free(p.mem, b->al.user);
    else hipFree(p.mem);
  }
  p.mem = nullptr;
}

// Rounds of p.seqs and their tables, written to device memory (synchronous copy).
cpal_status plan_build(cpal_batch *b, StagePlan &p) {
  p.rounds = plan_rounds(p.seqs);
  std::vector<unsigned char> tab;
  auto place = [&tab](size_t bytes) {
    const size_t off = (tab.size() + 255) / 256 * 256;
    tab.resize(off + bytes);
    return off;
  };
  for (StageRound &r : p.rounds)
    for (MultiGroup &g : r.groups) {
      const DescLaunch &h0 = p.seqs[g.members[0].first][g.members[0].second];
      const size_t stride = (h0.pack.size() + h0.align - 1) / h0.align * h0.align;
      g.packs_off = place(stride * g.members.size());
      for (size_t m = 0; m < g.members.size(); ++m) {
        const DescLaunch &l = p.seqs[g.members[m].first][g.members[m].second];
        std::memcpy(tab.data() + g.packs_off + m * stride, l.pack.data(), l.pack.size());
      }
      g.pre_off = place(sizeof(unsigned) * (g.members.size() + 1));
      unsigned acc = 0;
      for (size_t m = 0; m <= g.members.size(); ++m) {
        std::memcpy(tab.data() + g.pre_off + m * sizeof(unsigned), &acc, sizeof(unsigned));
        if (m < g.members.size()) {
          const DescLaunch &l = p.seqs[g.members[m].first][g.members[m].second];
          acc += l.grid;
          g.shmem = std::max(g.shmem, l.shmem);
        }
      }
      g.blocks = acc;
    }
  if (tab.empty()) return CPAL_OK;
  if (b->al.alloc) p.mem = b->al.alloc(tab.size(), b->al.user);
  else if (hipMalloc(&p.mem, tab.size()) != hipSuccess) p.mem = nullptr;
  if (!p.mem) return CPAL_E_NOMEM;
  return hipMemcpy(p.mem, tab.data(), tab.size(), hipMemcpyHostToDevice) == hipSuccess
             ? CPAL_OK : CPAL_E_DEVICE;
}

// The rounds in order on streams[0] (batched launches) and the batch's other
// streams (solo launches, by decomposition), each round joined back into
// streams[0] before the next; capturable.
void plan_issue(cpal_batch *b, const StagePlan &p) {
  hipStream_t s0 = b->streams[0];
  const size_t ns = b->streams.size();
  for (const StageRound &r : p.rounds) {
    std::vector<char> used(ns, 0);
    if (!r.solos.empty() && ns > 1) {
      hipEventRecord(b->start, s0);
      for (const auto &q : r.solos) {
        const size_t j = 1 + (size_t)q.first % (ns - 1);
        if (!used[j]) hipStreamWaitEvent(b->streams[j], b->start, 0);
        used[j] = 1;
      }
    }
    for (const auto &q : r.solos)
      p.seqs[q.first][q.second].solo(ns > 1 ? b->streams[1 + (size_t)q.first % (ns - 1)] : s0);
    for (const MultiGroup &g : r.groups)
      if (g.blocks > 0)
        g.ml((const unsigned char *)p.mem + g.packs_off,
             (const unsigned *)((const unsigned char *)p.mem + g.pre_off),
             (unsigned)g.members.size(), g.blocks, g.block, g.shmem, s0);
    for (size_t j = 1; j < ns; ++j)
      if (used[j]) {
        hipEventRecord(b->done[j], b->streams[j]);
        hipStreamWaitEvent(s0, b->done[j], 0);
      }
  }
}

cpal_status batch_stage_capture(cpal_batch *b, int mode) {
  const size_t n = b->ctx.size();
  // 1. describe every decomposition's update
  StagePlan p;
  p.seqs.resize(n);
  cpal_status res = CPAL_OK;
  for (size_t i = 0; i < n; ++i) {
    cpal_ctx *c = b->ctx[i];
    if (mode >= c->D) continue;
    const u64 t = c->t;
    const unsigned timing = c->timing;
    c->timing = 0;
    SeqSink sink;
    launch_sink() = &sink;
    const cpal_status st = cp_arls_lev_mode_update(c, mode, b->stats + i);
    launch_sink() = nullptr;
    c->timing = timing;
    c->t = t;
    if (st != CPAL_OK && res == CPAL_OK) res = st;
    p.seqs[i] = std::move(sink.seq);
  }
  if (res != CPAL_OK) return res;
  // 2. rounds and their tables (kept until the graph is dropped)
  drop_stage_graph(b, mode);
  res = plan_build(b, p);
  b->plan_mem[mode] = p.mem;
  if (res != CPAL_OK) return res;
  // 3. capture the rounds
  hipStream_t s0 = b->streams[0];
  if (hipStreamBeginCapture(s0, hipStreamCaptureModeRelaxed) != hipSuccess) return CPAL_E_DEVICE;
  plan_issue(b, p);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(s0, &g);
  if (e != hipSuccess || !g) return CPAL_E_DEVICE;
  b->kernels[1][mode] = kernel_nodes(g);
  if (hipGraphInstantiate(&b->exec2[mode], g, nullptr, nullptr, 0) != hipSuccess)
    res = CPAL_E_DEVICE;
  hipGraphDestroy(g);
  return res;
}

// Milliseconds per run of the gather stage of mode `mode` of every
// decomposition (with the launch shapes they hold), issued as stage-major
// rounds: M cleared, then the gather; the best of `reps` runs.  Runs on the
// sampled system each decomposition's last update_front left.
cpal_status time_batch_gathers(cpal_batch *b, int mode, int reps, double *ms) {
  const size_t n = b->ctx.size();
  StagePlan p;
  p.seqs.resize(n);
  for (size_t i = 0; i < n; ++i) {
    cpal_ctx *c = b->ctx[i];
    if (mode >= c->D || c->dense) continue;
    Mode &md = c->mode[mode];
    SeqSink sink;
    launch_sink() = &sink;
    launch_zero_words(c->M, (i64)m_copies(md.n) * md.n * c->ldz * (c->f64 ? 2 : 1), c->stream);
    update_gather(c, mode, md.g_grid, md.g_sort_min);
    launch_sink() = nullptr;
    p.seqs[i] = std::move(sink.seq);
  }
  cpal_status res = plan_build(b, p);
  if (res == CPAL_OK) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      res = CPAL_E_DEVICE;
    } else {
      double best = 1e30;
      for (int r = 0; r < reps; ++r) {
        hipEventRecord(e0, b->streams[0]);
        plan_issue(b, p);
        hipEventRecord(e1, b->streams[0]);
        float t = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
          res = CPAL_E_DEVICE;
          break;
        }
        best = std::min(best, (double)t);
      }
      *ms = best;
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  }
  for (hipStream_t st : b->streams) hipStreamSynchronize(st);
  plan_free(b, p);
  return res;
}

}  // namespace

extern "C" {

cpal_status cp_arls_lev_init_batch(int32_t m, const cpal_tensor *Xs, int32_t n,
                                   const int32_t *tensor_of, const cpal_options *opts,
                                   double *const *const *factors, void *hip_stream,
                                   const cpal_allocator *alloc, cpal_batch **out) {
  if (!out) return CPAL_E_ARG;
  *out = nullptr;
  if (m < 1 || n < 1 || !Xs || !tensor_of || !opts || !factors) return CPAL_E_ARG;
  if (alloc && (!alloc->alloc || !alloc->free)) return CPAL_E_ARG;
  for (int i = 0; i < n; ++i)
    if (tensor_of[i] < 0 || tensor_of[i] >= m || !factors[i]) return CPAL_E_ARG;
  cpal_batch *b = new cpal_batch();
  if (alloc) b->al = *alloc;
  b->user = (hipStream_t)hip_stream;
  const int ns = std::min(n, kBatchStreams);
  for (int j = 0; j < ns; ++j) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      if (s) hipStreamDestroy(s);
      batch_free(b);
      return CPAL_E_DEVICE;
    }
    b->streams.push_back(s);
    b->done.push_back(e);
  }
  if (hipEventCreateWithFlags(&b->start, hipEventDisableTiming) != hipSuccess) {
    batch_free(b);
    return CPAL_E_DEVICE;
  }
  {
    const size_t bytes = sizeof(cpal_mode_stats) * (size_t)n;
    void *p = nullptr;
    if (b->al.alloc) p = b->al.alloc(bytes, b->al.user);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (!p) {
      batch_free(b);
      return CPAL_E_NOMEM;
    }
    b->stats = (cpal_mode_stats *)p;
  }
  b->tensor_of.assign(tensor_of, tensor_of + n);
  // init runs on the batch streams after the caller's pending work
  batch_fork(b);
  std::vector<cpal_ctx *> owner(m, nullptr);
  b->ctx.assign(n, nullptr);
  for (int i = 0; i < n; ++i) {
    const int t = tensor_of[i];
    const cpal_status st = init_impl(&Xs[t], &opts[i], factors[i], b->streams[i % ns], alloc,
                                     owner[t], &b->ctx[i]);
    if (st != CPAL_OK) {
      batch_free(b);
      return st;
    }
    if (!owner[t]) owner[t] = b->ctx[i];
  }
  *out = b;
  return CPAL_OK;
}

cpal_status cp_arls_lev_mode_step_batch(cpal_batch *b, int32_t mode, cpal_mode_stats *stats_dev) {
  if (!b || mode < 0 || mode >= CPAL_MAXORDER) return CPAL_E_ARG;
  if (b->graphs) {
    hipGraphExec_t &ex = b->graphs == 2 ? b->exec2[mode] : b->exec[mode];
    if (!ex) {
      const cpal_status st = b->graphs == 2 ? batch_stage_capture(b, mode) : batch_capture(b, mode);
      if (st != CPAL_OK) return st;
    }
    hipEventRecord(b->start, b->user);
    hipStreamWaitEvent(b->streams[0], b->start, 0);
    if (hipGraphLaunch(ex, b->streams[0]) != hipSuccess) return CPAL_E_DEVICE;
    for (cpal_ctx *c : b->ctx)
      if (mode < c->D) {   // host state an eager step would have left
        c->t += 1;
        c->last_key_bits = c->mode[mode].key_bits;
        c->samples_valid = true;
      }
    hipEventRecord(b->done[0], b->streams[0]);
    hipStreamWaitEvent(b->user, b->done[0], 0);
    if (stats_dev)
      hipMemcpyAsync(stats_dev, b->stats, sizeof(cpal_mode_stats) * b->ctx.size(),
                     hipMemcpyDeviceToDevice, b->user);
    return hipGetLastError() == hipSuccess ? CPAL_OK : CPAL_E_DEVICE;
  }
  batch_fork(b);
  cpal_status res = CPAL_OK;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    cpal_ctx *c = b->ctx[i];
    if (mode >= c->D) continue;
    const cpal_status st = cp_arls_lev_mode_update(c, mode, stats_dev ? stats_dev + i : nullptr);
    if (st != CPAL_OK && res == CPAL_OK) res = st;
  }
  batch_join(b);
  return res;
}

cpal_status cp_arls_lev_fit_estimate_batch(cpal_batch *b, double *fits_dev) {
  if (!b || !fits_dev) return CPAL_E_ARG;
  batch_fork(b);
  cpal_status res = CPAL_OK;
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    const cpal_status st = cp_arls_lev_fit_estimate(b->ctx[i], fits_dev + i);
    if (st != CPAL_OK && res == CPAL_OK) res = st;
  }
  batch_join(b);
  return res;
}

cpal_status cp_arls_lev_autotune_batch(cpal_batch *b, int32_t reps) {
  if (!b) return CPAL_E_ARG;
  for (hipStream_t s : b->streams) hipStreamSynchronize(s);
  // tune the first decomposition of every tensor; the others of that tensor
  // (restarts: same shapes and sampled-fiber statistics) take its choice
  std::vector<int> tuned(b->ctx.size(), -1);
  for (size_t i = 0; i < b->ctx.size(); ++i) {
    int src = -1;
    for (size_t j = 0; j < i; ++j)
      if (b->tensor_of[j] == b->tensor_of[i] && tuned[j] == (int)j) { src = (int)j; break; }
    cpal_ctx *c = b->ctx[i];
    if (src < 0) {
      const cpal_status st = cp_arls_lev_autotune(c, reps);
      if (st != CPAL_OK) return st;
      tuned[i] = (int)i;
    } else {
      // a restart takes the tuned shapes; the bucketed gather needs its own
      // buffers, and where they cannot be had the restart keeps the default
      bool need_bkt = false, need_own = false, need_tile = false;
      for (int k = 0; k < c->D; ++k) {
        need_bkt |= b->ctx[src]->mode[k].g_sort_min == -1 || b->ctx[src]->mode[k].g_sort_min == -4;
        need_own |= b->ctx[src]->mode[k].g_sort_min == -2;
        need_tile |= b->ctx[src]->mode[k].g_sort_min == -3 || b->ctx[src]->mode[k].g_sort_min == -5;
        need_bkt |= b->ctx[src]->mode[k].g_sort_min == -5;
      }
      const bool bkt_ok = need_bkt && ensure_bucket_buffers(c) == CPAL_OK;
      const bool own_ok = need_own && ensure_owner_buffers(c) == CPAL_OK;
      const bool tile_ok = need_tile && ensure_tile_buffers(c) == CPAL_OK;
      for (int k = 0; k < c->D; ++k) {
        const int sm = b->ctx[src]->mode[k].g_sort_min;
        if ((sm == -1 && !(bkt_ok && bucket_capable(c, k))) ||
            (sm == -4 && !(bkt_ok && bucket_lds_capable(c, k))) ||
            (sm == -2 && !(own_ok && owner_capable(c, k))) ||
            (sm == -3 && !(tile_ok && tile_capable(c, k))) ||
            (sm == -5 && !(tile_ok && bkt_ok && tile_capable(c, k) && bucket_lds_capable(c, k)))) {
          c->mode[k].g_grid = 0;
          c->mode[k].g_sort_min = 0;
        } else {
          c->mode[k].g_grid = b->ctx[src]->mode[k].g_grid;
          c->mode[k].g_sort_min = sm;
        }
      }
      tuned[i] = src;
    }
  }
  // In a batch the decompositions' gathers run together (the stage-major
  // graph launches each gather kernel once for all of them), which the
  // per-tensor timings above (one decomposition alone) cannot see: forms whose
  // grids are small alone fill the chip in a batch.  Per mode, the gather
  // stage of all decompositions is timed as stage-major rounds with the shapes
  // chosen so far and with the shared-block bucketed gather in every mode that
  // takes it; the latter is kept when at least 3% faster.  The sampled systems
  // are those of one more update_front (the step counters are restored).
  cpal_status res = CPAL_OK;
  for (int k = 0; k < CPAL_MAXORDER && res == CPAL_OK; ++k) {
    bool any = false;
    for (cpal_ctx *c : b->ctx) any |= k < c->D && !c->dense;
    if (!any) continue;
    for (cpal_ctx *c : b->ctx)
      if (k < c->D) update_front(c, k);
    for (hipStream_t s : b->streams) hipStreamSynchronize(s);
    double t_kept = 0.0, t_bktl = 0.0;
    cpal_status st = time_batch_gathers(b, k, std::max(reps, 1) + 1, &t_kept);
    std::vector<std::pair<int, int>> saved(b->ctx.size());
    int switched = 0;
    for (size_t i = 0; i < b->ctx.size(); ++i) {
      cpal_ctx *c = b->ctx[i];
      if (k >= c->D || c->dense) continue;
      saved[i] = {c->mode[k].g_grid, c->mode[k].g_sort_min};
      if (st == CPAL_OK && c->mode[k].g_sort_min != -4 && ensure_bucket_buffers(c) == CPAL_OK &&
          bucket_lds_capable(c, k)) {
        c->mode[k].g_grid = 0;
        c->mode[k].g_sort_min = -4;
        ++switched;
      }
    }
    if (switched > 0) st = time_batch_gathers(b, k, std::max(reps, 1) + 1, &t_bktl);
    if (!(switched > 0 && st == CPAL_OK && t_bktl < 0.97 * t_kept))
      for (size_t i = 0; i < b->ctx.size(); ++i) {
        cpal_ctx *c = b->ctx[i];
        if (k >= c->D || c->dense) continue;
        c->mode[k].g_grid = saved[i].first;
        c->mode[k].g_sort_min = saved[i].second;
      }
    for (cpal_ctx *c : b->ctx) {
      launch_set_step(c->st, c->t, c->stream);
      c->samples_valid = false;
    }
    res = st;   // on an error the shapes chosen so far stay
  }
  // captured graphs hold the old launch shapes
  for (hipStream_t s : b->streams) hipStreamSynchronize(s);
  for (int m = 0; m < CPAL_MAXORDER; ++m) {
    if (b->exec[m]) hipGraphExecDestroy(b->exec[m]);
    b->exec[m] = nullptr;
    b->kernels[0][m] = 0;
    drop_stage_graph(b, m);
  }
  return res;
}

cpal_status cp_arls_lev_batch_set_graphs(cpal_batch *b, int32_t on) {
  if (!b) return CPAL_E_ARG;
  if (on < 0 || on > 2) return CPAL_E_ARG;
  b->graphs = on;
  return CPAL_OK;
}

cpal_status cp_arls_lev_batch_graph_kernels(const cpal_batch *b, int32_t kind, int32_t mode,
                                            int64_t *kernels) {
  if (!b || !kernels || kind < 1 || kind > 2 || mode < 0 || mode >= CPAL_MAXORDER)
    return CPAL_E_ARG;
  *kernels = b->kernels[kind - 1][mode];
  return CPAL_OK;
}

cpal_status cp_arls_lev_batch_ctx(const cpal_batch *b, int32_t i, cpal_ctx **ctx) {
  if (!b || !ctx || i < 0 || i >= (int32_t)b->ctx.size()) return CPAL_E_ARG;
  *ctx = b->ctx[i];
  return CPAL_OK;
}

void cp_arls_lev_destroy_batch(cpal_batch *b) {
  if (!b) return;
  for (hipStream_t s : b->streams) hipStreamSynchronize(s);
  batch_free(b);
}

}  // extern "C"
