"""Python face of the gfx950 CP-ARLS-LEV library (thin wrapper over the C ABI).

A :class:`CpArlsLev` owns one library context: a COO (or dense) tensor, FP64 factor
matrices on the device, and the options of Alg. 3 (rank R, samples s,
threshold tau, seed).  ``mode_update(k)`` runs one sampled least-squares
update of factor k entirely in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class TorchAllocator:
    """A cpal_allocator whose device memory comes from torch's caching
    allocator (on one device, associated with one stream).  It counts the
    calls and the live allocations, and must outlive every context using it."""

    def __init__(self, device=None, stream=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.device = dev.index if dev.index is not None else torch.cuda.current_device()
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.n_alloc = 0
        self.n_free = 0
        self.live = {}

        def _alloc(nbytes, user):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:   # out of memory: the library reports CPAL_E_NOMEM
                return None
            self.live[int(p)] = int(nbytes)
            self.n_alloc += 1
            return p

        def _free(ptr, user):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            finally:
                self.live.pop(int(ptr), None)
                self.n_free += 1

        self._fa = L.ALLOC_FN(_alloc)
        self._ff = L.FREE_FN(_free)
        self.struct = L.cpal_allocator(self._fa, self._ff, None)

    @property
    def live_bytes(self):
        return sum(self.live.values())


def _allocator_arg(allocator, device, stream):
    """(allocator object or None, pointer for the C call).  "torch": torch's
    caching allocator; None: the library's hipMalloc."""
    if allocator == "torch":
        allocator = TorchAllocator(device, stream)
    if allocator is None:
        return None, None
    return allocator, C.byref(allocator.struct)


def _check(code, ctx_ptr=None, contextless=False):
    if code != L.CPAL_OK:
        msg = ""
        if ctx_ptr or contextless:
            m = L.load().cp_arls_lev_last_error(ctx_ptr if ctx_ptr else None)
            msg = m.decode() if m else ""
        raise L.CpalError(code, msg)


def leverage_noalloc(A, out=None, stream=None):
    """Leverage scores of the rows of a CUDA FP64 n x R matrix through
    cp_arls_lev_leverage_noalloc (no allocation by the library; the scores a
    context keeps for the same factor matrix, bit for bit).  out: optional
    FP64 CUDA tensor of n entries."""
    assert A.is_cuda and A.dtype == torch.float64 and A.dim() == 2 and A.is_contiguous()
    if out is None:
        out = torch.empty(A.shape[0], dtype=torch.float64, device=A.device)
    code = L.load().cp_arls_lev_leverage_noalloc(A.data_ptr(), int(A.shape[0]), int(A.shape[1]),
                                                 out.data_ptr(), _stream_ptr(stream))
    _check(code, None, contextless=True)
    return out


class CpArlsLev:
    def __init__(self, dims, coords, values, factors, rank, samples, tau=None, seed=0,
                 stream_id=0, gather_dtype="f64", fit_samples=0, fit_alpha=0.5,
                 det_enum_cap=0, stream=None, allocator="torch", sampling="leverage"):
        lib = L.load()
        self.order = len(dims)
        self.dims = tuple(int(n) for n in dims)
        self.rank = int(rank)
        self.samples = int(samples)
        self.tau = (1.0 / samples if samples > 0 else 1.0) if tau is None else float(tau)
        if values.dtype not in (torch.float32, torch.float64) or not values.is_cuda:
            raise ValueError("values must be a float32/float64 CUDA tensor")
        self.dense = coords is None
        if self.dense:
            # every entry stored: values[i_0, ..., i_{D-1}] handed over with mode 0 fastest
            if tuple(values.shape) != self.dims:
                raise ValueError("a dense tensor (coords=None) must have shape dims")
            self.coords = None
            self.values = values.permute(*reversed(range(self.order))).contiguous().reshape(-1)
            self.nnz = 0
        else:
            if (coords.dtype != torch.int32 or not coords.is_cuda
                    or coords.shape[0] != self.order):
                raise ValueError("coords must be an int32 CUDA tensor of shape [order, nnz]")
            self.coords = coords.contiguous()
            self.values = values.contiguous()
            self.nnz = int(self.coords.shape[1])
        if len(factors) != self.order:
            raise ValueError("one factor matrix per mode")
        for m, f in enumerate(factors):
            if (f.dtype != torch.float64 or not f.is_cuda or not f.is_contiguous()
                    or tuple(f.shape) != (self.dims[m], self.rank)):
                raise ValueError(f"factor {m} must be a contiguous float64 CUDA tensor "
                                 f"of shape ({self.dims[m]}, {self.rank})")
        self.factors = list(factors)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._dims_c = (C.c_int64 * self.order)(*self.dims)
        t = L.cpal_tensor(self.order, self._dims_c, self.nnz,
                          self.coords.data_ptr() if self.coords is not None else None,
                          self.values.data_ptr(),
                          L.CPAL_F64 if self.values.dtype == torch.float64 else L.CPAL_F32,
                          1 if self.dense else 0)
        gdt = {"f64": L.CPAL_F64, "f32": L.CPAL_F32, "bf16": L.CPAL_BF16}[gather_dtype]
        self.gather_dtype = gather_dtype
        self.sampling = sampling
        o = L.cpal_options(self.rank, self.samples, self.tau, seed, stream_id, gdt,
                           int(fit_samples), float(fit_alpha), int(det_enum_cap),
                           L.SAMPLING[sampling], 0)
        fp = (C.c_void_p * self.order)(*[f.data_ptr() for f in self.factors])
        self._ctx = C.c_void_p()
        self.allocator, aptr = _allocator_arg(allocator, self.values.device, self.stream)
        code = lib.cp_arls_lev_init(C.byref(t), C.byref(o), fp, _stream_ptr(self.stream), aptr,
                                    C.byref(self._ctx))
        _check(code)
        self._stats = torch.zeros(L.STATS_BYTES // 8, dtype=torch.int64,
                                  device=self.values.device)

    # ---------------------------------------------------------------- calls
    def mode_update(self, k, stats=True, stats_buf=None):
        """One mode update of factor k.  stats_buf: optional int64 CUDA tensor
        of >= 7 entries receiving this update's cpal_mode_stats."""
        if stats_buf is not None:
            ptr = C.c_void_p(stats_buf.data_ptr())
        else:
            ptr = C.c_void_p(self._stats.data_ptr()) if stats else None
        _check(L.load().cp_arls_lev_mode_update(self._ctx, int(k), ptr), self._ctx)

    @staticmethod
    def parse_stats(buf):
        """Decode a cpal_mode_stats held in an int64 tensor (host or device)."""
        b = buf.detach().cpu().contiguous()
        v = b.numpy()
        f = b.view(torch.float64).numpy()
        i32 = b.view(torch.int32).numpy()
        return dict(s_det=int(v[0]), s_rnd=int(v[1]), s_bar=int(v[2]), draws=int(v[3]),
                    gathered_nnz=int(v[4]), p_det=float(f[5]), flags=int(i32[12]))

    def set_timing(self, on=True, stages=None):
        """Time every stage (on=True), none (on=False) or the named stages
        (stages = iterable of names from STAGES)."""
        if stages is not None:
            mask = 0
            for name in stages:
                mask |= 1 << L.STAGES.index(name)
        else:
            mask = (1 << len(L.STAGES)) - 1 if on else 0
        _check(L.load().cp_arls_lev_set_timing(self._ctx, mask), self._ctx)

    def stage_times(self, reset=True):
        """{stage: (ms_total, count)} of the timed updates (synchronizes)."""
        ms = (C.c_double * 5)()
        cnt = (C.c_int64 * 5)()
        _check(L.load().cp_arls_lev_stage_times(self._ctx, ms, cnt, 1 if reset else 0), self._ctx)
        return {name: (ms[i], cnt[i]) for i, name in enumerate(L.STAGES)}

    def last_stats(self):
        """Stats of the last mode_update (synchronizes)."""
        return self.parse_stats(self._stats)

    def samples_view(self):
        """(idx uint64 as int64, omega, w) of the last update, s_bar rows (synchronizes)."""
        dev = self.values.device
        idx = torch.empty(self.samples, dtype=torch.int64, device=dev)
        om = torch.empty(self.samples, dtype=torch.float64, device=dev)
        w = torch.empty(self.samples, dtype=torch.float64, device=dev)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        _check(L.load().cp_arls_lev_samples(self._ctx, idx.data_ptr(), om.data_ptr(), w.data_ptr(),
                                            self.samples, cnt.data_ptr()), self._ctx)
        n = int(cnt.item())
        return idx[:n], om[:n], w[:n]

    def leverage(self, m):
        out = torch.empty(self.dims[m], dtype=torch.float64, device=self.values.device)
        _check(L.load().cp_arls_lev_leverage(self._ctx, int(m), out.data_ptr()), self._ctx)
        return out

    def refresh(self, m):
        _check(L.load().cp_arls_lev_refresh(self._ctx, int(m)), self._ctx)

    def set_gather_config(self, k, grid=0, sort_min=0):
        """Launch shape of mode k's gather (grid 0: default; sort_min >= 0:
        segmented gather, chunks spanning at most this many fibers skip the
        row sort; -1 bucketed, -2 owner, -3 tile, -4 bucketed with
        shared-memory buckets, -5 tile for long fibers + -4 for the rest, grid
        = the long-fiber factor)."""
        _check(L.load().cp_arls_lev_set_gather_config(self._ctx, int(k), int(grid),
                                                       int(sort_min)), self._ctx)

    def gather_config(self, k):
        g, sm = C.c_int32(0), C.c_int32(0)
        _check(L.load().cp_arls_lev_get_gather_config(self._ctx, int(k), C.byref(g),
                                                       C.byref(sm)), self._ctx)
        return g.value, sm.value

    def autotune(self, reps=2):
        """Time the gather launch shapes of every mode on this decomposition's
        current state and keep the fastest (factors and step unchanged).
        Returns [(grid, sort_min)] per mode."""
        _check(L.load().cp_arls_lev_autotune(self._ctx, int(reps)), self._ctx)
        return [self.gather_config(k) for k in range(self.order)]

    def rrf_init(self, s_init, omega):
        """Randomized range finder initialisation (App. F): every factor is
        overwritten by a random linear combination of s_init uniformly drawn
        nonempty fibers, omega[k] (a CUDA FP64 s_init x R tensor per mode)
        holding the combination weights."""
        assert len(omega) == self.order
        for o in omega:
            assert o.is_cuda and o.dtype == torch.float64 and o.is_contiguous()
            assert o.shape[0] >= s_init and o.shape[1] == self.rank
        ptrs = (C.c_void_p * self.order)(*[o.data_ptr() for o in omega])
        _check(L.load().cp_arls_lev_rrf_init(self._ctx, int(s_init), ptrs), self._ctx)

    def fit_estimate(self, out=None):
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.values.device)
        _check(L.load().cp_arls_lev_fit_estimate(self._ctx, out.data_ptr()), self._ctx)
        return out

    def fit_exact(self, out=None):
        """Exact fit of the current factors (eq. (6.1)), on the device."""
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.values.device)
        _check(L.load().cp_arls_lev_fit_exact(self._ctx, out.data_ptr()), self._ctx)
        return out

    def run(self, eta=5, pi=3, tol=1e-4, max_epochs=100, exact_fit=False):
        """CP-ARLS-LEV (Alg. 3) until pi epochs of eta iterations fail to
        improve the fit by more than tol.  Returns a dict: trace (fit after
        each epoch), epochs, stopped, best_fit, final_exact_fit and, for the
        estimated fit, the bias-corrected trace (shifted so that its last
        entry equals the final exact fit)."""
        import numpy as np
        ro = L.cpal_run_options(int(eta), int(pi), float(tol), int(max_epochs),
                                1 if exact_fit else 0)
        trace = (C.c_double * int(max_epochs))()
        res = L.cpal_run_result()
        _check(L.load().cp_arls_lev_run(self._ctx, C.byref(ro), trace, C.byref(res)), self._ctx)
        tr = np.array(trace[:res.epochs])
        out = dict(trace=tr, epochs=res.epochs, stopped=bool(res.stopped), best_fit=res.best_fit,
                   final_exact_fit=res.final_exact_fit)
        if not exact_fit and res.epochs > 0:
            out["trace_bias_corrected"] = tr - (tr[-1] - res.final_exact_fit)
        return out

    @property
    def step(self):
        t = C.c_uint64(0)
        _check(L.load().cp_arls_lev_get_step(self._ctx, C.byref(t)), self._ctx)
        return t.value

    @step.setter
    def step(self, t):
        _check(L.load().cp_arls_lev_set_step(self._ctx, int(t)), self._ctx)

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            L.load().cp_arls_lev_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Member(CpArlsLev):
    """One decomposition of a CpArlsLevBatch (samples, leverage, step
    counter); the batch owns the context."""

    def __init__(self, ptr, dims, rank, samples, device):
        self._ctx = C.c_void_p(ptr)
        self.order = len(dims)
        self.dims = tuple(dims)
        self.rank = rank
        self.samples = samples
        self.values = torch.empty(0, device=device)
        self._stats = torch.zeros(L.STATS_BYTES // 8, dtype=torch.int64, device=device)

    # the context's work runs on one of the batch's streams: synchronize the
    # device before reading what the library wrote
    def samples_view(self):
        dev = self.values.device
        idx = torch.empty(self.samples, dtype=torch.int64, device=dev)
        om = torch.empty(self.samples, dtype=torch.float64, device=dev)
        w = torch.empty(self.samples, dtype=torch.float64, device=dev)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        torch.cuda.synchronize()
        _check(L.load().cp_arls_lev_samples(self._ctx, idx.data_ptr(), om.data_ptr(), w.data_ptr(),
                                            self.samples, cnt.data_ptr()), self._ctx)
        torch.cuda.synchronize()
        n = int(cnt.item())
        return idx[:n], om[:n], w[:n]

    def leverage(self, m):
        out = torch.empty(self.dims[m], dtype=torch.float64, device=self.values.device)
        torch.cuda.synchronize()
        _check(L.load().cp_arls_lev_leverage(self._ctx, int(m), out.data_ptr()), self._ctx)
        torch.cuda.synchronize()
        return out

    def close(self):
        self._ctx = C.c_void_p()


class CpArlsLevBatch:
    """Many independent decompositions (restarts, tensors of different shape
    and rank) stepped together: ``mode_step(k)`` updates mode k of every
    decomposition whose tensor has more than k modes.

    tensors: list of (dims, coords or None, values) as for CpArlsLev;
    tensor_of[i]: the tensor of decomposition i; factors[i]: its FP64 factor
    matrices; ranks, samples, taus, seeds, stream_ids: per decomposition
    (scalars broadcast)."""

    def __init__(self, tensors, tensor_of, factors, ranks, samples, taus=None, seeds=0,
                 stream_ids=0, gather_dtype="f32", fit_samples=0, fit_alpha=0.5,
                 det_enum_cap=0, stream=None, use_graphs=False, allocator="torch",
                 sampling="leverage"):
        lib = L.load()
        n = len(tensor_of)
        per = lambda v: list(v) if isinstance(v, (list, tuple)) else [v] * n
        ranks, samples, seeds, stream_ids = per(ranks), per(samples), per(seeds), per(stream_ids)
        taus = [1.0 / s for s in samples] if taus is None else per(taus)
        self._keep = []
        tens = (L.cpal_tensor * len(tensors))()
        self.tdims = []
        for t, (dims, coords, values) in enumerate(tensors):
            dims = tuple(int(x) for x in dims)
            self.tdims.append(dims)
            if coords is None:
                vals = values.permute(*reversed(range(len(dims)))).contiguous().reshape(-1)
                crd, nnz, dense = None, 0, 1
            else:
                crd, vals = coords.contiguous(), values.contiguous()
                nnz, dense = int(crd.shape[1]), 0
            dc = (C.c_int64 * len(dims))(*dims)
            self._keep += [dc, crd, vals]
            tens[t] = L.cpal_tensor(len(dims), dc, nnz, crd.data_ptr() if crd is not None else None,
                                    vals.data_ptr(),
                                    L.CPAL_F64 if vals.dtype == torch.float64 else L.CPAL_F32,
                                    dense)
            self.device = vals.device
        gdt = {"f64": L.CPAL_F64, "f32": L.CPAL_F32, "bf16": L.CPAL_BF16}[gather_dtype]
        opts = (L.cpal_options * n)()
        fptrs = (C.c_void_p * n)()
        self.factors = [list(f) for f in factors]
        for i in range(n):
            opts[i] = L.cpal_options(int(ranks[i]), int(samples[i]), float(taus[i]), int(seeds[i]),
                                     int(stream_ids[i]), gdt, int(fit_samples), float(fit_alpha),
                                     int(det_enum_cap), L.SAMPLING[sampling], 0)
            arr = (C.c_void_p * len(self.factors[i]))(*[f.data_ptr() for f in self.factors[i]])
            self._keep.append(arr)
            fptrs[i] = C.cast(arr, C.c_void_p)
        tof = (C.c_int32 * n)(*[int(t) for t in tensor_of])
        self.tensor_of = list(tensor_of)
        self.ranks, self.samples = ranks, samples
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._b = C.c_void_p()
        self.allocator, aptr = _allocator_arg(allocator, self.device, self.stream)
        _check(lib.cp_arls_lev_init_batch(len(tensors), tens, n, tof, opts, fptrs,
                                          _stream_ptr(self.stream), aptr, C.byref(self._b)))
        self.n = n
        self._stats = torch.zeros((n, L.STATS_BYTES // 8), dtype=torch.int64, device=self.device)
        if use_graphs:
            self.set_graphs(use_graphs)

    def autotune(self, reps=2):
        """cp_arls_lev_autotune_batch: tune the first decomposition of every
        tensor, the restarts take its launch shapes."""
        _check(L.load().cp_arls_lev_autotune_batch(self._b, int(reps)))

    def set_graphs(self, on):
        """on: each later mode step replays the HIP graph captured for that
        mode on its first step.  True or 1: every decomposition's kernels as
        a branch of the graph; "stages" or 2: stage-major (one launch per
        stage for all decompositions where the kernel has a batched form);
        False or 0: kernels launched step by step."""
        kind = 2 if on in ("stages", 2) else (1 if on else 0)
        _check(L.load().cp_arls_lev_batch_set_graphs(self._b, kind))

    def graph_kernels(self, k, kind=2):
        """Kernel launches in the captured graph of mode k (kind 1: branches,
        2: stage-major; 0 while none is captured)."""
        out = C.c_int64()
        _check(L.load().cp_arls_lev_batch_graph_kernels(self._b, int(kind), int(k), C.byref(out)))
        return out.value

    def mode_step(self, k, stats_buf=None):
        """Update mode k of every decomposition (whose tensor has > k modes);
        stats_buf: optional int64 CUDA tensor (n, >= 7) for the statistics."""
        buf = stats_buf if stats_buf is not None else self._stats
        _check(L.load().cp_arls_lev_mode_step_batch(self._b, int(k), C.c_void_p(buf.data_ptr())))

    def fit_estimate(self, out=None):
        if out is None:
            out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(L.load().cp_arls_lev_fit_estimate_batch(self._b, C.c_void_p(out.data_ptr())))
        return out

    def member(self, i):
        p = C.c_void_p()
        _check(L.load().cp_arls_lev_batch_ctx(self._b, int(i), C.byref(p)))
        return _Member(p.value, self.tdims[self.tensor_of[i]], self.ranks[i], self.samples[i],
                       self.device)

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            L.load().cp_arls_lev_destroy_batch(self._b)
            self._b = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
