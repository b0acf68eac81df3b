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


def _check(code, ctx_ptr=None):
    if code != L.CPAL_OK:
        msg = ""
        if ctx_ptr:
            m = L.load().cp_arls_lev_last_error(ctx_ptr)
            msg = m.decode() if m else ""
        raise L.CpalError(code, msg)


class CpArlsLev:
    def __init__(self, dims, coords, values, factors, rank, samples, tau=None, seed=0,
                 stream_id=0, gather_dtype="f64", fit_samples=0, fit_alpha=0.5,
                 det_enum_cap=0, stream=None):
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
        o = L.cpal_options(self.rank, self.samples, self.tau, seed, stream_id, gdt,
                           int(fit_samples), float(fit_alpha), int(det_enum_cap))
        fp = (C.c_void_p * self.order)(*[f.data_ptr() for f in self.factors])
        self._ctx = C.c_void_p()
        code = lib.cp_arls_lev_init(C.byref(t), C.byref(o), fp, _stream_ptr(self.stream),
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

    def fit_estimate(self, out=None):
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.values.device)
        _check(L.load().cp_arls_lev_fit_estimate(self._ctx, out.data_ptr()), self._ctx)
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
