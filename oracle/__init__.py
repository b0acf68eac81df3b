"""ctypes wrapper around the FP64 CPU oracle (``cpal_oracle.c``).

TEST INFRASTRUCTURE ONLY: used by ``tests/``, the smoke check and the
benchmark's CPU baseline.  The product library never imports it.

The shared object is compiled with gcc (``-O2 -ffp-contract=off``) by
``build()`` and, if missing, on first use.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpal_oracle.c")
_SO = os.path.join(_HERE, "libcpal_oracle.so")
_lib = None

FLAG_PINV, FLAG_DETCAP, FLAG_DET_TRUNC, FLAG_PDET_ONE, FLAG_DRAWCAP = 1, 2, 4, 8, 16


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-Wall",
                               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Tensor(C.Structure):
    _fields_ = [("order", C.c_int32), ("dims", C.POINTER(C.c_int64)), ("nnz", C.c_int64),
                ("coords", C.POINTER(C.c_int32)), ("vals", C.POINTER(C.c_double))]


class _Opts(C.Structure):
    _fields_ = [("rank", C.c_int32), ("samples", C.c_int64), ("tau", C.c_double),
                ("seed", C.c_uint64), ("stream_id", C.c_uint64), ("det_cap", C.c_int64),
                ("sampling", C.c_int32), ("pad", C.c_int32)]

SAMPLING = {"leverage": 0, "uniform": 1, "length_squared": 2}


class _Stats(C.Structure):
    _fields_ = [("s_det", C.c_int64), ("s_rnd", C.c_int64), ("s_bar", C.c_int64),
                ("draws", C.c_int64), ("gathered_nnz", C.c_int64), ("p_det", C.c_double),
                ("flags", C.c_int32), ("pad", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_SO)
        P = C.POINTER
        L.orc_philox4x64_10.argtypes = [P(C.c_uint64), P(C.c_uint64), P(C.c_uint64)]
        L.orc_scale128.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        L.orc_scale128.restype = C.c_uint64
        L.orc_upper_bound.argtypes = [P(C.c_uint64), C.c_int64, C.c_uint64]
        L.orc_upper_bound.restype = C.c_int64
        L.orc_gram.argtypes = [P(C.c_double), C.c_int64, C.c_int32, P(C.c_double)]
        L.orc_leverage.argtypes = [P(C.c_double), C.c_int64, C.c_int32, P(C.c_double)]
        L.orc_leverage.restype = C.c_int32
        L.orc_sampling_vectors.argtypes = [P(C.c_double), C.c_int64, C.c_int32,
                                           P(C.c_uint64), P(C.c_uint64), P(C.c_double)]
        L.orc_sampling_vectors.restype = C.c_uint64
        L.orc_scores.argtypes = [P(C.c_double), C.c_int64, C.c_int32, C.c_int32, P(C.c_double)]
        L.orc_scores.restype = C.c_double
        L.orc_sampling_vectors_norm.argtypes = [P(C.c_double), C.c_int64, C.c_double,
                                                P(C.c_uint64), P(C.c_uint64), P(C.c_double)]
        L.orc_sampling_vectors_norm.restype = C.c_uint64
        L.orc_index_build.argtypes = [P(_Tensor)]
        L.orc_index_build.restype = C.c_void_p
        L.orc_index_free.argtypes = [C.c_void_p]
        L.orc_det_set.argtypes = [C.c_int32, P(C.c_int64), P(P(C.c_double)), C.c_int32,
                                  C.c_int64, C.c_double, C.c_int64, P(C.c_uint64),
                                  P(C.c_double), C.c_int64, P(C.c_double), P(C.c_int32)]
        L.orc_det_set.restype = C.c_int64
        L.orc_mode_update.argtypes = [P(_Tensor), C.c_void_p, P(P(C.c_double)), P(_Opts),
                                      C.c_int32, C.c_uint64, P(C.c_uint64), P(C.c_double),
                                      P(C.c_double), P(C.c_uint64), P(_Stats)]
        L.orc_mode_update.restype = C.c_int32
        L.orc_fit_exact.argtypes = [P(_Tensor), P(P(C.c_double)), C.c_int32]
        L.orc_fit_exact.restype = C.c_double
        L.orc_fit_sample.argtypes = [P(_Tensor), C.c_uint64, C.c_uint64, C.c_int64, C.c_double,
                                     P(C.c_int32), P(C.c_double), P(C.c_double), C.c_int64,
                                     P(C.c_int32)]
        L.orc_fit_sample.restype = C.c_int64
        L.orc_fit_estimate.argtypes = [C.c_int32, C.c_int64, P(C.c_int32), C.c_int64,
                                       P(C.c_double), P(C.c_double), P(P(C.c_double)),
                                       C.c_int32, C.c_double]
        L.orc_fit_estimate.restype = C.c_double
        L.orc_model_entry.argtypes = [C.c_int32, P(P(C.c_double)), C.c_int32, P(C.c_int32)]
        L.orc_model_entry.restype = C.c_double
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Threads of the oracle's independent loops (1 = the sequential loops);
    every sum keeps its sequential order, so results do not depend on n."""
    L = lib()
    L.orc_set_threads.argtypes = [C.c_int32]
    L.orc_set_threads(int(n))


def get_threads() -> int:
    L = lib()
    L.orc_get_threads.restype = C.c_int32
    return int(L.orc_get_threads())


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c, C.c_uint64), _p(k, C.c_uint64), _p(out, C.c_uint64))
    return out


def scale128(u0, u1, W):
    return int(lib().orc_scale128(int(u0), int(u1), int(W)))


def upper_bound(Cdf, v):
    c = np.ascontiguousarray(Cdf, dtype=np.uint64)
    return int(lib().orc_upper_bound(_p(c, C.c_uint64), c.size, int(v)))


def gram(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n, R = A.shape
    G = np.zeros((R, R))
    lib().orc_gram(_p(A, C.c_double), n, R, _p(G, C.c_double))
    return G


def leverage(A):
    """Returns (lev, flags)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n, R = A.shape
    lev = np.zeros(n)
    fl = lib().orc_leverage(_p(A, C.c_double), n, R, _p(lev, C.c_double))
    return lev, int(fl)


def sampling_vectors(lev, R):
    """Returns (w, C, q, W)."""
    lev = np.ascontiguousarray(lev, dtype=np.float64)
    n = lev.size
    w = np.zeros(n, dtype=np.uint64)
    Cdf = np.zeros(n, dtype=np.uint64)
    q = np.zeros(n)
    W = lib().orc_sampling_vectors(_p(lev, C.c_double), n, R, _p(w, C.c_uint64),
                                   _p(Cdf, C.c_uint64), _p(q, C.c_double))
    return w, Cdf, q, int(W)


def scores(A, kind):
    """Row scores of App. B's distributions: returns (score, total)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n, R = A.shape
    sc = np.zeros(n)
    S = lib().orc_scores(_p(A, C.c_double), n, R, SAMPLING[kind] if isinstance(kind, str) else kind,
                         _p(sc, C.c_double))
    return sc, float(S)


def sampling_vectors_norm(score, S):
    """(w, C, q, W) with the scores normalised by S."""
    score = np.ascontiguousarray(score, dtype=np.float64)
    n = score.size
    w = np.zeros(n, dtype=np.uint64)
    Cdf = np.zeros(n, dtype=np.uint64)
    q = np.zeros(n)
    W = lib().orc_sampling_vectors_norm(_p(score, C.c_double), n, S, _p(w, C.c_uint64),
                                        _p(Cdf, C.c_uint64), _p(q, C.c_double))
    return w, Cdf, q, int(W)


def det_set(dims, qs, k, s, tau, det_cap=1 << 26, cap=None):
    """Returns (idx, p, p_det, flags)."""
    order = len(dims)
    d = np.ascontiguousarray(dims, dtype=np.int64)
    qarr = [np.ascontiguousarray(q if q is not None else np.zeros(1), dtype=np.float64) for q in qs]
    qp = (C.POINTER(C.c_double) * order)(*[_p(q, C.c_double) for q in qarr])
    cap = s if cap is None else cap
    idx = np.zeros(max(cap, 1), dtype=np.uint64)
    p = np.zeros(max(cap, 1))
    pdet = C.c_double(0)
    fl = C.c_int32(0)
    n = lib().orc_det_set(order, _p(d, C.c_int64), qp, k, s, tau, det_cap, _p(idx, C.c_uint64),
                          _p(p, C.c_double), cap, C.byref(pdet), C.byref(fl))
    if n < 0:
        raise RuntimeError("det_set capacity too small")
    return idx[:n].copy(), p[:n].copy(), pdet.value, fl.value


class Tensor:
    """Oracle-side COO tensor with its per-mode fiber index."""

    def __init__(self, dims, coords, values):
        self.dims = np.ascontiguousarray(dims, dtype=np.int64)
        self.coords = np.ascontiguousarray(coords, dtype=np.int32)
        self.vals = np.ascontiguousarray(values, dtype=np.float64)
        self.order = len(dims)
        self.nnz = self.coords.shape[1]
        self._c = _Tensor(self.order, _p(self.dims, C.c_int64), self.nnz,
                          _p(self.coords, C.c_int32), _p(self.vals, C.c_double))
        self._ix = None

    @classmethod
    def from_synth(cls, T):
        return cls(T.dims, T.coords, T.values)

    @property
    def index(self):
        if self._ix is None:
            self._ix = lib().orc_index_build(C.byref(self._c))
            if not self._ix:
                raise RuntimeError("oracle index build failed")
        return self._ix

    def __del__(self):
        if getattr(self, "_ix", None):
            try:
                lib().orc_index_free(self._ix)
            except Exception:
                pass
            self._ix = None

    @property
    def norm(self):
        return float(np.sqrt(np.sum(self.vals * self.vals)))


def _fac_ptrs(factors):
    for f in factors:
        assert f.dtype == np.float64 and f.flags["C_CONTIGUOUS"]
    return (C.POINTER(C.c_double) * len(factors))(*[_p(f, C.c_double) for f in factors])


def mode_update(T: Tensor, factors, k, t, rank, samples, tau=None, seed=0, stream_id=0,
                det_cap=1 << 26, sampling="leverage"):
    """One mode update, in place on factors[k].  Returns a dict with idx, omega,
    wgt (the s_bar sampled rows), raw (accepted random draws, draw order) and
    the stats."""
    if tau is None:
        tau = 1.0 / samples
    opts = _Opts(rank, samples, tau, seed, stream_id, det_cap, SAMPLING[sampling], 0)
    idx = np.zeros(samples, dtype=np.uint64)
    om = np.zeros(samples)
    wg = np.zeros(samples)
    raw = np.zeros(samples, dtype=np.uint64)
    st = _Stats()
    rc = lib().orc_mode_update(C.byref(T._c), T.index, _fac_ptrs(factors), C.byref(opts), k, t,
                               _p(idx, C.c_uint64), _p(om, C.c_double), _p(wg, C.c_double),
                               _p(raw, C.c_uint64), C.byref(st))
    if rc != 0:
        raise RuntimeError(f"oracle mode_update failed rc={rc}")
    sb = st.s_bar
    stats = dict(s_det=st.s_det, s_rnd=st.s_rnd, s_bar=sb, draws=st.draws,
                 gathered_nnz=st.gathered_nnz, p_det=st.p_det, flags=st.flags)
    return dict(idx=idx[:sb].copy(), omega=om[:sb].copy(), wgt=wg[:sb].copy(),
                raw=raw[:st.s_rnd].copy(), stats=stats)


def rrf_init(T: Tensor, k, s_init, omega, seed=0, stream_id=0):
    """Randomized range finder initial factor of mode k (App. F): the sum
    over s_init uniform draws of nonempty mode-k fibers of the fiber times
    the draw's row of omega (s_init x R, given).  Returns (A, nfib)."""
    L = lib()
    L.orc_rrf_init.argtypes = [C.POINTER(_Tensor), C.c_void_p, C.c_int32, C.c_int64,
                               C.c_void_p, C.c_int32, C.c_uint64, C.c_uint64, C.c_void_p]
    L.orc_rrf_init.restype = C.c_int64
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    R = omega.shape[1]
    assert omega.shape[0] >= s_init
    A = np.zeros((int(T.dims[k]), R))
    nfib = L.orc_rrf_init(C.byref(T._c), T.index, int(k), int(s_init), omega.ctypes.data, R,
                          int(seed), int(stream_id), A.ctypes.data)
    return A, int(nfib)


def fit_exact(T: Tensor, factors, rank):
    return float(lib().orc_fit_exact(C.byref(T._c), _fac_ptrs(factors), rank))


def model_entry(factors, coord):
    c = np.ascontiguousarray(coord, dtype=np.int32)
    R = factors[0].shape[1]
    return float(lib().orc_model_entry(len(factors), _fac_ptrs(factors), R, _p(c, C.c_int32)))


class FitSample:
    def __init__(self, T: Tensor, s_fit, alpha=0.5, seed=0, stream_id=0):
        cap = int(s_fit) + 1
        self.order = T.order
        self.coords = np.zeros((T.order, cap), dtype=np.int32)
        self.x = np.zeros(cap)
        self.phi = np.zeros(cap)
        fl = C.c_int32(0)
        n = lib().orc_fit_sample(C.byref(T._c), seed, stream_id, s_fit, alpha,
                                 _p(self.coords, C.c_int32), _p(self.x, C.c_double),
                                 _p(self.phi, C.c_double), cap, C.byref(fl))
        if n < 0:
            raise RuntimeError("oracle fit_sample failed")
        self.n = int(n)
        self.cap = cap
        self.flags = fl.value
        self.normX = T.norm

    def estimate(self, factors):
        R = factors[0].shape[1]
        return float(lib().orc_fit_estimate(self.order, self.n, _p(self.coords, C.c_int32),
                                            self.cap, _p(self.x, C.c_double),
                                            _p(self.phi, C.c_double), _fac_ptrs(factors), R,
                                            self.normX))


def cp_arls_lev(T: Tensor, factors, rank, samples, iters, tau=None, seed=0, stream_id=0,
                det_cap=1 << 26, t0=0):
    """Outer iterations of Alg. 3 (fixed count, modes in ascending order);
    factors are updated in place.  Returns the list of per-update stats."""
    t = t0
    log = []
    for _ in range(iters):
        for k in range(T.order):
            out = mode_update(T, factors, k, t, rank, samples, tau, seed, stream_id, det_cap)
            log.append(out["stats"])
            t += 1
    return log


def cp_arls_lev_run(T: Tensor, factors, rank, samples, eta=5, pi=3, tol=1e-4, max_epochs=100,
                    tau=None, seed=0, stream_id=0, fit_sample=None, det_cap=1 << 26, t0=0):
    """The full loop of Alg. 3: epochs of eta outer iterations (every mode
    once per iteration, ascending), the fit after each epoch -- the estimate
    of Sec. 6.4 from `fit_sample` (a FitSample drawn once), or the exact fit
    when it is None -- and the stop when pi consecutive epochs fail to beat
    the best earlier fit by more than tol (or after max_epochs).  Factors are
    updated in place; the step counter starts at t0 and advances by one per
    mode update.  Returns dict(trace, epochs, stopped, best_fit,
    final_exact_fit)."""
    t = t0
    trace = []
    best = -np.inf
    fails = 0
    stopped = False
    while len(trace) < max_epochs:
        for _ in range(eta):
            for k in range(T.order):
                mode_update(T, factors, k, t, rank, samples, tau, seed, stream_id, det_cap)
                t += 1
        fit = fit_sample.estimate(factors) if fit_sample is not None else fit_exact(T, factors, rank)
        trace.append(fit)
        fails = 0 if fit > best + tol else fails + 1
        best = max(best, fit)
        if fails >= pi:
            stopped = True
            break
    return dict(trace=np.array(trace), epochs=len(trace), stopped=stopped, best_fit=best,
                final_exact_fit=fit_exact(T, factors, rank))
