"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random data: COO coordinates, values and initial
factor matrices.  It contains none of the decomposition's arithmetic and is
shared, as data, by the HIP path, the CPU oracle, the tests and the bench.

Workloads (the real FROSTT tensors of Section 7 are not available, so these
stand in for them):

* ``small3``  -- 3-way 100x80x60, 20,000 distinct coordinates drawn uniformly
  without replacement, values from a planted rank-5 CP model (U(0,1) factor
  entries, unit 2-norm columns) plus N(0, 0.01^2) noise; R = 5.
* ``uber4``   -- 4-way 183x24x1140x1717 (the shape of the Uber tensor of
  Section 7.3), 3.3e6 distinct coordinates with Zipf(1.1) indices per mode,
  values log(1 + c) with c ~ Poisson(3) conditioned on c >= 1; R = 25.
* ``planted`` -- any shape, every entry stored (dense as COO) or a random
  subset, planted rank-R model plus relative Gaussian noise; used for
  recovery tests.
* ``coherent`` -- the dense tensor of App. C: N(0,1) factors whose first
  three columns are zero except `spread` rows each (distinct rows, value
  `magnitude` + U(0, jitter)), so that a few rows carry most of the leverage;
  the rank-R model plus relative Gaussian noise, every entry stored.

Zipf(a) on {0..n-1}: P(i) proportional to (i+1)^-a, then mapped through a
seeded random permutation so that hot indices are scattered.  Distinct
coordinates: draws are taken in order, the first occurrence of each
coordinate is kept, and generation stops at the target count.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class SparseTensor:
    dims: tuple            # n_0..n_{D-1}
    coords: np.ndarray     # int32 [D, nnz], 0-based, distinct
    values: np.ndarray     # float64 [nnz]

    @property
    def order(self) -> int:
        return len(self.dims)

    @property
    def nnz(self) -> int:
        return int(self.coords.shape[1])


def _full_keys(coords: np.ndarray, dims) -> np.ndarray:
    """Column-major linear index over all modes (first mode fastest)."""
    key = np.zeros(coords.shape[1], dtype=np.uint64)
    stride = 1
    for m, n in enumerate(dims):
        key += coords[m].astype(np.uint64) * np.uint64(stride)
        stride *= int(n)
    return key


def _zipf_sampler(rng: np.random.Generator, n: int, a: float):
    w = np.arange(1, n + 1, dtype=np.float64) ** (-a)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    perm = rng.permutation(n).astype(np.int32)

    def draw(size: int) -> np.ndarray:
        u = rng.random(size)
        r = np.searchsorted(cdf, u, side="right")
        np.minimum(r, n - 1, out=r)
        return perm[r]
    return draw


def _distinct_first(dims, draw_batch, target: int, batch: int) -> np.ndarray:
    """Draw coordinate batches until `target` distinct ones exist; keep the
    first occurrence of each, in draw order."""
    chunks = []
    have = 0
    keys_seen = np.empty(0, dtype=np.uint64)
    while have < target:
        c = draw_batch(batch)
        chunks.append(c)
        allc = np.concatenate(chunks, axis=1)
        keys = _full_keys(allc, dims)
        _, first = np.unique(keys, return_index=True)
        have = first.size
        keys_seen = keys
        if len(chunks) > 4096:
            raise RuntimeError("coordinate generator did not reach the target count")
    allc = np.concatenate(chunks, axis=1)
    _, first = np.unique(keys_seen, return_index=True)
    first.sort()
    return np.ascontiguousarray(allc[:, first[:target]]).astype(np.int32)


def gaussian_factors(dims, rank: int, seed: int):
    """Initial guesses with N(0,1) entries (Section 7 setup)."""
    rng = np.random.default_rng([seed, 0x1F])
    return [rng.standard_normal((int(n), rank)) for n in dims]


def _planted_factors(rng, dims, rank, law="uniform"):
    fac = []
    for n in dims:
        if law == "uniform":
            a = rng.random((int(n), rank))
        else:
            a = rng.standard_normal((int(n), rank))
        a /= np.linalg.norm(a, axis=0, keepdims=True)
        fac.append(a)
    return fac


def _model_at(fac, coords):
    """Entries of the planted CP model at the given coordinates."""
    prod = np.ones((coords.shape[1], fac[0].shape[1]))
    for m, a in enumerate(fac):
        prod *= a[coords[m]]
    return prod.sum(axis=1)


def small3(seed: int = 0, noise_std: float = 0.01):
    """100x80x60, 20,000 nnz, planted rank 5 (+ N(0, noise_std^2))."""
    dims = (100, 80, 60)
    rank = 5
    rng = np.random.default_rng([seed, 1])
    total = dims[0] * dims[1] * dims[2]
    lin = np.sort(rng.choice(total, size=20000, replace=False))
    coords = np.empty((3, lin.size), dtype=np.int32)
    rem = lin
    for m, n in enumerate(dims):
        coords[m] = rem % n
        rem = rem // n
    fac = _planted_factors(rng, dims, rank, "uniform")
    vals = _model_at(fac, coords) + noise_std * rng.standard_normal(lin.size)
    return SparseTensor(dims, coords, vals), fac, rank


def uber4(seed: int = 0, nnz: int = 3_300_000, a: float = 1.1):
    """183x24x1140x1717 Zipf(1.1) coordinates, log(1+c) values, c>=1."""
    dims = (183, 24, 1140, 1717)
    rng = np.random.default_rng([seed, 2])
    samplers = [_zipf_sampler(rng, n, a) for n in dims]

    def draw_batch(b):
        return np.stack([s(b) for s in samplers]).astype(np.int32)

    coords = _distinct_first(dims, draw_batch, nnz, batch=1 << 21)
    vals = _log1p_poisson_ge1(rng, 3.0, coords.shape[1])
    return SparseTensor(dims, coords, vals)


def _log1p_poisson_ge1(rng, lam, size):
    kmax = 64
    k = np.arange(1, kmax + 1)
    logp = -lam + k * math.log(lam) - np.cumsum(np.log(k))
    p = np.exp(logp)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    u = rng.random(size)
    c = np.searchsorted(cdf, u, side="right") + 1
    return np.log1p(c.astype(np.float64))


def planted(dims, rank: int, seed: int = 0, density: float = 1.0,
            rel_noise: float = 0.01, law: str = "uniform"):
    """Planted rank-`rank` model; `density` of all entries stored as COO.

    noise = rel_noise * ||model values|| / ||G|| * G with G ~ N(0,1)."""
    rng = np.random.default_rng([seed, 3])
    total = int(np.prod(dims))
    if density >= 1.0:
        lin = np.arange(total, dtype=np.int64)
    else:
        lin = np.sort(rng.choice(total, size=max(1, int(density * total)), replace=False))
    coords = np.empty((len(dims), lin.size), dtype=np.int32)
    rem = lin
    for m, n in enumerate(dims):
        coords[m] = rem % n
        rem = rem // n
    fac = _planted_factors(rng, dims, rank, law)
    clean = _model_at(fac, coords)
    g = rng.standard_normal(lin.size)
    vals = clean + rel_noise * (np.linalg.norm(clean) / np.linalg.norm(g)) * g
    return SparseTensor(tuple(int(n) for n in dims), coords, vals), fac


def coherent_factors(rng, dims, rank: int, spread: int = 5, magnitude: float = 3.0,
                     jitter: float = 0.05):
    """Factor matrices of App. C: N(0,1) entries; columns 0, 1, 2 zeroed, then
    column c gets magnitude + U(0, jitter) in rows [c spread, (c+1) spread)
    (every row has at most one nonzero among the three columns)."""
    fac = []
    for n in dims:
        a = rng.standard_normal((int(n), rank))
        a[:, :min(3, rank)] = 0.0
        for c in range(min(3, rank)):
            rows = slice(c * spread, (c + 1) * spread)
            a[rows, c] = magnitude + jitter * rng.random(spread)
        fac.append(a)
    return fac


def coherent(dims, rank: int = 25, spread: int = 5, magnitude: float = 3.0,
             jitter: float = 0.05, noise: float = 0.05, seed: int = 0):
    """App. C's dense test tensor on any shape: the rank-`rank` model of
    coherent_factors plus noise * ||X0|| / ||G|| * G, G ~ N(0,1); every entry
    stored, in linear order with mode 0 fastest.  Returns (tensor, factors)."""
    rng = np.random.default_rng([seed, 5])
    fac = coherent_factors(rng, dims, rank, spread, magnitude, jitter)
    total = int(np.prod(dims))
    lin = np.arange(total, dtype=np.int64)
    coords = np.empty((len(dims), total), dtype=np.int32)
    rem = lin
    for m, n in enumerate(dims):
        coords[m] = rem % n
        rem = rem // n
    clean = _model_at(fac, coords)
    g = rng.standard_normal(total)
    vals = clean + noise * (np.linalg.norm(clean) / np.linalg.norm(g)) * g
    return SparseTensor(tuple(int(n) for n in dims), coords, vals), fac


def random_sparse(dims, nnz: int, seed: int = 0):
    """Uniform distinct coordinates, N(0,1) values (shape/edge-case tests)."""
    rng = np.random.default_rng([seed, 4])
    total = int(np.prod(dims))
    nnz = min(nnz, total)
    lin = np.sort(rng.choice(total, size=nnz, replace=False))
    coords = np.empty((len(dims), lin.size), dtype=np.int32)
    rem = lin
    for m, n in enumerate(dims):
        coords[m] = rem % n
        rem = rem // n
    perm = rng.permutation(lin.size)
    return SparseTensor(tuple(int(n) for n in dims),
                        np.ascontiguousarray(coords[:, perm]),
                        rng.standard_normal(lin.size))
