"""Seeded synthetic tensors generated on the GPU with torch's own generator,
for workloads too large to build on the host: the 10^9-nonzero 3-way tensor,
the batch of 64 sparse tensors and the dense 1000^3 tensor.  Like synth.py
this module holds input recipes only (none of the method's arithmetic).

Zipf(a) on {0..n-1}: p(i) proportional to (i+1)^-a, mapped through a seeded
random permutation so that the hot indices are scattered.  Distinct
coordinates: draws are taken in order, the first occurrence of a coordinate
is kept (with the value drawn for that draw) and generation stops at the
target count."""
from __future__ import annotations

import sys
import time

import torch


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _zipf_table(n, a, g, dev):
    p = torch.arange(1, n + 1, device=dev, dtype=torch.float64).pow_(-a)
    cdf = torch.cumsum(p / p.sum(), 0)
    perm = torch.randperm(n, generator=g, device=dev)
    return cdf, perm


def _zipf_draw(cdf, perm, count, g, dev):
    u = torch.rand(count, generator=g, device=dev, dtype=torch.float64)
    i = torch.searchsorted(cdf, u, right=True)
    del u
    i.clamp_(max=cdf.numel() - 1)
    return perm[i]


def zipf_distinct(dims, nnz, a, seed, value_fn, chunk=1 << 28, max_chunks=64, verbose=False,
                  device="cuda:0"):
    """First `nnz` distinct coordinates of a stream of per-mode Zipf(a) draws
    (mode 0 fastest in the linear key), with value_fn(count, g) drawing one
    value per draw.  Returns (coords int32 [D, nnz], values float32 [nnz]) on
    `device`, ordered by linear key."""
    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    tables = [_zipf_table(n, a, g, dev) for n in dims]
    total = 1
    for n in dims:
        total *= n
    if nnz > total:
        raise ValueError("more nonzeros than entries")
    U = torch.empty(0, dtype=torch.int64, device=dev)     # distinct keys so far, sorted
    V = torch.empty(0, dtype=torch.float32, device=dev)
    t0 = time.time()
    for c in range(max_chunks):
        key = torch.zeros(chunk, dtype=torch.int64, device=dev)
        stride = 1
        for (cdf, perm), n in zip(tables, dims):
            key.add_(_zipf_draw(cdf, perm, chunk, g, dev), alpha=stride)
            stride *= n
        vals = value_fn(chunk, g)
        sk, pos = torch.sort(key, stable=True)   # equal keys keep draw order
        del key
        first = torch.ones(chunk, dtype=torch.bool, device=dev)
        first[1:] = sk[1:] != sk[:-1]
        uk, up = sk[first], pos[first]
        del sk, pos, first
        if U.numel():
            at = torch.searchsorted(U, uk).clamp_(max=U.numel() - 1)
            fresh = U[at] != uk
            del at
            uk, up = uk[fresh], up[fresh]
            del fresh
        need = nnz - U.numel()
        if uk.numel() >= need:   # the needed new keys are the earliest drawn ones
            o = torch.argsort(up)[:need]
            uk, up = uk[o], up[o]
        uv = vals[up]
        del vals, up
        U = torch.cat([U, uk])
        V = torch.cat([V, uv])
        del uk, uv
        U, o = torch.sort(U)
        V = V[o]
        del o
        if verbose:
            _log(f"  zipf chunk {c}: {U.numel()} distinct of {nnz} ({time.time() - t0:.1f}s)")
        if U.numel() >= nnz:
            break
    else:
        raise RuntimeError(f"only {U.numel()} distinct coordinates after {max_chunks} chunks")
    coords = torch.empty((len(dims), nnz), dtype=torch.int32, device=dev)
    rem = U
    for m, n in enumerate(dims):
        coords[m] = (rem % n).to(torch.int32)
        rem = rem // n
    del U, rem
    return coords, V


def large3(seed=0, nnz=1_000_000_000, dims=(8211, 176962, 8116), a=1.2, verbose=True):
    """The 3-way tensor standing in for the large Reddit-like case: dims
    8211 x 176962 x 8116, `nnz` distinct Zipf(1.2) coordinates, values
    log(1 + c), c ~ Geometric(0.3) on {1, 2, ...}, FP32."""
    def value_fn(count, g):
        v = torch.empty(count, dtype=torch.float32, device="cuda:0").geometric_(0.3, generator=g)
        return v.log1p_()
    chunk = 1 << 29 if nnz >= (1 << 28) else 1 << 26
    coords, vals = zipf_distinct(dims, nnz, a, seed, value_fn, chunk=chunk, verbose=verbose)
    return tuple(dims), coords, vals


def batch_tensors(n_tensors, seed, nnz_lo=100_000, nnz_hi=5_000_000):
    """Sparse 3-way tensors: dims uniform in [200, 5000], nnz uniform in
    [nnz_lo, nnz_hi] capped at 5% of the entries, per-mode Zipf(1.1)
    coordinates, planted rank uniform in 8..32 with U(0,1) unit-norm-column
    factors, values = model + 1% relative Gaussian noise.  Returns a list of
    (dims, coords int32 [3, nnz], values float32, planted rank) on cuda:0."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    out = []
    for _ in range(n_tensors):
        dims = [int(x) for x in torch.randint(200, 5001, (3,), generator=g, device=dev)]
        total = dims[0] * dims[1] * dims[2]
        want = int(torch.randint(nnz_lo, nnz_hi + 1, (1,), generator=g, device=dev))
        want = min(want, total // 20)
        sub_seed = int(torch.randint(0, 2 ** 62, (1,), generator=g, device=dev))
        coords, _ = zipf_distinct(dims, want, 1.1, sub_seed,
                                  lambda count, gg: torch.zeros(count, dtype=torch.float32,
                                                                device=dev),
                                  chunk=max(1 << 20, 1 << (int(want * 8) - 1).bit_length()))
        c0, c1, c2 = (coords[m].long() for m in range(3))
        rank = int(torch.randint(8, 33, (1,), generator=g, device=dev))
        fac = []
        for n in dims:
            f = torch.rand(n, rank, generator=g, device=dev, dtype=torch.float64)
            fac.append(f / f.norm(dim=0, keepdim=True))
        model = (fac[0][c0] * fac[1][c1] * fac[2][c2]).sum(1)
        noise = torch.randn(model.shape, generator=g, device=dev, dtype=torch.float64)
        vals = (model + 0.01 * (model.norm() / noise.norm()) * noise).float().contiguous()
        out.append((tuple(dims), coords, vals, rank))
    return out


def dense_planted(n, rank, seed, noise=0.01):
    """n^3 FP32 tensor: planted rank-`rank` CP model with N(0,1) factors plus
    `noise` relative Gaussian noise, scaled to noise * ||X0|| / ||G||."""
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    dev = torch.device("cuda:0")
    A = [torch.randn(n, rank, generator=g, device=dev) for _ in range(3)]
    X = torch.einsum("ir,jr,kr->ijk", A[0], A[1], A[2])
    E = torch.randn(X.shape, generator=g, device=dev)
    X.add_(E, alpha=noise * (X.norm() / E.norm()).item())
    del E
    return X


def coherent_dense(n=500, rank=25, spread=5, magnitude=3.0, jitter=0.05, noise=0.05, seed=0):
    """App. C's n^3 dense tensor on the GPU (FP32, indexed [i0, i1, i2]):
    N(0,1) factors whose first three columns are zero except `spread` rows
    each (column c: rows [c spread, (c+1) spread), value magnitude +
    U(0, jitter)), the rank-`rank` model plus noise * ||X0|| / ||G|| * G.
    Returns (X, factors) with the factors as FP64 CPU tensors."""
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    dev = torch.device("cuda:0")
    A = []
    for _ in range(3):
        a = torch.randn(n, rank, generator=g, device=dev, dtype=torch.float64)
        a[:, :min(3, rank)] = 0.0
        for c in range(min(3, rank)):
            a[c * spread:(c + 1) * spread, c] = magnitude + jitter * torch.rand(
                spread, generator=g, device=dev, dtype=torch.float64)
        A.append(a)
    Af = [a.float() for a in A]
    X = torch.einsum("ir,jr,kr->ijk", Af[0], Af[1], Af[2])
    E = torch.randn(X.shape, generator=g, device=dev)
    X.add_(E, alpha=noise * (X.norm() / E.norm()).item())
    del E
    return X, [a.cpu() for a in A]
