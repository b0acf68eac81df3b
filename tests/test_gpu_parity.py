"""GPU parity: the HIP mode update against the FP64 CPU oracle, per update
with identical inputs (see gpu_util.run_parity).  Sample indices, omega,
weights, statistics and leverage scores are compared bit for bit; factors
within 1e-10 relative (max-norm) in FP64 gather mode; in FP32 mode within
the bound derived per update from the rounding of the operands, the number
of terms summed and the condition number of G_s (gpu_util.derived_tolerance).
Edge cases whose G_s is ill-conditioned (s = 1, R = 64) take the larger of
1e-10 and that bound in FP64 too."""
import numpy as np
import pytest

import oracle
from paper_2006_16438_amd import synth
from tests.gpu_util import log, make_ctx, rel_err, run_parity

pytestmark = pytest.mark.gpu


def concentrated(dims, R, seed):
    rng = np.random.default_rng(seed)
    fac = []
    for n in dims:
        A = rng.standard_normal((n, R)) * 0.05
        hot = rng.choice(n, size=min(n, R), replace=False)
        for j, h in enumerate(hot):
            A[h, j % R] += 3.0 + j
        fac.append(A)
    return fac


def test_small3_fp64_hybrid_ten_iterations():
    """100x80x60, 20,000 nnz, R=5, s=1024, tau=1/s, 10 iterations, FP64."""
    T, _, R = synth.small3(0)
    fac = synth.gaussian_factors(T.dims, R, 0)
    log("small3 fp64 hybrid: 30 updates")
    res = run_parity(T, fac, R, 1024, 1 / 1024, 30, "f64", 1e-10, label="small3")
    assert all(r[0] is not None for r in res)
    assert sum(r[0]["s_det"] for r in res) > 0, "hybrid sampling never found a deterministic row"


def test_small3_fp32_gather():
    T, _, R = synth.small3(0)
    fac = synth.gaussian_factors(T.dims, R, 0)
    log("small3 fp32 gather: 9 updates")
    run_parity(T, fac, R, 1024, 1 / 1024, 9, "f32", "derived", label="small3-f32")


def test_small3_random_only():
    T, _, R = synth.small3(0)
    fac = synth.gaussian_factors(T.dims, R, 1)
    log("small3 tau=1: 6 updates")
    res = run_parity(T, fac, R, 1024, 1.0, 6, "f64", 1e-10, seed=5, stream_id=3, label="tau1")
    assert all(r[0]["s_det"] == 0 and r[0]["draws"] == 1024 for r in res)


def test_multi_tile_ragged():
    """Several Gram blocks (700 = 2*256 + 188 rows), sort tiles, draw chunks."""
    dims = (700, 300, 257)
    T = synth.random_sparse(dims, 150_000, seed=21)
    R = 8
    fac = concentrated(dims, R, 22)
    log("multi-tile 700x300x257: 6 updates")
    run_parity(T, fac, R, 8192 + 77, 1 / 8192, 6, "f64", 1e-10, label="multitile")


def test_rank_above_mode_size_uses_pinv():
    """Uber shape with 200k nnz: mode 1 has 24 rows < R = 25, so its leverage
    takes the pseudo-inverse path on both sides."""
    T = synth.uber4(0, nnz=200_000)
    R = 25
    fac = synth.gaussian_factors(T.dims, R, 0)
    log("uber-shape 200k nnz R=25: 8 updates")
    res = run_parity(T, fac, R, 1 << 14, 2.0 ** -14, 8, "f64", 1e-10, label="uber200k")
    assert any(r[1]["flags"] & oracle.FLAG_PINV for r in res)


def test_all_rows_matches_cp_als():
    dims = (9, 7, 5)
    T = synth.random_sparse(dims, 120, seed=7)
    R = 3
    fac = synth.gaussian_factors(dims, R, 8)
    log("all rows (tau=0)")
    res = run_parity(T, fac, R, 80, 0.0, 3, "f64", 1e-10, det_cap=1000, label="allrows")
    for rs, st, _ in res:
        assert rs is not None and st["flags"] & oracle.FLAG_PDET_ONE and st["s_rnd"] == 0


def test_detcap_and_truncation():
    dims = (12, 10, 9)
    T = synth.random_sparse(dims, 300, seed=9)
    R = 3
    fac = concentrated(dims, R, 10)
    log("det cap")
    res = run_parity(T, fac, R, 64, 1e-6, 3, "f64", 1e-10, det_cap=5, label="detcap")
    assert all(r[1]["flags"] & oracle.FLAG_DETCAP for r in res)
    log("det truncation")
    res = run_parity(T, fac, R, 16, 1e-9, 3, "f64", 1e-10, det_cap=100000, label="trunc")
    assert all(r[1]["flags"] & oracle.FLAG_DET_TRUNC for r in res)


@pytest.mark.parametrize("dims,R,s,nnz", [
    ((40, 30), 4, 64, 500),          # order 2: the KRP is one factor
    ((6, 5, 4, 3, 2), 2, 50, 200),   # order 5
    ((50, 40, 30), 1, 256, 2000),    # R = 1
    ((300, 200, 100), 64, 4096, 60_000),  # R = 64 (maximum)
    ((20, 20, 20), 4, 1, 800),       # s = 1
    ((20, 20, 20), 3, 32, 1),        # a single nonzero
])
def test_shapes_and_edges(dims, R, s, nnz):
    T = synth.random_sparse(dims, nnz, seed=sum(dims) + R)
    fac = synth.gaussian_factors(dims, R, R + s)
    log(f"edge case dims={dims} R={R} s={s} nnz={nnz}")
    run_parity(T, fac, R, s, 1.0 / s if s > 1 else 1.0, 2 * len(dims), "f64", "derived",
               label=f"edge{dims}")


def test_values_given_in_fp32():
    T, _, R = synth.small3(3)
    T.values = T.values.astype(np.float32).astype(np.float64)
    fac = synth.gaussian_factors(T.dims, R, 3)
    from paper_2006_16438_amd._lib import CpalError  # noqa: F401
    log("fp32 input values")
    OT = oracle.Tensor.from_synth(T)
    ctx, F = make_ctx(T, fac, R, 512, values_f32=True)
    host = [f.copy() for f in fac]
    ref = oracle.mode_update(OT, host, 0, 0, R, 512)
    ctx.mode_update(0)
    assert np.array_equal(ctx.samples_view()[0].cpu().numpy().view(np.uint64), ref["idx"])
    assert rel_err(F[0].cpu().numpy(), host[0]) < 1e-10
    ctx.close()


def test_init_errors():
    import torch
    from paper_2006_16438_amd._lib import CpalError
    dims = (5, 4, 3)
    T = synth.random_sparse(dims, 20, seed=1)
    fac = synth.gaussian_factors(dims, 2, 1)
    log("init errors")
    # duplicate coordinate
    T2 = synth.SparseTensor(dims, np.concatenate([T.coords, T.coords[:, :1]], axis=1),
                            np.concatenate([T.values, T.values[:1]]))
    with pytest.raises(CpalError) as e:
        make_ctx(T2, fac, 2, 8)
    assert e.value.code == 1
    # coordinate out of range
    T3 = synth.SparseTensor(dims, T.coords.copy(), T.values)
    T3.coords[1, 0] = 4
    with pytest.raises(CpalError) as e:
        make_ctx(T3, fac, 2, 8)
    assert e.value.code == 1
    # all-zero factor
    f0 = [f.copy() for f in fac]
    f0[2][:] = 0
    with pytest.raises(CpalError) as e:
        make_ctx(T, f0, 2, 8)
    assert e.value.code == 4
    # bad options
    with pytest.raises(CpalError):
        make_ctx(T, fac, 2, 0)
    with pytest.raises(CpalError):
        make_ctx(T, fac, 2, 8, tau=1.5)
    torch.cuda.synchronize()


def test_uber4_full_size_fp32():
    """The benchmark workload at full size: 183x24x1140x1717, 3.3e6 nnz,
    R = 25, s = 2^17, tau = 2^-17, FP32 gather: one outer iteration."""
    T = synth.uber4(0)
    R = 25
    fac = synth.gaussian_factors(T.dims, R, 0)
    log("uber4 full size fp32: 4 updates")
    res = run_parity(T, fac, R, 1 << 17, 2.0 ** -17, 4, "f32", "derived", label="uber4")
    for rs, st, err in res:
        assert rs is not None
        log(f"  s_bar={st['s_bar']} nnz(X~)={st['gathered_nnz']} err={err:.2e}")


@pytest.mark.parametrize("which", ["small3", "uber4"])
def test_fit_estimate_matches_oracle(which):
    """Sec. 6.4 stratified estimate: the device draws the same sample as the
    oracle (same Philox counters), so the estimates agree to rounding."""
    if which == "small3":
        T, _, R = synth.small3(0)
        s_fit, s = 4096, 1024
    else:
        T = synth.uber4(0)
        R, s_fit, s = 25, 1 << 20, 1 << 17
    fac = synth.gaussian_factors(T.dims, R, 0)
    log(f"fit estimate {which} s_fit={s_fit}")
    OT = oracle.Tensor.from_synth(T)
    fs = oracle.FitSample(OT, s_fit, 0.5, seed=0, stream_id=0)
    ctx, F = make_ctx(T, fac, R, s, gather="f32", fit_samples=s_fit)
    for it in range(2):
        host = [f.cpu().numpy().copy() for f in F]
        ref = fs.estimate(host)
        got = float(ctx.fit_estimate().item())
        log(f"  fit gpu={got!r} oracle={ref!r}")
        assert abs(got - ref) <= 1e-10 * max(1.0, abs(ref))
        for k in range(len(T.dims)):
            ctx.mode_update(k)
    ctx.close()


@pytest.mark.parametrize("gather", ["f64", "f32"])
def test_large_mode_gather_paths(gather):
    """A 5000-row mode: the chunk-local sort by output row takes two 6-bit
    radix passes (13-bit row indices), the short modes one."""
    dims = (5000, 60, 50)
    T = synth.random_sparse(dims, 300_000, seed=31)
    R = 16
    fac = concentrated(dims, R, 32)
    log(f"large mode gather paths ({gather})")
    run_parity(T, fac, R, 4096, 1 / 4096, 6, gather, 1e-10 if gather == "f64" else "derived",
               label=f"large-{gather}")


@pytest.mark.parametrize("gather", ["f64", "f32"])
def test_tall_mode_atomic_gather(gather):
    """A mode with more than 2^20 rows has row indices too wide for the
    chunk-local sort keys; its gather adds straight into M (global atomics)."""
    dims = ((1 << 20) + 4099, 7, 5)
    T = synth.random_sparse(dims, 120_000, seed=41)
    R = 8
    fac = concentrated(dims, R, 43)
    log(f"tall mode atomic gather ({gather})")
    run_parity(T, fac, R, 2048, 1 / 2048, 3, gather, 1e-10 if gather == "f64" else "derived",
               label=f"tall-{gather}")


@pytest.mark.parametrize("grid,sort_min", [(64, 0), (1024, 1 << 30), (300, 4)])
def test_gather_launch_shapes(grid, sort_min):
    """Results do not depend on the gather's launch shape: a tensor whose
    mode-0 fibers are long (a 2048-position chunk spans one or two fibers,
    the case that skips the row sort) and whose other modes have short ones
    (many fibers per chunk, sorted), FP64, under grids smaller and larger
    than the chip and every sort threshold."""
    dims = (3000, 4, 3)
    T = synth.random_sparse(dims, 30_000, seed=51)
    R = 3
    fac = concentrated(dims, R, 52)
    log(f"gather launch shape grid={grid} sort_min={sort_min}")
    run_parity(T, fac, R, 256, 1 / 256, 6, "f64", 1e-10, label=f"shape-{grid}-{sort_min}",
               gather_config=(grid, sort_min))


@pytest.mark.parametrize("gather", ["f64", "f32"])
def test_autotune_then_parity(gather):
    """The autotuner times the launch shapes on the decomposition's own state
    and leaves factors, leverage and step unchanged; the updates after it
    match the oracle."""
    dims = (700, 300, 257)
    T = synth.random_sparse(dims, 150_000, seed=21)
    R = 8
    fac = concentrated(dims, R, 22)
    log(f"autotune then parity ({gather})")
    run_parity(T, fac, R, 8192, 1 / 8192, 6, gather, 1e-10 if gather == "f64" else "derived",
               label=f"autotune-{gather}", autotune=True)


@pytest.mark.parametrize("case", ["long_short", "multitile", "uber4"])
def test_bucketed_gather_fp32(case):
    """The bucketed gather (sampled nonzeros moved into 4096 buckets of
    output rows before the chunked reduction), FP32: bucket widths of one
    row (modes up to 4096 rows) and more, long-fiber and short-fiber modes,
    the benchmark workload at full size."""
    if case == "long_short":
        dims = (3000, 4, 3)
        T = synth.random_sparse(dims, 30_000, seed=51)
        R, s, tau, n = 3, 256, 1 / 256, 6
        fac = concentrated(dims, R, 52)
    elif case == "multitile":
        dims = (700, 300, 257)
        T = synth.random_sparse(dims, 150_000, seed=21)
        R, s, tau, n = 8, 8192 + 77, 1 / 8192, 6
        fac = concentrated(dims, R, 22)
    else:
        T = synth.uber4(0)
        R, s, tau, n = 25, 1 << 17, 2.0 ** -17, 4
        fac = synth.gaussian_factors(T.dims, R, 0)
    log(f"bucketed gather, {case}")
    run_parity(T, fac, R, s, tau, n, "f32", "derived", label=f"bucketed-{case}",
               gather_config=(512, -1))


@pytest.mark.parametrize("case", ["long_short", "multitile"])
def test_bucketed_gather_fp64(case):
    """The bucketed gather in FP64 (16-byte records {row, KRP row, value}),
    held to the 1e-10 parity bar."""
    if case == "long_short":
        dims = (3000, 4, 3)
        T = synth.random_sparse(dims, 30_000, seed=51)
        R, s, tau, n = 3, 256, 1 / 256, 6
        fac = concentrated(dims, R, 52)
    else:
        dims = (700, 300, 257)
        T = synth.random_sparse(dims, 150_000, seed=21)
        R, s, tau, n = 8, 8192 + 77, 1 / 8192, 6
        fac = concentrated(dims, R, 22)
    log(f"bucketed gather FP64, {case}")
    run_parity(T, fac, R, s, tau, n, "f64", 1e-10, label=f"bucketed64-{case}",
               gather_config=(512, -1))


@pytest.mark.parametrize("case", ["long_short", "multitile", "uber4"])
def test_owner_gather_fp32(case):
    """The owner gather (no atomic operation: workgroup (row block, fiber
    part) alone forms its rows of one copy of M in shared memory, from the
    fibers' per-block segments), FP32: long-fiber and short-fiber modes,
    several row blocks and fiber groups, the benchmark workload at full
    size."""
    if case == "long_short":
        dims = (3000, 4, 3)
        T = synth.random_sparse(dims, 30_000, seed=51)
        R, s, tau, n = 3, 256, 1 / 256, 6
        fac = concentrated(dims, R, 52)
    elif case == "multitile":
        dims = (700, 300, 257)
        T = synth.random_sparse(dims, 150_000, seed=21)
        R, s, tau, n = 8, 8192 + 77, 1 / 8192, 6
        fac = concentrated(dims, R, 22)
    else:
        T = synth.uber4(0)
        R, s, tau, n = 25, 1 << 17, 2.0 ** -17, 4
        fac = synth.gaussian_factors(T.dims, R, 0)
    log(f"owner gather, {case}")
    run_parity(T, fac, R, s, tau, n, "f32", "derived", label=f"owner-{case}",
               gather_config=(0, -2))


def _rowblock_case(case):
    """Workloads of the row-block gathers (modes of at least 1024 rows take
    them): one long-fiber 3000-row mode; 2100- and 1100-row modes of 66 and
    35 blocks with a 300-row mode beside them; R = 40 (three 16-column
    groups) on a 1500-row mode; the Uber-shaped workload at full size."""
    if case == "long_short":
        dims = (3000, 4, 3)
        T = synth.random_sparse(dims, 30_000, seed=51)
        return T, 3, 256, 1 / 256, 6, concentrated(dims, 3, 52)
    if case == "multiblock":
        dims = (2100, 300, 1100)
        T = synth.random_sparse(dims, 150_000, seed=21)
        return T, 8, 8192 + 77, 1 / 8192, 6, concentrated(dims, 8, 22)
    if case == "rank40":
        dims = (1500, 40, 35)
        T = synth.random_sparse(dims, 200_000, seed=23)
        return T, 40, 4096, 1 / 4096, 6, concentrated(dims, 40, 22)
    T = synth.uber4(0)
    return T, 25, 1 << 17, 2.0 ** -17, 4, synth.gaussian_factors(T.dims, 25, 0)


@pytest.mark.parametrize("gather,case", [("f64", "long_short"), ("f64", "multiblock"),
                                          ("f64", "rank40"), ("f64", "uber4"),
                                          ("f32", "multiblock"), ("f32", "uber4")])
def test_tile_gather(gather, case):
    """The tile gather (workgroup (row block, fiber part) adds the segments of
    its part's fibers in its block into a shared FP64 row block, one
    nonzero per lane): row blocks of 32 to 512 rows, windows of more than
    one workgroup of fibers, R > 32, the benchmark workload at full size;
    FP64 at the 1e-10 bar."""
    T, R, s, tau, n, fac = _rowblock_case(case)
    log(f"tile gather {gather}, {case}")
    run_parity(T, fac, R, s, tau, n, gather, 1e-10 if gather == "f64" else "derived",
               label=f"tile-{gather}-{case}", gather_config=(0, -3))


@pytest.mark.parametrize("gather,case", [("f64", "long_short"), ("f64", "multiblock"),
                                          ("f64", "rank40"), ("f64", "uber4"),
                                          ("f32", "multiblock"), ("f32", "uber4")])
def test_bucketed_shared_block_gather(gather, case):
    """The bucketed gather with shared-memory bucket blocks (buckets of up to
    512 rows; the records of a bucket cut into slices, each slice added into
    a shared FP64 block and then into M): one-bucket and many-bucket modes,
    slices of several workgroup passes, R > 32, the benchmark workload at
    full size; FP64 at the 1e-10 bar."""
    T, R, s, tau, n, fac = _rowblock_case(case)
    log(f"shared-block bucketed gather {gather}, {case}")
    run_parity(T, fac, R, s, tau, n, gather, 1e-10 if gather == "f64" else "derived",
               label=f"bktl-{gather}-{case}", gather_config=(0, -4))


def test_bucketed_shared_block_gather_full_records():
    """The shared-block bucketed gather with 2^23 samples: a KRP row (slot
    index) no longer fits the compact record's 23 bits, so the records are
    the full 16-byte ones (row, KRP row, value); 1100- and 4096-row modes,
    FP64 at the 1e-10 bar."""
    T = synth.random_sparse((1100, 4096, 4096), 1_000_000, seed=71)
    fac = synth.gaussian_factors(T.dims, 8, 3)
    s = 1 << 23
    log("shared-block bucketed gather, 2^23 samples")
    run_parity(T, fac, 8, s, 1.0 / s, 3, "f64", 1e-10, label="bktl-full-records",
               gather_config=(0, -4))


def _zipf3(seed=61):
    """3-way Zipf(1.2) coordinates (3000 x 1200 x 300, 4e5 nonzeros): fiber
    lengths from one to thousands in every mode."""
    dims = (3000, 1200, 300)
    rng = np.random.default_rng([seed, 5])
    samplers = [synth._zipf_sampler(rng, n, 1.2) for n in dims]
    coords = synth._distinct_first(dims, lambda b: np.stack([sm(b) for sm in samplers]).astype(np.int32),
                                   400_000, batch=1 << 19)
    vals = rng.random(coords.shape[1]) + 0.5
    return synth.SparseTensor(dims, coords, vals)


@pytest.mark.parametrize("gather,lfac,case", [("f64", 8, "zipf3"), ("f64", 32, "zipf3"),
                                               ("f64", 16, "long_short"), ("f64", 16, "uber4"),
                                               ("f32", 16, "zipf3")])
def test_hybrid_gather(gather, lfac, case):
    """The hybrid gather: fibers of at least lfac x (row blocks) nonzeros
    through the tile gather, which stores every row of M, then the shorter
    ones through the shared-block bucketed gather, which adds into it (its
    count and scatter passes skip the long fibers, its reduction takes the
    record count from the scan); FP64 at the 1e-10 bar."""
    if case == "zipf3":
        T = _zipf3()
        R, s, tau, n = 8, 4096, 1 / 4096, 6
        fac = concentrated(T.dims, R, 62)
    elif case == "long_short":
        dims = (3000, 4, 3)
        T = synth.random_sparse(dims, 30_000, seed=51)
        R, s, tau, n = 3, 256, 1 / 256, 6
        fac = concentrated(dims, R, 52)
    else:
        T = synth.uber4(0)
        R, s, tau, n = 25, 1 << 17, 2.0 ** -17, 4
        fac = synth.gaussian_factors(T.dims, R, 0)
    log(f"hybrid gather {gather}, threshold factor {lfac}, {case}")
    run_parity(T, fac, R, s, tau, n, gather, 1e-10 if gather == "f64" else "derived",
               label=f"hyb-{gather}-{lfac}-{case}", gather_config=(lfac, -5))


@pytest.mark.parametrize("which", ["multitile", "rank40"])
def test_fp64_updates_bit_reproducible(which):
    """FP64 mode updates (owner gather, earliest draw carrying each repeated
    row) are bit-reproducible: two contexts built from the same inputs, run
    through the same updates, hold bit-identical factors after every update,
    although repeated rows and many fibers per output row occur."""
    if which == "multitile":
        dims = (700, 300, 257)
        T = synth.random_sparse(dims, 150_000, seed=21)
        R, s = 8, 8192
    else:   # R > 32: 64-wide rows
        dims = (900, 40, 35)
        T = synth.random_sparse(dims, 200_000, seed=23)
        R, s = 40, 4096
    fac = concentrated(dims, R, 22)
    a, Fa = make_ctx(T, fac, R, s, 1.0 / s, "f64")
    b, Fb = make_ctx(T, fac, R, s, 1.0 / s, "f64")
    assert all(a.gather_config(m)[1] == -2 for m in range(3))
    for u in range(9):
        k = u % 3
        a.mode_update(k)
        b.mode_update(k)
        st = a.last_stats()
        assert np.array_equal(Fa[k].cpu().numpy().view(np.uint64), Fb[k].cpu().numpy().view(np.uint64)), \
            f"update {u}: factors differ between identical runs"
        log(f"  update {u}: s_bar {st['s_bar']} of {s} (repeats combined), bit-identical")
    a.close()
    b.close()


def test_gather_config_errors():
    """Argument checks of the launch-shape calls: negative grids, sort
    thresholds below -5, row-block gathers (-3 to -5) on modes of fewer than
    1024 rows, a dense split beyond the default, modes out of range; FP64
    contexts start on the owner gather (-2)."""
    from paper_2006_16438_amd._lib import CpalError
    T, _, R = synth.small3(0)
    fac = synth.gaussian_factors(T.dims, R, 0)
    ctx, _ = make_ctx(T, fac, R, 1024, gather="f64")
    for args in ((0, -1, 0), (0, 64, -6), (0, 300, -5), (3, 64, 0), (-1, 64, 0)):
        with pytest.raises(CpalError):
            ctx.set_gather_config(*args)
    assert ctx.gather_config(0)[1] == -2
    ctx.set_gather_config(0, 64, 4)
    assert ctx.gather_config(0) == (64, 4)
    ctx.set_gather_config(0, 256, -1)   # the bucketed gather exists in FP64 mode too
    assert ctx.gather_config(0) == (256, -1)
    for args in ((2, 0, -3), (1, 0, -4), (0, 16, -5)):   # modes of fewer than 1024 rows
        with pytest.raises(CpalError):
            ctx.set_gather_config(*args)
    ctx.close()
    W = synth.random_sparse((1100, 50, 40), 20_000, seed=9)   # a 1100-row mode takes them
    ctx, _ = make_ctx(W, synth.gaussian_factors(W.dims, R, 0), R, 1024, gather="f64")
    ctx.set_gather_config(0, 0, -3)     # the tile gather
    assert ctx.gather_config(0)[1] == -3
    ctx.set_gather_config(0, 0, -4)     # the shared-block bucketed gather
    assert ctx.gather_config(0)[1] == -4
    ctx.set_gather_config(0, 16, -5)    # the hybrid gather
    assert ctx.gather_config(0) == (16, -5)
    with pytest.raises(CpalError):
        ctx.set_gather_config(1, 16, -5)
    ctx.close()
    ctx, _ = make_ctx(T, fac, R, 1024, gather="f32")
    ctx.set_gather_config(1, 256, -1)   # the bucketed gather exists in FP32 mode
    assert ctx.gather_config(1) == (256, -1)
    ctx.close()
    D, _ = synth.planted((12, 10, 8), 3, seed=8, density=1.0, law="normal")
    ctx, _ = make_ctx(D, synth.gaussian_factors(D.dims, 3, 0), 3, 256, gather="f32", dense=True)
    default = ctx.gather_config(0)[0]
    with pytest.raises(CpalError):
        ctx.set_gather_config(0, default + 1, 0)
    with pytest.raises(CpalError):
        ctx.set_gather_config(0, 1, -1)   # no bucketed gather for dense tensors
    with pytest.raises(CpalError):
        ctx.set_gather_config(0, 1, -2)   # nor an owner gather
    with pytest.raises(CpalError):
        ctx.set_gather_config(0, 1, -3)   # nor a tile gather
    with pytest.raises(CpalError):
        ctx.set_gather_config(0, 1, -4)
    with pytest.raises(CpalError):
        ctx.set_gather_config(0, 1, -5)
    ctx.close()
