"""The large sparse 3-way shape (8211 x 176962 x 8116, Zipf(1.2)
coordinates, log(1 + Geometric(0.3)) values) through the C ABI with 10^8
nonzeros: every index structure at these mode sizes (44-bit full keys,
fiber keys up to 1.4e9, a 176,962-row mode through the segmented gather).

Per mode update: the sample (idx, omega, w) equals the oracle's (sampling
depends only on the factors, step and seed, so the oracle runs it on a
one-entry tensor of the same shape), and the new factor equals an FP64
solve of the sampled system built by plain torch operations from the same
sampled fibers: within 1e-10 for the FP64 gather, 1e-4 for FP32 (values and
weighted KRP rows rounded to FP32, FP32 sums)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2006_16438_amd import synth
from tests.gpu_util import log, rel_err, sampled_solve_torch

pytestmark = pytest.mark.gpu

NNZ = 100_000_000
FTOL = {"f64": 1e-10, "f32": 1e-4}


@pytest.fixture(scope="module")
def large_tensor():
    from paper_2006_16438_amd import synth_gpu
    log(f"generating the large 3-way shape with {NNZ} nonzeros")
    dims, coords, vals = synth_gpu.large3(0, nnz=NNZ, verbose=False)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    yield dims, coords, vals
    del coords, vals
    torch.cuda.empty_cache()


@pytest.mark.parametrize("gather", ["f64", "f32", "f32-bucketed", "f64-tile", "f32-tile",
                                    "f64-bktl"])
def test_large3_shape_parity(large_tensor, gather):
    from paper_2006_16438_amd.api import CpArlsLev
    dims, coords, vals = large_tensor
    R, s = 25, 1 << 17
    dev = coords.device
    fac = synth.gaussian_factors(dims, R, 3)
    F = [torch.from_numpy(f.copy()).to(dev) for f in fac]
    log(f"large3 {dims} nnz={NNZ} R={R} s={s} gather={gather}: init")
    bucketed = gather == "f32-bucketed"
    tile = gather.endswith("-tile")
    bktl = gather.endswith("-bktl")
    gather = gather.split("-")[0]
    ctx = CpArlsLev(dims, coords, vals, F, R, s, tau=1.0 / s, seed=0, stream_id=0,
                    gather_dtype=gather)
    if bucketed:   # nonzeros moved into row buckets before the reduction
        for k in range(3):
            ctx.set_gather_config(k, 512, -1)
    elif tile:     # row blocks in shared memory (512 rows in the long mode)
        for k in range(3):
            ctx.set_gather_config(k, 0, -3)
    elif bktl:     # 512-row buckets reduced in shared memory
        for k in range(3):
            ctx.set_gather_config(k, 0, -4)
    elif gather == "f32":   # the tuned launch shapes
        log(f"  autotuned gather shapes {ctx.autotune()}")
    OT = oracle.Tensor(np.array(dims), np.zeros((3, 1), dtype=np.int32), np.ones(1))
    for k in range(3):
        host = [f.cpu().numpy().copy() for f in F]
        t = ctx.step
        ref = oracle.mode_update(OT, [h.copy() for h in host], k, t, R, s, 1.0 / s)
        ctx.mode_update(k)
        st = ctx.last_stats()
        idx, om, w = ctx.samples_view()
        assert np.array_equal(idx.cpu().numpy().view(np.uint64), ref["idx"]), \
            f"mode {k}: sample indices differ"
        assert np.array_equal(om.cpu().numpy(), ref["omega"]), f"mode {k}: omega differs"
        assert np.array_equal(w.cpu().numpy(), ref["wgt"]), f"mode {k}: weights differ"
        Fh = [torch.from_numpy(h).to(dev) for h in host]
        A_ref, nnz_g = sampled_solve_torch(dims, coords, vals, Fh, k, idx, om)
        assert nnz_g == st["gathered_nnz"], f"mode {k}: gathered {st['gathered_nnz']} != {nnz_g}"
        err = rel_err(F[k].cpu().numpy(), A_ref.cpu().numpy())
        log(f"  mode {k}: s_bar={idx.numel()} gathered nnz={nnz_g} factor rel err {err:.3e}")
        assert err <= FTOL[gather], f"mode {k}: factor rel err {err:.3e}"
        del A_ref, Fh
    ctx.close()
    torch.cuda.empty_cache()


def test_large3_full_size_fp32():
    """The benchmark's 10^9-nonzero tensor in the benchmark's launch
    configuration (FP32 gather, default launch shapes), one iteration from
    the benchmark's initial factors: per mode the sample equals the
    oracle's and the factor an FP64 solve of the same sampled system built
    with torch from its definition (1e-4)."""
    from paper_2006_16438_amd import synth_gpu
    from paper_2006_16438_amd.api import CpArlsLev
    torch.cuda.empty_cache()
    log("generating the 1e9-nonzero tensor")
    dims, coords, vals = synth_gpu.large3(0, verbose=False)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    R, s = 25, 1 << 17
    dev = coords.device
    fac = synth.gaussian_factors(dims, R, 0)
    F = [torch.from_numpy(f.copy()).to(dev) for f in fac]
    ctx = CpArlsLev(dims, coords, vals, F, R, s, tau=1.0 / s, seed=0, stream_id=0,
                    gather_dtype="f32")
    OT = oracle.Tensor(np.array(dims), np.zeros((3, 1), dtype=np.int32), np.ones(1))
    for k in range(3):
        host = [f.cpu().numpy().copy() for f in F]
        ref = oracle.mode_update(OT, [h.copy() for h in host], k, ctx.step, R, s, 1.0 / s)
        ctx.mode_update(k)
        st = ctx.last_stats()
        idx, om, w = ctx.samples_view()
        assert np.array_equal(idx.cpu().numpy().view(np.uint64), ref["idx"]), \
            f"mode {k}: sample indices differ"
        assert np.array_equal(om.cpu().numpy(), ref["omega"]), f"mode {k}: omega differs"
        assert np.array_equal(w.cpu().numpy(), ref["wgt"]), f"mode {k}: weights differ"
        Fh = [torch.from_numpy(h).to(dev) for h in host]
        A_ref, nnz_g = sampled_solve_torch(dims, coords, vals, Fh, k, idx, om)
        assert nnz_g == st["gathered_nnz"]
        err = rel_err(F[k].cpu().numpy(), A_ref.cpu().numpy())
        log(f"  mode {k}: s_bar={idx.numel()} gathered nnz={nnz_g} factor rel err {err:.3e}")
        assert err <= FTOL["f32"], f"mode {k}: factor rel err {err:.3e}"
        del A_ref, Fh
        torch.cuda.empty_cache()
    ctx.close()
    del coords, vals, F
    torch.cuda.empty_cache()
