"""Dense tensors through the C ABI on the GPU (sampled fibers are whole
mode-k columns; the contraction M = X~^T diag(omega) Z runs on the matrix
cores in FP64, FP32, or BF16 with FP32 accumulation).

Parity protocol as for sparse tensors (tests/gpu_util.py): per update, the
oracle gets the device's current factors and runs the same update on the
COO form of the tensor with every entry stored; sample indices, omega,
weights, statistics and leverage must match bit for bit, the new factor
within the precision's tolerance:
  FP64: 1e-10 (rounding order only);
  FP32, BF16: the bound derived per update (gpu_util.derived_tolerance):
        both operands rounded once (2^-24 each in FP32, 2^-9 each in BF16),
        FP32 sums over the sampled fibers, amplified by cond(G_s) and by the
        cancellation in M = X~^T Omega Z."""
import numpy as np
import pytest
import torch

import oracle
from paper_2006_16438_amd import synth
from tests.gpu_util import bound_from_system, fro_rel_err, log, make_ctx, rel_err, run_parity

pytestmark = pytest.mark.gpu

FTOL = {"f64": 1e-10, "f32": "derived", "bf16": "derived"}


@pytest.mark.parametrize("gather", ["f64", "f32", "bf16"])
def test_dense_small3_parity(gather):
    T, _ = synth.planted((40, 30, 20), 4, seed=0, density=1.0, law="normal")
    R, s = 6, 2048
    fac = synth.gaussian_factors(T.dims, R, 0)
    log(f"dense 40x30x20 R={R} s={s} gather={gather}")
    out = run_parity(T, fac, R, s, 1.0 / s, 6, gather=gather, ftol=FTOL[gather],
                     label=f"dense-{gather}", dense=True)
    errs = [e for _, _, e in out]
    log(f"  factor rel errors {['%.2e' % e for e in errs]}")


def test_dense_4way_parity():
    T, _ = synth.planted((12, 10, 9, 7), 3, seed=1, density=1.0, law="normal")
    R, s = 5, 1024
    fac = synth.gaussian_factors(T.dims, R, 1)
    log("dense 12x10x9x7 R=5 s=1024 gather=f32")
    run_parity(T, fac, R, s, 1.0 / s, 8, gather="f32", ftol=FTOL["f32"], label="dense-4way",
               dense=True)


@pytest.mark.parametrize("gather", ["f64", "bf16"])
def test_dense_ragged_rank20(gather):
    """Mode sizes that are not multiples of the 16-row tiles, R = 20 (two
    column tiles), random-only sampling (tau = 1, many repeated rows).  With
    only 700 samples for 20 unknowns G_s is far less well conditioned than
    in the other cases; the BF16 bound is derived from its condition number
    per update."""
    T, _ = synth.planted((37, 23, 19), 5, seed=2, density=1.0, law="normal")
    R, s = 20, 700
    fac = synth.gaussian_factors(T.dims, R, 2)
    log(f"dense 37x23x19 R={R} s={s} tau=1 gather={gather}")
    ftol = FTOL[gather]
    out = run_parity(T, fac, R, s, 1.0, 6, gather=gather, ftol=ftol,
                     label=f"dense-ragged-{gather}", dense=True)
    log(f"  factor rel errors {['%.2e' % e for _, _, e in out]}")


@pytest.mark.parametrize("gather", ["bf16", "f32"])
def test_dense_1000cube_full_size(gather):
    """Dense 1000^3 FP32, planted rank 10 + 1% noise, R = 10, s = 2^14, in the
    launch configuration the benchmark uses.  Per mode: the sample (idx,
    omega, w) equals the oracle's (sampling depends on the factors, the step
    and the seed only, so the oracle runs it on a one-entry tensor of the
    same shape); the new factor equals an FP64 solve of the sampled system
    built from the same sampled fibers of X, within the precision's
    tolerance."""
    n, R, s = 1000, 10, 1 << 14
    dims = (n, n, n)
    from paper_2006_16438_amd import synth_gpu
    X = synth_gpu.dense_planted(n, 10, seed=4)
    fac = synth.gaussian_factors(dims, R, 4)
    log(f"dense 1000^3 R={R} s={s} gather={gather}: init")
    ctx, F = make_ctx(_Shape(dims), fac, R, s, 1.0 / s, gather, dense_values_gpu=X)
    OT = oracle.Tensor(np.array(dims), np.zeros((3, 1), dtype=np.int32), np.ones(1))
    for k in range(3):
        host = [f.cpu().numpy().copy() for f in F]
        t = ctx.step
        ref = oracle.mode_update(OT, [h.copy() for h in host], k, t, R, s, 1.0 / s)
        ctx.mode_update(k)
        idx, om, w = ctx.samples_view()
        idx = idx.cpu().numpy().view(np.uint64)
        assert np.array_equal(idx, ref["idx"]), f"mode {k}: sample indices differ"
        assert np.array_equal(om.cpu().numpy(), ref["omega"]), f"mode {k}: omega differs"
        assert np.array_equal(w.cpu().numpy(), ref["wgt"]), f"mode {k}: weights differ"
        # FP64 reference of the sampled system from the same fibers
        others = [m for m in range(3) if m != k]
        rem = idx.astype(np.int64)
        sub = []
        for m in others:
            sub.append(rem % dims[m])
            rem = rem // dims[m]
        Z = np.ones((idx.size, R))
        for m, i in zip(others, sub):
            Z *= host[m][i]
        ix = [None, None, None]
        for m, i in zip(others, sub):
            ix[m] = torch.from_numpy(i).to(X.device)
        ix[k] = slice(None)
        fib = X[tuple(ix)].double().cpu().numpy()   # (s_bar, n) or (n, s_bar)
        if fib.shape[0] != idx.size:
            fib = fib.T
        omg = om.cpu().numpy()
        M = fib.T @ (omg[:, None] * Z)
        G = Z.T @ (omg[:, None] * Z)
        A_ref = np.linalg.solve(G, M.T).T
        err = fro_rel_err(F[k].cpu().numpy(), A_ref)
        sy = dict(G=G, Ga=np.abs(Z).T @ (omg[:, None] * np.abs(Z)), M=M,
                  Ma=np.abs(fib).T @ (omg[:, None] * np.abs(Z)), n_terms=idx.size)
        bound = bound_from_system(sy, idx.size, gather)
        log(f"  mode {k}: s_bar={idx.size} factor rel err {err:.3e} (derived bound {bound:.2e})")
        assert err <= bound, f"mode {k}: factor rel err {err:.3e} > {bound:.2e}"
    ctx.close()
    del X
    torch.cuda.empty_cache()


class _Shape:
    def __init__(self, dims):
        self.dims = dims


@pytest.mark.parametrize("split", ["quarter", "autotune"])
def test_dense_split_shapes(split):
    """The split of the sampled fibers over workgroups (one partial M each)
    changes only the rounding order: FP64 parity under a quarter of the
    default split, and after the autotuner (which leaves factors, leverage
    and step unchanged)."""
    T, _ = synth.planted((40, 30, 20), 4, seed=0, density=1.0, law="normal")
    R, s = 6, 4096
    fac = synth.gaussian_factors(T.dims, R, 0)
    if split == "quarter":
        ctx, _ = make_ctx(T, fac, R, s, 1.0 / s, "f64", dense=True)
        default = ctx.gather_config(0)[0]
        ctx.close()
        log(f"dense split: default {default} workgroups along the fibers, running {default // 4}")
        run_parity(T, fac, R, s, 1.0 / s, 3, gather="f64", ftol=FTOL["f64"],
                   label="dense-split", dense=True, gather_config=(max(1, default // 4), 0))
    else:
        run_parity(T, fac, R, s, 1.0 / s, 3, gather="f64", ftol=FTOL["f64"],
                   label="dense-autotune", dense=True, autotune=True)
