"""Randomized range finder initialisation (App. F) through the C ABI
(cp_arls_lev_rrf_init) against the oracle (oracle.rrf_init): every factor
becomes the sum over s_init uniformly drawn nonempty fibers of the fiber
times the caller's Gaussian row.  The drawn fibers follow from the same
Philox counters on both sides, so the factors agree to the rounding of the
sums: 1e-12 relative in FP64, the FP32 bound of the stored values and rows
otherwise.  After the initialisation the mode updates keep the per-update
parity protocol (bit-exact samples)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2006_16438_amd import synth
from paper_2006_16438_amd._lib import CpalError
from tests.gpu_util import log, make_ctx, rel_err, run_parity

pytestmark = pytest.mark.gpu


def _omegas(dims, s_init, R, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((s_init, R)) for _ in dims]


# Bounds: FP64 sums over at most s_init terms, 1e-12; FP32 and BF16 round each
# stored value and Omega row once (u = 2^-24, 2^-8) and the sums then carry a
# random walk of roundings, sqrt(s_init) u relative to the sum of |terms|,
# which the Gaussian weights make ~sqrt(s_init) times the sum itself at most
# for the largest entries; 16x margin.
def _bound(gather, s_init):
    if gather == "f64":
        return 1e-12
    u = 2.0 ** -24 if gather == "f32" else 2.0 ** -8
    return 16 * u * (np.sqrt(s_init) if gather == "f32" else 1.0)


@pytest.mark.parametrize("case,gather", [("small3", "f64"), ("uber4", "f32"), ("dense", "f64"),
                                         ("dense", "bf16")])
def test_rrf_init_matches_oracle(case, gather):
    dense = case == "dense"
    if case == "small3":
        T, _, R = synth.small3(0)
        s, s_init = 1024, 700
    elif case == "uber4":
        T = synth.uber4(0, nnz=400_000)
        R, s, s_init = 25, 1 << 15, 20_000
    else:
        T, _ = synth.planted((30, 20, 16), 3, seed=2, density=1.0, law="normal")
        R, s, s_init = 4, 512, 300
    tol = _bound(gather, s_init)
    fac = synth.gaussian_factors(T.dims, R, 1)
    OT = oracle.Tensor.from_synth(T)
    om = _omegas(T.dims, s_init, R, 9)
    ctx, F = make_ctx(T, fac, R, s, gather=gather, dense=dense)
    ctx.rrf_init(s_init, [torch.from_numpy(o).cuda() for o in om])
    for k in range(len(T.dims)):
        ref, nfib = oracle.rrf_init(OT, k, s_init, om[k])
        got = F[k].cpu().numpy()
        err = rel_err(got, ref)
        log(f"  {case}/{gather} mode {k}: {nfib} nonempty fibers, rel err {err:.2e}")
        assert err <= tol
        lev_ref, _ = oracle.leverage(got)
        assert np.array_equal(ctx.leverage(k).cpu().numpy(), lev_ref)
    ctx.close()


def test_rrf_then_updates_keep_parity():
    T, _, R = synth.small3(0)
    s = 1024
    OT = oracle.Tensor.from_synth(T)
    fac = synth.gaussian_factors(T.dims, R, 1)
    om = _omegas(T.dims, 1000, R, 4)
    ctx, F = make_ctx(T, fac, R, s, gather="f64")
    ctx.rrf_init(1000, [torch.from_numpy(o).cuda() for o in om])
    start = [f.cpu().numpy().copy() for f in F]
    ctx.close()
    run_parity(T, start, R, s, 1.0 / s, 6, "f64", 1e-10, OT=OT, label="after-rrf")


def test_rrf_argument_errors():
    T, _, R = synth.small3(0)
    fac = synth.gaussian_factors(T.dims, R, 1)
    ctx, F = make_ctx(T, fac, R, 256, gather="f64")
    om = [torch.zeros((300, R), dtype=torch.float64, device="cuda:0") for _ in range(3)]
    with pytest.raises(CpalError):
        ctx.rrf_init(300, om)   # s_init above the context's sample count
    before = [f.cpu().numpy().copy() for f in F]
    for m in range(3):
        assert np.array_equal(F[m].cpu().numpy(), before[m])
    ctx.close()
