"""The full CP-ARLS-LEV loop of Alg. 3 through the C ABI (cp_arls_lev_run)
against the oracle's loop (oracle.cp_arls_lev_run): epochs of eta = 5
iterations, the estimated fit of Sec. 6.4 after each epoch from the same
stratified sample (same Philox counters on both sides), stop after pi = 3
epochs without an improvement above tol = 1e-4.  FP64 gather, both sides
from the same initial factors and seed, factors never exchanged: the fit
traces agree to 1e-10, the runs stop at the same epoch, and the exact fit of
the device's final factors (cp_arls_lev_fit_exact) equals the oracle's exact
fit of the same factors."""
import numpy as np
import pytest

import oracle
from paper_2006_16438_amd import synth
from tests.gpu_util import log, make_ctx

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which", ["small3", "uber4"])
def test_run_matches_oracle_loop(which):
    if which == "small3":
        T, _, R = synth.small3(0)
        s, s_fit, max_epochs = 1024, 1 << 14, 30
    else:
        T = synth.uber4(0)
        R, s, s_fit, max_epochs = 25, 1 << 17, 1 << 20, 8
    tau = 1.0 / s
    fac = synth.gaussian_factors(T.dims, R, 0)
    OT = oracle.Tensor.from_synth(T)
    fs = oracle.FitSample(OT, s_fit, 0.5, seed=0, stream_id=0)
    ctx, F = make_ctx(T, fac, R, s, tau, "f64", fit_samples=s_fit)
    log(f"{which}: device loop")
    got = ctx.run(eta=5, pi=3, tol=1e-4, max_epochs=max_epochs)
    log(f"  device: epochs {got['epochs']} stopped {got['stopped']} trace {np.round(got['trace'], 6)}")
    fo = [f.copy() for f in fac]
    ref = oracle.cp_arls_lev_run(OT, fo, R, s, eta=5, pi=3, tol=1e-4, max_epochs=max_epochs,
                                 tau=tau, fit_sample=fs)
    log(f"  oracle: epochs {ref['epochs']} stopped {ref['stopped']}")
    assert got["epochs"] == ref["epochs"] and got["stopped"] == ref["stopped"]
    d = np.max(np.abs(got["trace"] - ref["trace"]))
    log(f"  max |fit trace difference| {d:.2e}")
    assert d <= 1e-10
    exact_orc = oracle.fit_exact(OT, [f.cpu().numpy() for f in F], R)
    assert abs(got["final_exact_fit"] - exact_orc) <= 1e-10
    bc = got["trace_bias_corrected"]
    assert abs(bc[-1] - got["final_exact_fit"]) < 1e-12
    ctx.close()


@pytest.mark.parametrize("gather", ["f64", "f32"])
def test_exact_fit_matches_oracle(gather):
    T, _, R = synth.small3(0)
    fac = synth.gaussian_factors(T.dims, R, 3)
    OT = oracle.Tensor.from_synth(T)
    ctx, F = make_ctx(T, fac, R, 1024, gather=gather)
    for u in range(4):
        host = [f.cpu().numpy() for f in F]
        ref = oracle.fit_exact(OT, host, R)
        got = float(ctx.fit_exact().item())
        tol = 1e-10 if gather == "f64" else 1e-6   # FP32 copies of the values
        assert abs(got - ref) <= tol, (u, got, ref)
        ctx.mode_update(u % 3)
    ctx.close()


def test_exact_fit_dense_matches_oracle():
    T, _ = synth.planted((20, 15, 12), 3, seed=4, density=1.0, law="normal")
    R = 4
    fac = synth.gaussian_factors(T.dims, R, 5)
    OT = oracle.Tensor.from_synth(T)
    ctx, F = make_ctx(T, fac, R, 256, gather="f64", dense=True)
    got = float(ctx.fit_exact().item())
    ref = oracle.fit_exact(OT, [f.copy() for f in fac], R)
    assert abs(got - ref) <= 1e-10
    ctx.close()
