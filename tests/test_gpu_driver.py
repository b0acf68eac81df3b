"""The full CP-ARLS-LEV loop of Alg. 3 through the C ABI (cp_arls_lev_run)
against the oracle's loop (oracle.cp_arls_lev_run): epochs of eta = 5
iterations, the estimated fit of Sec. 6.4 after each epoch from the same
stratified sample (same Philox counters on both sides), stop after pi = 3
epochs without an improvement above tol = 1e-4.  FP64 gather.

Two protocols, chosen by what the loop's own dynamics allow:

* A planted, fully stored rank-4 tensor with 1% noise, where ALS contracts
  towards the planted model: a relative perturbation of 2^-50 of one initial
  entry stays at ~1e-14 through the whole loop (measured on the oracle), so
  both sides run the whole loop end to end from the same initial factors
  and must stop at the same epoch with fit traces within 1e-10.
* The 100x80x60 workload (planted model RMS below the noise) and the
  Uber-shaped tensor, where the loop amplifies rounding: on the oracle
  alone, the same 2^-50 perturbation grows about 2x per iteration (1e-10
  after 9 iterations, a different sample at iteration 24).  Two
  implementations that round differently cannot agree end to end there,
  so (a) the library's loop is checked against the stop rule applied to
  its own trace, and (b) the epochs are run through the per-update calls
  with the oracle re-fed the device factors at the start of every epoch:
  the epoch's samples, factors and fit estimate must match."""
import numpy as np
import pytest

import oracle
from paper_2006_16438_amd import synth
from tests.gpu_util import log, make_ctx, rel_err

pytestmark = pytest.mark.gpu


def _stop_rule(trace, pi, tol):
    """Epochs run and the stop flag that the rule of Alg. 3 gives for a
    sequence of epoch fits (the loop ends after the first epoch at which pi
    consecutive epochs failed to beat the best earlier fit by more than tol)."""
    best, fails = -np.inf, 0
    for e, f in enumerate(trace):
        fails = 0 if f > best + tol else fails + 1
        best = max(best, f)
        if fails >= pi:
            return e + 1, True
    return len(trace), False


def test_run_matches_oracle_loop_planted():
    T, _ = synth.planted((40, 30, 20), 4, seed=7, density=1.0, rel_noise=0.01, law="normal")
    R, s, s_fit = 4, 512, 1 << 12
    tau = 1.0 / s
    fac = synth.gaussian_factors(T.dims, R, 0)
    OT = oracle.Tensor.from_synth(T)
    fs = oracle.FitSample(OT, s_fit, 0.5, seed=0, stream_id=0)
    ctx, F = make_ctx(T, fac, R, s, tau, "f64", fit_samples=s_fit)
    got = ctx.run(eta=5, pi=3, tol=1e-4, max_epochs=30)
    fo = [f.copy() for f in fac]
    ref = oracle.cp_arls_lev_run(OT, fo, R, s, eta=5, pi=3, tol=1e-4, max_epochs=30,
                                 tau=tau, fit_sample=fs)
    log(f"  device: epochs {got['epochs']} stopped {got['stopped']} trace {np.round(got['trace'], 8)}")
    log(f"  oracle: epochs {ref['epochs']} stopped {ref['stopped']}")
    assert got["epochs"] == ref["epochs"] and got["stopped"] == ref["stopped"]
    d = np.max(np.abs(got["trace"] - ref["trace"]))
    log(f"  max |fit trace difference| {d:.2e}")
    assert d <= 1e-10
    for m in range(3):
        assert rel_err(F[m].cpu().numpy(), fo[m]) <= 1e-10
    exact_orc = oracle.fit_exact(OT, [f.cpu().numpy() for f in F], R)
    assert abs(got["final_exact_fit"] - exact_orc) <= 1e-10
    assert abs(got["trace_bias_corrected"][-1] - got["final_exact_fit"]) < 1e-12
    ctx.close()


@pytest.mark.parametrize("which", ["small3", "uber4"])
def test_run_stop_rule_and_epochwise_parity(which):
    if which == "small3":
        T, _, R = synth.small3(0)
        s, s_fit, max_epochs = 1024, 1 << 14, 30
    else:
        T = synth.uber4(0)
        R, s, s_fit, max_epochs = 25, 1 << 17, 1 << 20, 4
    tau = 1.0 / s
    eta, pi, tol = 5, 3, 1e-4
    fac = synth.gaussian_factors(T.dims, R, 0)
    OT = oracle.Tensor.from_synth(T)
    D = len(T.dims)

    # (a) the library's loop obeys the stop rule on its own trace
    ctx, F = make_ctx(T, fac, R, s, tau, "f64", fit_samples=s_fit)
    got = ctx.run(eta=eta, pi=pi, tol=tol, max_epochs=max_epochs)
    log(f"{which}: device loop epochs {got['epochs']} stopped {got['stopped']} "
        f"trace {np.round(got['trace'], 6)}")
    assert (got["epochs"], got["stopped"]) == _stop_rule(got["trace"], pi, tol)
    assert got["best_fit"] == np.max(got["trace"])
    exact_orc = oracle.fit_exact(OT, [f.cpu().numpy() for f in F], R)
    assert abs(got["final_exact_fit"] - exact_orc) <= 1e-10
    ctx.close()

    # (b) epoch by epoch through the per-update calls, the oracle re-fed the
    # device factors at every epoch start
    fs = oracle.FitSample(OT, s_fit, 0.5, seed=0, stream_id=0)
    ctx, F = make_ctx(T, fac, R, s, tau, "f64", fit_samples=s_fit)
    epochs = min(got["epochs"], 3)
    t = 0
    for e in range(epochs):
        fo = [f.cpu().numpy().copy() for f in F]
        worst = 0.0
        for _ in range(eta):
            for k in range(D):
                ref = oracle.mode_update(OT, fo, k, t, R, s, tau)
                ctx.mode_update(k)
                idx = ctx.samples_view()[0].cpu().numpy().view(np.uint64)
                assert np.array_equal(idx, ref["idx"]), (e, t)
                worst = max(worst, rel_err(F[k].cpu().numpy(), fo[k]))
                t += 1
        fit_d = float(ctx.fit_estimate().item())
        fit_o = fs.estimate(fo)
        log(f"  epoch {e}: fit device {fit_d:.12f} oracle {fit_o:.12f}; max factor error {worst:.1e}")
        assert worst <= 1e-10
        assert abs(fit_d - fit_o) <= 1e-10
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
