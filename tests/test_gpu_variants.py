"""The sampling distributions of App. B on the device (cpal_options.sampling):
uniform and length-squared row probabilities, in the random-only (tau = 1)
and hybrid (tau = 1/s) settings.  Only the probability vector changes, so the
parity protocol is the one of the leverage-score method: per update with
identical inputs, sample indices, omega, weights, statistics and the row
scores bit for bit; factors within 1e-10 (FP64 gather) or the derived bound
(FP32 gather)."""
import pytest

from paper_2006_16438_amd import synth
from tests.gpu_util import log, run_parity

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["uniform", "length_squared"])
@pytest.mark.parametrize("tau", ["random", "hybrid"])
def test_sampling_variants_small3(kind, tau):
    T, _, R = synth.small3(0)
    fac = synth.gaussian_factors(T.dims, R, 0)
    s = 1024
    log(f"small3 sampling={kind} tau={tau}")
    run_parity(T, fac, R, s, 1.0 if tau == "random" else 1.0 / s, 6, "f64", 1e-10,
               label=f"{kind}-{tau}", sampling=kind)


@pytest.mark.parametrize("kind", ["uniform", "length_squared"])
def test_sampling_variants_uber_shape_fp32(kind):
    """Uber-shaped 4-way tensor (200k nonzeros, R = 25 > n_1 = 24), FP32 gather."""
    T = synth.uber4(0, nnz=200_000)
    R = 25
    fac = synth.gaussian_factors(T.dims, R, 0)
    log(f"uber-shape sampling={kind}")
    run_parity(T, fac, R, 1 << 14, 1.0, 4, "f32", "derived", label=f"uber-{kind}",
               sampling=kind)
