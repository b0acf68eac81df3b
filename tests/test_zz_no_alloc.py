"""The allocation-free entry point cp_arls_lev_leverage_noalloc through the
C ABI: the leverage scores of a caller's matrix, computed with the static
per-GPU scratch array, equal bit for bit the scores a context computed for
the same factor matrix (cp_arls_lev_leverage), on two calls in a row with
the second matrix smaller than the first (the array keeps the first call's
contents), through the Cholesky branch, the row-space branch (fewer rows
than columns) and the pseudo-inverse branch; a matrix whose scratch exceeds
the array is rejected before anything is launched."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2006_16438_amd import _lib as L
from paper_2006_16438_amd import synth
from paper_2006_16438_amd.api import leverage_noalloc
from tests.gpu_util import log, make_ctx

pytestmark = pytest.mark.gpu


def _bits(t):
    return t.cpu().numpy().view(np.uint64)


def test_leverage_noalloc_matches_context_leverage():
    T = synth.uber4(0, nnz=200_000)            # modes of 183, 24, 1140, 1717 rows
    R = 25
    fac = synth.gaussian_factors(T.dims, R, 5)
    fac[2][:, 7] = fac[2][:, 3]                 # a rank-deficient factor: pseudo-inverse
    ctx, F = make_ctx(T, fac, R, 4096, gather="f64")
    torch.cuda.synchronize()
    # larger first, then smaller: 1717 rows, then 1140 (singular Gram), 183, 24 (< R)
    for m in (3, 2, 0, 1):
        ref = ctx.leverage(m)
        got = leverage_noalloc(F[m])
        torch.cuda.synchronize()
        same = np.array_equal(_bits(got), _bits(ref))
        log(f"  mode {m} ({F[m].shape[0]} x {R}): bit-identical {same}, "
            f"sum {float(got.sum()):.12f}")
        assert same
    # after updates the context's factors and scores change; the entry point follows
    for k in range(4):
        ctx.mode_update(k)
    for m in (3, 0):
        assert np.array_equal(_bits(leverage_noalloc(F[m])), _bits(ctx.leverage(m)))
    ctx.close()


def test_leverage_noalloc_many_gram_blocks_matches_oracle():
    """A 40,000-row factor (157 Gram blocks: the partials are summed by a
    separate kernel in the canonical order) gives the oracle's leverage
    scores bit for bit, twice in a row, then a smaller matrix."""
    import oracle
    rng = np.random.default_rng(12)
    for n, R in ((40_000, 25), (40_000, 25), (3000, 7)):
        A = rng.standard_normal((n, R))
        got = leverage_noalloc(torch.from_numpy(A).cuda())
        torch.cuda.synchronize()
        ref, _ = oracle.leverage(A)
        assert np.array_equal(_bits(got), ref.view(np.uint64)), (n, R)


def test_leverage_noalloc_rejects_oversized_matrix():
    A = torch.zeros((4, 64), dtype=torch.float64, device="cuda:0")
    out = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    lib = L.load()
    code = lib.cp_arls_lev_leverage_noalloc(A.data_ptr(), 1 << 24, 64, out.data_ptr(), None)
    assert code == L.CPAL_E_ARG
    msg = lib.cp_arls_lev_last_error(None).decode()
    assert "scratch" in msg
    assert lib.cp_arls_lev_leverage_noalloc(A.data_ptr(), 4, 65, out.data_ptr(), None) == L.CPAL_E_ARG
    assert lib.cp_arls_lev_leverage_noalloc(None, 4, 8, out.data_ptr(), None) == L.CPAL_E_ARG
    assert float(out.abs().sum()) == 0.0
