"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics (no GPU).  Every test here checks the oracle against something
other than itself: a library routine, a closed form, an invariant stated in
the paper, or brute force on tiny inputs."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2006_16438_amd import synth


# ----------------------------------------------------------------- helpers --
def krp_rows(factors, modes):
    """Explicit KRP of factors[modes] (first listed mode fastest), eq. (2.1)."""
    Z = factors[modes[0]].copy()
    for m in modes[1:]:
        A = factors[m]
        Z = (A[:, None, :] * Z[None, :, :]).reshape(A.shape[0] * Z.shape[0], -1)
    return Z


def unfold(dims, coords, vals, k):
    """Dense mode-k unfolding X_(k), columns indexed by the other modes'
    linear index (first other mode fastest)."""
    others = [m for m in range(len(dims)) if m != k]
    N = int(np.prod([dims[m] for m in others]))
    lin = np.zeros(coords.shape[1], dtype=np.int64)
    stride = 1
    for m in others:
        lin += coords[m].astype(np.int64) * stride
        stride *= dims[m]
    X = np.zeros((dims[k], N))
    np.add.at(X, (coords[k], lin), vals)
    return X


def q_vectors(factors, R):
    qs = []
    for A in factors:
        lev, _ = oracle.leverage(A)
        _, _, q, _ = oracle.sampling_vectors(lev, R)
        qs.append(q)
    return qs


def concentrated_factors(dims, R, seed):
    rng = np.random.default_rng(seed)
    fac = []
    for n in dims:
        A = rng.standard_normal((n, R)) * 0.05
        hot = rng.choice(n, size=min(n, R), replace=False)
        for j, h in enumerate(hot):
            A[h, j % R] += 3.0 + j
        fac.append(A)
    return fac


# ------------------------------------------------------------------ Philox --
@pytest.mark.parametrize("key", [(0, 0), (0x1234, 0x5678), (2**64 - 1, 7), (0xDEADBEEF, 2**63)])
def test_philox_matches_numpy(key):
    """numpy's Philox (4x64, 10 rounds) increments its 256-bit counter and
    then emits that block, so a numpy counter of c-1 yields block c."""
    for c0 in [0, 1, 2, 12345, 2**40 + 3]:
        for rest in [(0, 0, 0), (5 | (2 << 8), 9, 0), (2**64 - 1, 3, 1)]:
            ctr = [c0, *rest]
            v = sum(int(c) << (64 * i) for i, c in enumerate(ctr))
            v = (v - 1) % (1 << 256)
            prev = [(v >> (64 * i)) & (2**64 - 1) for i in range(4)]
            ref = np.random.Philox(key=np.array(key, dtype=np.uint64),
                                  counter=np.array(prev, dtype=np.uint64)).random_raw(4)
            assert np.array_equal(oracle.philox(ctr, key), ref), (ctr, key)


def test_scale128_exact():
    rng = np.random.default_rng(3)
    for _ in range(2000):
        u0, u1 = (int(x) for x in rng.integers(0, 2**64, size=2, dtype=np.uint64))
        W = int(rng.integers(1, 2**53, dtype=np.uint64))
        U = (u1 << 64) | u0
        assert oracle.scale128(u0, u1, W) == (U * W) >> 128
    # extremes
    assert oracle.scale128(2**64 - 1, 2**64 - 1, 2**53) == 2**53 - 1
    assert oracle.scale128(0, 0, 12345) == 0


def test_integer_cdf_map_is_exact():
    """Each v in [0, W) maps to the unique i with C[i-1] <= v < C[i], so a
    uniform v picks i with probability exactly w_i / W (multinomial draw)."""
    w = np.array([3, 0, 5, 1, 0, 7, 2], dtype=np.uint64)
    Cdf = np.cumsum(w).astype(np.uint64)
    counts = np.zeros(w.size, dtype=np.int64)
    for v in range(int(Cdf[-1])):
        i = oracle.upper_bound(Cdf, v)
        counts[i] += 1
        lo = 0 if i == 0 else int(Cdf[i - 1])
        assert lo <= v < int(Cdf[i])
    assert np.array_equal(counts, w.astype(np.int64))


# ---------------------------------------------------------------- leverage --
@pytest.mark.parametrize("n,R", [(7, 7), (50, 5), (300, 7), (513, 25), (1000, 64)])
def test_leverage_matches_qr(n, R):
    """Def. 3.4: l_i = ||Q(i,:)||^2 for an orthonormal basis Q of range(A);
    0 <= l <= 1 and sum l = r."""
    rng = np.random.default_rng(n * 100 + R)
    A = rng.standard_normal((n, R))
    lev, fl = oracle.leverage(A)
    Q, _ = np.linalg.qr(A)
    ref = (Q * Q).sum(axis=1)
    assert fl == 0
    assert np.max(np.abs(lev - ref)) <= 1e-12 * max(1.0, R)
    assert abs(lev.sum() - R) <= 1e-11 * R
    assert lev.min() >= 0 and lev.max() <= 1 + 1e-12


def test_leverage_rank_deficient_uses_pinv():
    """Rank-deficient A: leverage is the diagonal of the projector onto
    range(A), sum = rank(A)."""
    rng = np.random.default_rng(11)
    B = rng.standard_normal((120, 4))
    A = np.concatenate([B, B[:, :1] * 2.0], axis=1)      # rank 4, R = 5
    lev, fl = oracle.leverage(A)
    assert fl & oracle.FLAG_PINV
    U, S, _ = np.linalg.svd(A, full_matrices=False)
    Ur = U[:, :4]
    ref = (Ur * Ur).sum(axis=1)
    assert np.max(np.abs(lev - ref)) <= 1e-10
    assert abs(lev.sum() - 4.0) <= 1e-9


def test_gram_blocked_matches_numpy():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((1000, 9))
    G = oracle.gram(A)
    assert np.allclose(G, A.T @ A, rtol=1e-13, atol=1e-12)
    assert np.array_equal(G, G.T)


def test_sampling_vectors_integer_weights():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((400, 6))
    lev, _ = oracle.leverage(A)
    w, Cdf, q, W = oracle.sampling_vectors(lev, 6)
    assert W == int(Cdf[-1]) == int(w.astype(object).sum())
    assert np.array_equal(np.cumsum(w.astype(object)).astype(np.uint64), Cdf)
    # w_i / 2^52 underestimates l_i / R by less than 2^-52
    err = lev / 6 - w.astype(np.float64) / 2.0**52
    assert err.min() >= 0 and err.max() < 2.0**-52 * 1.0000001
    assert abs(q.sum() - 1.0) < 1e-13
    # total mass lost to flooring is below n * 2^-52
    assert 2**52 - W <= 400 + 1


def test_lemma51_krp_leverage_bound():
    """Lemma 5.1: l_i(Z) <= prod_k l_{i_k}(A_k) for Z a Khatri-Rao product."""
    rng = np.random.default_rng(21)
    for dims, R in [((6, 5, 4), 3), ((9, 7), 4), ((4, 3, 5, 2), 2)]:
        fac = [rng.standard_normal((n, R)) for n in dims]
        Z = krp_rows(fac, list(range(len(dims))))
        lz, _ = oracle.leverage(Z)
        levs = [oracle.leverage(A)[0] for A in fac]
        bound = krp_rows([l[:, None] for l in levs], list(range(len(dims))))[:, 0]
        assert np.all(lz <= bound + 1e-12)
        assert abs(lz.sum() - R) < 1e-10


# ---------------------------------------------------------------- sampling --
def test_lemma53_per_mode_draws_follow_product_distribution():
    """Lemma 5.3: independent per-mode draws from l(A_m)/r give KRP row i
    with probability prod q.  Chi-square over 2e5 draws on N = 4*6 rows."""
    dims = (5, 4, 6)
    R = 2
    rng = np.random.default_rng(31)
    fac = [rng.standard_normal((n, R)) for n in dims]
    T = synth.random_sparse(dims, 40, seed=2)
    OT = oracle.Tensor.from_synth(T)
    s = 200_000
    out = oracle.mode_update(OT, [f.copy() for f in fac], 0, 7, R, s, tau=1.0)
    raw = out["raw"].astype(np.int64)
    assert raw.size == s and out["stats"]["s_det"] == 0 and out["stats"]["draws"] == s
    qs = q_vectors(fac, R)
    p = (qs[2][:, None] * qs[1][None, :]).reshape(-1)   # lin = i1 + 4*i2
    counts = np.bincount(raw, minlength=p.size)
    chi2 = ((counts - s * p) ** 2 / (s * p)).sum()
    assert stats.chi2.sf(chi2, p.size - 1) > 1e-6


@pytest.mark.parametrize("tau", [1 / 8, 1 / 32, 1 / 128, 1 / 1024])
def test_det_set_bruteforce(tau):
    """Sec. 5.3: D = {i : p_i > tau} computed without visiting all N rows
    equals the brute-force set over all N; D is inside the product of the
    candidate sets; |D| < 1/tau."""
    dims = (7, 9, 8, 6)
    R = 3
    fac = concentrated_factors(dims, R, 41)
    qs = q_vectors(fac, R)
    k = 2
    others = [0, 1, 3]
    idx, p, pdet, fl = oracle.det_set(dims, qs, k, 10_000, tau)
    true = []
    for i3, i1, i0 in itertools.product(range(dims[3]), range(dims[1]), range(dims[0])):
        pr = qs[0][i0] * qs[1][i1]
        pr = pr * qs[3][i3]
        if pr > tau:
            true.append((i0 + dims[0] * (i1 + dims[1] * i3), pr))
    true.sort()
    assert fl == 0
    assert [int(x) for x in idx] == [t[0] for t in true]
    assert np.array_equal(p, np.array([t[1] for t in true]))
    assert len(true) < 1 / tau
    assert math.isclose(pdet, math.fsum(t[1] for t in true), rel_tol=1e-14, abs_tol=1e-300)
    assert others == [0, 1, 3]


def test_det_set_truncation_keeps_most_probable():
    dims = (5, 6, 4)
    R = 2
    fac = concentrated_factors(dims, R, 43)
    qs = q_vectors(fac, R)
    s = 16
    idx, p, pdet, fl = oracle.det_set(dims, qs, 0, s, 1e-12)
    assert fl & oracle.FLAG_DET_TRUNC
    allp = []
    for i2, i1 in itertools.product(range(dims[2]), range(dims[1])):
        allp.append((-(qs[1][i1] * qs[2][i2]), i1 + dims[1] * i2))
    allp.sort()
    keep = sorted(lin for _, lin in allp[:s])
    assert [int(x) for x in idx] == keep


def test_det_cap_falls_back_to_random():
    dims = (6, 5, 4)
    T = synth.random_sparse(dims, 60, seed=3)
    OT = oracle.Tensor.from_synth(T)
    fac = concentrated_factors(dims, 2, 44)
    out = oracle.mode_update(OT, fac, 0, 0, 2, 64, tau=1e-6, det_cap=3)
    assert out["stats"]["flags"] & oracle.FLAG_DETCAP
    assert out["stats"]["s_det"] == 0 and out["stats"]["p_det"] == 0.0
    assert out["stats"]["draws"] == 64


def test_combining_preserves_sketch_norm():
    """Sec. 4.1/4.3: ||Omega_bar x|| = ||Omega x|| for every x, where the
    uncombined random rows have weight^2 = (1 - p_det) / (s_rnd p_i)."""
    dims = (10, 8, 6)
    R = 3
    T = synth.random_sparse(dims, 200, seed=5)
    OT = oracle.Tensor.from_synth(T)
    fac = concentrated_factors(dims, R, 45)
    qs = q_vectors(fac, R)
    out = oracle.mode_update(OT, [f.copy() for f in fac], 1, 3, R, 300)
    st = out["stats"]
    assert st["s_det"] > 0 and st["s_rnd"] > 0
    N = dims[0] * dims[2]
    pfull = (qs[2][:, None] * qs[0][None, :]).reshape(-1)    # lin = i0 + 10*i2
    rng = np.random.default_rng(0)
    for _ in range(5):
        x = rng.standard_normal(N)
        raw = out["raw"].astype(np.int64)
        unc = np.sum((1 - st["p_det"]) / (st["s_rnd"] * pfull[raw]) * x[raw] ** 2)
        sd = st["s_det"]
        det = np.sum(x[out["idx"][:sd].astype(np.int64)] ** 2)
        comb = np.sum(out["omega"][sd:] * x[out["idx"][sd:].astype(np.int64)] ** 2)
        assert math.isclose(det + unc, det + comb, rel_tol=1e-12)
    # counts: omega_j = c_j (1 - p_det) / (s_rnd p_j) with c_j the multiplicity
    uniq, cnt = np.unique(out["raw"], return_counts=True)
    sd = st["s_det"]
    assert np.array_equal(uniq, out["idx"][sd:])
    expect = cnt * (1 - st["p_det"]) / (st["s_rnd"] * pfull[uniq.astype(np.int64)])
    assert np.allclose(out["omega"][sd:], expect, rtol=1e-14)
    assert np.array_equal(out["wgt"], np.sqrt(out["omega"]))
    # deterministic and random rows are disjoint and each part is ascending
    assert not set(out["idx"][:sd].tolist()) & set(uniq.tolist())
    assert np.all(np.diff(out["idx"][:sd].astype(np.int64)) > 0)


def test_hybrid_sketch_is_unbiased():
    """Lemma 3.2 with the hybrid reweighting of Sec. 4.2: E||Omega x||^2 =
    ||x||^2.  Monte Carlo over 600 seeds, 5 standard errors."""
    dims = (6, 5, 4)
    R = 2
    T = synth.random_sparse(dims, 30, seed=6)
    OT = oracle.Tensor.from_synth(T)
    fac = concentrated_factors(dims, R, 46)
    N = dims[1] * dims[2]
    x = np.random.default_rng(1).standard_normal(N)
    ests = []
    saw_det = False
    for seed in range(600):
        out = oracle.mode_update(OT, [f.copy() for f in fac], 0, 0, R, 8, tau=1 / 8, seed=seed)
        saw_det |= out["stats"]["s_det"] > 0
        ests.append(np.sum(out["omega"] * x[out["idx"].astype(np.int64)] ** 2))
    ests = np.array(ests)
    se = ests.std(ddof=1) / math.sqrt(ests.size)
    assert saw_det
    assert abs(ests.mean() - np.sum(x * x)) < 5 * se


# ----------------------------------------------------------- mode update --
@pytest.mark.parametrize("dims,k", [((9, 7, 5), 0), ((9, 7, 5), 2), ((6, 5, 4, 3), 1), ((40, 30), 0)])
def test_all_rows_update_equals_cp_als(dims, k):
    """tau = 0 and s > N: every KRP row is deterministic with weight 1 and
    the sampled update is the CP-ALS normal-equations step
    A_k = X_(k) Z (Z^T Z)^{-1}, Z^T Z = Hadamard product of the Grams."""
    R = 3
    T = synth.random_sparse(dims, int(0.4 * np.prod(dims)), seed=7)
    OT = oracle.Tensor.from_synth(T)
    fac = synth.gaussian_factors(dims, R, 8)
    others = [m for m in range(len(dims)) if m != k]
    N = int(np.prod([dims[m] for m in others]))
    Z = krp_rows(fac, others)
    Xk = unfold(dims, T.coords, T.values, k)
    V = np.ones((R, R))
    for m in others:
        V *= fac[m].T @ fac[m]
    assert np.allclose(Z.T @ Z, V, rtol=1e-12)
    ref = np.linalg.solve(V, (Xk @ Z).T).T
    f2 = [f.copy() for f in fac]
    out = oracle.mode_update(OT, f2, k, 0, R, N + 5, tau=0.0, det_cap=N + 1)
    st = out["stats"]
    assert st["s_det"] == N and st["s_rnd"] == 0 and st["flags"] & oracle.FLAG_PDET_ONE
    assert np.array_equal(out["idx"], np.arange(N, dtype=np.uint64))
    assert np.all(out["omega"] == 1.0)
    assert st["gathered_nnz"] == T.nnz
    err = np.max(np.abs(f2[k] - ref)) / np.max(np.abs(ref))
    assert err < 1e-12


def test_update_solves_the_explicit_sketched_problem():
    """Eq. (1.2): the update is argmin ||Omega Z B^T - Omega X_(k)^T|| with
    Omega given by the returned rows and weights; built explicitly here and
    solved by QR (numpy lstsq).  Sparse X, so some sampled fibers are empty
    and still enter the system as zero rows."""
    dims = (12, 10, 8)
    R = 4
    T = synth.random_sparse(dims, 60, seed=9)
    OT = oracle.Tensor.from_synth(T)
    fac = concentrated_factors(dims, R, 47)
    saw_empty = False
    for k in range(3):
        f2 = [f.copy() for f in fac]
        out = oracle.mode_update(OT, f2, k, 11 + k, R, 96)
        others = [m for m in range(3) if m != k]
        Z = krp_rows(fac, others)
        Xk = unfold(dims, T.coords, T.values, k)
        ii = out["idx"].astype(np.int64)
        wv = out["wgt"][:, None]
        Zs = wv * Z[ii]
        Xs = wv * Xk[:, ii].T
        saw_empty |= bool(np.any(np.all(Xk[:, ii] == 0, axis=0)))
        B, *_ = np.linalg.lstsq(Zs, Xs, rcond=None)
        ref = B.T
        err = np.max(np.abs(f2[k] - ref)) / np.max(np.abs(ref))
        assert err < 1e-9
        assert out["stats"]["gathered_nnz"] == int(np.count_nonzero(Xk[:, ii]))
    assert saw_empty, "want at least one empty sampled fiber"


def test_exact_model_is_recovered_from_any_sample():
    """Noise-free rank-R tensor, all entries stored, other factors exact:
    the sampled LS is consistent, so the true A_k comes back."""
    dims = (8, 7, 6)
    R = 3
    T, fac = synth.planted(dims, R, seed=12, rel_noise=0.0)
    OT = oracle.Tensor.from_synth(T)
    for k in range(3):
        f2 = [f.copy() for f in fac]
        f2[k] = np.random.default_rng(k).standard_normal(f2[k].shape)
        oracle.mode_update(OT, f2, k, k, R, 40)
        assert np.max(np.abs(f2[k] - fac[k])) < 1e-10


def _fms(A, B):
    """Factor match score over the best column permutation (congruence)."""
    R = A[0].shape[1]
    best = 0.0
    for perm in itertools.permutations(range(R)):
        sc = 0.0
        for r in range(R):
            prod = 1.0
            for Am, Bm in zip(A, B):
                a = Am[:, r] / np.linalg.norm(Am[:, r])
                b = Bm[:, perm[r]] / np.linalg.norm(Bm[:, perm[r]])
                prod *= abs(a @ b)
            sc += prod
        best = max(best, sc / R)
    return best


def test_planted_model_recovery():
    """Whole loop (Alg. 3 with fixed iterations): a fully stored planted
    rank-3 tensor with 1% noise is recovered (FMS >= 0.99, fit near 1 - noise)
    from at least one of four random starts."""
    dims = (30, 25, 20)
    R = 3
    T, fac = synth.planted(dims, R, seed=13, rel_noise=0.01)
    OT = oracle.Tensor.from_synth(T)
    results = []
    for restart in range(4):
        f = synth.gaussian_factors(dims, R, 100 + restart)
        oracle.cp_arls_lev(OT, f, R, 512, 25, seed=restart)
        results.append((oracle.fit_exact(OT, f, R), _fms(fac, f)))
    fit, fms = max(results)
    assert fms >= 0.99, results
    assert fit >= 1 - 1.5 * 0.01, results


def test_zero_factor_is_a_state_error():
    dims = (5, 4, 3)
    T = synth.random_sparse(dims, 20, seed=1)
    OT = oracle.Tensor.from_synth(T)
    fac = synth.gaussian_factors(dims, 2, 1)
    fac[1][:] = 0.0
    with pytest.raises(RuntimeError):
        oracle.mode_update(OT, fac, 0, 0, 2, 16)


# --------------------------------------------------------------------- fit --
def test_exact_fit_matches_dense():
    dims = (7, 6, 5)
    R = 3
    T = synth.random_sparse(dims, 80, seed=14)
    OT = oracle.Tensor.from_synth(T)
    fac = synth.gaussian_factors(dims, R, 15)
    X = np.zeros(dims)
    X[tuple(T.coords)] = T.values
    M = np.einsum("ir,jr,kr->ijk", *fac)
    ref = 1 - np.linalg.norm(X - M) / np.linalg.norm(X)
    assert math.isclose(oracle.fit_exact(OT, fac, R), ref, rel_tol=1e-11, abs_tol=1e-11)
    coord = T.coords[:, 3]
    assert math.isclose(oracle.model_entry(fac, coord), M[tuple(coord)], rel_tol=1e-13)


def test_fit_estimate_is_unbiased_and_stratified():
    """Sec. 6.4: ceil(alpha s_fit) nonzeros and floor((1-alpha) s_fit) zeros,
    zeros never stored coordinates, and E[F_hat] = ||X - M||^2."""
    dims = (8, 7, 6)
    R = 2
    T = synth.random_sparse(dims, 50, seed=16)
    OT = oracle.Tensor.from_synth(T)
    fac = synth.gaussian_factors(dims, R, 17)
    X = np.zeros(dims)
    X[tuple(T.coords)] = T.values
    M = np.einsum("ir,jr,kr->ijk", *fac)
    F = np.sum((X - M) ** 2)
    stored = set(map(tuple, T.coords.T.tolist()))
    ests = []
    for sid in range(300):
        fs = oracle.FitSample(OT, 33, 0.5, seed=4, stream_id=sid)
        assert fs.n == 33
        zc = fs.coords[:, 17:33]
        assert all(tuple(c) not in stored for c in zc.T.tolist())
        assert np.all(fs.x[17:33] == 0)
        assert np.all(fs.phi[:17] == 50 / 17) and np.all(fs.phi[17:33] == (336 - 50) / 16)
        fhat = (1 - fs.estimate(fac)) ** 2 * OT.norm ** 2
        ests.append(fhat)
    ests = np.array(ests)
    se = ests.std(ddof=1) / math.sqrt(ests.size)
    assert abs(ests.mean() - F) < 5 * se


def test_single_row_krp_is_always_accepted():
    """Degenerate N = 1 (every other mode has size 1): p = 1 = tau for the
    random-only setting, and Alg. 2 keeps rows with p <= tau, so all s draws
    are accepted and combine into one row of weight sqrt(s/s)."""
    dims = (5, 1)
    T = synth.random_sparse(dims, 4, seed=2)
    OT = oracle.Tensor.from_synth(T)
    fac = synth.gaussian_factors(dims, 1, 3)
    out = oracle.mode_update(OT, fac, 0, 0, 1, 7, tau=1.0)
    st = out["stats"]
    assert st["draws"] == 7 and st["s_rnd"] == 7 and st["s_bar"] == 1
    assert out["omega"][0] == 1.0 and st["flags"] == 0


def test_leverage_fewer_rows_than_rank():
    """n < R with full row rank: range(A) = R^n, so every leverage score is
    exactly 1 (the projector is the identity); with a repeated row the rank
    drops and the projector from the SVD applies."""
    rng = np.random.default_rng(12)
    A = rng.standard_normal((24, 25))
    lev, fl = oracle.leverage(A)
    assert fl & oracle.FLAG_PINV
    assert np.all(lev == 1.0)
    U, S, _ = np.linalg.svd(A, full_matrices=False)
    assert np.allclose((U * U).sum(axis=1), 1.0, atol=1e-12)
    B = A.copy()
    B[5] = B[3]                      # rank 23
    lev, fl = oracle.leverage(B)
    U, S, _ = np.linalg.svd(B, full_matrices=False)
    ref = (U[:, :23] ** 2).sum(axis=1)
    assert fl & oracle.FLAG_PINV
    assert np.max(np.abs(lev - ref)) < 1e-10
    assert abs(lev.sum() - 23) < 1e-9


# ------------------------------------- singular G_s, draw guards, zero stratum --
def _sketched_minimum_norm(dims, T, fac, k, out):
    """argmin ||Omega Z B^T - Omega X_(k)^T|| of eq. (1.2) built explicitly
    from the returned rows and weights; numpy's SVD-based lstsq returns the
    minimizer of least norm when the system is rank-deficient."""
    others = [m for m in range(len(dims)) if m != k]
    Z = krp_rows(fac, others)
    Xk = unfold(dims, T.coords, T.values, k)
    ii = out["idx"].astype(np.int64)
    wv = out["wgt"][:, None]
    B, *_ = np.linalg.lstsq(wv * Z[ii], wv * Xk[:, ii].T, rcond=None)
    return B.T


@pytest.mark.parametrize("case", ["collinear", "one_sample"])
def test_singular_sampled_gram_gives_minimum_norm_solution(case):
    """A singular G_s = Z~^T Z~ leaves the sketched problem (1.2) with many
    minimizers; the update takes the one of least norm, G_s^+ applied to M
    (the pseudo-inverse branch of the solve).  'collinear': two KRP columns
    are equal bit for bit (the null vector (1, -1, 0) is not a coordinate
    axis, so a transposed or mis-cut eigenbasis fails); 'one_sample': s = 1
    gives a rank-1 G_s."""
    dims = (9, 7, 6)
    R = 3
    T = synth.random_sparse(dims, 150, seed=21)
    OT = oracle.Tensor.from_synth(T)
    fac = synth.gaussian_factors(dims, R, 22)
    if case == "collinear":
        for m in (1, 2):
            fac[m][:, 1] = fac[m][:, 0]
        s, tau = 24, None
    else:
        s, tau = 1, 1.0
    for k in range(3):
        if case == "collinear" and k != 0:
            continue
        f2 = [f.copy() for f in fac]
        out = oracle.mode_update(OT, f2, k, 3 + k, R, s, tau)
        assert out["stats"]["flags"] & oracle.FLAG_PINV
        ref = _sketched_minimum_norm(dims, T, fac, k, out)
        err = np.max(np.abs(f2[k] - ref)) / np.max(np.abs(ref))
        assert err < 1e-10, (case, k, err)
        if case == "collinear":
            # the least-norm solution splits equally over the two equal columns
            assert np.max(np.abs(f2[k][:, 0] - f2[k][:, 1])) < 1e-12 * np.max(np.abs(f2[k]))


def test_draw_guard_stops_rejection_and_normalizes_by_accepted_draws():
    """One KRP row holds almost all probability (p ~ 0.99999 > tau), so it is
    deterministic and a random draw is accepted (p <= tau) only with
    probability 1 - p_det ~ 1e-5: the rejection loop of Alg. 2 stops at the
    guard of 64 s_rnd + 2^20 draws with fewer accepted draws than asked for.
    The weights then use the number of accepted draws (the draws are an
    i.i.d. sample of that size from p restricted to p <= tau), which makes
    sum_rnd omega_j p_j = 1 - p_det hold exactly: the random rows estimate
    the mass outside the deterministic set without bias (Lemma 3.2)."""
    dims = (6, 7, 8)
    R = 1
    T = synth.random_sparse(dims, 100, seed=5)
    OT = oracle.Tensor.from_synth(T)
    fac = [np.ones((n, 1)) for n in dims]
    fac[1][0, 0] = 1000.0
    fac[2][0, 0] = 1000.0
    s = 2048
    tau = 1.0 / s
    f2 = [f.copy() for f in fac]
    out = oracle.mode_update(OT, f2, 0, 0, R, s, tau)
    st = out["stats"]
    assert st["flags"] & oracle.FLAG_DRAWCAP
    assert st["s_det"] == 1 and out["idx"][0] == 0
    assert st["draws"] == 64 * (s - 1) + (1 << 20)
    assert 0 < st["s_rnd"] < s - 1
    assert out["raw"].size == st["s_rnd"]
    q = q_vectors(fac, R)
    lin = out["idx"][1:].astype(np.int64)
    p = q[1][lin % 7] * q[2][lin // 7]
    assert np.all(p <= tau)
    om = out["omega"][1:]
    assert abs(np.sum(om * p) - (1 - st["p_det"])) < 1e-12 * (1 - st["p_det"])
    counts = om * st["s_rnd"] * p / (1 - st["p_det"])
    assert np.allclose(counts, np.round(counts), atol=1e-9) and round(counts.sum()) == st["s_rnd"]


def test_fit_estimate_zero_stratum_weight_uses_the_zeros_drawn():
    """A nearly full tensor (998 of 1000 entries stored): the rejection
    sampling of zeros (Sec. 6.4) stops at its guard with fewer zeros than
    floor((1 - alpha) s_fit).  The zero stratum (2 entries) is then
    represented by the zeros actually drawn, phi = 2 / drawn, and F_hat
    still estimates ||X - M||^2 = the model's squares at the two zeros
    (the stored values equal the model, so the nonzero stratum adds 0)."""
    dims = (10, 10, 10)
    R = 2
    fac = synth.gaussian_factors(dims, R, 5)
    full = np.array(np.unravel_index(np.arange(1000), dims, order="F"), dtype=np.int32)
    missing = [137, 802]
    keep = np.setdiff1d(np.arange(1000), missing)
    coords = np.ascontiguousarray(full[:, keep])
    M = np.einsum("ir,jr,kr->ijk", *fac)
    vals = M[tuple(coords)]
    OT = oracle.Tensor(dims, coords, vals)
    fs = oracle.FitSample(OT, 20000, 0.5, seed=0)
    assert fs.flags & oracle.FLAG_DRAWCAP
    got = fs.n - 10000
    assert 0 < got < 10000
    assert np.all(fs.phi[10000:fs.n] == 2.0 / got)
    F = sum(M[tuple(full[:, e])] ** 2 for e in missing)
    fhat = ((1 - fs.estimate(fac)) * OT.norm) ** 2
    assert abs(fhat / F - 1) < 0.1, (fhat, F)


# ------------------------------------------------------------- Alg. 3 loop --
def _first_stop(trace, pi, tol):
    """Epoch count at which 'pi consecutive epochs without beating the best
    earlier fit by more than tol' first holds (None if it never does)."""
    best, fails = -np.inf, 0
    for e, f in enumerate(trace):
        fails = 0 if f > best + tol else fails + 1
        best = max(best, f)
        if fails >= pi:
            return e + 1
    return None


@pytest.mark.parametrize("fit", ["exact", "estimated"])
def test_full_loop_stops_by_the_epoch_rule_at_the_noise_floor(fit):
    """Alg. 3 with epochs (eta = 5), pi = 3 and tol = 1e-4 on a fully stored
    planted rank-3 tensor with 1% noise: the run ends at the first epoch
    where the stopping rule holds for its recorded trace, it ends because of
    the rule (not the epoch limit), the final factors reach the fit of the
    planted model (1 - ||E||/||X||, up to what the sampled solves leave), and
    the trace's exact fits equal a dense numpy evaluation of ||X - M||."""
    dims = (30, 25, 20)
    R = 3
    T, planted = synth.planted(dims, R, seed=13, rel_noise=0.01)
    OT = oracle.Tensor.from_synth(T)
    X = np.zeros(dims)
    X[tuple(T.coords)] = T.values
    floor = 1 - np.linalg.norm(X - np.einsum("ir,jr,kr->ijk", *planted)) / np.linalg.norm(X)
    fs = oracle.FitSample(OT, 4096, 1.0, seed=3) if fit == "estimated" else None
    best_run = None
    for restart in range(4):
        f = synth.gaussian_factors(dims, R, 100 + restart)
        out = oracle.cp_arls_lev_run(OT, f, R, 512, eta=5, pi=3, tol=1e-4, max_epochs=60,
                                     seed=restart, fit_sample=fs)
        assert out["stopped"]
        assert _first_stop(out["trace"], 3, 1e-4) == out["epochs"]
        M = np.einsum("ir,jr,kr->ijk", *f)
        dense = 1 - np.linalg.norm(X - M) / np.linalg.norm(X)
        assert abs(out["final_exact_fit"] - dense) < 1e-10
        if fit == "exact":
            assert abs(out["trace"][-1] - dense) < 1e-10
        if best_run is None or out["final_exact_fit"] > best_run["final_exact_fit"]:
            best_run = out
    assert best_run["final_exact_fit"] > floor - 2e-3, (best_run["final_exact_fit"], floor)


def test_epoch_rule_counts_consecutive_failures_against_the_best_fit():
    """The rule on hand-made traces: improvements smaller than tol count as
    failures, a later improvement resets the count, and the reference is the
    best earlier fit (a dip and recovery to below best + tol is a failure)."""
    assert _first_stop([0.5, 0.50005, 0.5001, 0.50015], 3, 1e-4) == 4
    assert _first_stop([0.5, 0.50005, 0.5002, 0.50021, 0.50022, 0.50023], 3, 1e-4) == 6
    assert _first_stop([0.5, 0.4, 0.6, 0.59, 0.6, 0.6], 3, 1e-4) == 6
    assert _first_stop([0.1, 0.2, 0.3], 1, 1e-4) is None


# ------------------------------------------- sampling distributions of App. B --
def test_length_squared_probabilities_are_normalised_row_norms():
    """App. B: length-squared sampling takes row i of A with probability
    ||A(i,:)||^2 / ||A||_F^2; the integer weights reproduce it to the
    2^-52 resolution of the CDF."""
    rng = np.random.default_rng(41)
    A = rng.standard_normal((300, 7)) * rng.uniform(0.1, 3.0, size=(300, 1))
    sc, S = oracle.scores(A, "length_squared")
    ref = np.sum(A * A, axis=1)
    assert np.allclose(sc, ref, rtol=1e-14)
    assert math.isclose(S, np.sum(A * A), rel_tol=1e-13)
    _, Cdf, q, W = oracle.sampling_vectors_norm(sc, S)
    assert np.all(np.abs(q - ref / np.sum(ref)) <= (A.shape[0] + 2) * 2.0 ** -52)
    assert int(Cdf[-1]) == W


def test_uniform_probabilities_are_equal():
    A = np.random.default_rng(42).standard_normal((37, 4))
    sc, S = oracle.scores(A, "uniform")
    assert np.all(sc == 1.0) and S == 37.0
    w, _, q, _ = oracle.sampling_vectors_norm(sc, S)
    assert np.all(w == w[0]) and np.all(q == q[0]) and abs(q[0] - 1 / 37) < 1e-16


def test_length_squared_krp_row_bound():
    """App. B: ||Z(i,:)||^2 <= prod_k ||A_k(i_k,:)||^2 for the rows of the
    KRP (brute force over every row of a small KRP)."""
    rng = np.random.default_rng(43)
    fac = [rng.standard_normal((n, 5)) for n in (6, 7, 5)]
    Z = krp_rows(fac, [0, 1, 2])
    zn = np.sum(Z * Z, axis=1)
    bound = (np.sum(fac[2] ** 2, 1)[:, None, None] * np.sum(fac[1] ** 2, 1)[None, :, None]
             * np.sum(fac[0] ** 2, 1)[None, None, :]).reshape(-1)
    assert np.all(zn <= bound * (1 + 1e-13))


@pytest.mark.parametrize("kind", ["uniform", "length_squared"])
def test_other_distributions_draw_the_product_probabilities(kind):
    """The per-mode draws of Alg. 2 with App. B's row probabilities give KRP
    row i with probability prod q (chi-square over 2e5 draws, N = 24)."""
    dims = (5, 4, 6)
    R = 2
    rng = np.random.default_rng(31)
    fac = [rng.standard_normal((n, R)) for n in dims]
    T = synth.random_sparse(dims, 40, seed=2)
    OT = oracle.Tensor.from_synth(T)
    s = 200_000
    out = oracle.mode_update(OT, [f.copy() for f in fac], 0, 7, R, s, tau=1.0, sampling=kind)
    raw = out["raw"].astype(np.int64)
    qs = []
    for A in fac:
        sc = np.sum(A * A, axis=1) if kind == "length_squared" else np.ones(A.shape[0])
        qs.append(sc / sc.sum())
    p = (qs[2][:, None] * qs[1][None, :]).reshape(-1)
    counts = np.bincount(raw, minlength=p.size)
    chi2 = ((counts - s * p) ** 2 / (s * p)).sum()
    assert stats.chi2.sf(chi2, p.size - 1) > 1e-6


@pytest.mark.parametrize("kind", ["uniform", "length_squared"])
def test_other_distributions_solve_the_sketched_problem(kind):
    """Only the probability vector changes: the update is still the
    least-squares solution of the explicit sketched problem (1.2) with the
    returned rows and weights, and the weights follow Sec. 4.3 with the
    distribution's probabilities."""
    dims = (12, 10, 8)
    R = 4
    T = synth.random_sparse(dims, 60, seed=9)
    OT = oracle.Tensor.from_synth(T)
    fac = concentrated_factors(dims, R, 47)
    for k in range(3):
        f2 = [f.copy() for f in fac]
        out = oracle.mode_update(OT, f2, k, 11 + k, R, 96, sampling=kind)
        ref = _sketched_minimum_norm(dims, T, fac, k, out)
        err = np.max(np.abs(f2[k] - ref)) / np.max(np.abs(ref))
        assert err < 1e-9
        others = [m for m in range(3) if m != k]
        qk = {}
        for m in others:
            sc = np.sum(fac[m] ** 2, 1) if kind == "length_squared" else np.ones(dims[m])
            qk[m] = sc / sc.sum()
        lin = out["idx"].astype(np.int64)
        st = out["stats"]
        p = qk[others[0]][lin % dims[others[0]]] * qk[others[1]][lin // dims[others[0]]]
        rnd = slice(st["s_det"], None)
        assert np.all(p[:st["s_det"]] > 1 / 96) and np.all(p[rnd] <= 1 / 96 * (1 + 1e-12))
        assert abs(np.sum(out["omega"][rnd] * p[rnd]) - (1 - st["p_det"])) < 1e-9


def test_threaded_oracle_matches_sequential():
    """The oracle's threaded loops (blocks of draws, Gram rows, leverage
    rows, the sampled system summed row by row in sample order, solved rows)
    give the same bits as the sequential loops: the GPU parity bar never
    depends on how the oracle was run, and its all-thread timing measures the
    same computation."""
    import oracle
    from paper_2006_16438_amd import synth
    T = synth.random_sparse((300, 120, 90), 60_000, seed=9)
    R, s = 7, 2048
    OT = oracle.Tensor.from_synth(T)
    fac = synth.gaussian_factors(T.dims, R, 4)
    runs = []
    for threads in (1, 4):
        oracle.set_threads(threads)
        F = [f.copy() for f in fac]
        out = []
        for t in range(6):
            r = oracle.mode_update(OT, F, t % 3, t, R, s, 1.0 / s)
            out.append((r["idx"].copy(), r["omega"].copy(), r["stats"]["gathered_nnz"],
                        r["stats"]["draws"], [f.copy() for f in F]))
        runs.append(out)
    oracle.set_threads(1)
    for a, b in zip(*runs):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert a[2] == b[2] and a[3] == b[3]
        for fa, fb in zip(a[4], b[4]):
            assert np.array_equal(fa.view(np.uint64), fb.view(np.uint64))


# --------------------------------------------------------- RRF initialisation --
def _np_philox_block(ctr, key):
    v = (sum(int(c) << (64 * i) for i, c in enumerate(ctr)) - 1) % (1 << 256)
    prev = [(v >> (64 * i)) & (2**64 - 1) for i in range(4)]
    return np.random.Philox(key=np.array(key, dtype=np.uint64),
                            counter=np.array(prev, dtype=np.uint64)).random_raw(4)


@pytest.mark.parametrize("dims,nnz,k", [((9, 7, 5), 60, 0), ((9, 7, 5), 60, 2),
                                       ((6, 5, 4, 3), 90, 1)])
def test_rrf_init_matches_independent_recomputation(dims, nnz, k):
    """App. F: A_k = X_(k)(:, F) Omega for uniform draws F of nonempty
    fibers, recomputed here without the oracle: fibers from numpy's unique
    over the other-mode linear indices, draws from numpy's Philox and exact
    integer arithmetic, dense fiber vectors from the COO entries."""
    from paper_2006_16438_amd import synth
    T = synth.random_sparse(dims, nnz, seed=17)
    OT = oracle.Tensor.from_synth(T)
    R, s_init, seed, sid = 4, 40, 5, 2
    omega = np.random.default_rng(3).standard_normal((s_init, R))
    A, nfib = oracle.rrf_init(OT, k, s_init, omega, seed, sid)
    others = [m for m in range(len(dims)) if m != k]
    lin = np.zeros(T.coords.shape[1], dtype=np.int64)
    stride = 1
    for m in others:
        lin += T.coords[m].astype(np.int64) * stride
        stride *= dims[m]
    keys = np.unique(lin)
    assert nfib == keys.size
    ref = np.zeros((dims[k], R))
    for j in range(s_init):
        w = _np_philox_block([j, (k << 8) | (3 << 16), 0, 0], (seed, sid))
        U = (int(w[1]) << 64) | int(w[0])
        u = (U * keys.size) >> 128
        sel = lin == keys[u]
        fiber = np.zeros(dims[k])
        fiber[T.coords[k][sel]] = T.values[sel]
        ref += np.outer(fiber, omega[j])
    assert np.max(np.abs(A - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    # every column lies in the span of the drawn fibers (range finder)
    assert np.linalg.matrix_rank(np.hstack([A, ref])) == np.linalg.matrix_rank(ref)


def test_coherent_generator_concentrates_leverage():
    """App. C's generator: in every factor the 3 x spread seeded rows carry
    the leverage of the three sparse columns (each seeded row >= 1/spread up
    to the Gaussian columns' share), while a Gaussian row of an n x R
    matrix has leverage about R/n; the tensor holds every entry."""
    import oracle
    from paper_2006_16438_amd import synth
    dims, R, spread = (60, 50, 40), 6, 3
    T, fac = synth.coherent(dims, R, spread=spread, seed=1)
    assert T.coords.shape[1] == int(np.prod(dims))
    for A in fac:
        lev, _ = oracle.leverage(A)
        seeded = lev[:3 * spread]
        rest = lev[3 * spread:]
        assert np.all(seeded >= 1.0 / spread - 0.05)
        assert np.sum(seeded) >= 3.0 - 0.1
        assert np.max(rest) < np.min(seeded)
        assert np.all(A[3 * spread:, :3] == 0.0)
