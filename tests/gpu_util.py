"""Helpers shared by the GPU tests: build a library context and run the
per-update parity protocol against the CPU oracle.

Protocol (per mode update, identical inputs): the current device factors
are copied to the host, the oracle runs the same update (same step t, seed,
stream id) from those copies, then the device runs it.  Sample indices,
omega and weights, the statistics and the cached leverage scores must match
bit for bit; the new factor within a stated relative tolerance."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dense_values(T):
    """A fully stored tensor (every coordinate, linear order with mode 0
    fastest, as synth.planted(..., density=1.0) makes it) as an array of
    shape dims."""
    assert T.coords.shape[1] == int(np.prod(T.dims)), "every entry must be stored"
    return np.reshape(np.asarray(T.values), tuple(T.dims), order="F")


def make_ctx(T, fac, R, s, tau=None, gather="f64", seed=0, stream_id=0, det_cap=0,
             fit_samples=0, values_f32=False, dense=False, dense_values_gpu=None,
             sampling="leverage"):
    """dense_values_gpu: a dense CUDA tensor of shape T.dims handed over as is."""
    from paper_2006_16438_amd.api import CpArlsLev
    dev = torch.device("cuda:0")
    if dense_values_gpu is not None:
        coords = None
        vals = dense_values_gpu
    elif dense:
        coords = None
        vals = torch.from_numpy(np.ascontiguousarray(dense_values(T))).to(dev)
    else:
        coords = torch.from_numpy(np.ascontiguousarray(T.coords)).to(dev)
        vals = torch.from_numpy(np.ascontiguousarray(T.values)).to(dev)
    if values_f32:
        vals = vals.float()
    F = [torch.from_numpy(np.ascontiguousarray(f, dtype=np.float64).copy()).to(dev) for f in fac]
    ctx = CpArlsLev(T.dims, coords, vals, F, R, s, tau=tau, seed=seed, stream_id=stream_id,
                    gather_dtype=gather, det_enum_cap=det_cap, fit_samples=fit_samples,
                    sampling=sampling)
    return ctx, F


def rel_err(a, b):
    den = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / den)


# unit roundoff of the operands the gather rounds (fiber value and weighted
# KRP row, each rounded once) and of one accumulation step
_U_IN = {"f64": 2.0 ** -52, "f32": 2.0 ** -23, "bf16": 2.0 ** -8}
_U_ACC = {"f64": 2.0 ** -52, "f32": 2.0 ** -24, "bf16": 2.0 ** -24}


def sampled_system(OT, fac, k, idx, om):
    """The explicit sampled system of one update from the oracle's output:
    Z (s_bar x R), G_s = Z^T Omega Z, M = X~^T Omega Z, the same with
    absolute values (|X~|^T Omega |Z|, |Z|^T Omega |Z|), and the largest
    number of terms summed into one entry of M."""
    dims = [int(d) for d in OT.dims]
    others = [m for m in range(len(dims)) if m != k]
    idx = np.asarray(idx, dtype=np.uint64).astype(np.int64)
    om = np.asarray(om, dtype=np.float64)
    R = fac[0].shape[1]
    Z = np.ones((idx.size, R))
    stride = 1
    key = np.zeros(OT.nnz, dtype=np.int64)
    for m in others:
        Z *= fac[m][(idx // stride) % dims[m]]
        key += OT.coords[m].astype(np.int64) * stride
        stride *= dims[m]
    order = np.argsort(idx, kind="stable")
    sidx = idx[order]
    pos = np.searchsorted(sidx, key)
    pos_c = np.minimum(pos, max(idx.size - 1, 0))
    hit = (idx.size > 0) & (sidx[pos_c] == key) if idx.size else np.zeros(OT.nnz, bool)
    j = order[pos_c[hit]]
    ik = OT.coords[k][hit].astype(np.int64)
    x = OT.vals[hit]
    n_k = dims[k]
    M = np.zeros((n_k, R))
    Ma = np.zeros((n_k, R))
    np.add.at(M, ik, (om[j] * x)[:, None] * Z[j])
    np.add.at(Ma, ik, (om[j] * np.abs(x))[:, None] * np.abs(Z[j]))
    G = Z.T @ (om[:, None] * Z)
    Ga = np.abs(Z).T @ (om[:, None] * np.abs(Z))
    n_terms = int(np.bincount(ik, minlength=n_k).max()) if ik.size else 0
    return dict(Z=Z, G=G, Ga=Ga, M=M, Ma=Ma, n_terms=n_terms)


def derived_tolerance(OT, fac, k, ref, gather):
    """First-order bound on the relative Frobenius-norm difference of the new
    factor between the device and the FP64 oracle, from the arithmetic:
    A = M G_s^+ with M = X~^T Omega Z.  The device rounds each fiber value
    and each weighted KRP row once to the gather precision and sums in that
    precision (FP32 for BF16 operands), so every term of M carries a
    relative error of at most u_in + n u_acc (n = terms in the entry):
    ||dM||_F <= (u_in + n u_acc) || |X~|^T Omega |Z| ||_F.  G_s is FP64 on
    both sides, in different orders: ||dG||_F <= 2 n_G 2^-53 || |Z|^T Omega |Z| ||_F.
    With ||A||_F >= ||M||_F / ||G||_2 and dA = dM G^+ - A dG G^+,
      ||dA||_F / ||A||_F <= kappa(G_s) (||dM||_F/||M||_F + ||dG||_F/||G||_2),
    kappa over the nonzero spectrum (the pseudo-inverse when G_s is singular)."""
    sy = sampled_system(OT, fac, k, ref["idx"], ref["omega"])
    return bound_from_system(sy, len(ref["idx"]), gather)


def bound_from_system(sy, n_g, gather):
    """The bound of derived_tolerance from an explicit sampled system (keys
    G, Ga, M, Ma, n_terms as made by sampled_system) with n_g sampled rows."""
    ev = np.linalg.eigvalsh(sy["G"])
    top = ev.max() if ev.size else 0.0
    keep = ev > top * sy["G"].shape[0] * 2.0 ** -52
    if not np.any(keep):
        return np.inf
    kappa = ev[keep].max() / ev[keep].min()
    eps_m = _U_IN[gather] + sy["n_terms"] * _U_ACC[gather]
    mnorm = np.linalg.norm(sy["M"])
    rel_m = eps_m * np.linalg.norm(sy["Ma"]) / mnorm if mnorm > 0 else 0.0
    rel_g = 2 * n_g * 2.0 ** -53 * np.linalg.norm(sy["Ga"]) / top
    return float(kappa * (rel_m + rel_g))


def fro_rel_err(a, b):
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a))


def run_parity(T, fac, R, s, tau, updates, gather="f64", ftol=1e-10, seed=0, stream_id=0,
               det_cap=0, OT=None, check_lev=True, label="", dense=False, gather_config=None,
               autotune=False, sampling="leverage"):
    """Returns the list of (oracle stats, device stats) per update.  dense:
    hand the (fully stored) tensor to the library as a dense array; the
    oracle keeps the equivalent COO form with every entry.  gather_config:
    (grid, sort_min) set for every mode; autotune: run the autotuner first
    and check that it left factors, leverage and step as they were."""
    OT = OT or oracle.Tensor.from_synth(T)
    ctx, F = make_ctx(T, fac, R, s, tau, gather, seed, stream_id, det_cap, dense=dense,
                      sampling=sampling)
    D = len(T.dims)
    if gather_config is not None:
        from paper_2006_16438_amd._lib import CpalError
        took = []
        for m in range(D):
            try:
                ctx.set_gather_config(m, *gather_config)
                took.append(m)
            except CpalError:
                # the row-block gathers (sort_min -3 to -5) need modes of at
                # least 1024 rows; the other modes keep their default
                if gather_config[1] > -3:
                    raise
        assert took, f"no mode of {T.dims} takes gather form {gather_config}"
        log(f"  {label}: gather form {gather_config} in modes {took}")
    if autotune:
        before = [f.cpu().numpy().copy() for f in F]
        lev0 = [ctx.leverage(m).cpu().numpy() for m in range(D)]
        t0 = ctx.step
        cfg = ctx.autotune()
        log(f"  {label}: autotuned gather shapes {cfg}")
        assert ctx.step == t0, "autotune changed the step counter"
        for m in range(D):
            assert np.array_equal(F[m].cpu().numpy(), before[m]), "autotune changed a factor"
            assert np.array_equal(ctx.leverage(m).cpu().numpy(), lev0[m]), \
                "autotune changed a leverage vector"
    cap = det_cap if det_cap else (1 << 26)
    out = []
    for u in range(updates):
        k = u % D
        host = [f.cpu().numpy().copy() for f in F]
        inputs = [h.copy() for h in host]   # the update's input factors
        if check_lev:
            for m in range(D):
                if sampling == "leverage":
                    ref_lev, _ = oracle.leverage(host[m])
                else:
                    ref_lev, _ = oracle.scores(host[m], sampling)
                got = ctx.leverage(m).cpu().numpy()
                assert np.array_equal(got, ref_lev), f"{label} update {u}: leverage of mode {m} differs"
        t = ctx.step
        try:
            ref = oracle.mode_update(OT, host, k, t, R, s, tau, seed, stream_id, cap,
                                     sampling=sampling)
        except RuntimeError:
            # an all-zero probability vector: the oracle rejects the update; the
            # device flags it and leaves the factor unchanged
            before = F[k].cpu().numpy().copy()
            ctx.mode_update(k)
            st = ctx.last_stats()
            assert st["flags"] & 64 and st["s_bar"] == 0, f"{label} update {u}: state not flagged"
            assert np.array_equal(F[k].cpu().numpy(), before)
            out.append((None, st, 0.0))
            continue
        ctx.mode_update(k)
        st = ctx.last_stats()
        idx, om, w = ctx.samples_view()
        idx = idx.cpu().numpy().view(np.uint64)
        om = om.cpu().numpy()
        w = w.cpu().numpy()
        rs = ref["stats"]
        for key in ("s_det", "s_rnd", "s_bar", "draws", "gathered_nnz", "flags"):
            assert st[key] == rs[key], f"{label} update {u} (mode {k}): {key} {st[key]} != {rs[key]}"
        assert np.float64(st["p_det"]).tobytes() == np.float64(rs["p_det"]).tobytes(), \
            f"{label} update {u}: p_det {st['p_det']!r} != {rs['p_det']!r}"
        assert np.array_equal(idx, ref["idx"]), f"{label} update {u}: sample indices differ"
        assert np.array_equal(om, ref["omega"]), f"{label} update {u}: omega differs"
        assert np.array_equal(w, ref["wgt"]), f"{label} update {u}: weights differ"
        got = F[k].cpu().numpy()
        if ftol == "derived":
            # the bound of derived_tolerance on the Frobenius-norm error; in
            # FP64 the 1e-10 parity bar applies unless the bound is larger
            # (an ill-conditioned G_s), and then the bound does
            bound = derived_tolerance(OT, inputs, k, ref, gather)
            tol = max(bound, 1e-10) if gather == "f64" else bound
            err = fro_rel_err(got, host[k])
            assert err <= tol, (f"{label} update {u} (mode {k}): factor rel err {err:.3e} > "
                                f"derived bound {tol:.2e}")
            out.append((rs, st, err))
            continue
        err = rel_err(got, host[k])
        assert err <= ftol, f"{label} update {u} (mode {k}): factor rel err {err:.3e} > {ftol:.1e}"
        out.append((rs, st, err))
    ctx.close()
    return out


def sampled_solve_torch(dims, coords, vals, F, k, idx, om):
    """FP64 solve of a sampled system built directly from its definition,
    with plain torch operations on the GPU: the fiber of sampled row j is
    every stored entry whose coordinates on the other modes equal those of
    lin(j) (first other mode fastest); M = sum_j omega_j sum_{(i_k, x) in
    fiber j} x e_{i_k} z_j^T, G_s = sum_j omega_j z_j z_j^T, A_k = M G_s^{-1}."""
    D = len(dims)
    others = [m for m in range(D) if m != k]
    key = torch.zeros(coords.shape[1], dtype=torch.int64, device=coords.device)
    stride = 1
    strides = []
    for m in others:
        key += coords[m].long() * stride
        strides.append(stride)
        stride *= dims[m]
    sk, perm = torch.sort(key)
    del key
    lo = torch.searchsorted(sk, idx)
    hi = torch.searchsorted(sk, idx, right=True)
    del sk
    lens = hi - lo
    R = F[0].shape[1]
    Z = torch.ones((idx.numel(), R), dtype=torch.float64, device=idx.device)
    for m, st in zip(others, strides):
        Z *= F[m][(idx // st) % dims[m]]
    rep = torch.repeat_interleave(torch.arange(idx.numel(), device=idx.device), lens)
    start = torch.cumsum(lens, 0) - lens
    M = torch.zeros((dims[k], R), dtype=torch.float64, device=idx.device)
    step = 1 << 24   # entries per accumulation chunk (bounded temporaries)
    for a in range(0, rep.numel(), step):
        r = rep[a:a + step]
        pos = lo[r] + (torch.arange(a, a + r.numel(), device=idx.device) - start[r])
        e = perm[pos]
        M.index_add_(0, coords[k][e].long(), (om[r] * vals[e].double())[:, None] * Z[r])
        del r, pos, e
    G = Z.T @ (om[:, None] * Z)
    return torch.linalg.solve(G, M.T).T, int(rep.numel())
