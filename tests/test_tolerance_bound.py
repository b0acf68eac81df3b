"""The parity bound of the reduced-precision gathers (gpu_util.derived_tolerance)
checked on the CPU: the sampled system of an oracle update is solved again
with the fiber values and weighted KRP rows rounded to FP32 or BF16 and the
products summed in FP32 one term at a time (what the device's gather may
do), and the result must stay within the bound of the FP64 oracle factor."""
import numpy as np
import pytest

import oracle
from paper_2006_16438_amd import synth
from tests.gpu_util import derived_tolerance, fro_rel_err, sampled_system


def _bf16(a):
    """Round FP32 values to the nearest BF16 (ties to even), kept as FP32."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32)


def _reduced_update(OT, fac, k, ref, gather):
    dims = [int(d) for d in OT.dims]
    others = [m for m in range(len(dims)) if m != k]
    idx = ref["idx"].astype(np.int64)
    om = ref["omega"]
    R = fac[0].shape[1]
    Z = np.ones((idx.size, R))
    stride = 1
    key = np.zeros(OT.nnz, dtype=np.int64)
    for m in others:
        Z *= fac[m][(idx // stride) % dims[m]]
        key += OT.coords[m].astype(np.int64) * stride
        stride *= dims[m]
    rnd = _bf16 if gather == "bf16" else (lambda a: np.asarray(a, dtype=np.float32))
    wz = rnd((om[:, None] * Z).astype(np.float32) if gather == "bf16" else om[:, None] * Z)
    slot = {int(v): j for j, v in enumerate(idx)}
    M = np.zeros((dims[k], R), dtype=np.float32)
    for e in range(OT.nnz):
        j = slot.get(int(key[e]))
        if j is None:
            continue
        x = rnd(np.float32(OT.vals[e]) if gather == "bf16" else OT.vals[e])
        M[OT.coords[k][e]] += np.float32(x) * wz[j]          # FP32 product and sum
    G = sampled_system(OT, fac, k, ref["idx"], om)["G"]
    return np.linalg.lstsq(G, M.astype(np.float64).T, rcond=None)[0].T


@pytest.mark.parametrize("gather", ["f32", "bf16"])
@pytest.mark.parametrize("case", ["small3", "ragged-tau1"])
def test_reduced_precision_update_within_derived_bound(gather, case):
    if case == "small3":
        T, _, R = synth.small3(0)
        s, tau = 1024, 1.0 / 1024
    else:
        T, _ = synth.planted((37, 23, 19), 5, seed=2, density=1.0, law="normal")
        R, s, tau = 20, 700, 1.0
    OT = oracle.Tensor.from_synth(T)
    fac = synth.gaussian_factors(T.dims, R, 2)
    for k in range(3):
        f2 = [f.copy() for f in fac]
        ref = oracle.mode_update(OT, f2, k, k, R, s, tau)
        got = _reduced_update(OT, fac, k, ref, gather)
        err = fro_rel_err(got, f2[k])
        bound = derived_tolerance(OT, fac, k, ref, gather)
        assert err <= bound, (case, gather, k, err, bound)
        # a bound far above the error would pin nothing
        print(case, gather, k, f"err={err:.2e} bound={bound:.2e}")
        assert bound < 0.25, (case, gather, k, bound)
