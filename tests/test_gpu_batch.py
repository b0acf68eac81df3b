"""Batched decompositions through the C ABI on the GPU: sparse 3-way and
4-way tensors and a dense tensor of different shapes, ranks and sample
counts, two restarts (stream ids) per sparse tensor sharing its fiber
index, stepped together with cp_arls_lev_mode_step_batch.

Per step and decomposition the parity protocol of tests/gpu_util.py: the
oracle gets the decomposition's current factors and runs the same update;
sample indices, omega, weights and leverage match bit for bit, the new
factor within 1e-10 (FP64 gather)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2006_16438_amd import synth
from tests.gpu_util import dense_values, log, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("graphs", [False, True, "autotune", "stages", "stages_seg",
                                    "stages_autotune"])
def test_batch_mixed_parity(graphs):
    """graphs=True: every mode step after the first replays the captured
    graph of that mode; each replay is checked against the oracle.
    graphs="autotune": as True, and after the first iteration the autotuner
    changes the launch shapes, which drops the captured graphs (the next
    steps capture again with the new shapes).  "stages": the stage-major
    graph (one launch per stage for all decompositions where the kernel has
    a batched form; the owner gather of these FP64 decompositions and the
    dense contraction run per decomposition beside it); "stages_seg": every
    sparse decomposition on the segmented gather, which has a batched form
    too; "stages_autotune": stage-major with the autotuner's shapes."""
    from paper_2006_16438_amd.api import CpArlsLevBatch
    dev = torch.device("cuda:0")
    A = synth.random_sparse((30, 25, 20), 3000, seed=5)
    B = synth.random_sparse((50, 12, 40), 5000, seed=6)
    C4 = synth.random_sparse((10, 9, 8, 7), 2000, seed=7)
    Dn, _ = synth.planted((12, 10, 8), 3, seed=8, density=1.0, law="normal")
    tensors_np = [A, B, C4, Dn]
    tensors = []
    for t, T in enumerate(tensors_np):
        if t == 3:
            tensors.append((T.dims, None, torch.from_numpy(dense_values(T)).to(dev)))
        else:
            tensors.append((T.dims, torch.from_numpy(np.ascontiguousarray(T.coords)).to(dev),
                            torch.from_numpy(np.ascontiguousarray(T.values)).to(dev)))
    tensor_of = [0, 0, 1, 1, 2, 2, 3]
    ranks = [4, 4, 7, 7, 5, 5, 3]
    samples = [512, 512, 1024, 1024, 300, 300, 256]
    stream_ids = [0, 1, 0, 1, 0, 1, 0]
    factors = [[torch.from_numpy(f.copy()).to(dev)
                for f in synth.gaussian_factors(tensors_np[t].dims, ranks[i], 10 + i)]
               for i, t in enumerate(tensor_of)]
    stages = isinstance(graphs, str) and graphs.startswith("stages")
    b = CpArlsLevBatch(tensors, tensor_of, factors, ranks, samples, seeds=3,
                       stream_ids=stream_ids, gather_dtype="f64",
                       use_graphs="stages" if stages else bool(graphs))
    OTs = [oracle.Tensor.from_synth(T) for T in tensors_np]
    members = [b.member(i) for i in range(len(tensor_of))]
    if graphs == "stages_seg":
        for i, t in enumerate(tensor_of):
            if t != 3:
                for k in range(len(tensors_np[t].dims)):
                    members[i].set_gather_config(k, 0, 0)
    max_order = max(len(T.dims) for T in tensors_np)
    for it in range(3):
        if graphs in ("autotune", "stages_autotune") and it == 1:
            b.autotune()
            log("autotuned: " + str([members[i].gather_config(k) for i in range(len(tensor_of))
                                     for k in range(len(tensors_np[tensor_of[i]].dims))]))
            # a restart runs the launch shapes tuned on the first decomposition
            # of its tensor (the gather form's buffers allocated for it too)
            for i in range(1, len(tensor_of)):
                if tensor_of[i] == tensor_of[i - 1]:
                    for k in range(len(tensors_np[tensor_of[i]].dims)):
                        assert members[i].gather_config(k) == members[i - 1].gather_config(k), \
                            f"decomposition {i} mode {k}: launch shape not taken from its tensor"
        for k in range(max_order):
            refs = {}
            for i, t in enumerate(tensor_of):
                D = len(tensors_np[t].dims)
                if k >= D:
                    continue
                host = [f.cpu().numpy().copy() for f in factors[i]]
                for m in range(D):
                    ref_lev, _ = oracle.leverage(host[m])
                    assert np.array_equal(members[i].leverage(m).cpu().numpy(), ref_lev), \
                        f"decomposition {i}: leverage of mode {m} differs"
                ref = oracle.mode_update(OTs[t], host, k, members[i].step, ranks[i], samples[i],
                                         1.0 / samples[i], 3, stream_ids[i])
                refs[i] = (ref, host[k])
            b.mode_step(k)
            for i, (ref, new) in refs.items():
                idx, om, w = members[i].samples_view()
                assert np.array_equal(idx.cpu().numpy().view(np.uint64), ref["idx"]), \
                    f"iteration {it} mode {k} decomposition {i}: sample indices differ"
                assert np.array_equal(om.cpu().numpy(), ref["omega"])
                assert np.array_equal(w.cpu().numpy(), ref["wgt"])
                err = rel_err(factors[i][k].cpu().numpy(), new)
                assert err <= 1e-10, f"decomposition {i} mode {k}: factor rel err {err:.3e}"
            nk = b.graph_kernels(k, 2 if stages else 1) if graphs else 0
            log(f"iteration {it} mode {k}: {len(refs)} decompositions match (graphs={graphs}, "
                f"{nk} kernels in the step's graph)")
    b.close()


@pytest.mark.parametrize("graphs", [True, "stages"])
def test_batch256_full_size_members(graphs):
    """The benchmark's batch at full size (64 generated sparse tensors, nnz up
    to 5e6, x 4 restarts, FP32 gather, s = 2^15), stepped from captured graphs
    (graph of branches, or stage-major) after an autotuned warm-up iteration;
    two decompositions on different tensors are checked at every mode step of
    the next iteration against the oracle: bit-exact samples, factors within
    1e-4 (FP32 gather)."""
    from paper_2006_16438_amd import synth_gpu
    from paper_2006_16438_amd.api import CpArlsLevBatch
    dev = torch.device("cuda:0")
    tens = synth_gpu.batch_tensors(64, seed=0)
    restarts, s = 4, 1 << 15
    tensor_of = [t for t in range(len(tens)) for _ in range(restarts)]
    ranks = [tens[t][3] for t in tensor_of]
    stream_ids = [r for _ in range(len(tens)) for r in range(restarts)]
    factors = [[torch.from_numpy(f).to(dev)
                for f in synth.gaussian_factors(tens[t][0], ranks[i], 100 + i)]
               for i, t in enumerate(tensor_of)]
    b = CpArlsLevBatch([(d, c, v) for d, c, v, _ in tens], tensor_of, factors, ranks, s,
                       seeds=0, stream_ids=stream_ids, gather_dtype="f32")
    for k in range(3):   # warm-up iteration, kernel by kernel
        b.mode_step(k)
    b.autotune()
    b.set_graphs(graphs)
    check = [0, 4 * 37 + 2]
    OTs, members = {}, {}
    for i in check:
        d, c, v, _ = tens[tensor_of[i]]
        OTs[i] = oracle.Tensor(np.array(d), c.cpu().numpy(), v.cpu().numpy().astype(np.float64))
        members[i] = b.member(i)
        log(f"decomposition {i}: tensor {tensor_of[i]} dims {d} nnz {c.shape[1]} rank {ranks[i]}")
    for k in range(3):
        refs = {}
        for i in check:
            host = [f.cpu().numpy().copy() for f in factors[i]]
            ref = oracle.mode_update(OTs[i], host, k, members[i].step, ranks[i], s, 1.0 / s, 0,
                                     stream_ids[i])
            refs[i] = (ref, host[k])
        b.mode_step(k)
        for i, (ref, new) in refs.items():
            idx, om, w = members[i].samples_view()
            assert np.array_equal(idx.cpu().numpy().view(np.uint64), ref["idx"]), \
                f"mode {k} decomposition {i}: sample indices differ"
            assert np.array_equal(om.cpu().numpy(), ref["omega"])
            assert np.array_equal(w.cpu().numpy(), ref["wgt"])
            err = rel_err(factors[i][k].cpu().numpy(), new)
            log(f"  mode {k} decomposition {i}: s_bar={idx.numel()} factor rel err {err:.2e}")
            assert err <= 1e-4, f"decomposition {i} mode {k}: factor rel err {err:.3e}"
        log(f"  mode {k}: {b.graph_kernels(k, 2 if graphs == 'stages' else 1)} kernels in the "
            f"step's graph ({graphs})")
    b.close()


def test_batch_stage_major_rowblock_forms():
    """The stage-major graph with the row-block gathers in their batched form:
    two sparse 3-way tensors with modes of 1024 rows and more (2100 x 300 x
    1100, 1.5e5 nonzeros; Zipf(1.2) 3000 x 1200 x 300, 4e5 nonzeros), four
    restarts each, restart r of a tensor on the tile (r = 0), shared-block
    bucketed (r = 1), hybrid (r = 2, long-fiber factor 16) or segmented (r = 3)
    gather in every mode that takes it (the others keep the default), FP64.
    Two iterations, every mode step of every decomposition checked against
    the oracle: bit-exact samples, factors within 1e-10."""
    from paper_2006_16438_amd import _lib as L
    from paper_2006_16438_amd.api import CpArlsLevBatch
    from tests.test_gpu_parity import _zipf3
    dev = torch.device("cuda:0")
    tensors_np = [synth.random_sparse((2100, 300, 1100), 150_000, seed=21), _zipf3()]
    tensors = [(T.dims, torch.from_numpy(np.ascontiguousarray(T.coords)).to(dev),
                torch.from_numpy(np.ascontiguousarray(T.values)).to(dev)) for T in tensors_np]
    restarts = 4
    tensor_of = [t for t in range(2) for _ in range(restarts)]
    n = len(tensor_of)
    R = 8
    samples = [8192 + 77 if t == 0 else 4096 for t in tensor_of]
    taus = [1 / 8192 if t == 0 else 1 / 4096 for t in tensor_of]
    stream_ids = [i % restarts for i in range(n)]
    factors = [[torch.from_numpy(f.copy()).to(dev)
                for f in synth.gaussian_factors(tensors_np[t].dims, R, 30 + i)]
               for i, t in enumerate(tensor_of)]
    b = CpArlsLevBatch(tensors, tensor_of, factors, R, samples, taus=taus, seeds=3,
                       stream_ids=stream_ids, gather_dtype="f64")
    members = [b.member(i) for i in range(n)]
    forms = [(0, -3), (0, -4), (16, -5), (0, 0)]
    taken = {f: 0 for f in forms}
    for i in range(n):
        f = forms[i % restarts]
        for k in range(3):
            try:
                members[i].set_gather_config(k, *f)
                taken[f] += 1
            except L.CpalError:
                pass   # a mode below 1024 rows keeps its default gather
    assert all(v > 0 for v in taken.values()), taken
    b.set_graphs("stages")
    OTs = [oracle.Tensor.from_synth(T) for T in tensors_np]
    for it in range(2):
        for k in range(3):
            refs = {}
            for i, t in enumerate(tensor_of):
                host = [f.cpu().numpy().copy() for f in factors[i]]
                ref = oracle.mode_update(OTs[t], host, k, members[i].step, R, samples[i],
                                         taus[i], 3, stream_ids[i])
                refs[i] = (ref, host[k])
            b.mode_step(k)
            for i, (ref, new) in refs.items():
                idx, om, w = members[i].samples_view()
                assert np.array_equal(idx.cpu().numpy().view(np.uint64), ref["idx"]), \
                    f"iteration {it} mode {k} decomposition {i}: sample indices differ"
                assert np.array_equal(om.cpu().numpy(), ref["omega"])
                assert np.array_equal(w.cpu().numpy(), ref["wgt"])
                err = rel_err(factors[i][k].cpu().numpy(), new)
                assert err <= 1e-10, f"decomposition {i} mode {k}: factor rel err {err:.3e}"
            log(f"iteration {it} mode {k}: {n} decompositions match, "
                f"{b.graph_kernels(k, 2)} kernels in the step's graph, forms "
                f"{[members[i].gather_config(k) for i in range(n)]}")
    b.close()
