"""The GPU input recipe's distinct-coordinate rule, run on the CPU: the kept
coordinates are exactly the first `nnz` distinct ones of the draw stream, in
draw order, each with the value drawn for its first occurrence (checked
against a plain loop over the same draws, replayed from the same seed)."""
import torch

from paper_2006_16438_amd import synth_gpu


def _replay(dims, a, seed, chunk, nchunks):
    """The draw stream zipf_distinct consumes: per chunk, per mode, the Zipf
    index draws, then the chunk's values (same generator, same call order)."""
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    tables = [synth_gpu._zipf_table(n, a, g, torch.device("cpu")) for n in dims]
    keys, vals = [], []
    for _ in range(nchunks):
        key = torch.zeros(chunk, dtype=torch.int64)
        stride = 1
        for (cdf, perm), n in zip(tables, dims):
            key += synth_gpu._zipf_draw(cdf, perm, chunk, g, torch.device("cpu")) * stride
            stride *= n
        keys.append(key)
        vals.append(torch.rand(chunk, generator=g))
    return torch.cat(keys).tolist(), torch.cat(vals).tolist()


def test_first_occurrences_in_draw_order():
    dims, a, seed, chunk = (7, 5, 6), 1.2, 3, 64
    target = 150   # needs several chunks (hot coordinates repeat)
    coords, values = synth_gpu.zipf_distinct(dims, target, a, seed,
                                             lambda n, g: torch.rand(n, generator=g),
                                             chunk=chunk, device="cpu")
    keys, vals = _replay(dims, a, seed, chunk, 64)
    seen, want = {}, []
    for k, v in zip(keys, vals):
        if k not in seen:
            seen[k] = v
            want.append(k)
            if len(want) == target:
                break
    assert len(want) == target
    got = (coords[0].long() + dims[0] * (coords[1].long() + dims[1] * coords[2].long())).tolist()
    assert got == sorted(want), "kept coordinates differ from the first distinct draws"
    for k, v in zip(got, values.tolist()):
        assert v == seen[k], "value is not the one drawn at the first occurrence"
    for m, n in enumerate(dims):
        assert int(coords[m].min()) >= 0 and int(coords[m].max()) < n
