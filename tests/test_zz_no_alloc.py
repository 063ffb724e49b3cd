"""rerank_run_static, the allocation-free variant of rerank_run (working set in
the library's static device array), against rerank_run on the same inputs:
two calls in a row, the second on a smaller problem, each bit-identical to
rerank_run; no device memory taken by the calls; a problem whose working set
exceeds the array is refused before anything is enqueued. Every call goes
through the C-ABI library."""
import numpy as np
import pytest

from paper_2012_07620_amd import synth

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


CASES = [  # n, q, d, k1, k2, layers, seed
    (5000, 700, 512, 26, 7, 1, 31),
    (2100, 300, 128, 20, 6, 2, 32),  # smaller: the array still holds the first call's contents
]


@pytest.mark.parametrize("sim,final", [("f32", "f32"), ("bf16", "sparse")])
def test_static_working_set_matches_rerank_run(gpu_lib, sim, final):
    import torch
    from paper_2012_07620_amd import binding
    ctx = binding.Context(0)
    xs, ref, refk = [], [], []
    for n, q, d, k1, k2, layers, seed in CASES:
        x = _dev(synth.random_features(n, d, seed=seed, n_ids=n // 20))
        xs.append(x)
        dist, ki, kv = binding.run(x, q, k1, k2, layers, sim_prec=sim, final_prec=final, ctx=ctx, return_knn=True)
        ref.append(dist)
        refk.append((ki, kv))
    outs = [torch.full_like(r, float("nan")) for r in ref]
    kouts = [(torch.full_like(a, -1), torch.full_like(b, float("nan"))) for a, b in refk]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for (n, q, d, k1, k2, layers, _), x, o, ko in zip(CASES, xs, outs, kouts):
        print(f"case static n={n} q={q} d={d} k1={k1} k2={k2} L={layers} sim={sim} final={final}", flush=True)
        binding.run_static(x, q, k1, k2, layers, sim_prec=sim, final_prec=final, ctx=ctx, out=o, knn_out=ko)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    for r, o, (a, b), (ka, kb) in zip(ref, outs, refk, kouts):
        assert torch.equal(r, o)
        assert torch.equal(a, ka) and torch.equal(b, kb)
    assert free0 - free1 < (1 << 20), f"device free memory fell by {free0 - free1} bytes"
    ctx.close()


def test_static_refuses_a_working_set_beyond_the_array(gpu_lib):
    import torch
    from paper_2012_07620_amd import binding
    n, q, d = 6000, 900, 2048
    p = binding.make_params(n, q, d, 20, 6, 1)
    assert binding.workspace_bytes(p) > binding.STATIC_BYTES
    x = torch.zeros((n, d), device="cuda")
    out = torch.full((q, n - q), 7.0, device="cuda")
    with pytest.raises(binding.RerankError) as e:
        binding.run_static(x, q, 20, 6, 1, out=out)
    assert e.value.status == binding.E_NOMEM
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))  # nothing ran
