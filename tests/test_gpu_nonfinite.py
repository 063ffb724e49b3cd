"""Non-finite features (NaN, Inf) give undefined distances, but every
candidate list still holds columns of the row: the block-pruned selection and
the fused k-NN fall back to a whole-row selection when their bound admits
fewer than K values (NaN passes no bound), so nothing downstream indexes a
row outside the problem. The runs must complete and the lists stay in range.
Every call goes through the C-ABI library."""
import numpy as np
import pytest

from paper_2012_07620_amd import synth

pytestmark = pytest.mark.gpu


def _features(n, d, seed):
    import torch
    spec = synth.ProblemSpec("nonfinite", max(1, n // 7), n - max(1, n // 7), d, max(2, n // 20), 0.5, 0.05, 10, 3, 1,
                             "f32", seed)
    x = torch.from_numpy(synth.make_problem(spec).x32).cuda()
    x[5, 3] = float("nan")
    x[77, :] = float("inf")
    x[n - 1, 0] = float("-inf")
    return x, spec.n_query


# sizes where the selection is block-pruned (4 (K - 1) <= column blocks): FP32
# takes k1 + 8 candidates, BF16 / FP8 k1 + 16 and k1 + 32
@pytest.mark.parametrize("prec,fused,n", [("f32", False, 9000), ("f32", True, 9000), ("bf16", False, 13000),
                                          ("fp8", False, 21000), ("fp8", True, 9000)])
def test_non_finite_features_keep_the_lists_in_range(gpu_lib, prec, fused, n):
    import torch
    from paper_2012_07620_amd import binding
    print(f"case prec={prec} fused={fused} n={n}", flush=True)
    x, q = _features(n, 64, 11)
    ctx = binding.Context(0, fused_knn=fused)
    k1 = 10
    ki, kv = binding.knn(x, k1, ctx=ctx, sim_prec=prec)
    torch.cuda.synchronize()
    ki = ki.cpu().numpy()
    assert ki.shape == (n, k1)
    assert ki.min() >= 0 and ki.max() < n
    assert np.array_equal(ki[:, 0], np.arange(n))  # each row first in its own list
    if not fused:
        d = binding.run(x, q, k1, 3, 1, ctx=ctx, sim_prec=prec)
        torch.cuda.synchronize()
        assert d.shape == (q, n - q)
        # rows with finite features and no non-finite neighbour keep finite distances
        assert np.isfinite(d.cpu().numpy()).any()
    ctx.close()
