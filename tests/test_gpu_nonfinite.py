"""Non-finite features (NaN, Inf) and all-zero rows give undefined distances
for their own rows, but every candidate list still holds K columns of the
problem: the selection keys rank a NaN similarity after every number, and the
block-pruned selection and the fused k-NN fall back to a whole-row selection
when their bound admits fewer than K values (NaN passes no bound), so nothing
downstream indexes a row outside the problem and the other rows keep finite
distances. Every call goes through the C-ABI library."""
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
    x[10, :] = 0.0  # norm 0: its similarities are 0 * inf = NaN
    return x, spec.n_query


# k1 = 10 at sizes where the selection is block-pruned (4 (K - 1) <= column
# blocks): FP32 takes k1 + 8 candidates, BF16 / FP8 k1 + 16 and k1 + 32. The
# streaming selection with more than 64 candidates (k1 = 70, K = 78), and with
# fewer columns than 4 K (n = 200, K = 68), fills its list past the first
# chunk's 64 lane maxima, through the value filter that a NaN must pass.
@pytest.mark.parametrize("prec,fused,n,k1", [("f32", False, 9000, 10), ("f32", True, 9000, 10),
                                             ("bf16", False, 13000, 10), ("fp8", False, 21000, 10),
                                             ("fp8", True, 9000, 10), ("f32", False, 3000, 70),
                                             ("bf16", False, 200, 52)])
def test_non_finite_features_keep_the_lists_in_range(gpu_lib, prec, fused, n, k1):
    import torch
    from paper_2012_07620_amd import binding
    print(f"case prec={prec} fused={fused} n={n} k1={k1}", flush=True)
    x, q = _features(n, 64, 11)
    ctx = binding.Context(0, fused_knn=fused)
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
        # a NaN similarity ranks after every number, so the rows with finite
        # features keep finite neighbours, and only the rows and columns of the
        # four vectors without a direction have undefined distances
        assert np.isfinite(d.cpu().numpy()).mean() > 0.9
    ctx.close()


def test_non_finite_features_in_a_grouped_request(gpu_lib):
    """A request small enough for the grouped serving launches, with more than
    64 candidates per row: it completes, and the rows not reached by the
    non-finite ones keep finite distances."""
    import torch
    from paper_2012_07620_amd import binding
    n, k1 = 3000, 70
    print(f"case grouped request n={n} k1={k1}", flush=True)
    x, q = _features(n, 64, 12)
    out = torch.empty(q, n - q, device="cuda")
    ctx = binding.Context(0)
    t = binding.submit(ctx, x, out, q, k1, 3, 1)
    binding.wait(ctx, t)
    assert np.isfinite(out.cpu().numpy()).mean() > 0.9
    ctx.close()
