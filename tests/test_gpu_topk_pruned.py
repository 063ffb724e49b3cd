"""The block-pruned candidate selection (taken when the candidates per row
are few against the row's 128-column blocks: 4 (K - 1) <= ceil(N / 128)) vs
the FP64 oracle, through rerank_knn. These shapes are chosen so that it runs:
the similarity product records each row's block maxima and the selection
reads only the blocks that can hold a member."""
import numpy as np
import pytest

from oracle import rerank_oracle as orc
from paper_2012_07620_amd import synth
from tests.parity import TIE_TOL, compare_lists

pytestmark = pytest.mark.gpu


def _knn(x, k1, **kw):
    import torch
    from paper_2012_07620_amd import binding
    ki, kv = binding.knn(torch.from_numpy(np.ascontiguousarray(x)).cuda(), k1, **kw)
    torch.cuda.synchronize()
    return ki.cpu().numpy(), kv.cpu().numpy()


def _pruned(n, k1, extra):
    return 4 * (k1 + extra - 1) <= (n + 127) // 128


CASES = [
    # n, d, k1, extra, n_ids, dup
    (300, 16, 1, 0, 0, 0.0),        # K = 1: the row itself only
    (385, 24, 2, 0, 0, 0.0),        # K = 2, four blocks (ragged last block)
    (2000, 40, 4, 0, 80, 0.0),      # clustered rows
    (3000, 32, 5, 0, 100, 0.25),    # exact duplicates: ties at the bound
    (4100, 64, 6, 2, 0, 0.0),       # re-scored candidates, ragged N
    (9000, 48, 12, 4, 400, 0.05),   # several blocks per member, ties
]


@pytest.mark.parametrize("n,d,k1,extra,n_ids,dup", CASES)
def test_pruned_selection_f32_vs_oracle(gpu_lib, n, d, k1, extra, n_ids, dup):
    assert _pruned(n, k1, extra)
    x = synth.random_features(n, d, seed=n + 7 * d, n_ids=n_ids, dup_frac=dup)
    print(f"case n={n} d={d} k1={k1} extra={extra} n_ids={n_ids} dup={dup}", flush=True)
    ki, kv = _knn(x, k1, extra_cand=extra)
    assert np.all(ki[:, 0] == np.arange(n))
    g = orc.knn_lists(x, k1, min(k1, 3))
    f1, _ = compare_lists(ki, g, min(k1, 3), x=x)
    ok = ~np.isin(np.arange(n), f1)
    np.testing.assert_allclose(kv[ok], g.val[ok], atol=2e-6)


@pytest.mark.parametrize("prec,n,k1", [("bf16", 13000, 10), ("fp8", 13000, 4)])
def test_pruned_selection_low_precision(gpu_lib, prec, n, k1):
    extra = 16
    assert _pruned(n, k1, extra)
    x = synth.random_features(n, 64, seed=n + k1, n_ids=600)
    ki, kv = _knn(x, k1, sim_prec=prec, extra_cand=extra)
    rows = np.random.Generator(np.random.PCG64(11)).choice(n, 400, replace=False)
    g = orc.knn_lists(x, k1, min(k1, 3), rows=rows)
    same = np.mean([set(ki[i].tolist()) == set(g.idx[r].tolist()) for r, i in enumerate(rows)])
    print(f"{prec}: sampled rows with the oracle's k1 set {same:.4f}")
    assert np.all(ki[:, 0] == np.arange(n))
    assert same >= 0.99
    # every kept value is the FP32 re-score of its pair
    xhat = orc.unit_rows(x)
    for r, i in enumerate(rows[:50]):
        exact = xhat[ki[i]] @ xhat[i]
        exact[0] = 1.0
        np.testing.assert_allclose(kv[i], exact, atol=2e-6)


@pytest.mark.parametrize("n,k1,extra", [
    (33000, 60, 5),   # K - 1 = 64: the bound is the last lane maximum of the sort
    (36000, 66, 4),   # K = 70 (two keys per lane): no bound, every block read
])
def test_pruned_selection_many_candidates(gpu_lib, n, k1, extra):
    assert _pruned(n, k1, extra)
    x = synth.random_features(n, 16, seed=n, n_ids=n // 40)
    ki, kv = _knn(x, k1, extra_cand=extra)
    assert np.all(ki[:, 0] == np.arange(n))
    rows = np.random.Generator(np.random.PCG64(5)).choice(n, 300, replace=False)
    g = orc.knn_lists(x, k1, 3, rows=rows)
    xhat = orc.unit_rows(x)
    from tests.parity import check_alternative
    for r, i in enumerate(rows):
        if g.gap1[r] >= TIE_TOL:
            assert set(ki[i].tolist()) == set(g.idx[r].tolist()), f"row {i}"
            np.testing.assert_allclose(kv[i], g.val[r], atol=2e-6)
        else:
            check_alternative(xhat, int(i), ki[i], TIE_TOL, "k1 set")
