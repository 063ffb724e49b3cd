"""The fused similarity + candidate selection (RERANK_CTX_FUSED_KNN) vs the
FP64 oracle and vs the unfused path, through the C-ABI library."""
import numpy as np
import pytest

from oracle import rerank_oracle as orc
from paper_2012_07620_amd import synth
from tests.parity import TIE_TOL, check_alternative, check_run, compare_lists

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture(scope="module")
def fused_ctx(gpu_lib):
    from paper_2012_07620_amd import binding
    ctx = binding.Context(0, fused_knn=True)
    yield ctx
    ctx.close()


def _knn(x, k1, ctx, **kw):
    import torch
    from paper_2012_07620_amd import binding
    ki, kv = binding.knn(_dev(x), k1, ctx=ctx, **kw)
    torch.cuda.synchronize()
    return ki.cpu().numpy(), kv.cpu().numpy()


CASES = [
    # n, d, k1, extra_cand, n_ids, dup
    (2, 1, 1, -1, 0, 0.0),        # one tile, K = N
    (20, 7, 20, -1, 0, 0.0),      # k1 = N
    (100, 64, 9, -1, 5, 0.0),     # one row panel
    (129, 33, 5, 0, 4, 0.0),      # no re-score: the selected similarities are the output
    (300, 40, 12, -1, 10, 0.2),   # exact duplicates (ties on the product's values)
    (1000, 128, 10, -1, 50, 0.0),
    (2500, 96, 26, -1, 100, 0.0),  # several column ranges per row panel
    (3001, 130, 56, 8, 60, 0.05),  # K = 64, ragged K and N
]


@pytest.mark.parametrize("n,d,k1,extra,n_ids,dup", CASES)
def test_fused_knn_f32_vs_oracle_and_unfused(gpu_lib, fused_ctx, n, d, k1, extra, n_ids, dup):
    x = synth.random_features(n, d, seed=n * 11 + d, n_ids=n_ids, dup_frac=dup)
    print(f"case n={n} d={d} k1={k1} extra={extra} n_ids={n_ids} dup={dup}", flush=True)
    ki, kv = _knn(x, k1, fused_ctx, extra_cand=extra)
    g = orc.knn_lists(x, k1, min(k1, 3))
    f1, _ = compare_lists(ki, g, min(k1, 3), x=x)
    ok = ~np.isin(np.arange(n), f1)
    np.testing.assert_allclose(kv[ok], g.val[ok], atol=2e-6)
    ui, uv = _knn(x, k1, None, extra_cand=extra)
    if extra != 0:  # re-scored lists: the same candidates give the same bits
        assert np.array_equal(ki, ui) and np.array_equal(kv, uv)
    else:  # the selected values are the product's; allow its rounding order
        diff = np.flatnonzero(np.any(ki != ui, axis=1))
        assert np.all(g.gap1[diff] < TIE_TOL), f"fused / unfused lists differ on rows {diff[:10]}"
        np.testing.assert_allclose(kv, uv, atol=2e-7)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("n,d,k1,n_ids", [(1000, 128, 10, 50), (2500, 256, 20, 120)])
def test_fused_knn_low_precision(gpu_lib, fused_ctx, prec, n, d, k1, n_ids):
    x = synth.random_features(n, d, seed=n * 13 + d, n_ids=n_ids)
    ki, kv = _knn(x, k1, fused_ctx, sim_prec=prec)
    g = orc.knn_lists(x, k1, 3)
    overlap = np.mean([len(set(a) & set(b)) / k1 for a, b in zip(ki.tolist(), g.idx.tolist())])
    print(f"{prec} fused: top-k1 overlap {overlap:.5f}")
    assert overlap >= 0.995
    assert np.all(ki[:, 0] == np.arange(n))
    ui, uv = _knn(x, k1, None, sim_prec=prec)
    same = np.mean(np.all(ki == ui, axis=1))
    print(f"{prec}: rows identical to the unfused path: {same:.5f}")
    assert same >= 0.999


@pytest.mark.parametrize("sim,final", [("f32", "f32"), ("bf16", "f32"), ("f32", "sparse")])
def test_fused_run_matches_unfused(gpu_lib, fused_ctx, sim, final):
    import torch
    from paper_2012_07620_amd import binding
    p = synth.make_problem(synth.TINY)
    s = p.spec
    x = _dev(p.x32)
    a, ka, _ = binding.run(x, s.n_query, s.k1, s.k2, 2, sim_prec=sim, final_prec=final, return_knn=True,
                           ctx=fused_ctx)
    b, kb, _ = binding.run(x, s.n_query, s.k1, s.k2, 2, sim_prec=sim, final_prec=final, return_knn=True)
    torch.cuda.synchronize()
    assert torch.equal(ka, kb)
    assert torch.equal(a, b)
    if sim == "f32":
        ref = orc.rerank(p.x32, s.n_query, s.k1, s.k2, 2)
        r = check_run(p.x32, ref, ka.cpu().numpy(), a.cpu().numpy(), s.n_query, s.k2, 2, 1e-4)
        print(f"fused run D max err {r['max_err']:.2e}, pairs vs tie-breaks {r['pairs_vs_tie_breaks']}")


def test_fused_rejects_more_than_64_candidates(gpu_lib, fused_ctx):
    from paper_2012_07620_amd import binding
    x = synth.random_features(200, 16, seed=5)
    with pytest.raises(binding.RerankError) as e:
        _knn(x, 60, fused_ctx)  # 60 + 8 extra candidates
    assert e.value.status == 7


def test_fused_knn_without_an_n_by_n_buffer(gpu_lib):
    """N = 30000: S alone would take 3.6 GB; a 1 GiB context runs the fused
    path and refuses the unfused one. Sampled rows vs the oracle."""
    from paper_2012_07620_amd import binding
    n, d, k1 = 30000, 128, 20
    x = synth.random_features(n, d, seed=77, n_ids=1500)
    small = binding.Context(0, budget_bytes=1 << 30, fused_knn=True)
    plain = binding.Context(0, budget_bytes=1 << 30)
    try:
        with pytest.raises(binding.RerankError) as e:
            _knn(x, k1, plain)
        assert e.value.status == 2  # RERANK_E_NOMEM
        ki, kv = _knn(x, k1, small)
    finally:
        small.close()
        plain.close()
    rows = np.random.Generator(np.random.PCG64(3)).choice(n, 300, replace=False)
    g = orc.knn_lists(x, k1, 3, rows=rows)
    xhat = orc.unit_rows(x)
    for r, i in enumerate(rows):
        assert ki[i, 0] == i
        if g.gap1[r] >= TIE_TOL:
            assert set(ki[i].tolist()) == set(g.idx[r].tolist()), f"row {i}"
            np.testing.assert_allclose(kv[i], g.val[r], atol=2e-6)
        else:  # a tied row may keep the other tie-break, which must be a valid one
            check_alternative(xhat, int(i), ki[i], TIE_TOL, "k1 set")


@pytest.mark.parametrize("sim,final", [("f32", "f32"), ("bf16", "sparse"), ("fp8", "bf16")])
def test_fused_run_matches_unfused_above_the_batching_limit(gpu_lib, fused_ctx, sim, final):
    """N = 9000 (direct path, several column ranges, two layers): the fused
    similarity + selection leaves lists and distances bit-identical."""
    import torch
    from paper_2012_07620_amd import binding
    n, q, d = 9000, 1350, 256
    x = _dev(synth.random_features(n, d, seed=91, n_ids=450))
    a, ka, va = binding.run(x, q, 20, 6, 2, sim_prec=sim, final_prec=final, return_knn=True, ctx=fused_ctx)
    b, kb, vb = binding.run(x, q, 20, 6, 2, sim_prec=sim, final_prec=final, return_knn=True)
    torch.cuda.synchronize()
    same_rows = torch.all(ka == kb, dim=1).float().mean().item()
    print(f"{sim}/{final}: rows with identical lists {same_rows:.6f}")
    assert torch.equal(ka, kb) and torch.equal(va, vb)
    assert torch.equal(a, b)


def _sample_panels(n, K, sbytes):
    """Column panels (of 128) the fused path multiplies first, as the library
    lays them out: P panels spaced T // P apart from (T // P) // 2, with P the
    memory-balancing sample size (at least 8 panels, at most all of them)."""
    import math
    T = (n + 127) // 128
    f = 1.0 + 6.0 / math.sqrt(K)
    P = min(T, max(8, math.ceil(math.sqrt(8.0 * f * K * n / sbytes) / 128.0)))
    sp = T // P
    return [sp // 2 + t * sp for t in range(P)]


@pytest.mark.parametrize("sim", ["f32", "bf16"])
def test_fused_overflowing_rows_are_recomputed_by_their_row_panel(gpu_lib, fused_ctx, sim):
    """Rows of the sample panels form one cluster, every other row a second,
    orthogonal one: an outside row's bound comes from similarities near 0, so
    nearly all of its own cluster passes it and its candidate buffer
    overflows; those panels are recomputed by the row-panel kernel, the
    sample rows take the normal path. Both must give the exact lists."""
    n, d, k1 = 4096, 64, 20
    K = k1 + (8 if sim == "f32" else 16)
    panels = _sample_panels(n, K, 4 if sim == "f32" else 2)
    assert len(panels) < (n + 127) // 128  # some panels lie outside the sample
    rng = np.random.Generator(np.random.PCG64(2024))
    in_sample = np.zeros(n, bool)
    for p in panels:
        in_sample[p * 128:(p + 1) * 128] = True
    a = np.zeros(d, np.float32)
    a[0] = 1.0
    b = np.zeros(d, np.float32)
    b[1] = 1.0
    x = np.where(in_sample[:, None], a, b) + rng.standard_normal((n, d)).astype(np.float32) * 0.3
    x = np.ascontiguousarray(x.astype(np.float32))
    print(f"case {sim} n={n} K={K} sample panels {panels}", flush=True)
    ki, kv = _knn(x, k1, fused_ctx, sim_prec=sim)
    ui, uv = _knn(x, k1, None, sim_prec=sim)
    assert np.all(ki[:, 0] == np.arange(n))
    same = np.mean(np.all(ki == ui, axis=1))
    print(f"{sim}: rows identical to the unfused path: {same:.5f}")
    if sim == "f32":
        assert np.array_equal(ki, ui) and np.array_equal(kv, uv)
        g = orc.knn_lists(x, k1, 3)
        compare_lists(ki, g, 3, x=x)
    else:
        assert same >= 0.999
