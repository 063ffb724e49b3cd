"""GPU path vs the FP64 oracle on small problems (several tiles, ragged
tails, degenerate cases). Every call goes through the C-ABI library."""
import numpy as np
import pytest

from oracle import rerank_oracle as orc
from paper_2012_07620_amd import synth
from tests.parity import check_run, compare_lists

pytestmark = pytest.mark.gpu

D_TOL_F32 = 1e-4  # FP32 path: |D - D_oracle|
D_TOL_LOWP = 2e-2  # BF16 / FP8 similarity paths


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _run(gpu_lib, x, q, k1, k2, layers, **kw):
    import torch
    from paper_2012_07620_amd import binding
    d, ki, kv = binding.run(_dev(x), q, k1, k2, layers, return_knn=True, **kw)
    torch.cuda.synchronize()
    return d.cpu().numpy(), ki.cpu().numpy(), kv.cpu().numpy()


def _check_full(gpu_lib, x, q, k1, k2, layers, alpha=2, node="adj", tol=D_TOL_F32, **kw):
    print(f"case n={len(x)} q={q} d={x.shape[1]} k1={k1} k2={k2} L={layers} alpha={alpha} node={node} {kw}",
          flush=True)
    dg, ki, kv = _run(gpu_lib, x, q, k1, k2, layers, alpha=alpha, node=node, **kw)
    ref = orc.rerank(x, q, k1, k2, layers, alpha=alpha, node=node)
    r = check_run(x, ref, ki, dg, q, k2, layers, tol, alpha=alpha, node=node)
    ok = ~np.isin(np.arange(len(x)), r["flip1"])
    np.testing.assert_allclose(kv[ok], ref.graph.val[ok], atol=2e-6)
    return r["max_err"], r["mean_err"], r["pairs_vs_tie_breaks"]


def test_similarity_f32_tiny(gpu_lib):
    import torch
    from paper_2012_07620_amd import binding
    p = synth.make_problem(synth.TINY)
    s = binding.similarity(_dev(p.x32))
    torch.cuda.synchronize()
    s = s.cpu().numpy()
    ref = orc.similarity_rows(orc.unit_rows(p.x32), range(p.spec.n))
    err = np.abs(s - ref).max()
    print("max |S - S64| =", err)
    assert err < 2e-6
    assert np.array_equal(s, s.T)


def test_knn_f32_tiny(gpu_lib):
    import torch
    from paper_2012_07620_amd import binding
    p = synth.make_problem(synth.TINY)
    ki, kv = binding.knn(_dev(p.x32), 10)
    torch.cuda.synchronize()
    g = orc.knn_lists(p.x32, 10, 3)
    f1, f2 = compare_lists(ki.cpu().numpy(), g, 3, x=p.x32)
    assert f1.size == 0 and f2.size == 0
    np.testing.assert_allclose(kv.cpu().numpy(), g.val, atol=2e-7)


def test_run_f32_tiny(gpu_lib):
    p = synth.make_problem(synth.TINY)
    s = p.spec
    mx, mean, n_alt = _check_full(gpu_lib, p.x32, s.n_query, s.k1, s.k2, s.layers)
    print(f"tiny f32: max err {mx:.2e} mean {mean:.2e} pairs vs tie-breaks {n_alt}")
    assert n_alt == 0


EDGE = [
    # n, q, d, k1, k2, layers, alpha, node, dup, n_ids
    (2, 1, 1, 1, 1, 0, 2, "adj", 0.0, 0),
    (2, 1, 3, 2, 2, 1, 2, "adj", 0.0, 0),
    (5, 2, 2, 3, 2, 1, 2, "adj", 0.0, 0),
    (65, 7, 33, 5, 2, 2, 2, "adj", 0.0, 4),
    (130, 30, 64, 9, 4, 3, 2, "adj", 0.2, 6),
    (200, 50, 17, 200, 7, 1, 2, "adj", 0.0, 0),
    (257, 64, 128, 1, 1, 2, 2, "adj", 0.0, 5),
    (300, 100, 40, 12, 12, 0, 2, "adj", 0.0, 10),
    (300, 100, 40, 12, 5, 2, 0, "adj", 0.0, 10),
    (333, 33, 96, 20, 6, 0, 2, "raw", 0.0, 8),
    (333, 33, 96, 20, 6, 2, 2, "raw", 0.0, 8),
    (511, 200, 256, 64, 8, 1, 3, "adj", 0.1, 20),
    (700, 300, 24, 100, 10, 2, 2, "adj", 0.0, 7),
    (1029, 129, 130, 250, 30, 1, 2, "adj", 0.0, 9),
]


@pytest.mark.parametrize("n,q,d,k1,k2,layers,alpha,node,dup,n_ids", EDGE)
def test_edge_cases_f32(gpu_lib, n, q, d, k1, k2, layers, alpha, node, dup, n_ids):
    x = synth.random_features(n, d, seed=n * 7 + d, n_ids=n_ids, dup_frac=dup)
    mx, mean, excused = _check_full(gpu_lib, x, q, k1, k2, layers, alpha=alpha, node=node)
    print(f"max err {mx:.2e} mean {mean:.2e} pairs vs tie-breaks {excused}")


def test_integer_ties_hand_example(gpu_lib):
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_5pt.json")))
    x = np.array(g["x"], dtype=np.float32)
    for layers, key in ((0, "D_layers0"), (1, "D_layers1")):
        dg, ki, _ = _run(gpu_lib, x, g["n_query"], g["k1"], g["k2"], layers)
        assert ki.tolist() == g["lists"]
        np.testing.assert_allclose(dg, np.array(g[key]), atol=1e-6)


def test_bf16_input_matches_f32_of_same_values(gpu_lib):
    import torch
    spec = synth.ProblemSpec("b", 40, 260, 64, 12, 0.5, 0.05, 8, 3, 2, "bf16", 9)
    p = synth.make_problem(spec)
    xb = torch.from_numpy(p.x_bf16.view(np.int16)).cuda().view(torch.bfloat16)
    from paper_2012_07620_amd import binding
    d1 = binding.run(xb, 40, 8, 3, 2)
    d2 = binding.run(_dev(p.x32), 40, 8, 3, 2)
    torch.cuda.synchronize()
    assert torch.equal(d1, d2)
    _check_full(gpu_lib, p.x32, 40, 8, 3, 2)


def test_repeat_runs_bit_identical(gpu_lib):
    import torch
    from paper_2012_07620_amd import binding
    p = synth.make_problem(synth.TINY)
    x = _dev(p.x32)
    a = binding.run(x, 100, 10, 3, 2)
    b = binding.run(x, 100, 10, 3, 2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_low_precision_tiny(gpu_lib, prec):
    p = synth.make_problem(synth.TINY)
    s = p.spec
    dg, ki, kv = _run(gpu_lib, p.x32, s.n_query, s.k1, s.k2, s.layers, sim_prec=prec)
    ref = orc.rerank(p.x32, s.n_query, s.k1, s.k2, s.layers)
    overlap = np.mean([len(set(a) & set(b)) / s.k1 for a, b in zip(ki.tolist(), ref.graph.idx.tolist())])
    err = np.abs(dg - ref.dist)
    print(f"{prec}: top-k1 overlap {overlap:.5f}, D max err {err.max():.2e} mean {err.mean():.2e}")
    assert overlap >= 0.995
    assert err.max() <= D_TOL_LOWP


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_low_precision_similarity_error(gpu_lib, prec):
    import torch
    from paper_2012_07620_amd import binding
    p = synth.make_problem(synth.TINY)
    s = binding.similarity(_dev(p.x32), sim_prec=prec)
    torch.cuda.synchronize()
    ref = orc.similarity_rows(orc.unit_rows(p.x32), range(p.spec.n))
    err = np.abs(s.cpu().numpy() - ref)
    print(f"{prec}: max |S - S64| = {err.max():.3e}, mean {err.mean():.3e}")
    assert err.max() < (0.02 if prec == "bf16" else 0.08)


@pytest.mark.parametrize("n,q,d,k1,k2,layers,node", [
    (1000, 100, 128, 10, 3, 1, "adj"),
    (300, 100, 40, 12, 5, 0, "adj"),
    (333, 33, 96, 20, 6, 2, "raw"),
    (333, 33, 96, 20, 6, 0, "raw"),
    (130, 30, 64, 9, 4, 3, "adj"),
    (12000, 5000, 64, 20, 6, 1, "adj"),  # 40 x 55 tiles: the partly filled last round is split along K
])
def test_final_bf16x3_matches_fp64(gpu_lib, n, q, d, k1, k2, layers, node):
    # the split-bf16 final product must meet the FP32 path's tolerance
    x = synth.random_features(n, d, seed=n + d + layers, n_ids=8)
    mx, mean, excused = _check_full(gpu_lib, x, q, k1, k2, layers, node=node, final_prec="bf16x3")
    print(f"bf16x3: max err {mx:.2e} mean {mean:.2e}")


VARIANTS = [
    # n, q, d, k1, k2, layers, node, aggregator
    (300, 60, 48, 12, 5, 1, "adj", "mean"),
    (300, 60, 48, 12, 5, 2, "adj", "max"),
    (300, 60, 48, 12, 5, 0, "adj_raw", "sum"),
    (300, 60, 48, 12, 5, 1, "adj_raw", "sum"),
    (300, 60, 48, 12, 5, 2, "adj_raw", "mean"),
    (300, 60, 48, 12, 5, 1, "adj_raw", "max"),
    (333, 33, 96, 20, 6, 2, "raw", "max"),
    (333, 33, 96, 20, 6, 1, "raw", "mean"),
    (1000, 100, 128, 10, 3, 1, "adj", "max"),
]


@pytest.mark.parametrize("n,q,d,k1,k2,layers,node,agg", VARIANTS)
def test_variants_match_fp64(gpu_lib, n, q, d, k1, k2, layers, node, agg):
    # Eq. 13 aggregators and the Table 1 node-feature modes
    x = synth.random_features(n, d, seed=n + 3 * d + layers, n_ids=9)
    print(f"case {node}/{agg}", flush=True)
    dg, ki, kv = _run(gpu_lib, x, q, k1, k2, layers, node=node, aggregator=agg)
    ref = orc.rerank(x, q, k1, k2, layers, node=node, aggregator=agg)
    r = check_run(x, ref, ki, dg, q, k2, layers, D_TOL_F32, node=node, aggregator=agg)
    print(f"{node}/{agg} L={layers}: max err {r['max_err']:.2e}, pairs vs tie-breaks {r['pairs_vs_tie_breaks']}")


def test_hand_example_variants(gpu_lib):
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_5pt.json")))
    x = np.array(g["x"], dtype=np.float32)
    for agg, key in (("mean", "D_layers1_mean"), ("max", "D_layers1_max")):
        dg, _, _ = _run(gpu_lib, x, g["n_query"], g["k1"], g["k2"], 1, aggregator=agg)
        np.testing.assert_allclose(dg, np.array(g[key]), atol=1e-6)
    dg, _, _ = _run(gpu_lib, x, g["n_query"], g["k1"], g["k2"], 0, node="adj_raw")
    np.testing.assert_allclose(dg, np.array(g["D_layers0_A"]), atol=1e-6)


@pytest.mark.parametrize("q,g,r", [(1, 1, 1), (7, 300, 5), (33, 1000, 64), (5, 257, 200), (64, 5000, 256)])
def test_ranking_list(gpu_lib, q, g, r):
    # seeded distance matrices with many exact ties; the ranking list of
    # Algorithm 1 (ascending, ties to the lower position) must match exactly
    import torch
    from paper_2012_07620_amd import binding
    rng = np.random.default_rng(q * 1000 + g)
    d = (np.round(rng.random((q, g)) * 64) / 64).astype(np.float32)
    d[:, ::7] = 0.0
    d[:, 1::11] = -0.0
    got = binding.rank(torch.from_numpy(d).cuda(), r).cpu().numpy()
    ref = orc.ranking(d.astype(np.float64) + 0.0, r)
    assert np.array_equal(got, ref)


def test_ranking_of_a_rerank(gpu_lib):
    import torch
    from paper_2012_07620_amd import binding
    p = synth.make_problem(synth.TINY)
    s = p.spec
    d = binding.run(_dev(p.x32), s.n_query, s.k1, s.k2, s.layers)
    rk = binding.rank(d, 20).cpu().numpy()
    ref = orc.rerank(p.x32, s.n_query, s.k1, s.k2, s.layers)
    dref = ref.dist
    oref = orc.ranking(dref, 21)
    for qi in range(s.n_query):
        # positions whose oracle distances are separated by more than the FP32 error must agree
        for pos in range(20):
            a, b = dref[qi, oref[qi, pos]], dref[qi, oref[qi, pos + 1]]
            prev = dref[qi, oref[qi, pos - 1]] if pos else -np.inf
            if b - a > 1e-5 and a - prev > 1e-5:
                assert rk[qi, pos] == oref[qi, pos]


@pytest.mark.parametrize("layers", [64, 256])
@pytest.mark.parametrize("final_prec", ["f32", "sparse"])
def test_many_layers(gpu_lib, layers, final_prec):
    # Table 2 runs up to 256 layers: rows are renormalised after every layer,
    # so rounding does not grow with depth; the sparse layers turn dense once
    # their supports outgrow the slots, on the device
    x = synth.random_features(300, 32, seed=layers, n_ids=6)
    mx, mean, excused = _check_full(gpu_lib, x, 60, 12, 5, layers, final_prec=final_prec)
    print(f"L={layers} {final_prec}: max err {mx:.2e} mean {mean:.2e} pairs vs tie-breaks {excused}")


BF16_FINAL_CASES = [
    # n, q, d, k1, k2, layers, node, sim
    (1000, 100, 128, 10, 3, 1, "adj", "f32"),
    (300, 100, 40, 12, 5, 0, "adj", "f32"),
    (333, 33, 96, 20, 6, 2, "raw", "f32"),
    (333, 33, 96, 20, 6, 0, "raw", "bf16"),
    (2049, 333, 64, 20, 6, 2, "adj", "bf16"),
    (5000, 700, 64, 20, 6, 1, "adj", "fp8"),
]


@pytest.mark.parametrize("n,q,d,k1,k2,layers,node,sim", BF16_FINAL_CASES)
def test_final_bf16_within_low_precision_tolerance(gpu_lib, n, q, d, k1, k2, layers, node, sim):
    # bfloat16 operands for the final product: a low-precision mode, held to
    # the low-precision paths' bar (D within 2e-2 of the FP64 oracle); its
    # error is bounded by about 2 * 2^-8 of |h_q| |h_g|
    x = synth.random_features(n, d, seed=n + 3 * d + layers, n_ids=max(2, n // 20))
    print(f"case bf16 final n={n} q={q} d={d} k1={k1} k2={k2} L={layers} node={node} sim={sim}", flush=True)
    dg, ki, kv = _run(gpu_lib, x, q, k1, k2, layers, node=node, sim_prec=sim, final_prec="bf16")
    ref = orc.rerank(x, q, k1, k2, layers, node=node)
    err = np.abs(dg.astype(np.float64) - ref.dist)
    print(f"bf16 final: D vs FP64 max {err.max():.2e} mean {err.mean():.2e}")
    assert np.all(np.isfinite(dg)) and err.max() <= 2e-2


def test_features_read_in_place_and_copied_agree(gpu_lib):
    """FP32 rows whose length is a multiple of 64 on a 256-byte aligned address
    are read in place by the products and the re-score; the same values 16
    bytes further on are first copied into the working set. Both routes give
    bit-identical lists and distances in every similarity precision."""
    import torch
    from paper_2012_07620_amd import binding
    n, q, d = 1500, 300, 128
    x = synth.random_features(n, d, seed=5, n_ids=30)
    a = torch.from_numpy(x).cuda()
    buf = torch.empty(n * d + 4, device="cuda")
    b = buf[4:].view(n, d)
    b.copy_(a)
    assert a.data_ptr() % 256 == 0 and b.data_ptr() % 256 == 16
    for prec in ("f32", "bf16", "fp8"):
        print(f"case prec={prec}", flush=True)
        da, ia, va = binding.run(a, q, 20, 6, 1, sim_prec=prec, return_knn=True)
        db, ib, vb = binding.run(b, q, 20, 6, 1, sim_prec=prec, return_knn=True)
        torch.cuda.synchronize()
        assert torch.equal(ia, ib) and torch.equal(va, vb) and torch.equal(da, db)
        # the similarity entry point reads the rows the same two ways
        sa, sb = binding.similarity(a, sim_prec=prec), binding.similarity(b, sim_prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(sa, sb)
