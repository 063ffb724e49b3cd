"""Retrieval metrics (rerank_evaluate, Section 4.1) against the oracle.

Per-query list positions of the first true match and Recall@K are integer
results and must match exactly; AP and mAP are float64 sums whose terms the
kernel adds in gallery order and the oracle in list order, so they agree to
a few units in the last place (tolerance 1e-12). Every call goes through the
C-ABI library."""
import numpy as np
import pytest

from oracle import rerank_oracle as orc
from paper_2012_07620_amd import synth

pytestmark = pytest.mark.gpu

AP_TOL = 1e-12


def _gpu_eval(dist, ql, gl, ks, ld=None):
    import torch
    from paper_2012_07620_amd import binding
    q, g = dist.shape
    if ld is None:
        d = torch.from_numpy(np.ascontiguousarray(dist, dtype=np.float32)).cuda()
    else:  # rows inside a wider buffer
        buf = torch.full((q, ld), 7.0, dtype=torch.float32, device="cuda")
        buf[:, :g] = torch.from_numpy(np.ascontiguousarray(dist, dtype=np.float32)).cuda()
        d = buf[:, :g]
    res = binding.evaluate(d, torch.from_numpy(ql.astype(np.int32)).cuda(),
                           torch.from_numpy(gl.astype(np.int32)).cuda(), ks)
    torch.cuda.synchronize()
    return res


def _compare(dist, ql, gl, ks, ld=None):
    got = _gpu_eval(dist, ql, gl, ks, ld)
    ref = orc.evaluate(dist.astype(np.float32), ql, gl, ks)
    first = got["first"].cpu().numpy()
    ap = got["ap"].cpu().numpy()
    assert np.array_equal(first, ref["first"])
    np.testing.assert_allclose(ap, ref["ap"], rtol=0, atol=AP_TOL)
    assert got["queries"] == ref["queries"]
    assert got["map"] == pytest.approx(ref["map"], abs=AP_TOL)
    for k in ks:
        assert got["recall"][k] == ref["recall"][k]
    return got


CASES = [
    # q, g, distinct distance levels (few = many ties), labels, ld
    (1, 1, 3, 1, None),
    (3, 5, 2, 2, None),
    (40, 300, 7, 9, None),        # ties everywhere
    (25, 4097, 1000, 30, None),   # two LDS tiles, ragged second
    (10, 9000, 50, 3, 9100),      # > 1024 true matches per query: several passes; strided rows
    (64, 2500, 100000, 60, None),
]


@pytest.mark.parametrize("q,g,levels,labels,ld", CASES)
def test_evaluate_matches_oracle(gpu_lib, q, g, levels, labels, ld):
    print(f"case evaluate q={q} g={g} levels={levels} labels={labels} ld={ld}", flush=True)
    rng = np.random.default_rng(q * 1000 + g)
    dist = (rng.integers(0, levels, (q, g)) / levels).astype(np.float32)
    ql = rng.integers(0, labels + 1, q)      # label `labels` may be absent from the gallery
    gl = rng.integers(0, labels, g)
    if q > 1:
        ql[0] = 10 ** 6                      # a query without any true match
    _compare(dist, ql, gl, (1, 5, 10, g + 3), ld)


def test_evaluate_on_reranked_distances(gpu_lib):
    # the method's own output on the 1000-row shape, drawn noisier (sigma = 2)
    # so that retrieval is imperfect; labels from the generator
    import dataclasses
    import torch
    from paper_2012_07620_amd import binding
    p = synth.make_problem(dataclasses.replace(synth.TINY, sigma=2.0))
    s = p.spec
    ql, gl = p.labels[:s.n_query], p.labels[s.n_query:]
    x = torch.from_numpy(p.x32).cuda()
    for layers, node in ((0, "raw"), (s.layers, "adj")):
        dist = binding.run(x, s.n_query, s.k1, s.k2, layers, node=node).cpu().numpy()
        got = _compare(dist, ql, gl, (1, 5, 10))
        ref = orc.evaluate(orc.rerank(p.x32, s.n_query, s.k1, s.k2, layers, node=node).dist, ql, gl, (1, 5, 10))
        print(f"tiny sigma 2, L={layers} {node}: mAP {got['map']:.4f} (oracle pipeline {ref['map']:.4f}) "
              f"R@1 {got['recall'][1]:.4f}")
        assert got["map"] == pytest.approx(ref["map"], abs=2e-3)  # D within 1e-4 of FP64: at most near-tie flips


def test_evaluate_full_size_sampled(gpu_lib):
    # 19281-row workload: the whole matrix on the GPU, 150 sampled queries re-done by the oracle
    import torch
    from paper_2012_07620_amd import binding
    spec = synth.MID
    x, labels = synth.make_features_device(spec, "cuda", return_labels=True)
    dist = binding.run(x, spec.n_query, spec.k1, spec.k2, spec.layers)
    ql, gl = labels[:spec.n_query].contiguous(), labels[spec.n_query:].contiguous()
    got = binding.evaluate(dist, ql, gl, (1, 5, 10))
    torch.cuda.synchronize()
    rows = np.random.default_rng(0).choice(spec.n_query, 150, replace=False)
    d = dist[torch.from_numpy(rows).cuda()].cpu().numpy()
    gl_h = gl.cpu().numpy()
    ql_h = ql.cpu().numpy()[rows]
    ref = orc.evaluate(d, ql_h, gl_h, (1, 5, 10))
    assert np.array_equal(got["first"].cpu().numpy()[rows], ref["first"])
    np.testing.assert_allclose(got["ap"].cpu().numpy()[rows], ref["ap"], rtol=0, atol=AP_TOL)
    print(f"mid: mAP {got['map']:.4f} R@1 {got['recall'][1]:.4f} over {got['queries']} queries")
    assert got["queries"] == spec.n_query
