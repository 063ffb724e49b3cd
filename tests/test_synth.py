"""The seeded generators: shapes, determinism, and the recipe's statistics."""
import numpy as np

from paper_2012_07620_amd import synth


def test_tiny_problem_recipe():
    p = synth.make_problem(synth.TINY)
    s = p.spec
    assert p.x32.shape == (s.n, s.dim) and p.x32.dtype == np.float32
    np.testing.assert_allclose(np.linalg.norm(p.x32, axis=1), 1.0, atol=1e-6)
    q_lab, g_lab = p.labels[: s.n_query], p.labels[s.n_query:]
    assert np.bincount(q_lab).tolist() == [2] * 50
    assert np.bincount(g_lab).tolist() == [18] * 50
    # same identity: cos ~ 1/(1+sigma^2); different identities: ~0
    x = p.x32.astype(np.float64)
    same = [x[i] @ x[j] for i in range(40) for j in range(40, 400) if p.labels[i] == p.labels[j]]
    diff = [x[i] @ x[j] for i in range(40) for j in range(40, 400) if p.labels[i] != p.labels[j]]
    assert abs(np.mean(same) - 1 / (1 + 0.3 ** 2)) < 0.03
    assert abs(np.mean(diff)) < 0.02


def test_deterministic_and_seed_sensitive():
    a = synth.make_problem(synth.TINY).x32
    b = synth.make_problem(synth.TINY).x32
    c = synth.make_problem(synth.TINY, seed=5).x32
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_distractors_and_bf16():
    spec = synth.ProblemSpec("t", 30, 200, 64, 10, 0.5, 0.05, 8, 3, 1, "bf16", 3)
    p = synth.make_problem(spec)
    g_lab = p.labels[30:]
    assert (g_lab >= 10).sum() == 10 and len(set(g_lab[g_lab >= 10])) == 10
    assert p.x_bf16 is not None and p.x_bf16.dtype == np.uint16
    np.testing.assert_array_equal(synth.f32_from_bf16_bits(p.x_bf16), p.x32)


def test_bf16_rounding_is_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 1.0 + 2 ** -8 + 2 ** -20], dtype=np.float32)
    back = synth.f32_from_bf16_bits(synth.bf16_bits_from_f32(x))
    assert back.tolist() == [1.0, 1.0, 1.0 + 4 * 2 ** -8, -2.5, 1.0 + 2 ** -7]


def test_request_stream():
    reqs = synth.request_specs(synth.StreamSpec(), 50, qps=20.0)
    t = [a for a, _ in reqs]
    assert all(b > a for a, b in zip(t, t[1:]))
    for _, s in reqs:
        assert 1000 <= s.n <= 30000 and s.dim in (512, 2048)
        assert s.n_query == max(1, round(0.15 * s.n))
