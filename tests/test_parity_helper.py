"""The parity helper's exemptions follow the tie rule and nothing wider.

A hand-built problem has one exact tie at row 0's k1 boundary (rows 2 and 3
are equally similar to row 0) and a clear margin at its k2 boundary. The
helper must accept the other tie-break, with the distances that follow from
it, and must reject: a k2 prefix changed on that row (its k2 margin is not a
tie, whatever happened at k1), a k1 member swapped for one that is not tied,
distances that do not follow from the lists reported, and a distance error
on a pair that depends on the tie."""
import numpy as np
import pytest

from oracle import rerank_oracle as orc
from tests.parity import alternative_distances, check_run, compare_lists

X = np.array([
    [1.0, 0.0, 0.0],
    [0.9, 0.1, 0.0],
    [0.5, 0.5, 0.0],
    [0.5, 0.0, 0.5],  # a permutation of row 2's entries: S_02 == S_03 exactly
    [-1.0, 0.2, 0.1],
    [0.0, 1.0, 0.0],
    [0.0, 0.0, 1.0],
    [-0.5, -0.5, 0.3],
], dtype=np.float32)
Q, K1, K2, L = 1, 3, 2, 1


@pytest.fixture(scope="module")
def ref():
    r = orc.rerank(X, Q, K1, K2, L)
    assert r.graph.idx[0].tolist() == [0, 1, 2]  # tie broken by the lower index
    assert r.graph.gap1[0] == 0.0 and r.graph.gap2[0] > 0.1
    return r


def _lists(ref, row0):
    idx = ref.graph.idx.copy()
    idx[0] = row0
    return idx


def test_the_other_tie_break_is_accepted(ref):
    gpu = _lists(ref, [0, 1, 3])
    d = alternative_distances(X, ref.graph, gpu, [0], Q, K2, L).astype(np.float32)
    assert np.abs(d - ref.dist).max() > 1e-3  # the tie-break moves the distances
    r = check_run(X, ref, gpu, d, Q, K2, L, 1e-4)
    assert r["tied_rows_k1"] == 1 and r["pairs_vs_tie_breaks"] > 0
    assert r["max_err"] < 1e-6


def test_distances_must_follow_the_reported_tie_break(ref):
    gpu = _lists(ref, [0, 1, 3])
    with pytest.raises(AssertionError):
        check_run(X, ref, gpu, ref.dist.astype(np.float32), Q, K2, L, 1e-4)


def test_k2_prefix_checked_on_a_row_whose_k1_set_is_tied(ref):
    # same k1 set as the valid tie-break, but the k2 prefix {0, 3} is not {0, 1}
    with pytest.raises(AssertionError, match="k2 prefixes"):
        compare_lists(_lists(ref, [0, 3, 1]), ref.graph, K2, x=X)


def test_a_member_that_is_not_tied_is_rejected(ref):
    # row 0 has a tie at k1, but dropping member 1 (far above the boundary) is no tie-break
    with pytest.raises(AssertionError):
        compare_lists(_lists(ref, [0, 2, 3]), ref.graph, K2, x=X)


def test_error_on_a_tied_pair_is_caught(ref):
    gpu = _lists(ref, [0, 1, 3])
    d = alternative_distances(X, ref.graph, gpu, [0], Q, K2, L).astype(np.float32)
    d[0, 2] += 1e-3  # gallery row 3: a tied member of query 0
    with pytest.raises(AssertionError, match="max"):
        check_run(X, ref, gpu, d, Q, K2, L, 1e-4)


def test_exact_lists_need_no_tie_breaks(ref):
    r = check_run(X, ref, ref.graph.idx.copy(), ref.dist.astype(np.float32), Q, K2, L, 1e-4)
    assert r["tied_rows_k1"] == 0 and r["pairs_vs_tie_breaks"] == 0
