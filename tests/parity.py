"""Comparison helpers for GPU-vs-oracle parity (test infrastructure).

Expected values always come from the FP64 oracle. The method's result is
unique except where two neighbour sets are equally correct: a row whose
similarity margin at the k1 boundary (or the k2 boundary) is below the tie
tolerance may keep a different set there. The helpers below

* compare every row's k1 set and k2 prefix with the oracle's, and excuse a
  difference only on a row whose own margin at that boundary is below the
  tolerance (gap1 for the k1 set, gap2 for the k2 prefix, independently);
* check that every excused choice is itself a valid one: each member the GPU
  kept is within the tolerance of every row it left out, by the FP64
  similarities of that row (Eq. 7-8);
* compare every query x gallery distance: pairs that no excused choice can
  reach against the oracle's end-to-end result, the others against the
  oracle run again from the same features with the alternative sets the GPU
  chose at its tied rows (Eq. 9-14 on those lists, FP64 edge weights). No
  pair is left unchecked.
"""
from __future__ import annotations

import numpy as np

from oracle import rerank_oracle as orc

TIE_TOL = 1e-6  # similarity margin below which the k1 / k2 boundary is a tie


def check_alternative(xhat: np.ndarray, i: int, members: np.ndarray, tie_tol: float, what: str) -> None:
    """Row i's GPU-chosen members (self excluded) must beat every other row
    by at least -tie_tol in FP64 similarity."""
    s = xhat @ xhat[i]
    s[i] = np.nan
    inside = np.zeros(s.shape[0], dtype=bool)
    inside[members] = True
    inside[i] = False
    out = ~inside
    out[i] = False
    if not inside.any() or not out.any():
        return
    lo_in = float(np.min(s[inside]))
    hi_out = float(np.max(s[out]))
    assert lo_in >= hi_out - tie_tol, (f"row {i}: the GPU's {what} keeps a member at S = {lo_in:.9f} but leaves out "
                                       f"one at S = {hi_out:.9f} (more than {tie_tol:g} apart)")


def compare_lists(gpu_idx: np.ndarray, graph, k2: int, x=None, tie_tol: float = TIE_TOL):
    """Check the GPU's N x k1 lists against the oracle graph.

    Returns (flip1, flip2): rows whose k1 set / k2 prefix set differ. Raises
    AssertionError when a differing row is not exempt by its own margin at
    that boundary, when member 0 is not the row itself, or when a list holds
    a repeated index. With ``x`` (the features) every differing row's
    choice is also checked to be a valid tie-break against its FP64 row."""
    n, k1 = graph.idx.shape
    assert gpu_idx.shape == (n, k1)
    assert np.all(gpu_idx[:, 0] == np.arange(n)), "member 0 must be the row itself"
    assert gpu_idx.min() >= 0 and gpu_idx.max() < n
    srt = np.sort(gpu_idx, axis=1)
    assert np.all(srt[:, 1:] != srt[:, :-1]), "repeated neighbour"
    flip1 = np.flatnonzero(np.any(np.sort(graph.idx, 1) != srt, axis=1))
    bad1 = flip1[graph.gap1[flip1] >= tie_tol]
    assert bad1.size == 0, f"k1 sets differ on non-tied rows {bad1[:10]} (gaps {graph.gap1[bad1[:10]]})"
    g2 = np.sort(gpu_idx[:, :k2], 1)
    o2 = np.sort(graph.idx[:, :k2], 1)
    flip2 = np.flatnonzero(np.any(g2 != o2, axis=1))
    bad2 = flip2[graph.gap2[flip2] >= tie_tol]
    assert bad2.size == 0, f"k2 prefixes differ on non-tied rows {bad2[:10]} (gaps {graph.gap2[bad2[:10]]})"
    if x is not None and (flip1.size or flip2.size):
        xhat = orc.unit_rows(x)
        for i in flip1:
            check_alternative(xhat, int(i), gpu_idx[i], tie_tol, "k1 set")
        for i in flip2:
            check_alternative(xhat, int(i), gpu_idx[i, :k2], tie_tol, "k2 prefix")
    return flip1, flip2


def tainted_rows(oracle_idx: np.ndarray, gpu_idx: np.ndarray, flip1, flip2, k2: int, layers: int) -> np.ndarray:
    """Rows whose final feature can depend on a tied (excused) list choice."""
    n = oracle_idx.shape[0]
    t = np.zeros(n, dtype=bool)
    for f in flip1:  # A* row f and every row it touches (either list) change
        t[f] = True
        t[oracle_idx[f]] = True
        t[gpu_idx[f]] = True
    t[np.asarray(flip2, dtype=np.int64)] = True
    nb = oracle_idx[:, :k2]
    gb = gpu_idx[:, :k2]
    for _ in range(layers):
        t = t | np.any(t[nb], axis=1) | np.any(t[gb], axis=1)
    return t


def alternative_distances(x, graph, gpu_idx: np.ndarray, rows, n_query: int, k2: int, layers: int,
                          alpha: int = 2, node: str = "adj", aggregator: str = "sum", q_rows=None, g_rows=None):
    """The oracle's distances for the neighbour lists the GPU chose: the
    oracle's lists with ``rows`` (tied rows, already checked to be valid
    tie-breaks) replaced by the GPU's, every edge weight the FP64 similarity
    of its pair (Eq. 12, 14), then Eq. 9-14 and the final cosine."""
    idx = graph.idx.copy()
    val = graph.val.copy()
    rows = np.asarray(rows, dtype=np.int64)
    if rows.size:
        xhat = orc.unit_rows(x)
        for i in rows:
            m = gpu_idx[i].astype(np.int64)
            idx[i] = m
            v = xhat[m] @ xhat[i]
            v[0] = 1.0
            val[i] = v
    h0 = orc.initial_features(x, idx, node)
    w = orc.edge_weights(idx, val, k2, alpha)
    h = orc.propagate(h0, w, layers, aggregator=aggregator)
    return orc.distances(h, n_query, q_rows=q_rows, g_rows=g_rows)


def compare_distances(d_gpu: np.ndarray, d_ref: np.ndarray, n_query: int, taint: np.ndarray, tol: float,
                      q_rows=None, g_rows=None, d_alt=None):
    """Every |D_gpu - D_expected| <= tol: pairs with no tainted endpoint
    against ``d_ref`` (the oracle end to end), the rest against ``d_alt``
    (the oracle on the GPU's tie-breaks; required when any pair is tainted).
    Returns (max_err, mean_err, pairs compared against d_alt)."""
    nq, ng = d_ref.shape
    assert d_gpu.shape == d_ref.shape
    assert np.all(np.isfinite(d_gpu)), "non-finite distances"
    q = np.arange(nq) if q_rows is None else np.asarray(q_rows)
    g = np.arange(ng) if g_rows is None else np.asarray(g_rows)
    tainted = taint[q][:, None] | taint[n_query + g][None, :]
    n_alt = int(tainted.sum())
    err = np.abs(d_gpu.astype(np.float64) - d_ref)
    if n_alt:
        assert d_alt is not None and d_alt.shape == d_ref.shape, \
            f"{n_alt} pairs depend on tied rows: the oracle on the GPU's tie-breaks is needed to check them"
        err = np.where(tainted, np.abs(d_gpu.astype(np.float64) - d_alt), err)
    max_err = float(err.max()) if err.size else 0.0
    assert max_err <= tol, f"max |D - D_oracle| = {max_err:.3e} > {tol:.1e}"
    return max_err, float(err.mean()) if err.size else 0.0, n_alt


def check_run(x, ref, gpu_idx: np.ndarray, d_gpu: np.ndarray, n_query: int, k2: int, layers: int, tol: float,
              alpha: int = 2, node: str = "adj", aggregator: str = "sum", q_rows=None, graph=None, d_ref=None):
    """Lists and distances of one GPU run against the oracle, every pair
    checked. ``ref`` is an oracle result (or pass ``graph`` and ``d_ref``).
    Returns a dict with the errors and the counts of tied rows and pairs."""
    graph = ref.graph if graph is None else graph
    d_ref = ref.dist if d_ref is None else d_ref
    f1, f2 = compare_lists(gpu_idx, graph, k2, x=x)
    taint = tainted_rows(graph.idx, gpu_idx, f1, f2, k2, layers)
    d_alt = None
    rows = np.union1d(f1, f2)
    if rows.size:
        d_alt = alternative_distances(x, graph, gpu_idx, rows, n_query, k2, layers, alpha, node, aggregator,
                                      q_rows=q_rows)
    mx, mean, n_alt = compare_distances(d_gpu, d_ref, n_query, taint, tol, q_rows=q_rows, d_alt=d_alt)
    return {"max_err": mx, "mean_err": mean, "tied_rows_k1": int(f1.size), "tied_rows_k2": int(f2.size),
            "pairs_vs_tie_breaks": n_alt, "flip1": f1, "flip2": f2}
