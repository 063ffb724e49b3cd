"""Comparison helpers for GPU-vs-oracle parity (test infrastructure).

Expected values always come from the FP64 oracle on the same inputs. The
GPU's lists only decide which comparisons are excused: a list may differ from
the oracle's only at a row whose similarity margin at the list boundary is
below the stated tie tolerance, and distances that depend on such a row are
then compared against nothing (they are counted and reported).
"""
from __future__ import annotations

import numpy as np

TIE_TOL = 1e-6  # similarity margin below which the k1 / k2 boundary is a tie


def compare_lists(gpu_idx: np.ndarray, graph, k2: int, tie_tol: float = TIE_TOL):
    """Check the GPU's N x k1 lists against the oracle graph.

    Returns (flip1, flip2): rows whose k1 set / k2 prefix set differ. Raises
    AssertionError when a differing row is not exempt, when member 0 is not
    the row itself, or when a list holds a repeated index."""
    n, k1 = graph.idx.shape
    assert gpu_idx.shape == (n, k1)
    assert np.all(gpu_idx[:, 0] == np.arange(n)), "member 0 must be the row itself"
    srt = np.sort(gpu_idx, axis=1)
    assert np.all(srt[:, 1:] != srt[:, :-1]), "repeated neighbour"
    assert gpu_idx.min() >= 0 and gpu_idx.max() < n
    flip1 = np.flatnonzero(np.any(np.sort(graph.idx, 1) != srt, axis=1))
    bad1 = flip1[graph.gap1[flip1] >= tie_tol]
    assert bad1.size == 0, f"k1 sets differ on non-tied rows {bad1[:10]} (gaps {graph.gap1[bad1[:10]]})"
    g2 = np.sort(gpu_idx[:, :k2], 1)
    o2 = np.sort(graph.idx[:, :k2], 1)
    flip2 = np.flatnonzero(np.any(g2 != o2, axis=1))
    bad2 = flip2[(graph.gap2[flip2] >= tie_tol) & ~np.isin(flip2, flip1)]
    assert bad2.size == 0, f"k2 prefixes differ on non-tied rows {bad2[:10]}"
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
    for _ in range(layers):
        t = t | np.any(t[nb], axis=1)
    return t


def compare_distances(d_gpu: np.ndarray, d_ref: np.ndarray, n_query: int, taint: np.ndarray, tol: float,
                      q_rows=None, g_rows=None):
    """Max |D_gpu - D_oracle| over pairs with no tainted endpoint; returns
    (max_err, mean_err, excused_pairs)."""
    nq, ng = d_ref.shape
    q = np.arange(nq) if q_rows is None else np.asarray(q_rows)
    g = np.arange(ng) if g_rows is None else np.asarray(g_rows)
    ok = ~(taint[q][:, None] | taint[n_query + g][None, :])
    err = np.abs(d_gpu.astype(np.float64) - d_ref)
    assert np.all(np.isfinite(d_gpu)), "non-finite distances"
    e = err[ok]
    max_err = float(e.max()) if e.size else 0.0
    assert max_err <= tol, f"max |D - D_oracle| = {max_err:.3e} > {tol:.1e}"
    return max_err, float(e.mean()) if e.size else 0.0, int((~ok).sum())
