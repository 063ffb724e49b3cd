"""FP64 CPU oracle for GNN-based re-ranking (Zhang et al., "Understanding Image
Retrieval Re-Ranking: A Graph Neural Network Perspective", Section 3.3,
Equations 7-14 and Algorithm 1).

TEST INFRASTRUCTURE. Only the test-suite, the package smoke check and the
CPU-baseline leg of the benchmark may import or run this module. The product
path never calls it and shares no code with it: the GPU library has its own
kernels, the oracle is plain NumPy/SciPy in float64.

The method reaches a defined result (no approximation), so each function is
the definition written out in float64, taken from the exact input values:

  Eq. 7      S_ij = cos(x_i, x_j) over the union of queries and gallery.
  Eq. 8      A_ij = 1 iff j is one of the k1 most similar rows of row i.
  Eq. 9-10   A* = (A + A^T) / 2, entries in {0, 0.5, 1}.
  Eq. 11     h_i^(0) = row i of A*  (vertex feature).
  Eq. 12     edges e_ij = S_ij for j among the k2 most similar rows of i.
  Eq. 14     h_i^(l+1) = h_i^(l) + sum_{j in N(i,k2)} e_ij^alpha h_j^(l)
             (aggregator "sum", alpha = 2 in the paper's experiments),
             followed by an L2 normalisation of every row (Section 3.3,
             paragraph after Eq. 14).
  Final      ranking by cosine similarity of the refined features; the
             oracle returns the query x gallery distance 1 - cos.

Readings taken where the paper is silent (each is also the GPU library's;
R11 and R12 concern arguments and test tolerances, not arithmetic):
  R1  cos is a true cosine: rows are divided by their norm.
  R2  row i itself is always member 0 of N(i, k) with similarity exactly 1,
      so every row has exactly k1 neighbours including itself.
  R3  the order inside N(i, k) is similarity descending, ties to the lower
      column index, -0.0 equal to +0.0.
  R4  candidates are all N rows (queries and gallery alike).
  R5  N(i, k2) is the first k2 members of N(i, k1) (k2 <= k1), self
      included, so the self coefficient in Eq. 14 is 1 (residual) + 1.
  R6  h^(0) is the raw A* row; normalisation happens after each layer.
  R7  the edge weights use the original S and stay fixed for all layers.
  R8  alpha is a non-negative integer; e^alpha is the plain power.
  R9  output D_qg = 1 - cos(h_q, h_g) for q < Q <= g < N.
  R10 node mode "raw" uses h^(0)_i = x_i (the Table 1 ablation column with
      original features); with zero layers it gives the initial ranking.
  R13 aggregators (Eq. 13): "sum" (the paper's choice), "mean" = the sum of
      the k2 messages divided by k2, "max" = element-wise maximum of the k2
      messages e_ij^alpha h_j; the residual h_i is added in every case.
  R14 node mode "adj_raw" uses h^(0)_i = row i of A (Table 1, A_i column).
  R15 the ranking list L of Algorithm 1: per query, gallery rows by
      ascending distance, ties to the lower gallery index.

Retrieval metrics (Section 4.1, Evaluation Metrics), applied to synthetic
identity labels: the true matches of a query are the gallery rows carrying
its label.
  R16 AP is the area under the query's precision-recall curve taken over the
      ranking list R15 with the trapezoid rule: the curve starts at recall 0,
      precision 1, and every list position adds a point (recall, precision)
      of the list's prefix up to it. With P true matches, the i-th (0-based)
      at list position r_i contributes (1/P) * (p_before + p_at) / 2, where
      p_at = (i+1)/(r_i+1) and p_before = i/r_i (1 when r_i = 0); positions
      that are not true matches add no area. mAP is the mean AP over the
      queries with at least one true match.
  R17 Recall@K is 1 for a query whose first true match is among the first K
      positions of its list, else 0; averaged over the queries with at least
      one true match. No junk or same-camera filtering (the synthetic data
      has neither).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Iterable, Optional, Sequence

import numpy as np
import scipy.sparse as sp

__all__ = [
    "unit_rows", "similarity_rows", "knn_of_row", "knn_lists", "adjacency",
    "symmetric_adjacency", "edge_weights", "initial_features", "propagate",
    "row_norms", "distances", "rerank", "ranking", "Graph", "OracleResult",
    "average_precision", "evaluate",
]


# ----------------------------------------------------------------------- Eq. 7
def unit_rows(x: np.ndarray) -> np.ndarray:
    """Rows of ``x`` in float64 divided by their Euclidean norm (reading R1)."""
    x = np.asarray(x, dtype=np.float64)
    return x / np.sqrt(np.einsum("ij,ij->i", x, x))[:, None]


def similarity_rows(xhat: np.ndarray, rows: Sequence[int]) -> np.ndarray:
    """Rows ``rows`` of the cosine-similarity matrix S (Eq. 7); ``xhat`` are
    unit rows. A float64 matrix product serves as the dot products."""
    return xhat[np.asarray(rows)] @ xhat.T


# ----------------------------------------------------------------------- Eq. 8
def knn_of_row(s_row: np.ndarray, i: int, k: int, k_gap: Sequence[int] = ()):
    """N(i, k) of Eq. 8 under readings R2-R4.

    Returns ``(idx, val, gaps)``: ``idx[0] = i`` with ``val[0] = 1``, then the
    k-1 other columns ordered by (S desc, column asc). ``gaps[m]`` for each
    ``m`` in ``k_gap`` is T_(m-1) - T_(m), where T_1 >= T_2 >= ... are the
    similarities of the other columns in that order: the margin by which the
    m-th member of N(i, m) beats the first row left out. It is +inf when
    m == 1 (self alone) or when no row is left out."""
    n = s_row.shape[0]
    s = np.asarray(s_row, dtype=np.float64) + 0.0  # -0.0 -> +0.0
    s = s.copy()
    s[i] = -np.inf
    m_take = min(max(k, max(k_gap, default=1)), n - 1)  # other rows to order
    if m_take > 0:
        t = -np.partition(-s, m_take - 1)[m_take - 1]  # m_take-th largest value
        cand = np.flatnonzero(s >= t)  # every row tied with it is a candidate
        order = cand[np.lexsort((cand, -s[cand]))][:m_take]
    else:
        order = np.zeros(0, dtype=np.int64)
    idx = np.concatenate([[i], order[: k - 1]]).astype(np.int64)
    val = np.concatenate([[1.0], s[order[: k - 1]]])
    gaps = {}
    tv = s[order]
    for m in k_gap:
        if m <= 1 or m > n - 1:
            gaps[m] = math.inf
        else:
            gaps[m] = float(tv[m - 2] - tv[m - 1])
    return idx, val, gaps


@dataclass
class Graph:
    """Neighbour lists of every requested row, in rank order."""

    idx: np.ndarray  # (R, k1) int64
    val: np.ndarray  # (R, k1) float64 similarities, val[:, 0] == 1
    gap1: np.ndarray  # (R,) margin at the k1 boundary
    gap2: np.ndarray  # (R,) margin at the k2 boundary


def knn_lists(x: np.ndarray, k1: int, k2: Optional[int] = None,
              rows: Optional[Iterable[int]] = None, block: int = 1024) -> Graph:
    """N(i, k1) for the given rows (all rows by default), from float64 S rows
    computed ``block`` rows at a time."""
    xhat = unit_rows(x)
    n = xhat.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(list(rows), dtype=np.int64)
    k2 = k1 if k2 is None else k2
    idx = np.empty((len(rows), k1), dtype=np.int64)
    val = np.empty((len(rows), k1), dtype=np.float64)
    g1 = np.empty(len(rows))
    g2 = np.empty(len(rows))
    for b0 in range(0, len(rows), block):
        rb = rows[b0:b0 + block]
        s_blk = similarity_rows(xhat, rb)
        for r, i in enumerate(rb):
            ii, vv, gg = knn_of_row(s_blk[r], int(i), k1, (k1, k2))
            idx[b0 + r], val[b0 + r] = ii, vv
            g1[b0 + r], g2[b0 + r] = gg[k1], gg[k2]
    return Graph(idx, val, g1, g2)


# --------------------------------------------------------------- Eq. 8 - 11
def adjacency(idx: np.ndarray, n: int) -> sp.csr_matrix:
    """A of Eq. 8 from complete neighbour lists (one row per vertex)."""
    rows = np.repeat(np.arange(n), idx.shape[1])
    return sp.csr_matrix((np.ones(idx.size), (rows, idx.ravel())), shape=(n, n))


def symmetric_adjacency(idx: np.ndarray, n: int) -> sp.csr_matrix:
    """A* = (A + A^T) / 2 (Eq. 9); its entries are those of Eq. 10."""
    a = adjacency(idx, n)
    return ((a + a.T) * 0.5).tocsr()


# ------------------------------------------------------------- Eq. 12 and 14
def edge_weights(idx: np.ndarray, val: np.ndarray, k2: int, alpha: int) -> sp.csr_matrix:
    """W_ij = e_ij^alpha for j in N(i, k2) (Eq. 12 and the weight function of
    Eq. 14), with N(i, k2) the first k2 members of N(i, k1) (reading R5)."""
    n = idx.shape[0]
    nb = idx[:, :k2]
    e = val[:, :k2].astype(np.float64)
    w = e ** int(alpha)
    rows = np.repeat(np.arange(n), k2)
    return sp.csr_matrix((w.ravel(), (rows, nb.ravel())), shape=(n, n))


def initial_features(x: np.ndarray, idx: np.ndarray, node: str = "adj"):
    """h^(0): rows of A* (Eq. 11, node mode "adj"), rows of A (Eq. 8, node
    mode "adj_raw") or the raw features x_i (node mode "raw", reading R10).
    Not normalised (reading R6)."""
    n = x.shape[0]
    if node == "adj":
        return symmetric_adjacency(idx, n)
    if node == "adj_raw":
        return adjacency(idx, n)
    if node == "raw":
        return np.asarray(x, dtype=np.float64).copy()
    raise ValueError(node)


def row_norms(h) -> np.ndarray:
    if sp.issparse(h):
        return np.sqrt(np.asarray(h.multiply(h).sum(axis=1)).ravel())
    return np.sqrt(np.einsum("ij,ij->i", h, h))


def _scale_rows(h, f):
    if sp.issparse(h):
        return (sp.diags(f) @ h).tocsr()
    return h * f[:, None]


def _aggregate_max(h, w: sp.csr_matrix):
    """Element-wise maximum over the k2 messages e_ij^alpha h_j of each row
    (Eq. 13 with aggregate = max); plain loops over rows, dense rows."""
    hd = h.toarray() if sp.issparse(h) else np.asarray(h)
    out = np.empty_like(hd)
    for i in range(w.shape[0]):
        lo, hi = w.indptr[i], w.indptr[i + 1]
        msgs = w.data[lo:hi, None] * hd[w.indices[lo:hi]]
        out[i] = msgs.max(axis=0)
    return out


def propagate(h0, w: sp.csr_matrix, layers: int, keep_all: bool = False, aggregator: str = "sum"):
    """Eq. 13/14: h <- h + aggregate(e_ij^alpha h_j, j in N(i,k2)), ``layers``
    times, each followed by the row L2 normalisation. Aggregators per reading
    R13. ``keep_all`` also returns every intermediate h."""
    h = h0
    hist = [h0]
    k2 = np.diff(w.indptr)
    for _ in range(layers):
        if aggregator == "sum":
            u = h + w @ h
        elif aggregator == "mean":
            u = h + sp.diags(1.0 / k2) @ (w @ h)
        elif aggregator == "max":
            hd = h.toarray() if sp.issparse(h) else np.asarray(h)
            u = hd + _aggregate_max(hd, w)
        else:
            raise ValueError(aggregator)
        if sp.issparse(u):
            u = u.tocsr()
        h = _scale_rows(u, 1.0 / row_norms(u))
        hist.append(h)
    return (h, hist) if keep_all else h


def distances(h, n_query: int, q_rows: Optional[Sequence[int]] = None,
              g_rows: Optional[Sequence[int]] = None) -> np.ndarray:
    """D_qg = 1 - cos(h_q, h_g), queries ``q_rows`` (default all q < Q) by
    gallery rows ``g_rows`` (default all Q <= g < N), as a dense array."""
    n = h.shape[0]
    q = np.arange(n_query) if q_rows is None else np.asarray(q_rows)
    g = np.arange(n_query, n) if g_rows is None else np.asarray(g_rows)
    nrm = row_norms(h)
    hq, hg = h[q], h[g]
    dot = hq @ hg.T
    if sp.issparse(dot):
        dot = dot.toarray()
    dot = np.asarray(dot, dtype=np.float64)
    return 1.0 - dot / (nrm[q][:, None] * nrm[g][None, :])


# ------------------------------------------------------------- Algorithm 1
@dataclass
class OracleResult:
    graph: Graph
    h: object  # final features (scipy CSR for "adj", ndarray for "raw")
    dist: np.ndarray  # (len(q_rows), len(g_rows))


def ranking(dist: np.ndarray, r: int) -> np.ndarray:
    """The first ``r`` entries of the ranking list L (Algorithm 1, reading
    R15): per query row of ``dist``, gallery positions by ascending distance,
    ties to the lower position (a stable sort)."""
    return np.argsort(dist, axis=1, kind="stable")[:, :r]


def rerank(x: np.ndarray, n_query: int, k1: int, k2: int, layers: int,
           alpha: int = 2, node: str = "adj", q_rows=None, g_rows=None,
           aggregator: str = "sum") -> OracleResult:
    """Algorithm 1 end to end: similarity, k1 lists, A*, h^(0) and k2 edges,
    ``layers`` propagation steps, query x gallery distances."""
    x = np.asarray(x)
    n = x.shape[0]
    if not (1 <= n_query <= n - 1):
        raise ValueError("need 1 <= n_query <= N-1")
    if not (1 <= k2 <= k1 <= n):
        raise ValueError("need 1 <= k2 <= k1 <= N")
    g = knn_lists(x, k1, k2)
    h0 = initial_features(x, g.idx, node)
    w = edge_weights(g.idx, g.val, k2, alpha)
    h = propagate(h0, w, layers, aggregator=aggregator)
    return OracleResult(g, h, distances(h, n_query, q_rows, g_rows))


def average_precision(dist_row: np.ndarray, match: np.ndarray):
    """AP of one query (reading R16) and the list position of its first true
    match (-1 without matches). ``match`` flags the true matches among the
    gallery positions of ``dist_row``."""
    order = np.argsort(np.asarray(dist_row, dtype=np.float64), kind="stable")
    hits = np.asarray(match, dtype=bool)[order]
    p = int(hits.sum())
    if p == 0:
        return 0.0, -1
    ap = 0.0
    i = 0  # true matches before the current position
    for r in np.flatnonzero(hits):
        p_before = 1.0 if r == 0 else i / r
        p_at = (i + 1) / (r + 1)
        ap += (1.0 / p) * (p_before + p_at) / 2.0
        i += 1
    return ap, int(np.flatnonzero(hits)[0])


def evaluate(dist: np.ndarray, q_labels, g_labels, ks: Iterable[int] = (1, 5, 10)) -> dict:
    """mAP and Recall@K of a query x gallery distance matrix (Section 4.1,
    readings R16-R17). Returns per-query ``ap`` and ``first`` (list position
    of the first true match, -1 without one) and the means over the queries
    that have a true match."""
    dist = np.asarray(dist)
    q_labels = np.asarray(q_labels)
    g_labels = np.asarray(g_labels)
    ks = [int(k) for k in ks]
    ap = np.zeros(dist.shape[0])
    first = np.full(dist.shape[0], -1, dtype=np.int64)
    for q in range(dist.shape[0]):
        ap[q], first[q] = average_precision(dist[q], g_labels == q_labels[q])
    valid = first >= 0
    nv = int(valid.sum())
    out = {"ap": ap, "first": first, "queries": nv,
           "map": float(ap[valid].mean()) if nv else 0.0,
           "recall": {k: (float((first[valid] < k).mean()) if nv else 0.0) for k in ks}}
    return out
