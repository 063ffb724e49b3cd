"""Seeded synthetic re-ranking problems (clustered retrieval features).

This module only makes inputs. It holds none of the re-ranking arithmetic:
no similarity, no neighbour selection, no propagation. Both the FP64 oracle
tests and the GPU path receive the arrays it returns.

The features stand in for the backbone descriptors of the retrieval
datasets the paper evaluates on (Section 4.1: person re-id, vehicle re-id,
landmarks, drone geo-localisation). Those datasets and trained backbones are
not available, so every problem here is drawn from a seeded mixture:

* identity centres ``c ~ N(0, I_d)``, then scaled to unit length (uniform
  on the sphere);
* a sample of identity ``y`` is ``c_y + eps`` with ``eps ~ N(0, sigma^2/d I_d)``
  (``sigma`` is the expected norm of the noise relative to the unit
  centre), then scaled to unit length and cast to the storage dtype
  (``bf16`` uses round-to-nearest-even);
* query and gallery identities are assigned round-robin, distractors (a
  fraction of the gallery) each get a fresh centre, then queries and
  gallery are shuffled separately so row order carries no identity
  information. Queries are rows ``0..Q-1``, gallery rows ``Q..N-1``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass(frozen=True)
class ProblemSpec:
    """Shape and generation recipe of one re-ranking problem."""

    name: str
    n_query: int
    n_gallery: int
    dim: int
    n_ids: int
    sigma: float
    distractor_frac: float = 0.0
    k1: int = 20
    k2: int = 6
    layers: int = 1
    dtype: str = "f32"  # storage dtype of the features: "f32" or "bf16"
    seed: int = 0

    @property
    def n(self) -> int:
        return self.n_query + self.n_gallery


# The workloads that the benchmark and the parity tests run. Shapes follow
# the paper's datasets (Market-1501: 3,368 queries and 19,732 test images,
# k1=26 and k2=7; University-1652: 512-d features) scaled as stated.
TINY = ProblemSpec("tiny_n1000_d128", 100, 900, 128, 50, 0.3, 0.0, 10, 3, 1, "f32", 1001)
MID = ProblemSpec("mid_n19281_d2048", 3368, 15913, 2048, 751, 0.5, 0.05, 26, 7, 1, "f32", 1002)
LARGE = ProblemSpec("large_n50000_d512", 10000, 40000, 512, 5000, 0.5, 0.0, 20, 6, 2, "bf16", 1004)

SPECS = {s.name: s for s in (TINY, MID, LARGE)}


def bf16_bits_from_f32(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); return the
    16-bit patterns as uint16. Inputs must be finite."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    rounding = ((b >> np.uint32(16)) & np.uint32(1)) + np.uint32(0x7FFF)
    return ((b + rounding) >> np.uint32(16)).astype(np.uint16)


def f32_from_bf16_bits(b: np.ndarray) -> np.ndarray:
    """Exact float32 values of bfloat16 bit patterns."""
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def _unit_rows(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@dataclass
class Problem:
    spec: ProblemSpec
    x32: np.ndarray  # (N, d) float32: the exact values the method sees
    x_bf16: Optional[np.ndarray]  # (N, d) uint16 bit patterns when dtype == "bf16"
    labels: np.ndarray  # (N,) int64 identity label, distractors get unique ids >= n_ids
    extra: dict = field(default_factory=dict)


def make_problem(spec: ProblemSpec, seed: Optional[int] = None) -> Problem:
    """Draw one problem following the recipe in the module docstring."""
    rng = np.random.Generator(np.random.PCG64(spec.seed if seed is None else seed))
    d = spec.dim
    n_dis = int(round(spec.distractor_frac * spec.n_gallery))
    n_gal_ids = spec.n_gallery - n_dis
    centres = _unit_rows(rng.standard_normal((spec.n_ids, d)))
    q_lab = np.arange(spec.n_query) % spec.n_ids
    g_lab = np.arange(n_gal_ids) % spec.n_ids
    rng.shuffle(q_lab)
    rng.shuffle(g_lab)
    dis_centres = _unit_rows(rng.standard_normal((n_dis, d))) if n_dis else np.zeros((0, d))
    dis_lab = spec.n_ids + np.arange(n_dis)
    base = np.concatenate([centres[q_lab], centres[g_lab], dis_centres], axis=0)
    labels = np.concatenate([q_lab, g_lab, dis_lab]).astype(np.int64)
    # shuffle the gallery block so distractors are not at the end
    perm = spec.n_query + rng.permutation(spec.n_gallery)
    order = np.concatenate([np.arange(spec.n_query), perm])
    base, labels = base[order], labels[order]
    noise = rng.standard_normal(base.shape) * (spec.sigma / np.sqrt(d))
    x = _unit_rows(base + noise).astype(np.float32)
    xb = None
    if spec.dtype == "bf16":
        xb = bf16_bits_from_f32(x)
        x = f32_from_bf16_bits(xb)
    elif spec.dtype != "f32":
        raise ValueError(f"unknown dtype {spec.dtype}")
    return Problem(spec, np.ascontiguousarray(x), xb, labels)


def random_features(n: int, d: int, seed: int, *, n_ids: int = 0, sigma: float = 0.5,
                    dup_frac: float = 0.0) -> np.ndarray:
    """Small float32 feature sets for edge-case tests.

    ``n_ids > 0`` draws clustered features as above, otherwise i.i.d.
    Gaussian rows. ``dup_frac`` replaces that fraction of rows by exact copies
    of other rows (exact similarity ties)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if n_ids > 0:
        centres = _unit_rows(rng.standard_normal((n_ids, d)))
        lab = rng.integers(0, n_ids, n)
        x = centres[lab] + rng.standard_normal((n, d)) * (sigma / np.sqrt(d))
    else:
        x = rng.standard_normal((n, d))
    x = x.astype(np.float32)
    n_dup = int(dup_frac * n)
    if n_dup:
        dst = rng.choice(n, n_dup, replace=False)
        src = rng.integers(0, n, n_dup)
        x[dst] = x[src]
    return np.ascontiguousarray(x)


# ---------------------------------------------------------------- serving stream
@dataclass(frozen=True)
class StreamSpec:
    """Open-loop request stream: Poisson arrivals, N uniform in [n_min, n_max],
    15% queries, d drawn from ``dims``; clustered bf16 features with
    C = max(2, N // 20) identities (the paper's k1 = n / C rule with k1 = 20)."""

    n_min: int = 1000
    n_max: int = 30000
    query_frac: float = 0.15
    dims: tuple = (512, 2048)
    sigma: float = 0.5
    distractor_frac: float = 0.05
    k1: int = 20
    k2: int = 6
    layers: int = 1
    seed: int = 1005


def request_specs(stream: StreamSpec, count: int, qps: float):
    """Return ``count`` (arrival_time_s, ProblemSpec) pairs."""
    rng = np.random.Generator(np.random.PCG64(stream.seed))
    t = np.cumsum(rng.exponential(1.0 / qps, count))
    out = []
    for r in range(count):
        n = int(rng.integers(stream.n_min, stream.n_max + 1))
        q = max(1, int(round(stream.query_frac * n)))
        d = int(stream.dims[int(rng.integers(0, len(stream.dims)))])
        spec = ProblemSpec(f"req{r}", q, n - q, d, max(2, n // 20), stream.sigma,
                           stream.distractor_frac, stream.k1, stream.k2, stream.layers,
                           "bf16", int(stream.seed * 100003 + r))
        out.append((float(t[r]), spec))
    return out


def make_features_device(spec: ProblemSpec, device, seed: Optional[int] = None, return_labels: bool = False):
    """Same recipe as :func:`make_problem`, drawn with torch's generator on
    ``device`` (fast; used for the many requests of a serving stream). Returns
    the features as a contiguous (N, d) tensor in the spec's storage dtype,
    and with ``return_labels`` also the (N,) int32 identity labels
    (distractors get unique labels >= n_ids)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(spec.seed if seed is None else seed))
    d = spec.dim
    n_dis = int(round(spec.distractor_frac * spec.n_gallery))
    n_gal_ids = spec.n_gallery - n_dis

    def unit(v):
        return v / v.norm(dim=1, keepdim=True)

    centres = unit(torch.randn(spec.n_ids, d, generator=g, device=device))
    q_lab = torch.arange(spec.n_query, device=device) % spec.n_ids
    g_lab = torch.arange(n_gal_ids, device=device) % spec.n_ids
    q_lab = q_lab[torch.randperm(spec.n_query, generator=g, device=device)]
    g_lab = g_lab[torch.randperm(n_gal_ids, generator=g, device=device)]
    dis = unit(torch.randn(n_dis, d, generator=g, device=device)) if n_dis else torch.zeros(0, d, device=device)
    perm = torch.randperm(spec.n_gallery, generator=g, device=device)
    gal = torch.cat([centres[g_lab], dis])[perm]
    base = torch.cat([centres[q_lab], gal])
    x = unit(base + torch.randn(base.shape, generator=g, device=device) * (spec.sigma / d ** 0.5))
    x = (x.to(torch.bfloat16) if spec.dtype == "bf16" else x.float()).contiguous()
    if not return_labels:
        return x
    dis_lab = spec.n_ids + torch.arange(n_dis, device=device)
    labels = torch.cat([q_lab, torch.cat([g_lab, dis_lab])[perm]]).to(torch.int32).contiguous()
    return x, labels
