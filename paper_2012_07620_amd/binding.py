"""ctypes binding of ``librerank.so`` (argument marshalling only).

Every step of the method runs in the library's HIP kernels; this module
passes device pointers of PyTorch tensors and the current HIP stream. There
is no fallback: if the library is missing or no GPU is visible, calls raise.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librerank.so")

OK, E_INVALID, E_NOMEM, E_HIP, E_BUSY, E_TIMEOUT, E_CANCELLED, E_UNSUPPORTED = range(8)
IN_F32, IN_BF16 = 0, 1
SIM = {"f32": 0, "bf16": 1, "fp8": 2}
NODE = {"adj": 0, "raw": 1, "adj_raw": 2}
AGG = {"sum": 0, "mean": 1, "max": 2}
FINAL = {"f32": 0, "bf16x3": 1, "sparse": 2, "bf16": 3}

EXPORTS = (
    "rerank_default_params", "rerank_validate", "rerank_workspace_bytes", "rerank_knn_workspace_bytes",
    "rerank_create", "rerank_destroy",
    "rerank_run", "rerank_run_static", "rerank_knn", "rerank_similarity", "rerank_submit", "rerank_poll", "rerank_wait",
    "rerank_cancel", "rerank_status_str", "rerank_last_error", "rerank_stage_times", "rerank_stage_name",
    "rerank_rank", "rerank_evaluate",
)
CTX_STAGE_TIMING = 1
CTX_DENSE_LAYERS = 2
CTX_FUSED_KNN = 4
STAGES = ("prep", "similarity", "topk", "rescore", "adjacency", "propagate", "final")


class Params(ctypes.Structure):
    """Mirror of ``rerank_params``."""

    _fields_ = [(n, ctypes.c_int32) for n in (
        "n", "n_query", "dim", "k1", "k2", "layers", "alpha", "sim_prec", "extra_cand", "node", "final_prec",
        "aggregator")]


class RerankError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rerank status {status}: {msg}")
        self.status = status


_lib = None
_lock = threading.Lock()


def library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library once and declare the C signatures."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2012_07620_amd.build_lib`")
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER(Params)
        vp, i32, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_size_t
        sig = {
            "rerank_default_params": (None, [P, i32, i32, i32, i32, i32]),
            "rerank_validate": (ctypes.c_int, [P]),
            "rerank_workspace_bytes": (ctypes.c_int, [P, ctypes.POINTER(sz)]),
            "rerank_knn_workspace_bytes": (ctypes.c_int, [P, ctypes.c_uint32, ctypes.POINTER(sz)]),
            "rerank_create": (ctypes.c_int, [ctypes.POINTER(vp), ctypes.c_int, sz, ctypes.c_uint32]),
            "rerank_destroy": (ctypes.c_int, [vp]),
            "rerank_run": (ctypes.c_int, [vp, P, vp, i32, vp, vp, vp, vp]),
            "rerank_run_static": (ctypes.c_int, [vp, P, vp, i32, vp, vp, vp, vp]),
            "rerank_knn": (ctypes.c_int, [vp, P, vp, i32, vp, vp, vp]),
            "rerank_similarity": (ctypes.c_int, [vp, P, vp, i32, vp, ctypes.c_int64, vp]),
            "rerank_submit": (ctypes.c_int, [vp, P, vp, i32, vp, vp, ctypes.POINTER(u64)]),
            "rerank_poll": (ctypes.c_int, [vp, u64, ctypes.POINTER(ctypes.c_int)]),
            "rerank_wait": (ctypes.c_int, [vp, u64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
            "rerank_cancel": (ctypes.c_int, [vp, u64]),
            "rerank_status_str": (ctypes.c_char_p, [ctypes.c_int]),
            "rerank_last_error": (ctypes.c_char_p, []),
            "rerank_stage_times": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double)]),
            "rerank_stage_name": (ctypes.c_char_p, [i32]),
            "rerank_rank": (ctypes.c_int, [vp, vp, i32, i32, i32, vp, vp]),
            "rerank_evaluate": (ctypes.c_int, [vp, vp, i32, i32, ctypes.c_int64, vp, vp,
                                               ctypes.POINTER(i32), i32, vp, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def _check(status: int) -> None:
    if status != OK:
        lib = library()
        raise RerankError(status, f"{lib.rerank_status_str(status).decode()}: {lib.rerank_last_error().decode()}")


def make_params(n: int, n_query: int, dim: int, k1: int, k2: int, layers: int = 2, alpha: int = 2,
                sim_prec: str = "f32", extra_cand: int = -1, node: str = "adj", final_prec: str = "f32",
                aggregator: str = "sum") -> Params:
    return Params(n, n_query, dim, k1, k2, layers, alpha, SIM[sim_prec], extra_cand, NODE[node], FINAL[final_prec],
                  AGG[aggregator])


def validate(p: Params) -> int:
    return library().rerank_validate(ctypes.byref(p))


def workspace_bytes(p: Params) -> int:
    out = ctypes.c_size_t(0)
    _check(library().rerank_workspace_bytes(ctypes.byref(p), ctypes.byref(out)))
    return out.value


def knn_workspace_bytes(p: Params, fused_knn: bool = False) -> int:
    """Device bytes rerank_knn needs for ``p`` (with the fused similarity + selection: no N x N buffer)."""
    out = ctypes.c_size_t(0)
    _check(library().rerank_knn_workspace_bytes(ctypes.byref(p), CTX_FUSED_KNN if fused_knn else 0,
                                                ctypes.byref(out)))
    return out.value


class Context:
    """A library context on one HIP device (owns the working memory)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, stage_timing: bool = False,
                 dense_layers: bool = False, fused_knn: bool = False):
        lib = library()
        h = ctypes.c_void_p()
        flags = ((CTX_STAGE_TIMING if stage_timing else 0) | (CTX_DENSE_LAYERS if dense_layers else 0)
                 | (CTX_FUSED_KNN if fused_knn else 0))
        _check(lib.rerank_create(ctypes.byref(h), device, budget_bytes, flags))
        self.handle = h
        self.device = device

    def stage_times(self) -> dict:
        """Mean device ms per stage over the direct calls since the last query
        (needs stage_timing)."""
        arr = (ctypes.c_double * len(STAGES))()
        _check(library().rerank_stage_times(self.handle, arr))
        return dict(zip(STAGES, list(arr)))

    def close(self) -> None:
        if self.handle:
            _check(library().rerank_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def _stream_ptr(torch, device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _x_args(x):
    import torch
    if not x.is_cuda or x.dim() != 2 or not x.is_contiguous():
        raise ValueError("x must be a contiguous 2-D device tensor")
    if x.dtype == torch.float32:
        return IN_F32
    if x.dtype == torch.bfloat16:
        return IN_BF16
    raise ValueError("x must be float32 or bfloat16")


def run(x, n_query: int, k1: int, k2: int, layers: int = 2, alpha: int = 2, sim_prec: str = "f32",
        extra_cand: int = -1, node: str = "adj", final_prec: str = "f32", return_knn: bool = False,
        ctx: Optional[Context] = None, out=None, aggregator: str = "sum"):
    """Full method on device tensor ``x`` (N x d, queries first). Returns the
    Q x G distance tensor (and the N x k1 lists and similarities)."""
    import torch
    dt = _x_args(x)
    n, d = x.shape
    p = make_params(n, n_query, d, k1, k2, layers, alpha, sim_prec, extra_cand, node, final_prec, aggregator)
    ctx = ctx or default_context(x.device.index or 0)
    dist = out if out is not None else torch.empty((n_query, n - n_query), dtype=torch.float32, device=x.device)
    ki = kv = None
    if return_knn:
        ki = torch.empty((n, k1), dtype=torch.int32, device=x.device)
        kv = torch.empty((n, k1), dtype=torch.float32, device=x.device)
    _check(library().rerank_run(ctx.handle, ctypes.byref(p), x.data_ptr(), dt, dist.data_ptr(),
                                ki.data_ptr() if ki is not None else None, kv.data_ptr() if kv is not None else None,
                                _stream_ptr(torch, x.device)))
    return (dist, ki, kv) if return_knn else dist


STATIC_BYTES = 256 << 20  # RERANK_STATIC_BYTES


def run_static(x, n_query: int, k1: int, k2: int, layers: int = 2, alpha: int = 2, sim_prec: str = "f32",
               extra_cand: int = -1, node: str = "adj", final_prec: str = "f32", ctx: Optional[Context] = None,
               out=None, knn_out=None, aggregator: str = "sum"):
    """rerank_run_static: the full method with the working set in the
    library's static device array (no device allocation by the library).
    ``out`` (Q x G float32) and ``knn_out`` (a pair of N x k1 int32 / float32
    tensors, optional) are caller-owned; returns ``out``."""
    import torch
    dt = _x_args(x)
    n, d = x.shape
    p = make_params(n, n_query, d, k1, k2, layers, alpha, sim_prec, extra_cand, node, final_prec, aggregator)
    ctx = ctx or default_context(x.device.index or 0)
    if out is None:
        raise ValueError("run_static needs a caller-owned `out` tensor")
    ki, kv = knn_out if knn_out is not None else (None, None)
    _check(library().rerank_run_static(ctx.handle, ctypes.byref(p), x.data_ptr(), dt, out.data_ptr(),
                                       ki.data_ptr() if ki is not None else None,
                                       kv.data_ptr() if kv is not None else None, _stream_ptr(torch, x.device)))
    return out


def knn(x, k1: int, sim_prec: str = "f32", extra_cand: int = -1, ctx: Optional[Context] = None):
    """Phase 1 only: N x k1 neighbour lists (int32) and similarities."""
    import torch
    dt = _x_args(x)
    n, d = x.shape
    p = make_params(n, 1, d, k1, 1, 0, 2, sim_prec, extra_cand)
    ctx = ctx or default_context(x.device.index or 0)
    ki = torch.empty((n, k1), dtype=torch.int32, device=x.device)
    kv = torch.empty((n, k1), dtype=torch.float32, device=x.device)
    _check(library().rerank_knn(ctx.handle, ctypes.byref(p), x.data_ptr(), dt, ki.data_ptr(), kv.data_ptr(),
                                _stream_ptr(torch, x.device)))
    return ki, kv


def similarity(x, sim_prec: str = "f32", ctx: Optional[Context] = None, out=None):
    """Eq. 7 only: the N x N cosine matrix in the chosen arithmetic."""
    import torch
    dt = _x_args(x)
    n, d = x.shape
    p = make_params(n, 1, d, 1, 1, 0, 2, sim_prec)
    ctx = ctx or default_context(x.device.index or 0)
    s = out if out is not None else torch.empty((n, n), dtype=torch.float32, device=x.device)
    _check(library().rerank_similarity(ctx.handle, ctypes.byref(p), x.data_ptr(), dt, s.data_ptr(), s.stride(0),
                                       _stream_ptr(torch, x.device)))
    return s


def rank(dist, r: int, ctx: Optional[Context] = None):
    """First r entries of the ranking list per query row of ``dist``
    (ascending distance, ties to the lower gallery position), int32."""
    import torch
    if not dist.is_cuda or dist.dim() != 2 or not dist.is_contiguous() or dist.dtype != torch.float32:
        raise ValueError("dist must be a contiguous 2-D float32 device tensor")
    q, g = dist.shape
    ctx = ctx or default_context(dist.device.index or 0)
    out = torch.empty((q, r), dtype=torch.int32, device=dist.device)
    _check(library().rerank_rank(ctx.handle, dist.data_ptr(), q, g, r, out.data_ptr(),
                                 _stream_ptr(torch, dist.device)))
    return out


def evaluate(dist, q_labels, g_labels, ks=(1, 5, 10), ctx: Optional[Context] = None) -> dict:
    """mAP and Recall@K of the distance rows ``dist`` (Q x G float32 device
    tensor, row stride >= G) under int32 device label vectors. Returns
    ``{"map", "recall": {K: value}, "queries", "ap", "first"}`` with the
    per-query tensors on the device; waits for the result."""
    import torch
    if not dist.is_cuda or dist.dim() != 2 or dist.dtype != torch.float32 or dist.stride(1) != 1:
        raise ValueError("dist must be a 2-D float32 device tensor with unit column stride")
    q, g = dist.shape
    for t, n in ((q_labels, q), (g_labels, g)):
        if not t.is_cuda or t.dtype != torch.int32 or t.dim() != 1 or t.numel() != n or not t.is_contiguous():
            raise ValueError("labels must be contiguous int32 device vectors of Q and G entries")
    ks = [int(k) for k in ks]
    ctx = ctx or default_context(dist.device.index or 0)
    ap = torch.empty(q, dtype=torch.float64, device=dist.device)
    first = torch.empty(q, dtype=torch.int32, device=dist.device)
    summary = torch.empty(len(ks) + 2, dtype=torch.float64, device=dist.device)
    karr = (ctypes.c_int32 * len(ks))(*ks)
    _check(library().rerank_evaluate(ctx.handle, dist.data_ptr(), q, g, dist.stride(0), q_labels.data_ptr(),
                                     g_labels.data_ptr(), karr, len(ks), ap.data_ptr(), first.data_ptr(),
                                     summary.data_ptr(), _stream_ptr(torch, dist.device)))
    s = summary.cpu().tolist()
    return {"map": s[0], "recall": dict(zip(ks, s[1:1 + len(ks)])), "queries": int(s[-1]), "ap": ap, "first": first}


def submit(ctx: Context, x, out, n_query: int, k1: int, k2: int, layers: int = 1, alpha: int = 2,
           sim_prec: str = "f32", extra_cand: int = -1, node: str = "adj", final_prec: str = "f32",
           aggregator: str = "sum") -> int:
    """Asynchronous request; ``out`` (Q x G float32) must stay alive until
    done. The request starts after the work already enqueued on the current
    stream of ``x``'s device (the stream that produced ``x``)."""
    import torch
    dt = _x_args(x)
    n, d = x.shape
    p = make_params(n, n_query, d, k1, k2, layers, alpha, sim_prec, extra_cand, node, final_prec, aggregator)
    t = ctypes.c_uint64(0)
    _check(library().rerank_submit(ctx.handle, ctypes.byref(p), x.data_ptr(), dt, out.data_ptr(),
                                   _stream_ptr(torch, x.device), ctypes.byref(t)))
    return t.value


def poll(ctx: Context, ticket: int) -> bool:
    done = ctypes.c_int(0)
    _check(library().rerank_poll(ctx.handle, ticket, ctypes.byref(done)))
    return bool(done.value)


def wait(ctx: Context, ticket: int, timeout_us: int = -1) -> float:
    """Block until done; returns the request latency in ms. Raises on failure."""
    lat = ctypes.c_double(0.0)
    _check(library().rerank_wait(ctx.handle, ticket, timeout_us, ctypes.byref(lat)))
    return lat.value


def cancel(ctx: Context, ticket: int) -> None:
    _check(library().rerank_cancel(ctx.handle, ticket))
