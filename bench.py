"""Benchmark of the GNN re-ranking hot path on one MI355X.

One step = one whole re-ranking request (similarity product, top-k lists,
FP32 re-score, A*, propagation layers, final query x gallery product) on a
resident synthetic problem. Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload mid|tiny|large]

``value`` is N^2-elements per second of the FP32 path (N^2 / request time);
``ms_per_step`` the FP32 request time. The same line carries the BF16 / FP8
similarity variants on the same arrays, per-stage device times measured with
HIP events on the launch stream, the roofline fraction of the dominant
kernel, and the FP64 oracle timed on the host cores on the same problem.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "re-rank ms/request + N²-elem/s (FP32 vs BF16), p50/p99 at fixed QPS"
PEAK = {"fp32_mfma_tflops": 157.3, "bf16_mfma_tflops": 2500.0, "fp8_mfma_tflops": 5000.0, "hbm_gbs": 8000.0}


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def stage_work(spec, prec: str):
    """Algorithmic work of one request per stage: (unit, amount)."""
    n, q, g, d = spec.n, spec.n_query, spec.n_gallery, spec.dim
    k1, k2, L = spec.k1, spec.k2, spec.layers
    kc = min(k1 + {"f32": 8, "bf16": 16, "fp8": 32}[prec], n, 256)
    return {
        "similarity": ("flop", 1.0 * n * (n + 1) * d),  # unique entries of the symmetric S
        "topk": ("byte", 4.0 * n * n),
        "rescore": ("flop", 2.0 * n * kc * d),
        "adjacency": ("byte", 4.0 * n * n),
        "propagate": ("byte", L * (k2 + 2) * 4.0 * n * n),
        "final": ("flop", 2.0 * q * g * n),
    }


def roofline_entry(stage, unit, amount, ms, prec):
    if ms <= 0:
        return None
    if unit == "flop":
        ach = amount / (ms * 1e-3) / 1e12
        peak = PEAK["fp32_mfma_tflops"]
        if stage == "similarity" and prec == "bf16":
            peak = PEAK["bf16_mfma_tflops"]
        if stage == "similarity" and prec == "fp8":
            peak = PEAK["fp8_mfma_tflops"]
        if stage == "rescore":
            return {"bound": "alu", "achieved": ach, "unit": "TFLOP/s"}
        return {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak}
    ach = amount / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": ach / PEAK["hbm_gbs"]}


# Source files each stage's kernels are compiled from: measured counters stay
# valid while these files are unchanged.
KERNEL_SOURCES = {
    "similarity": ("common.h", "gemm_body.h", "k_gemm.hip"),
    "final": ("common.h", "gemm_body.h", "k_gemm.hip"),
    "topk": ("common.h", "rows_body.h", "k_topk.hip"),
    "rescore": ("common.h", "rows_body.h", "k_graph.hip"),
    "propagate": ("common.h", "rows_body.h", "k_graph.hip"),
    "prep": ("common.h", "rows_body.h", "k_prep.hip"),
    "sparse_final": ("common.h", "kernels.h", "gemm_body.h", "rows_body.h", "k_sparse.hip"),
    "sparse_layers": ("common.h", "kernels.h", "gemm_body.h", "rows_body.h", "k_sparse.hip", "k_graph.hip"),
}


def kernel_src_hash(role: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[role]:
        with open(os.path.join(ROOT, "paper_2012_07620_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, path: str, role: str):
    """HBM bytes per launch of the kernel playing `role`, from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when that summary is
    missing or the kernel sources changed since the counters were taken."""
    f = os.path.join(ROOT, "profiles", f"traffic_{workload}_{path}.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        t = json.load(fh)
    k = t.get("kernels", {}).get(role)
    if k is None or k.get("src_sha256") != kernel_src_hash(role):
        return None
    return {"read_bytes": k["read_bytes"], "write_bytes": k["write_bytes"],
            "bytes": k["read_bytes"] + k["write_bytes"], "source": os.path.relpath(f, ROOT)}


def time_path(binding, torch, ctx, x, spec, prec, steps, warmup, out, final_prec="f32"):
    kw = dict(sim_prec=prec, ctx=ctx, out=out, final_prec=final_prec)
    for _ in range(warmup):
        binding.run(x, spec.n_query, spec.k1, spec.k2, spec.layers, **kw)
    torch.cuda.synchronize()
    ctx.stage_times()  # restart the per-stage averages
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        binding.run(x, spec.n_query, spec.k1, spec.k2, spec.layers, **kw)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return ms, ctx.stage_times()


def serve_stream(binding, torch, synth, count, warmup, qps=None, prec="f32", reqs=None):
    """Submit the requests of a serving stream and wait for all of them.

    qps None: closed loop (everything submitted at once; the throughput is the
    saturation rate). Otherwise requests are submitted at their Poisson arrival
    times. Latency = submit -> completion, as measured by the library."""
    ctx = binding.Context(0)
    xs, outs, specs = reqs
    # warm-up requests: compile graphs, fill the working-set cache
    for i in range(warmup):
        s = specs[i]
        t = binding.submit(ctx, xs[i], outs[i], s.n_query, s.k1, s.k2, s.layers, sim_prec=prec)
        binding.wait(ctx, t)
    meas = range(warmup, warmup + count)
    rng = np.random.default_rng(17)
    gaps = rng.exponential(1.0 / qps, len(meas)) if qps else np.zeros(len(meas))
    arrivals = np.cumsum(gaps) - gaps[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = []
    for k, i in enumerate(meas):
        if qps:
            delay = t0 + arrivals[k] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
        s = specs[i]
        tickets.append(binding.submit(ctx, xs[i], outs[i], s.n_query, s.k1, s.k2, s.layers, sim_prec=prec))
    lat = [binding.wait(ctx, t) for t in tickets]
    t1 = time.perf_counter()
    ctx.close()
    n2 = sum(specs[i].n ** 2 for i in meas)
    return {"requests": len(meas), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(np.mean(lat)), "req_per_s": len(meas) / (t1 - t0), "n2_per_s": n2 / (t1 - t0)}


def serving_bench(binding, torch, synth, count, warmup):
    stream = synth.StreamSpec()
    specs = [s for _, s in synth.request_specs(stream, count + warmup, qps=1.0)]
    dev = torch.device("cuda:0")
    xs = [synth.make_features_device(s, dev) for s in specs]
    outs = [torch.empty((s.n_query, s.n_gallery), dtype=torch.float32, device=dev) for s in specs]
    torch.cuda.synchronize()
    reqs = (xs, outs, specs)
    sat = serve_stream(binding, torch, synth, count, warmup, None, "f32", reqs)
    qps = 0.7 * sat["req_per_s"]
    res = {"stream": "N ~ U[1000, 30000], 15% queries, d in {512, 2048}, bf16, k1=20 k2=6 L=1, Poisson arrivals",
           "saturation_f32_req_per_s": sat["req_per_s"], "qps": qps}
    for prec in ("f32", "bf16"):
        res[prec] = serve_stream(binding, torch, synth, count, warmup, qps, prec, reqs)
    del xs, outs
    return res


def quality_check(binding, torch, synth, spec, dev):
    """Retrieval quality (mAP, Recall@K of Section 4.1, computed on the GPU by
    rerank_evaluate) of plain cosine ranking and of the re-ranked distances,
    on a noisier draw of the benchmark's shape: sigma = 2 (d/128)^(1/4) puts
    the same-identity cosine ~1/(1+sigma^2) near the cross-identity spread
    ~1/sqrt(d), where cosine ranking alone is far from perfect."""
    import dataclasses
    sigma = 2.0 * (spec.dim / 128.0) ** 0.25
    qs = dataclasses.replace(spec, sigma=sigma, seed=spec.seed + 1)
    x, lab = synth.make_features_device(qs, dev, return_labels=True)
    ql, gl = lab[:qs.n_query].contiguous(), lab[qs.n_query:].contiguous()
    out = {"sigma": sigma, "seed": qs.seed}
    for name, layers, node in (("cosine", 0, "raw"), ("reranked", qs.layers, "adj")):
        d = binding.run(x, qs.n_query, qs.k1, qs.k2, layers, node=node)
        ev = binding.evaluate(d, ql, gl, (1, 5, 10))
        out[name] = {"map": ev["map"], "recall_at": {str(k): v for k, v in ev["recall"].items()},
                     "queries": ev["queries"]}
        del d
    torch.cuda.synchronize()
    return out


def cpu_baseline(x32, spec):
    """The FP64 oracle (as it stands) on the same problem, on this host."""
    from oracle import rerank_oracle as orc
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    ref = orc.rerank(x32, spec.n_query, spec.k1, spec.k2, spec.layers)
    t = time.perf_counter() - t0
    return ref, {"value": spec.n * spec.n / t, "unit": "N^2-elem/s", "ms_per_request": t * 1e3,
                 "cores": int(threads), "kind": "oracle",
                 "sample": f"the whole {spec.name} request (float64 NumPy/SciPy oracle, one pass)"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mid", choices=["tiny", "mid", "large"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lowp", action="store_true", help="skip every variant line")
    ap.add_argument("--variants", default="", help="comma-separated variant names to time (default: all)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-quality", action="store_true", help="skip the mAP / Recall@K check")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after timing, copy a 1 GiB float32 tensor once (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the library has no multi-GPU path", file=sys.stderr)
        return 2

    import torch
    from paper_2012_07620_amd import binding, synth

    spec = {"tiny": synth.TINY, "mid": synth.MID, "large": synth.LARGE}[args.workload]
    log(f"workload {spec.name}: generating")
    prob = synth.make_problem(spec)
    dev = torch.device("cuda:0")
    if spec.dtype == "bf16":
        x = torch.from_numpy(prob.x_bf16.view(np.int16)).to(dev).view(torch.bfloat16)
    else:
        x = torch.from_numpy(prob.x32).to(dev)
    ctx = binding.Context(0, stage_timing=True)
    out = torch.empty((spec.n_query, spec.n_gallery), dtype=torch.float32, device=dev)

    log("timing fp32 path")
    ms, stages = time_path(binding, torch, ctx, x, spec, "f32", args.steps, args.warmup, out)
    d_f32 = out.cpu().numpy()
    work = stage_work(spec, "f32")
    roof = {k: roofline_entry(k, *work[k], stages[k], "f32") for k in work}
    dominant = max(work, key=lambda k: stages[k])
    dom = dict(roof[dominant])
    tr = measured_traffic(spec.name, "f32", dominant)
    dom.update({"kernel": dominant, "traffic": tr["bytes"] if tr else None, "traffic_detail": tr,
                "ms_per_launch": stages[dominant]})

    lowp = {}
    if not args.no_lowp:
        ctx_fused = None  # similarity fused with the candidate selection (S never written)
        for name, prec, fprec in (("bf16", "bf16", "f32"), ("fp8", "fp8", "f32"),
                                  ("f32_final_bf16x3", "f32", "bf16x3"), ("bf16_final_bf16x3", "bf16", "bf16x3"),
                                  ("f32_final_sparse", "f32", "sparse"), ("bf16_final_sparse", "bf16", "sparse"),
                                  ("fp8_final_sparse", "fp8", "sparse"), ("bf16_final_bf16", "bf16", "bf16"),
                                  ("fp8_final_bf16", "fp8", "bf16"), ("f32_fused_knn", "f32", "f32"),
                                  ("bf16_fused_knn_final_sparse", "bf16", "sparse"),
                                  ("fp8_fused_knn_final_sparse", "fp8", "sparse")):
            if args.variants and name not in args.variants.split(","):
                continue
            log(f"timing {name} path")
            fused = "_fused_knn" in name
            if fused and ctx_fused is None:
                ctx_fused = binding.Context(0, stage_timing=True, fused_knn=True)
            out_l = torch.empty_like(out)
            ms_l, st_l = time_path(binding, torch, ctx_fused if fused else ctx, x, spec, prec, args.steps, args.warmup,
                                   out_l, fprec)
            wl = stage_work(spec, prec)
            entry = {"similarity": prec, "final": fprec, "fused_knn": fused, "ms_per_request": ms_l,
                     "value": spec.n ** 2 / (ms_l * 1e-3),
                     "speedup_vs_f32": ms / ms_l, "stages_ms": st_l,
                     "similarity_roofline": roofline_entry("similarity", *wl["similarity"], st_l["similarity"], prec),
                     "dist": out_l.cpu().numpy()}
            if fprec == "bf16x3":
                fl = wl["final"][1] / (st_l["final"] * 1e-3) / 1e12
                entry["final_roofline"] = {"bound": "mfma", "achieved": fl, "peak": PEAK["bf16_mfma_tflops"] / 3,
                                           "unit": "TFLOP/s (FP32-equivalent; 3 bf16 products per FP32 product)",
                                           "frac": fl / (PEAK["bf16_mfma_tflops"] / 3)}
            if fprec == "bf16":
                fl = wl["final"][1] / (st_l["final"] * 1e-3) / 1e12
                entry["final_roofline"] = {"bound": "mfma", "achieved": fl, "peak": PEAK["bf16_mfma_tflops"],
                                           "unit": "TFLOP/s", "frac": fl / PEAK["bf16_mfma_tflops"]}
            if fprec == "sparse":
                # the rows reach the product as CSR (a few hundred bytes each), so the floor is writing D once
                nbytes = 4.0 * spec.n_query * spec.n_gallery
                gbs = nbytes / (st_l["final"] * 1e-3) / 1e9
                tr = measured_traffic(spec.name, name, "sparse_final")
                entry["final_roofline"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                                           "frac": gbs / PEAK["hbm_gbs"], "algorithmic_bytes": nbytes,
                                           "traffic": tr["bytes"] if tr else None, "traffic_detail": tr}
            if fused:  # the similarity stage also selects the candidates; the full product is computed
                entry["similarity_roofline"]["note"] = ("fused similarity + top-k: every tile of the N x N product "
                                                        "(twice the symmetric product's flops), S never written")
                kp = binding.make_params(spec.n, spec.n_query, spec.dim, spec.k1, spec.k2, spec.layers, sim_prec=prec)
                entry["knn_workspace_bytes"] = {"unfused": binding.knn_workspace_bytes(kp),
                                                "fused": binding.knn_workspace_bytes(kp, fused_knn=True)}
            lowp[name] = entry
        if ctx_fused is not None:
            ctx_fused.close()

    quality = None
    if not args.no_quality:
        log("retrieval quality (cosine vs re-ranked)")
        quality = quality_check(binding, torch, synth, spec, dev)

    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 2.0, out=b)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del a, b

    serving = None
    if not args.no_serve:
        log("serving stream")
        del out
        serving = serving_bench(binding, torch, synth, args.serve_requests, 20)

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host")
        ref, cpu = cpu_baseline(prob.x32, spec)
        parity = {"f32_max_abs_err_vs_fp64": float(np.abs(d_f32 - ref.dist).max())}
        for prec, r in lowp.items():
            parity[f"{prec}_max_abs_err_vs_fp64"] = float(np.abs(r["dist"] - ref.dist).max())
    for r in lowp.values():
        r.pop("dist", None)

    phase1 = sum(stages[k] for k in ("prep", "similarity", "topk", "rescore", "adjacency"))
    phase2 = stages["propagate"] + stages["final"]
    line = {
        "metric": METRIC,
        "value": spec.n ** 2 / (ms * 1e-3),
        "unit": "N^2-elem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "ms_per_request": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": spec.name, "n": spec.n, "n_query": spec.n_query, "n_gallery": spec.n_gallery,
                   "dim": spec.dim, "k1": spec.k1, "k2": spec.k2, "layers": spec.layers, "alpha": 2,
                   "input_dtype": spec.dtype, "parallelism": "single GPU"},
        "roofline": dom,
        "cpu_baseline": cpu,
        "stages_ms": stages,
        "phase_ms": {"phase1_graph": phase1, "phase2_propagate_rank": phase2},
        "stage_roofline": roof,
        "variants": lowp,
        "parity": parity,
        "serving": serving,
        "quality": quality,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
