// C entry points declared in include/rerank.h.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>

#include "ctx.h"
#include "eval.h"
#include "pipeline.h"
#include "serve.h"

namespace rr {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

rerank_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what ? what : "HIP call") + ": " + hipGetErrorString(e));
  return (e == hipErrorOutOfMemory) ? RERANK_E_NOMEM : RERANK_E_HIP;
}

// Grow the direct-call working set to `bytes` (device memory, within budget).
// Blocks the serving pool keeps cached are given back first when the budget
// needs them; memory held by running serving requests is not waited for.
static rerank_status ensure_ws(rerank_ctx* c, size_t bytes) {
  if (bytes <= c->ws_bytes) return RERANK_OK;
  if (bytes > c->budget) {
    set_error("working set of " + std::to_string(bytes) + " bytes exceeds the context budget of " +
              std::to_string(c->budget));
    return RERANK_E_NOMEM;
  }
  if (c->ws) {
    hipError_t e = hipEventSynchronize(c->ws_free);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    e = hipFree(c->ws);
    if (e != hipSuccess) return hip_fail(e, "hipFree");
    c->reserved -= c->ws_bytes;
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  if (!try_reserve(c->reserved, c->budget, bytes)) {
    server_release_cache(c);
    if (!try_reserve(c->reserved, c->budget, bytes)) {
      set_error("working set does not fit next to the running serving requests");
      return RERANK_E_NOMEM;
    }
  }
  hipError_t e = hipMalloc(&c->ws, bytes);
  if (e != hipSuccess) {
    c->ws = nullptr;
    c->reserved -= bytes;
    return hip_fail(e, "hipMalloc(working set)");
  }
  c->ws_bytes = bytes;
  return RERANK_OK;
}

static bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

static rerank_status check_common(rerank_ctx* ctx, const rerank_params* p, const void* d_x, int32_t in_dtype) {
  std::string why;
  if (!ctx) {
    set_error("ctx is NULL");
    return RERANK_E_INVALID;
  }
  rerank_status st = validate_params(p, &why);
  if (st != RERANK_OK) {
    set_error(why);
    return st;
  }
  if (in_dtype != RERANK_IN_F32 && in_dtype != RERANK_IN_BF16) {
    set_error("unknown in_dtype");
    return RERANK_E_INVALID;
  }
  if (!d_x || !aligned(d_x, in_dtype == RERANK_IN_F32 ? 4 : 2)) {
    set_error("d_x is NULL or misaligned");
    return RERANK_E_INVALID;
  }
  return RERANK_OK;
}

// Run `body` on the context's working set, serialised after earlier direct calls.
template <typename F>
static rerank_status with_ws(rerank_ctx* ctx, const Plan& P, void* hip_stream, F body) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  rerank_status st = ensure_ws(ctx, P.total);
  if (st != RERANK_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  e = hipStreamWaitEvent(s, ctx->ws_free, 0);
  if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  const char* where = nullptr;
  if (ctx->clock) {
    e = ctx->clock->begin_call();
    if (e != hipSuccess) return hip_fail(e, "stage clock");
  }
  e = body(s, &where);
  // recorded after a failure too: whatever was enqueued still uses the working
  // set, and later calls (any stream) and its reallocation wait for this event
  const hipError_t er = hipEventRecord(ctx->ws_free, s);
  if (e != hipSuccess) return hip_fail(e, where);
  if (er != hipSuccess) return hip_fail(er, "hipEventRecord");
  return RERANK_OK;
}

// Argument checks and plan of rerank_run (shared with rerank_run_static).
rerank_status prepare_run(rerank_ctx* ctx, const rerank_params* p, const void* d_x, int32_t in_dtype, float* d_dist,
                          int32_t* d_knn_idx, float* d_knn_val, Plan* P) {
  rerank_status st = check_common(ctx, p, d_x, in_dtype);
  if (st != RERANK_OK) return st;
  if (!d_dist || !aligned(d_dist, 4)) {
    set_error("d_dist is NULL or misaligned");
    return RERANK_E_INVALID;
  }
  if ((d_knn_idx && !aligned(d_knn_idx, 4)) || (d_knn_val && !aligned(d_knn_val, 4))) {
    set_error("knn output misaligned");
    return RERANK_E_INVALID;
  }
  make_plan(p, false, P, (ctx->flags & RERANK_CTX_DENSE_LAYERS) != 0, (ctx->flags & RERANK_CTX_FUSED_KNN) != 0);
  if (P->fused && P->kc > KNN_LIST_MAX) {
    set_error("RERANK_CTX_FUSED_KNN: k1 + extra_cand above 64 is outside the fused path's limits");
    return RERANK_E_UNSUPPORTED;
  }
  return RERANK_OK;
}

// The kernels of rerank_run on working set `ws` (P.total bytes), then the
// optional copies of the neighbour lists.
hipError_t enqueue_run(const Plan& P, void* ws, const void* d_x, int32_t in_dtype, float* d_dist, int32_t* d_knn_idx,
                       float* d_knn_val, hipStream_t s, const char** where, StageClock* clk) {
  hipError_t e = enqueue_rerank(P, ws, d_x, in_dtype == RERANK_IN_BF16, d_dist, s, where, clk);
  if (e != hipSuccess) return e;
  const int64_t cnt = (int64_t)P.n * P.k1;
  if (d_knn_idx) {
    e = launch_copy_i32((const int32_t*)((char*)ws + P.o_ki), d_knn_idx, cnt, s);
    if (e != hipSuccess) {
      *where = "launch_copy_i32";
      return e;
    }
  }
  if (d_knn_val) {
    e = launch_copy_f32((const float*)((char*)ws + P.o_kv), d_knn_val, cnt, s);
    if (e != hipSuccess) *where = "launch_copy_f32";
  }
  return e;
}

}  // namespace rr

using namespace rr;

extern "C" {

void rerank_default_params(rerank_params* p, int32_t n, int32_t q, int32_t d, int32_t k1, int32_t k2) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n = n;
  p->n_query = q;
  p->dim = d;
  p->k1 = k1;
  p->k2 = k2;
  p->layers = 2;
  p->alpha = 2;
  p->sim_prec = RERANK_SIM_F32;
  p->extra_cand = -1;
  p->node = RERANK_NODE_ADJ_SYM;
  p->final_prec = RERANK_FINAL_F32;
  p->aggregator = RERANK_AGG_SUM;
}

rerank_status rerank_validate(const rerank_params* p) {
  std::string why;
  rerank_status st = validate_params(p, &why);
  if (st != RERANK_OK) set_error(why);
  return st;
}

rerank_status rerank_workspace_bytes(const rerank_params* p, size_t* bytes) {
  std::string why;
  rerank_status st = validate_params(p, &why);
  if (st != RERANK_OK) {
    set_error(why);
    return st;
  }
  if (!bytes) {
    set_error("bytes is NULL");
    return RERANK_E_INVALID;
  }
  Plan P;
  make_plan(p, false, &P);
  *bytes = P.total;
  return RERANK_OK;
}

// The fused similarity + top-k keeps at most 64 candidates per row.
static rerank_status check_fused(const Plan& P) {
  if (P.fused && P.kc > KNN_LIST_MAX) {
    set_error("RERANK_CTX_FUSED_KNN: k1 + extra_cand above 64 is outside the fused path's limits");
    return RERANK_E_UNSUPPORTED;
  }
  return RERANK_OK;
}

rerank_status rerank_knn_workspace_bytes(const rerank_params* p, uint32_t flags, size_t* bytes) {
  std::string why;
  rerank_status st = validate_params(p, &why);
  if (st != RERANK_OK) {
    set_error(why);
    return st;
  }
  if (!bytes || (flags & ~(RERANK_CTX_STAGE_TIMING | RERANK_CTX_DENSE_LAYERS | RERANK_CTX_FUSED_KNN))) {
    set_error("bytes is NULL or unknown flags");
    return RERANK_E_INVALID;
  }
  Plan P;
  make_plan(p, true, &P, false, (flags & RERANK_CTX_FUSED_KNN) != 0);
  if ((st = check_fused(P)) != RERANK_OK) return st;
  *bytes = P.total;
  return RERANK_OK;
}

rerank_status rerank_create(rerank_ctx** out, int hip_device, size_t hbm_budget_bytes, uint32_t flags) {
  if (!out) {
    set_error("out is NULL");
    return RERANK_E_INVALID;
  }
  *out = nullptr;
  if (flags & ~(RERANK_CTX_STAGE_TIMING | RERANK_CTX_DENSE_LAYERS | RERANK_CTX_FUSED_KNN)) {
    set_error("unknown flags");
    return RERANK_E_INVALID;
  }
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (hip_device < 0 || hip_device >= count) {
    set_error("no such HIP device");
    return RERANK_E_INVALID;
  }
  e = hipSetDevice(hip_device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  size_t free_b = 0, total_b = 0;
  e = hipMemGetInfo(&free_b, &total_b);
  if (e != hipSuccess) return hip_fail(e, "hipMemGetInfo");
  rerank_ctx* c = new (std::nothrow) rerank_ctx();
  if (!c) {
    set_error("host allocation failed");
    return RERANK_E_NOMEM;
  }
  e = static_scratch_setup(hip_device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipGetSymbolAddress(static working set)");
  }
  c->device = hip_device;
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)free_b);
  c->flags = flags;
  e = hipEventCreateWithFlags(&c->ws_free, hipEventDisableTiming);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipEventCreate");
  }
  if (flags & RERANK_CTX_STAGE_TIMING) {
    c->clock = new StageClock();
    e = c->clock->init();
    if (e != hipSuccess) {
      c->clock->destroy();
      delete c->clock;
      hipEventDestroy(c->ws_free);
      delete c;
      return hip_fail(e, "hipEventCreate(stage clock)");
    }
  }
  *out = c;
  return RERANK_OK;
}

rerank_status rerank_destroy(rerank_ctx* ctx) {
  if (!ctx) {
    set_error("ctx is NULL");
    return RERANK_E_INVALID;
  }
  rerank_status st = RERANK_OK;
  hipSetDevice(ctx->device);
  if (ctx->server) {
    server_stop(ctx->server);
    ctx->server = nullptr;
  }
  if (ctx->ws) {
    hipError_t e = hipEventSynchronize(ctx->ws_free);
    if (e != hipSuccess) st = hip_fail(e, "hipEventSynchronize");
    hipFree(ctx->ws);
  }
  if (ctx->ws_free) hipEventDestroy(ctx->ws_free);
  if (ctx->clock) {
    ctx->clock->destroy();
    delete ctx->clock;
  }
  delete ctx;
  return st;
}

rerank_status rerank_run(rerank_ctx* ctx, const rerank_params* p, const void* d_x, int32_t in_dtype, float* d_dist,
                         int32_t* d_knn_idx, float* d_knn_val, void* hip_stream) {
  Plan P;
  rerank_status st = prepare_run(ctx, p, d_x, in_dtype, d_dist, d_knn_idx, d_knn_val, &P);
  if (st != RERANK_OK) return st;
  return with_ws(ctx, P, hip_stream, [&](hipStream_t s, const char** where) -> hipError_t {
    return enqueue_run(P, ctx->ws, d_x, in_dtype, d_dist, d_knn_idx, d_knn_val, s, where, ctx->clock);
  });
}

rerank_status rerank_knn(rerank_ctx* ctx, const rerank_params* p, const void* d_x, int32_t in_dtype,
                         int32_t* d_knn_idx, float* d_knn_val, void* hip_stream) {
  rerank_status st = check_common(ctx, p, d_x, in_dtype);
  if (st != RERANK_OK) return st;
  if (!d_knn_idx || !d_knn_val || !aligned(d_knn_idx, 4) || !aligned(d_knn_val, 4)) {
    set_error("knn outputs are NULL or misaligned");
    return RERANK_E_INVALID;
  }
  Plan P;
  make_plan(p, true, &P, false, (ctx->flags & RERANK_CTX_FUSED_KNN) != 0);
  if ((st = check_fused(P)) != RERANK_OK) return st;
  return with_ws(ctx, P, hip_stream, [&](hipStream_t s, const char** where) -> hipError_t {
    hipError_t e = enqueue_knn(P, ctx->ws, d_x, in_dtype == RERANK_IN_BF16, s, where, ctx->clock);
    if (e != hipSuccess) return e;
    const int64_t cnt = (int64_t)P.n * P.k1;
    e = launch_copy_i32((const int32_t*)((char*)ctx->ws + P.o_ki), d_knn_idx, cnt, s);
    if (e != hipSuccess) return e;
    return launch_copy_f32((const float*)((char*)ctx->ws + P.o_kv), d_knn_val, cnt, s);
  });
}

rerank_status rerank_similarity(rerank_ctx* ctx, const rerank_params* p, const void* d_x, int32_t in_dtype,
                                float* d_s, int64_t ld_s, void* hip_stream) {
  rerank_status st = check_common(ctx, p, d_x, in_dtype);
  if (st != RERANK_OK) return st;
  if (!d_s || !aligned(d_s, 4) || ld_s < p->n) {
    set_error("d_s is NULL/misaligned or ld_s < n");
    return RERANK_E_INVALID;
  }
  Plan P;
  make_plan(p, true, &P);
  return with_ws(ctx, P, hip_stream, [&](hipStream_t s, const char** where) -> hipError_t {
    const int in_bf16 = in_dtype == RERANK_IN_BF16;
    const float* xp = feature_rows(P, ctx->ws, d_x, in_bf16);
    float* rn = (float*)((char*)ctx->ws + P.o_rn);
    float* sl = (float*)((char*)ctx->ws + P.o_sl);
    void* xl = P.lbytes ? (char*)ctx->ws + P.o_xl : nullptr;
    float* copy = features_in_place(P, d_x, in_bf16) ? nullptr : (float*)((char*)ctx->ws + P.o_xp);
    hipError_t e = launch_prep(d_x, in_bf16, P.n, P.d, copy, P.ldp, rn, P.prec, xl, P.ldl, sl, s);
    if (e != hipSuccess) {
      *where = "launch_prep";
      return e;
    }
    if (P.prec == SimPrec::F32)
      e = launch_gemm_sim(SimPrec::F32, xp, P.n, P.ldp * 4, P.ldp * 4, rn, d_s, ld_s, false, nullptr, 0, s);
    else
      e = launch_gemm_sim(P.prec, xl, P.n, P.ldl * P.lbytes, P.ldl * P.lbytes, sl, d_s, ld_s, false, nullptr, 0, s);
    if (e != hipSuccess) *where = "launch_gemm_sim";
    return e;
  });
}

rerank_status rerank_rank(rerank_ctx* ctx, const float* d_dist, int32_t q, int32_t g, int32_t r, int32_t* d_rank,
                          void* hip_stream) {
  if (!ctx || !d_dist || !d_rank || ((uintptr_t)d_dist & 3) || ((uintptr_t)d_rank & 3)) {
    set_error("ctx / d_dist / d_rank NULL or misaligned");
    return RERANK_E_INVALID;
  }
  if (q < 1 || g < 1 || r < 1 || r > g) {
    set_error("need q >= 1, g >= 1, 1 <= r <= g");
    return RERANK_E_INVALID;
  }
  if (r > kMaxCand) {
    set_error("r above 256 is outside this library's limits");
    return RERANK_E_UNSUPPORTED;
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  e = launch_rank(d_dist, q, g, r, d_rank, (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "launch_rank");
  return RERANK_OK;
}

rerank_status rerank_evaluate(rerank_ctx* ctx, const float* d_dist, int32_t q, int32_t g, int64_t ld_dist,
                              const int32_t* d_q_labels, const int32_t* d_g_labels, const int32_t* ks, int32_t n_ks,
                              double* d_ap, int32_t* d_first, double* d_summary, void* hip_stream) {
  if (!ctx || !d_dist || !d_q_labels || !d_g_labels || !ks || !d_ap || !d_first || !d_summary ||
      ((uintptr_t)d_dist & 3) || ((uintptr_t)d_q_labels & 3) || ((uintptr_t)d_g_labels & 3) ||
      ((uintptr_t)d_first & 3) || ((uintptr_t)d_ap & 7) || ((uintptr_t)d_summary & 7)) {
    set_error("a pointer is NULL or misaligned");
    return RERANK_E_INVALID;
  }
  if (q < 1 || g < 1 || ld_dist < g || n_ks < 1 || n_ks > kEvalMaxK) {
    set_error("need q >= 1, g >= 1, ld_dist >= g, 1 <= n_ks <= 16");
    return RERANK_E_INVALID;
  }
  for (int j = 0; j < n_ks; j++)
    if (ks[j] < 1) {
      set_error("every cut-off K must be >= 1");
      return RERANK_E_INVALID;
    }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  e = launch_evaluate(d_dist, q, g, ld_dist, d_q_labels, d_g_labels, ks, n_ks, d_ap, d_first, d_summary,
                      (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "launch_evaluate");
  return RERANK_OK;
}

rerank_status rerank_stage_times(rerank_ctx* ctx, double* ms_out) {
  if (!ctx || !ms_out || !ctx->clock) {
    set_error("stage timing is off for this context");
    return RERANK_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(ctx->mu);
  hipError_t e = ctx->clock->totals(ms_out);
  if (e != hipSuccess) return hip_fail(e, "stage clock");
  return RERANK_OK;
}

const char* rerank_stage_name(int32_t stage) {
  static const char* names[RERANK_STAGE_COUNT] = {"prep",      "similarity", "topk", "rescore",
                                                  "adjacency", "propagate",  "final"};
  return (stage >= 0 && stage < RERANK_STAGE_COUNT) ? names[stage] : nullptr;
}

const char* rerank_status_str(rerank_status s) {
  switch (s) {
    case RERANK_OK: return "ok";
    case RERANK_E_INVALID: return "invalid argument";
    case RERANK_E_NOMEM: return "out of memory budget";
    case RERANK_E_HIP: return "HIP error";
    case RERANK_E_BUSY: return "busy";
    case RERANK_E_TIMEOUT: return "timeout";
    case RERANK_E_CANCELLED: return "cancelled";
    case RERANK_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* rerank_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
