// The context object behind the opaque rerank_ctx handle.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <string>

#include "pipeline.h"

namespace rr {
class Server;
void set_error(const std::string& msg);
rerank_status hip_fail(hipError_t e, const char* what);

// Take `bytes` out of the budget if they fit next to what is already held
// (atomic: direct calls and the serving scheduler reserve from two threads).
inline bool try_reserve(std::atomic<size_t>& reserved, size_t budget, size_t bytes) {
  size_t cur = reserved.load();
  do {
    if (bytes > budget || cur > budget - bytes) return false;
  } while (!reserved.compare_exchange_weak(cur, cur + bytes));
  return true;
}
}  // namespace rr

struct rerank_ctx;

namespace rr {
// Shared by rerank_run and rerank_run_static (rerank_api.cpp).
rerank_status prepare_run(rerank_ctx* ctx, const rerank_params* p, const void* d_x, int32_t in_dtype, float* d_dist,
                          int32_t* d_knn_idx, float* d_knn_val, Plan* P);
hipError_t enqueue_run(const Plan& P, void* ws, const void* d_x, int32_t in_dtype, float* d_dist, int32_t* d_knn_idx,
                       float* d_knn_val, hipStream_t s, const char** where, StageClock* clk);
// Device address of the static working set of rerank_run_static on `device`
// (the current device), looked up once per device (static_ws.cpp).
hipError_t static_scratch_setup(int device);
}  // namespace rr

struct rerank_ctx {
  int device = 0;
  size_t budget = 0;
  std::mutex mu;             // guards the direct-call working set below
  void* ws = nullptr;        // working set of rerank_run / rerank_knn / rerank_similarity
  size_t ws_bytes = 0;
  hipEvent_t ws_free = nullptr;  // recorded after the last direct call's kernels
  std::atomic<size_t> reserved{0};  // bytes held by the direct working set + the serving pool
  uint32_t flags = 0;
  rr::StageClock* clock = nullptr;  // set with RERANK_CTX_STAGE_TIMING
  rr::Server* server = nullptr;     // serving scheduler, started on first submit
  std::mutex server_mu;
};
