// rerank_run_static: rerank_run for callers that cannot allocate device
// memory. The working set of one problem lives in a static device array of
// RERANK_STATIC_BYTES per GPU instead of memory the library allocates; the
// kernels are rerank_run's, given that array as their working set.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ctx.h"

namespace rr {

// Module-scope device memory: every GPU that loads the library holds its own
// copy until the process ends. Host code never uses this name as an address
// (it is a host-side stand-in there): the device address comes from
// hipGetSymbolAddress, once per device, in static_scratch_setup.
static __device__ __align__(256) unsigned char scratch[RERANK_STATIC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` per device
}  // namespace

// Called by rerank_create with `device` current.
hipError_t static_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p || ((uintptr_t)p & 255)) return hipErrorInvalidSymbol;  // the working set needs 256-byte alignment
  g_scratch[device] = p;
  return hipSuccess;
}

static void* static_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch[device] : nullptr;
}

}  // namespace rr

using namespace rr;

extern "C" rerank_status rerank_run_static(rerank_ctx* ctx, const rerank_params* p, const void* d_x,
                                           int32_t in_dtype, float* d_dist, int32_t* d_knn_idx, float* d_knn_val,
                                           void* hip_stream) {
  Plan P;
  rerank_status st = prepare_run(ctx, p, d_x, in_dtype, d_dist, d_knn_idx, d_knn_val, &P);
  if (st != RERANK_OK) return st;
  if (P.total > RERANK_STATIC_BYTES) {
    set_error("working set of " + std::to_string(P.total) + " bytes exceeds the static array of " +
              std::to_string((size_t)RERANK_STATIC_BYTES) + " bytes (rerank_workspace_bytes gives the figure)");
    return RERANK_E_NOMEM;
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  void* ws = static_scratch(ctx->device);
  if (!ws) {
    set_error("the static working set of this device was not set up");
    return RERANK_E_HIP;
  }
  const char* where = "rerank_run_static";
  e = enqueue_run(P, ws, d_x, in_dtype, d_dist, d_knn_idx, d_knn_val, (hipStream_t)hip_stream, &where, nullptr);
  if (e != hipSuccess) return hip_fail(e, where);
  return RERANK_OK;
}
