// Serving entry points (placeholder until the scheduler lands).
#include "serve.h"

namespace rr {
void server_stop(Server*) {}
}  // namespace rr

using namespace rr;

extern "C" {
rerank_status rerank_submit(rerank_ctx*, const rerank_params*, const void*, int32_t, float*, uint64_t*) {
  set_error("serving is not built yet");
  return RERANK_E_UNSUPPORTED;
}
rerank_status rerank_poll(rerank_ctx*, uint64_t, int*) { return RERANK_E_UNSUPPORTED; }
rerank_status rerank_wait(rerank_ctx*, uint64_t, int64_t, double*) { return RERANK_E_UNSUPPORTED; }
rerank_status rerank_cancel(rerank_ctx*, uint64_t) { return RERANK_E_UNSUPPORTED; }
}
