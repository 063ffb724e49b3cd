// Serving scheduler: admission by working-set bytes, continuous batching of
// requests over the context's streams.
#pragma once
#include "ctx.h"

namespace rr {

void server_stop(Server* s);
// Free the device blocks the serving pool keeps cached for later requests
// (no-op without a server). Called by direct calls that need the memory;
// takes the server's lock, never the context's.
void server_release_cache(rerank_ctx* ctx);

}  // namespace rr
