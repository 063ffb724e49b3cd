// Serving scheduler: admission by working-set bytes, continuous batching of
// requests over the context's streams.
#pragma once
#include "ctx.h"

namespace rr {

void server_stop(Server* s);

}  // namespace rr
