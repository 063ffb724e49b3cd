// Device-side table of a batch of small problems for the persistent grouped
// launches of the serving path. The host fills the table in pinned memory; a
// captured graph copies it to the device and runs one persistent launch per
// stage, whose workgroups walk the work items of every problem in the batch.
#pragma once
#include <stdint.h>

#include "../../include/rerank.h"
#include "kernels.h"

namespace rr {

constexpr int kMaxBatch = 32;

enum GStage : int {
  GS_PREP = 0,   // 4 rows per item
  GS_SIM,        // one upper-triangle 128x128 similarity tile per item
  GS_TOPK,       // 4 rows per item
  GS_RESCORE,    // 4 rows per item
  GS_FILL,       // FILL_ITEM floats of A* per item, plus one item for the counts
  GS_SCATTER,    // 256 (i, r) pairs per item
  GS_SIGMA,      // 256 rows per item (zero-layer norms)
  GS_PROP,       // one row per item (per layer)
  GS_FINAL,      // one 128x128 distance tile per item
  GS_MUTUAL,     // 256 (i, r) pairs per item (sparse first layer)
  GS_SCAN,       // one item per problem
  GS_CSR,        // 256 (i, r) pairs per item
  GS_COUNT
};

struct ProbDesc {
  int32_t n, q, g, d, k1, k2, kc, alpha, in_bf16, lbytes;
  int32_t tiles_sim, tiles_fin_m, tiles_fin_n, node, agg;
  int64_t ldp, ldl, ldN, ldH, fill_items_a;
  const void* x;
  float* dist;
  float* xp;
  void* xl;
  float* rn;
  float* sl;
  float* A;
  float* B;
  int32_t* ci;
  float* cv;
  int32_t* ki;
  float* kv;
  float* sa;
  float* sb;
  int32_t* cnt;
  uint8_t* mflag;  // sparse first layer (A* mode, layers >= 1), else null
  int32_t* off;
  int32_t* inl;
};

struct BatchTable {
  int32_t count;
  int32_t layers;
  int32_t start[GS_COUNT][kMaxBatch + 1];  // prefix sums of items; start[s][count] = total
  ProbDesc p[kMaxBatch];
};

// Batch key: requests batched together share these (they select the
// kernels of the captured graph); everything else is per problem.
struct BatchKey {
  int prec;    // SimPrec
  int r;       // wave list width for top-k / re-score (kc <= 64 r)
  int layers;  // propagation launches
  int node;    // rerank_node
  int agg;     // rerank_aggregator
  bool operator<(const BatchKey& o) const {
    if (prec != o.prec) return prec < o.prec;
    if (r != o.r) return r < o.r;
    if (layers != o.layers) return layers < o.layers;
    if (node != o.node) return node < o.node;
    return agg < o.agg;
  }
};

// Enqueue the persistent grouped pipeline for the table at d_tab (already on
// the device, stream-ordered before these launches).
hipError_t enqueue_grouped(const BatchKey& key, const BatchTable* d_tab, hipStream_t s);

}  // namespace rr
