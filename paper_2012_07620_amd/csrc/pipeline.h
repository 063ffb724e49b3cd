// Enqueue the kernels of one problem on a stream, given its working set.
#pragma once
#include "plan.h"

namespace rr {

// Optional per-stage device timing. Each direct call takes the next of a pool
// of event sets (start/stop per stage, recorded on the call's stream); a set
// is read back only when it is reused or when the totals are requested, so
// timing adds no host synchronisation to back-to-back calls.
struct StageClock {
  static constexpr int kSets = 64;
  struct Set {
    hipEvent_t ev[RERANK_STAGE_COUNT][2] = {};
    bool ran[RERANK_STAGE_COUNT] = {};
    bool pending = false;
  };
  Set sets[kSets];
  int next = 0;
  Set* cur = nullptr;
  double sum_ms[RERANK_STAGE_COUNT] = {};
  int runs[RERANK_STAGE_COUNT] = {};
  hipError_t init();
  void destroy();
  hipError_t harvest(Set& st);      // wait for a pending set and add its times
  hipError_t begin_call();          // select (and if needed harvest) the next set
  hipError_t mark(int stage, int edge, hipStream_t s) {
    if (edge == 0) cur->ran[stage] = true;
    cur->pending = true;
    return hipEventRecord(cur->ev[stage][edge], s);
  }
  hipError_t totals(double* mean_ms);  // mean per call since the last totals(), then reset
};

// The FP32 feature rows that the products, the re-score and raw-feature
// layers read: the caller's rows in place when they already have the padded
// layout (FP32 input, d a multiple of 64, 256-byte aligned), so prep only
// reads them; else the zero-padded copy prep writes into the working set.
inline bool features_in_place(const Plan& P, const void* x, int in_bf16) {
  return !in_bf16 && P.ldp == P.d && ((uintptr_t)x & 255u) == 0;
}
inline const float* feature_rows(const Plan& P, void* ws, const void* x, int in_bf16) {
  return features_in_place(P, x, in_bf16) ? (const float*)x : (const float*)((char*)ws + P.o_xp);
}

// Phase 1: features -> neighbour lists (in the working set at P.o_ki/P.o_kv).
hipError_t enqueue_knn(const Plan& P, void* ws, const void* x, int in_bf16, hipStream_t s, const char** where,
                       StageClock* clk = nullptr);
// Full method: writes the Q x G distances to `dist` (row stride G).
hipError_t enqueue_rerank(const Plan& P, void* ws, const void* x, int in_bf16, float* dist, hipStream_t s,
                          const char** where, StageClock* clk = nullptr);

}  // namespace rr
