// Launch of the retrieval-metric kernels (Section 4.1, Evaluation Metrics).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rr {

constexpr int kEvalMaxK = 16;  // Recall@K cut-offs per call

// Per query (q rows of dist, row stride ld floats, g gallery columns): ap[i]
// and first[i] (list position of the first true match, -1 without one);
// then summary[0] = mAP, summary[1 + j] = Recall@ks[j] (j < nk) and
// summary[nk + 1] = number of queries with a true match. ks is a host array.
hipError_t launch_evaluate(const float* dist, int q, int g, int64_t ld, const int32_t* qlab, const int32_t* glab,
                           const int32_t* ks, int nk, double* ap, int32_t* first, double* summary, hipStream_t s);

}  // namespace rr
