// a1 -- feature preparation for the Eq. 7 similarity product (direct launch).
//
// S_ij is a cosine, so it only needs 1/|x_i| per row; the product itself runs
// on the raw values (exact FP32 copies of f32 or bf16 inputs) and the norms
// are applied in the GEMM epilogue. One wavefront per row.
#include "rows_body.h"

namespace rr {

template <SimPrec P, bool IN_BF16>
__global__ __launch_bounds__(256) void prep_kernel(const void* __restrict__ x, int n, int d, float* __restrict__ xp,
                                                   int64_t ldp, float* __restrict__ rn, void* __restrict__ xl,
                                                   int64_t ldl, float* __restrict__ sl) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  prep_row<P, IN_BF16>(x, i, d, xp, ldp, rn, xl, ldl, sl);
}

template <SimPrec P>
static hipError_t launch_prep_t(const void* x, int in_bf16, int n, int d, float* xp, int64_t ldp, float* rn,
                                void* xl, int64_t ldl, float* sl, hipStream_t s) {
  dim3 grid((n + 3) / 4), block(256);
  if (in_bf16)
    hipLaunchKernelGGL((prep_kernel<P, true>), grid, block, 0, s, x, n, d, xp, ldp, rn, xl, ldl, sl);
  else
    hipLaunchKernelGGL((prep_kernel<P, false>), grid, block, 0, s, x, n, d, xp, ldp, rn, xl, ldl, sl);
  return hipGetLastError();
}

hipError_t launch_prep(const void* x, int in_bf16, int n, int d, float* xp, int64_t ldp, float* rn, SimPrec prec,
                       void* xl, int64_t ldl, float* sl, hipStream_t s) {
  switch (prec) {
    case SimPrec::F32: return launch_prep_t<SimPrec::F32>(x, in_bf16, n, d, xp, ldp, rn, xl, ldl, sl, s);
    case SimPrec::BF16: return launch_prep_t<SimPrec::BF16>(x, in_bf16, n, d, xp, ldp, rn, xl, ldl, sl, s);
    case SimPrec::FP8: return launch_prep_t<SimPrec::FP8>(x, in_bf16, n, d, xp, ldp, rn, xl, ldl, sl, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace rr
