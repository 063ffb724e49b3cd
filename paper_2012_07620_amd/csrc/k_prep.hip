// a1 -- feature preparation for the Eq. 7 similarity product.
//
// S_ij is a cosine, so it only needs 1/|x_i| per row; the product itself runs
// on the raw values (exact FP32 copies of f32 or bf16 inputs) and the norms
// are applied in the GEMM epilogue. One wavefront per row.
#include "common.h"
#include "kernels.h"

namespace rr {

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

// OCP FP8 E4M3 (bias 7, largest finite 448, no infinities): round to nearest
// even, saturate at 448. Input finite.
__device__ __forceinline__ uint32_t e4m3_rne_sat(float f) {
  const uint32_t sign = (__float_as_uint(f) >> 24) & 0x80u;
  const float a = fabsf(f);
  uint32_t code;
  if (a >= 448.0f) {
    code = 0x7Eu;
  } else if (a < 0.015625f) {  // below 2^-6: subnormal steps of 2^-9 (8 = smallest normal)
    code = (uint32_t)__builtin_rintf(a * 512.0f);
  } else {
    uint32_t b = __float_as_uint(a);
    b += 0x7FFFFu + ((b >> 20) & 1u);  // keep 3 mantissa bits
    code = ((((b >> 23) - 127u + 7u)) << 3) | ((b >> 20) & 7u);
    if (code > 0x7Eu) code = 0x7Eu;
  }
  return sign | code;
}

template <SimPrec P, bool IN_BF16>
__global__ __launch_bounds__(256) void prep_kernel(const void* __restrict__ x, int n, int d, float* __restrict__ xp,
                                                   int64_t ldp, float* __restrict__ rn, void* __restrict__ xl,
                                                   int64_t ldl, float* __restrict__ sl) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int64_t src = (int64_t)i * d;
  float* xr = xp + (int64_t)i * ldp;
  DF acc{0.f, 0.f};
  float amax = 0.f;
  for (int k = lane; k < ldp; k += 64) {
    float v = 0.f;
    if (k < d) {
      if (IN_BF16)
        v = __uint_as_float((uint32_t)((const uint16_t*)x)[src + k] << 16);
      else
        v = ((const float*)x)[src + k];
    }
    xr[k] = v;
    dot2_acc(acc, v, v);
    amax = fmaxf(amax, fabsf(v));
  }
  acc = wave_sum_df(acc);
  const float n2 = acc.hi + acc.lo;
  const float r = __fdiv_rn(1.0f, __fsqrt_rn(n2));
  if (P == SimPrec::BF16) {
    uint16_t* xb = (uint16_t*)xl + (int64_t)i * ldl;
    for (int k = lane; k < ldl; k += 64) {
      uint16_t b = 0;
      if (k < d) b = IN_BF16 ? ((const uint16_t*)x)[src + k] : bf16_rne(xr[k]);
      xb[k] = b;
    }
    if (lane == 0) sl[i] = r;
  } else if (P == SimPrec::FP8) {
    amax = wave_max_f32(amax);
    const float scale = amax > 0.f ? amax / 448.0f : 1.0f;
    const float inv = amax > 0.f ? 448.0f / amax : 1.0f;
    uint8_t* xq = (uint8_t*)xl + (int64_t)i * ldl;
    for (int k = lane; k < ldl; k += 64) xq[k] = (uint8_t)(k < d ? e4m3_rne_sat(xr[k] * inv) : 0u);
    if (lane == 0) sl[i] = r * scale;
  }
  if (lane == 0) rn[i] = r;
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
