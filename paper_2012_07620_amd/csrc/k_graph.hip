// a3b, a4, a5, a6 -- neighbour re-score, A* vertex features, propagation.
#include "common.h"
#include "kernels.h"

#pragma clang fp contract(off)

namespace rr {

// ---------------------------------------------------------------- a3b
// Candidates of row i re-scored as cos(x_i, x_j) with a compensated FP32 dot
// product (error about one rounding of the result, far below the spacing of
// distinct similarities the tie rule has to resolve), then sorted under
// (similarity desc, column asc) with the row itself first; the first k1 are
// N(i, k1) of Eq. 8. One wavefront per row.
template <int R>
__global__ __launch_bounds__(256) void rescore_kernel(const float* __restrict__ xp, int64_t ldp,
                                                      const float* __restrict__ rn, int n,
                                                      const int32_t* __restrict__ cand, int Kc, int k1,
                                                      int32_t* __restrict__ kidx, float* __restrict__ kval) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const float* xi = xp + (int64_t)i * ldp;
  const float rni = rn[i];
  uint64_t keys[R];
#pragma unroll
  for (int r = 0; r < R; r++) keys[r] = 0;
  for (int c = 0; c < Kc; c++) {
    const int j = cand[(int64_t)i * Kc + c];
    uint64_t key;
    if (j == i) {
      key = self_key((uint32_t)i);
    } else {
      const float* xj = xp + (int64_t)j * ldp;
      DF acc{0.f, 0.f};
      for (int k = lane * 4; k < ldp; k += 256) {
        const f32x4 a = *(const f32x4*)(xi + k);
        const f32x4 b = *(const f32x4*)(xj + k);
        dot2_acc(acc, a.x, b.x);
        dot2_acc(acc, a.y, b.y);
        dot2_acc(acc, a.z, b.z);
        dot2_acc(acc, a.w, b.w);
      }
      acc = wave_sum_df(acc);
      const float dot = acc.hi + acc.lo;
      key = sel_key((dot * rni) * rn[j], (uint32_t)j);
    }
#pragma unroll
    for (int r = 0; r < R; r++)
      if ((c >> 6) == r && lane == (c & 63)) keys[r] = key;
  }
  wave_sort_desc<R>(keys);
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int e = r * 64 + lane;
    if (e < k1) {
      const uint32_t j = key_col(keys[r]);
      kidx[(int64_t)i * k1 + e] = (int32_t)j;
      kval[(int64_t)i * k1 + e] = (j == (uint32_t)i) ? 1.0f : key_val(keys[r]);
    }
  }
}

hipError_t launch_rescore(const float* xp, int64_t ldp, int d, const float* rn, int n, const int32_t* cand, int Kc,
                          int k1, int32_t* knn_idx, float* knn_val, hipStream_t s) {
  (void)d;
  if (Kc < k1 || Kc > 256 || (ldp & 3)) return hipErrorInvalidValue;
  dim3 grid((n + 3) / 4), block(256);
  if (Kc <= 64)
    hipLaunchKernelGGL(rescore_kernel<1>, grid, block, 0, s, xp, ldp, rn, n, cand, Kc, k1, knn_idx, knn_val);
  else if (Kc <= 128)
    hipLaunchKernelGGL(rescore_kernel<2>, grid, block, 0, s, xp, ldp, rn, n, cand, Kc, k1, knn_idx, knn_val);
  else
    hipLaunchKernelGGL(rescore_kernel<4>, grid, block, 0, s, xp, ldp, rn, n, cand, Kc, k1, knn_idx, knn_val);
  return hipGetLastError();
}

__global__ void take_prefix_kernel(const int32_t* __restrict__ ci, const float* __restrict__ cv, int n, int Kc, int k1,
                                   int32_t* __restrict__ ki, float* __restrict__ kv) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * k1) return;
  const int64_t i = t / k1, r = t % k1;
  ki[t] = ci[i * Kc + r];
  kv[t] = cv[i * Kc + r];
}

hipError_t launch_take_prefix(const int32_t* cand_idx, const float* cand_val, int n, int Kc, int k1,
                              int32_t* knn_idx, float* knn_val, hipStream_t s) {
  const int64_t total = (int64_t)n * k1;
  hipLaunchKernelGGL(take_prefix_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, cand_idx, cand_val,
                     n, Kc, k1, knn_idx, knn_val);
  return hipGetLastError();
}

// ---------------------------------------------------------------- a4
__global__ void fill_zero_kernel(f32x4* __restrict__ p, int64_t n4) {
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n4; t += (int64_t)gridDim.x * blockDim.x)
    p[t] = z;
}

__global__ void fill_f32_kernel(float* __restrict__ p, float v, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    p[t] = v;
}

static unsigned grid_for(int64_t n, int per_thread) {
  int64_t g = (n / per_thread + 255) / 256;
  if (g < 1) g = 1;
  if (g > 256 * 1024) g = 256 * 1024;
  return (unsigned)g;
}

hipError_t launch_fill_zero(float* buf, int64_t count, hipStream_t s) {
  if (count & 3) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(count / 4, 4)), dim3(256), 0, s, (f32x4*)buf, count / 4);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* dst, float v, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(count, 4)), dim3(256), 0, s, dst, v, count);
  return hipGetLastError();
}

// H[i][j] = H[j][i] = A*_ij for every j in N(i, k1): 1 when i is also in
// N(j, k1), else 1/2 (Eq. 10). When both directions exist both writers store
// the same value, so plain stores suffice.
__global__ void astar_scatter_kernel(const int32_t* __restrict__ knn, int n, int k1, float* __restrict__ H,
                                     int64_t ldH, int32_t* __restrict__ indeg, int32_t* __restrict__ mutual) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * k1) return;
  const int i = (int)(t / k1);
  const int j = knn[t];
  const int32_t* lj = knn + (int64_t)j * k1;
  bool mut = false;
  for (int s = 0; s < k1; s++) mut |= (lj[s] == i);
  const float v = mut ? 1.0f : 0.5f;
  H[(int64_t)i * ldH + j] = v;
  H[(int64_t)j * ldH + i] = v;
  atomicAdd(indeg + j, 1);
  if (mut) atomicAdd(mutual + i, 1);
}

hipError_t launch_astar_scatter(const int32_t* knn_idx, int n, int k1, float* H, int64_t ldH, int32_t* indeg,
                                int32_t* mutual, hipStream_t s) {
  const int64_t total = (int64_t)n * k1;
  hipLaunchKernelGGL(astar_scatter_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, knn_idx, n, k1, H,
                     ldH, indeg, mutual);
  return hipGetLastError();
}

// |A*_i|^2 = (#mutual) * 1 + (#one-way) * 1/4, one-way = out-only + in-only.
__global__ void astar_sigma_kernel(const int32_t* __restrict__ indeg, const int32_t* __restrict__ mutual, int n,
                                   int k1, float* __restrict__ sigma) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int m = mutual[i];
  const float sq = (float)m + 0.25f * (float)(k1 - m + indeg[i] - m);
  sigma[i] = __fdiv_rn(1.0f, __fsqrt_rn(sq));
}

hipError_t launch_astar_sigma(const int32_t* indeg, const int32_t* mutual, int n, int k1, float* sigma,
                              hipStream_t s) {
  hipLaunchKernelGGL(astar_sigma_kernel, dim3((n + 255) / 256), dim3(256), 0, s, indeg, mutual, n, k1, sigma);
  return hipGetLastError();
}

// ---------------------------------------------------------------- a5 + a6
__device__ __forceinline__ uint16_t bf16_rne_g(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

// One workgroup per output row: gather the row itself and its k2 - 1 other
// edge rows (Eq. 12: the first k2 members of N(i, k1), member 0 = i), sum
// with weights (Eq. 14, sum aggregator), reduce the squared norm. Rows are
// kept unnormalised and the norm is carried as sigma = 1/|u| (the next layer
// and the final product fold it in), so each layer is one streaming pass.
__global__ __launch_bounds__(256) void propagate_kernel(const float* __restrict__ hin, const float* __restrict__ sin,
                                                        int n, int64_t ld, int64_t cols,
                                                        const int32_t* __restrict__ knn, const float* __restrict__ kv,
                                                        int k1, int k2, int alpha, float* __restrict__ hout,
                                                        float* __restrict__ sout, uint16_t* __restrict__ hi,
                                                        uint16_t* __restrict__ lo) {
  __shared__ int nb[256];
  __shared__ float cf[256];
  __shared__ float red[4];
  const int i = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid < k2) {
    const int j = knn[(int64_t)i * k1 + tid];
    float w = 1.0f;
    if (tid > 0) {  // member 0 is the row itself with e_ii = 1
      const float e = kv[(int64_t)i * k1 + tid];
      for (int a = 0; a < alpha; a++) w *= e;
    }
    const float sj = sin ? sin[j] : 1.0f;
    // member 0: residual h_i plus the self edge (weight 1)
    cf[tid] = (tid == 0) ? 2.0f * sj : w * sj;
    nb[tid] = j;
  }
  __syncthreads();
  float ss = 0.f;
  const int64_t c4 = cols >> 2;
  for (int64_t c = tid; c < c4; c += 256) {
    f32x4 acc = cf[0] * ((const f32x4*)(hin + (int64_t)nb[0] * ld))[c];
    for (int r = 1; r < k2; r++) acc += cf[r] * ((const f32x4*)(hin + (int64_t)nb[r] * ld))[c];
    ((f32x4*)(hout + (int64_t)i * ld))[c] = acc;
    ss += acc.x * acc.x + acc.y * acc.y + acc.z * acc.z + acc.w * acc.w;
    if (hi) {
      uint16_t h4[4], l4[4];
#pragma unroll
      for (int e = 0; e < 4; e++) {
        h4[e] = bf16_rne_g(acc[e]);
        l4[e] = bf16_rne_g(acc[e] - __uint_as_float((uint32_t)h4[e] << 16));
      }
      uint16_t* ph = hi + (int64_t)i * ld + c * 4;
      uint16_t* pl = lo + (int64_t)i * ld + c * 4;
      *(uint2*)ph = make_uint2(h4[0] | ((uint32_t)h4[1] << 16), h4[2] | ((uint32_t)h4[3] << 16));
      *(uint2*)pl = make_uint2(l4[0] | ((uint32_t)l4[1] << 16), l4[2] | ((uint32_t)l4[3] << 16));
    }
  }
  ss = wave_sum_f32(ss);
  if ((tid & 63) == 0) red[tid >> 6] = ss;
  __syncthreads();
  if (tid == 0) {
    const float t = (red[0] + red[1]) + (red[2] + red[3]);
    sout[i] = __fdiv_rn(1.0f, __fsqrt_rn(t));
  }
}

hipError_t launch_propagate(const float* hin, const float* sin, int n, int64_t ld, int64_t cols,
                            const int32_t* knn_idx, const float* knn_val, int k1, int k2, int alpha, float* hout,
                            float* sout, uint16_t* hi, uint16_t* lo, hipStream_t s) {
  if (k2 < 1 || k2 > 256 || (cols & 3) || (ld & 3)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(propagate_kernel, dim3(n), dim3(256), 0, s, hin, sin, n, ld, cols, knn_idx, knn_val, k1, k2,
                     alpha, hout, sout, hi, lo);
  return hipGetLastError();
}

__global__ void split_bf16_kernel(const float* __restrict__ h, int64_t total, uint16_t* __restrict__ hi,
                                  uint16_t* __restrict__ lo) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const float v = h[t];
    const uint16_t a = bf16_rne_g(v);
    hi[t] = a;
    lo[t] = bf16_rne_g(v - __uint_as_float((uint32_t)a << 16));
  }
}

hipError_t launch_split_bf16(const float* h, int n, int64_t ld, uint16_t* hi, uint16_t* lo, hipStream_t s) {
  const int64_t total = (int64_t)n * ld;
  hipLaunchKernelGGL(split_bf16_kernel, dim3(grid_for(total, 4)), dim3(256), 0, s, h, total, hi, lo);
  return hipGetLastError();
}

__global__ void copy_i32_kernel(const int32_t* __restrict__ a, int32_t* __restrict__ b, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    b[t] = a[t];
}
__global__ void copy_f32_kernel(const float* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    b[t] = a[t];
}

hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(copy_i32_kernel, dim3(grid_for(count, 4)), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}
hipError_t launch_copy_f32(const float* src, float* dst, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(copy_f32_kernel, dim3(grid_for(count, 4)), dim3(256), 0, s, src, dst, count);
  return hipGetLastError();
}

}  // namespace rr
