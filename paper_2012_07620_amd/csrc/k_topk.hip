// a3 -- per-row top-K of the similarity matrix (Eq. 8 neighbour lists),
// direct launch: four rows (one per wavefront) per workgroup.
#include "rows_body.h"

namespace rr {

template <int R, typename T>
__global__ __launch_bounds__(256) void topk_kernel(const T* __restrict__ S, int64_t ldS, int N, int rows, int K,
                                                   int32_t* __restrict__ oidx, float* __restrict__ oval, int ldo) {
  __shared__ uint64_t ring_all[4][128];
  const int w = threadIdx.x >> 6;
  const int i = blockIdx.x * 4 + w;
  if (i >= rows) return;  // no block-level barriers in the body: waves are independent
  topk_row<R, false, T>(S, ldS, N, i, K, oidx, oval, ldo, ring_all[w]);
}

template <typename T>
static void launch_topk_t(const T* S, int64_t ldS, int N, int rows, int K, int32_t* idx, float* val, int ldo,
                          hipStream_t s) {
  dim3 grid((rows + 3) / 4), block(256);
  if (K <= 64)
    hipLaunchKernelGGL((topk_kernel<1, T>), grid, block, 0, s, S, ldS, N, rows, K, idx, val, ldo);
  else if (K <= 128)
    hipLaunchKernelGGL((topk_kernel<2, T>), grid, block, 0, s, S, ldS, N, rows, K, idx, val, ldo);
  else
    hipLaunchKernelGGL((topk_kernel<4, T>), grid, block, 0, s, S, ldS, N, rows, K, idx, val, ldo);
}

hipError_t launch_topk(const void* S, bool half, int64_t ldS, int N, int rows, int K, int32_t* idx, float* val,
                       int ldo, hipStream_t s) {
  if (K < 1 || K > 256 || K > N || (ldS & 3)) return hipErrorInvalidValue;
  if (half)
    launch_topk_t((const _Float16*)S, ldS, N, rows, K, idx, val, ldo, s);
  else
    launch_topk_t((const float*)S, ldS, N, rows, K, idx, val, ldo, s);
  return hipGetLastError();
}

template <int R, typename T>
__global__ __launch_bounds__(256) void topk_pruned_kernel(const T* __restrict__ S, int64_t ldS, int N, int rows, int K,
                                                          const float* __restrict__ bm, int64_t ldbm,
                                                          int32_t* __restrict__ oidx, float* __restrict__ oval,
                                                          int ldo) {
  __shared__ uint64_t ring_all[4][128];
  __shared__ int list_all[4][512];
  __shared__ float bm_all[4][512];  // the four rows' block maxima
  const int w = threadIdx.x >> 6;
  // consecutive row groups on one XCD, which then shares the maxima's lines
  const int i0 = xcd_linear(blockIdx.x, gridDim.x) * 4;
  // one 16-byte load per column block covers the workgroup's four rows
  // (ldbm and i0 are multiples of 4; rows past the last are padding, unused)
  const int TB = (N + 127) / 128;
  for (int t = threadIdx.x; t < TB; t += 256) {
    const f32x4 v = *(const f32x4*)(bm + (int64_t)t * ldbm + i0);
#pragma unroll
    for (int r = 0; r < 4; r++) bm_all[r][t] = v[r];
  }
  __syncthreads();
  const int i = i0 + w;
  if (i >= rows) return;  // no block-level barriers after this point
  topk_pruned_row<R, T>(S, ldS, N, i, K, bm_all[w], oidx, oval, ldo, ring_all[w], list_all[w]);
}

// Rows the pruned selection left marked (first index -1) are selected again
// over the whole row. One wavefront checks 64 rows with one load, so a launch
// over finite inputs, where no row is marked, reads 4 bytes per row.
template <int R, typename T>
__global__ __launch_bounds__(256) void topk_redo_kernel(const T* __restrict__ S, int64_t ldS, int N, int rows, int K,
                                                        int32_t* __restrict__ oidx, float* __restrict__ oval,
                                                        int ldo) {
  __shared__ uint64_t ring_all[4][128];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i0 = (blockIdx.x * 4 + w) * 64;
  if (i0 >= rows) return;  // waves are independent
  const int i = i0 + lane;
  uint64_t m = __ballot(i < rows && oidx[(int64_t)i * ldo] < 0);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // every lane has read its marker
  while (m) {
    const int r = __builtin_ctzll(m);
    m &= m - 1;
    topk_row<R, false, T>(S, ldS, N, i0 + r, K, oidx, oval, ldo, ring_all[w]);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the ring is reused by the next row
  }
}

template <typename T>
static void launch_topk_pruned_t(const T* S, int64_t ldS, int N, int rows, int K, const float* bm, int64_t ldbm,
                                 int32_t* idx, float* val, int ldo, hipStream_t s) {
  dim3 grid((rows + 3) / 4), block(256), grid_redo((rows + 255) / 256);
  if (K <= 64) {
    hipLaunchKernelGGL((topk_pruned_kernel<1, T>), grid, block, 0, s, S, ldS, N, rows, K, bm, ldbm, idx, val, ldo);
    hipLaunchKernelGGL((topk_redo_kernel<1, T>), grid_redo, block, 0, s, S, ldS, N, rows, K, idx, val, ldo);
  } else {  // K <= 128 (checked by the launcher)
    hipLaunchKernelGGL((topk_pruned_kernel<2, T>), grid, block, 0, s, S, ldS, N, rows, K, bm, ldbm, idx, val, ldo);
    hipLaunchKernelGGL((topk_redo_kernel<2, T>), grid_redo, block, 0, s, S, ldS, N, rows, K, idx, val, ldo);
  }
}

hipError_t launch_topk_pruned(const void* S, bool half, int64_t ldS, int N, int rows, int K, const float* bm,
                              int64_t ldbm, int32_t* idx, float* val, int ldo, hipStream_t s) {
  if (K < 1 || K > kPrunedMaxK || K > N || N > kPrunedMaxN || (ldS & 3) || !bm || (ldbm & 3) || ldbm < (rows + 3) / 4 * 4 ||
      ((uintptr_t)bm & 15))
    return hipErrorInvalidValue;
  if (half)
    launch_topk_pruned_t((const _Float16*)S, ldS, N, rows, K, bm, ldbm, idx, val, ldo, s);
  else
    launch_topk_pruned_t((const float*)S, ldS, N, rows, K, bm, ldbm, idx, val, ldo, s);
  return hipGetLastError();
}

// Ranking list (Algorithm 1): per row of D, the r smallest in ascending order.
template <int R>
__global__ __launch_bounds__(256) void rank_kernel(const float* __restrict__ D, int q, int g, int r,
                                                   int32_t* __restrict__ out) {
  __shared__ uint64_t ring_all[4][128];
  const int w = threadIdx.x >> 6;
  const int i = blockIdx.x * 4 + w;
  if (i >= q) return;
  topk_row<R, true>(D, g, g, i, r, out, nullptr, r, ring_all[w]);
}

hipError_t launch_rank(const float* D, int q, int g, int r, int32_t* out, hipStream_t s) {
  if (r < 1 || r > 256 || r > g || q < 1) return hipErrorInvalidValue;
  dim3 grid((q + 3) / 4), block(256);
  if (r <= 64)
    hipLaunchKernelGGL(rank_kernel<1>, grid, block, 0, s, D, q, g, r, out);
  else if (r <= 128)
    hipLaunchKernelGGL(rank_kernel<2>, grid, block, 0, s, D, q, g, r, out);
  else
    hipLaunchKernelGGL(rank_kernel<4>, grid, block, 0, s, D, q, g, r, out);
  return hipGetLastError();
}

}  // namespace rr
