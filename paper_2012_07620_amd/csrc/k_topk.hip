// a3 -- per-row top-K of the similarity matrix (Eq. 8 neighbour lists).
//
// One wavefront owns one row and streams it once from HBM in 1024-column
// chunks (four coalesced 1 KB loads per lane-group). The wave keeps the K
// best keys seen so far as a sorted list spread over its lanes (64*R keys,
// R = 1, 2 or 4) and a running threshold tau = the K-th best key. Columns
// whose key beats tau are appended to a 128-entry LDS ring; every 64 entries
// the ring is bitonic-sorted and merged into the list, which raises tau.
// The first chunk seeds the list with the per-lane maxima so the threshold
// is tight from the start.
//
// Key = (order-preserving bits of S_ij) << 32 | ~j: one 64-bit compare gives
// "similarity descending, column ascending" (the tie rule), -0.0 == +0.0.
// The row's own column gets the largest key, so it is always member 0.
#include "common.h"
#include "kernels.h"

namespace rr {

template <int R>
__global__ __launch_bounds__(256) void topk_kernel(const float* __restrict__ S, int64_t ldS, int N, int rows, int K,
                                                   int32_t* __restrict__ oidx, float* __restrict__ oval, int ldo) {
  __shared__ uint64_t ring_all[4][128];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 4 + w;
  if (i >= rows) return;  // no block-level barriers below: waves are independent
  uint64_t* ring = ring_all[w];
  const float* srow = S + (int64_t)i * ldS;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;

  uint64_t best[R];
#pragma unroll
  for (int r = 0; r < R; r++) best[r] = 0;
  uint64_t tau = 0;
  int head = 0, cnt = 0;

  constexpr int U = 4;
  constexpr int CH = 64 * 4 * U;
  for (int c0 = 0; c0 < N; c0 += CH) {
    f32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int col = c0 + u * 256 + lane * 4;
      v[u] = (col < N) ? *(const f32x4*)(srow + col) : f32x4{0.f, 0.f, 0.f, 0.f};
    }
    uint64_t lm = 0;
    if (c0 == 0) {
#pragma unroll
      for (int u = 0; u < U; u++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int col = u * 256 + lane * 4 + e;
          if (col < N) lm = umax64(lm, col == i ? self_key(i) : sel_key(v[u][e], (uint32_t)col));
        }
      best[0] = lm;
      wave_sort_desc<R>(best);
      tau = wave_rank_key<R>(best, K - 1);
    }
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int col = c0 + u * 256 + lane * 4 + e;
        uint64_t key = 0;
        if (col < N) key = (col == i) ? self_key(i) : sel_key(v[u][e], (uint32_t)col);
        const bool pass = key > tau && key != lm;
        const uint64_t m = __ballot(pass);
        if (m) {
          if (pass) ring[(head + cnt + __popcll(m & below)) & 127] = key;
          cnt += __popcll(m);
          if (cnt >= 64) {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            const uint64_t b = ring[(head + lane) & 127];
            head = (head + 64) & 127;
            cnt -= 64;
            wave_merge_batch<R>(best, b);
            tau = wave_rank_key<R>(best, K - 1);
          }
        }
      }
  }
  if (cnt > 0) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const uint64_t b = lane < cnt ? ring[(head + lane) & 127] : 0ull;
    wave_merge_batch<R>(best, b);
  }
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int e = r * 64 + lane;
    if (e < K) {
      const uint32_t j = key_col(best[r]);
      oidx[(int64_t)i * ldo + e] = (int32_t)j;
      oval[(int64_t)i * ldo + e] = (j == (uint32_t)i) ? 1.0f : key_val(best[r]);
    }
  }
}

hipError_t launch_topk(const float* S, int64_t ldS, int N, int rows, int K, int32_t* idx, float* val, int ldo,
                       hipStream_t s) {
  if (K < 1 || K > 256 || K > N || (ldS & 3)) return hipErrorInvalidValue;
  dim3 grid((rows + 3) / 4), block(256);
  if (K <= 64)
    hipLaunchKernelGGL(topk_kernel<1>, grid, block, 0, s, S, ldS, N, rows, K, idx, val, ldo);
  else if (K <= 128)
    hipLaunchKernelGGL(topk_kernel<2>, grid, block, 0, s, S, ldS, N, rows, K, idx, val, ldo);
  else
    hipLaunchKernelGGL(topk_kernel<4>, grid, block, 0, s, S, ldS, N, rows, K, idx, val, ldo);
  return hipGetLastError();
}

}  // namespace rr
