// a2 + a3 fused: the Eq. 7 similarity product with the Eq. 8 candidate
// selection in its epilogue, so S is never written. Each workgroup owns a
// panel of 128 rows and one range of column tiles; it computes those tiles
// one after another on the matrix cores and merges each tile into the K best
// keys of each of its rows (knn_epilogue: lists in the workgroup's slice of
// the per-range list buffer, thresholds in LDS). A second kernel merges the
// per-range lists of every row. The symmetric tile skip is given up (every tile of the full
// N x N product is computed), so this path trades twice the product's flops
// for no N x N buffer and no S traffic.
#include "gemm_body.h"
#include "kernels.h"

namespace rr {

static_assert(KNN_LIST == KNN_LIST_MAX, "one merging wave holds the largest K the host admits");

// Two workgroups per CU (like the similarity product): one LDS stage buffer
// with the next stage prefetched into registers.
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void knn_fused_kernel(GemmArgs g, int tiles_m, int tiles_n, int ranges, int tpr, int K, uint64_t* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[knn_lds_bytes(MODE)];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // groups of 8 row panels x all ranges: the workgroups of one XCD share
  // their panels' rows and the column tiles of their ranges in its L2
  const int pid = xcd_linear(blockIdx.x, gridDim.x);
  constexpr int G = 8;
  const int per = G * ranges;
  const int grp = pid / per, in = pid - grp * per;
  const int gsz = min(tiles_m - grp * G, G);
  const int tm = grp * G + in % gsz, rg = in / gsz;
  KnnShared& ks = *(KnnShared*)(lds + knn_stage_bytes(MODE));
  if (tid < BM) {
    ks.tau[tid] = 0ull;
    ks.have[tid] = 0;
  }
  if (tid == 0) {
    ks.lists = part;
    ks.K = K;
    ks.range = rg;
  }
  __syncthreads();
  const int t0 = rg * tpr, t1 = min(tiles_n, t0 + tpr);
  for (int tn = t0; tn < t1; tn++) {
    if (tid == 0) ks.first = tn == t0;  // read after the tile's first barrier
    gemm_tile<MODE, EPI_KNN, 1, 1>(g, tm, tn, lds);
  }
  for (int lr = wave * 32; lr < wave * 32 + 32; lr++) {  // empty entries of lists shorter than K
    const int i = tm * BM + lr;
    if (i >= g.M) break;
    if (lane >= ks.have[lr] && lane < K) part[((int64_t)rg * g.M + i) * K + lane] = 0ull;
  }
}

// One wavefront per row: the K best of its per-range lists, written as the
// candidate list (column, similarity; the row itself first with 1).
__global__ __launch_bounds__(256) void knn_merge_kernel(const uint64_t* __restrict__ part, int n, int ranges, int K,
                                                        int32_t* __restrict__ idx, float* __restrict__ val) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  uint64_t best[1] = {0ull};
  for (int r = 0; r < ranges; r++) {
    const uint64_t b = lane < K ? part[((int64_t)r * n + i) * K + lane] : 0ull;
    wave_merge_batch<1>(best, b);
  }
  if (lane < K) {
    const uint32_t j = key_col(best[0]);
    idx[(int64_t)i * K + lane] = (int32_t)j;
    val[(int64_t)i * K + lane] = (j == (uint32_t)i) ? 1.0f : key_val(best[0]);
  }
}

template <int MODE>
static int fused_slots() {  // resident fused workgroups on the current device
  static const int slots = [] {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)knn_fused_kernel<MODE>, 256, 0) !=
            hipSuccess)
      return 0;
    return cus * per;
  }();
  return slots;
}

int knn_fused_ranges(int tiles_m, int tiles_n, int slots) {
  // the range count with the least (rounds of workgroups) x (tiles per range)
  int best = 1;
  int64_t cost = -1;
  const int rmax = tiles_n < kKnnMaxRanges ? tiles_n : kKnnMaxRanges;
  for (int r = 1; r <= rmax; r++) {
    const int64_t w = (int64_t)tiles_m * r;
    const int64_t rounds = slots > 0 ? (w + slots - 1) / slots : 1;
    const int64_t c = rounds * ((tiles_n + r - 1) / r);
    if (cost < 0 || c < cost) {
      cost = c;
      best = r;
    }
  }
  return best;
}

template <int MODE>
static hipError_t launch_fused_t(const void* a, int M, int64_t lda, int64_t kbytes, const float* sa, int K,
                                 uint64_t* part, int32_t* idx, float* val, hipStream_t s) {
  const int T = (M + BM - 1) / BM;
  const int ranges = knn_fused_ranges(T, T, fused_slots<MODE>());
  const int tpr = (T + ranges - 1) / ranges;
  GemmArgs g{(const uint8_t*)a, (const uint8_t*)a, M, M, lda, lda, (int)(kbytes / BKB), sa, sa, nullptr, 0};
  hipLaunchKernelGGL(knn_fused_kernel<MODE>, dim3((unsigned)(T * ranges)), dim3(256), 0, s, g, T, T, ranges, tpr, K,
                     part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(knn_merge_kernel, dim3((unsigned)((M + 3) / 4)), dim3(256), 0, s, (const uint64_t*)part, M,
                     ranges, K, idx, val);
  return hipGetLastError();
}

hipError_t launch_knn_fused(SimPrec prec, const void* a, int M, int64_t lda_bytes, int64_t kbytes, const float* sa,
                           int K, uint64_t* part, int32_t* idx, float* val, hipStream_t s) {
  if (M < 1 || K < 1 || K > KNN_LIST || K > M || kbytes % BKB || lda_bytes < kbytes || lda_bytes % 16)
    return hipErrorInvalidValue;
  switch (prec) {
    case SimPrec::F32:
      return launch_fused_t<MODE_F32>(a, M, lda_bytes, kbytes, sa, K, part, idx, val, s);
    case SimPrec::BF16:
      return launch_fused_t<MODE_BF16>(a, M, lda_bytes, kbytes, sa, K, part, idx, val, s);
    case SimPrec::FP8:
      return launch_fused_t<MODE_FP8>(a, M, lda_bytes, kbytes, sa, K, part, idx, val, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace rr
