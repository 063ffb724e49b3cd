// a3b, a4, a5, a6 -- direct launches of the re-score, A* and propagation
// kernels; the per-item bodies are in rows_body.h.
#include "rows_body.h"

#pragma clang fp contract(off)

namespace rr {

// ---------------------------------------------------------------- a3b
// Cluster order: rows whose lists overlap (a cluster of mutual neighbours)
// share the key min(i, entries of row i); a counting sort by key puts them
// next to each other. Kernels that walk rows in this order with consecutive
// rows on one XCD (xcd_linear) fetch the rows a cluster shares into that
// XCD's L2 once instead of once per row.
__global__ void order_key_kernel(const int32_t* __restrict__ lists, int rows, int w, int32_t* __restrict__ key,
                                 int32_t* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  int m = i;
#pragma unroll 8
  for (int c = 0; c < w; c++) m = min(m, lists[(int64_t)i * w + c]);  // eight loads in flight per step
  key[i] = m;
  atomicAdd(cnt + m, 1);
}

__global__ void order_place_kernel(const int32_t* __restrict__ key, int rows, const int32_t* __restrict__ off,
                                   int32_t* __restrict__ cursor, int32_t* __restrict__ order) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const int k = key[i];
  order[off[k] + atomicAdd(cursor + k, 1)] = i;
}

hipError_t launch_cluster_order(const int32_t* lists, int rows, int w, int n, int32_t* scratch, int32_t* order,
                                hipStream_t s) {
  if (rows < 1 || rows > n || w < 1 || ((uintptr_t)scratch & 15)) return hipErrorInvalidValue;
  int32_t* cnt = scratch;  // cnt[n], cursor[n], key[rows], off[n + 1], scan parts
  int32_t* cursor = cnt + n;
  int32_t* key = cursor + n;
  int32_t* off = key + rows;
  int32_t* part = off + n + 1;
  hipError_t e = launch_fill_zero((float*)cnt, 2 * (int64_t)n, s);
  if (e != hipSuccess) return e;
  const unsigned g = (unsigned)((rows + 255) / 256);
  hipLaunchKernelGGL(order_key_kernel, dim3(g), dim3(256), 0, s, lists, rows, w, key, cnt);
  e = launch_scan(cnt, n, off, part, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(order_place_kernel, dim3(g), dim3(256), 0, s, key, rows, off, cursor, order);
  return hipGetLastError();
}

// W: wavefronts per SIMD the register allocation must allow (1: the
// compiler's choice, two for the 2048-feature blocks). None spills.
template <int R, int U, int W>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W)))
void rescore_kernel(const float* __restrict__ xp, int64_t ldp,
                                                      const float* __restrict__ rn, int n,
                                                      const int32_t* __restrict__ cand,
                                                      const float* __restrict__ cval, int Kc, int k1, float skip2,
                                                      int32_t* __restrict__ kidx, float* __restrict__ kval,
                                                      const int32_t* __restrict__ order) {
  const int p = (order ? xcd_linear(blockIdx.x, gridDim.x) : (int)blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (p >= n) return;
  const int i = order ? order[p] : p;
  rescore_row_u<R, U>(xp, ldp, rn, i, cand, cval, Kc, k1, skip2, kidx, kval);
}

// Rows that re-score every candidate (no skip bound) run best with fewer
// rows in flight on the 2048-feature blocks (the L2 keeps more of the
// candidates those rows share): 0.86 against 0.98 ms for 58 candidates of
// 19281 rows; rows that re-score only the prefix the bound leaves run best
// with three wavefronts per SIMD (0.43 against 0.48 ms).
template <int R>
static void launch_rescore_r(dim3 grid, dim3 block, hipStream_t s, const float* xp, int64_t ldp, const float* rn,
                             int n, const int32_t* cand, const float* cval, int Kc, int k1, float skip2,
                             int32_t* knn_idx, float* knn_val, const int32_t* order) {
  constexpr int W8 = R > 2 ? 1 : 3;
  switch (rescore_u(ldp)) {  // as rescore_row picks it
    case 8:
      if (skip2 < 0.f || R > 2)
        hipLaunchKernelGGL((rescore_kernel<R, 8, 1>), grid, block, 0, s, xp, ldp, rn, n, cand, cval, Kc, k1, skip2,
                           knn_idx, knn_val, order);
      else
        hipLaunchKernelGGL((rescore_kernel<R, 8, W8>), grid, block, 0, s, xp, ldp, rn, n, cand, cval, Kc, k1, skip2,
                           knn_idx, knn_val, order);
      break;
    case 4:
      hipLaunchKernelGGL((rescore_kernel<R, 4, 3>), grid, block, 0, s, xp, ldp, rn, n, cand, cval, Kc, k1, skip2,
                         knn_idx, knn_val, order);
      break;
    case 2:
      hipLaunchKernelGGL((rescore_kernel<R, 2, 3>), grid, block, 0, s, xp, ldp, rn, n, cand, cval, Kc, k1, skip2,
                         knn_idx, knn_val, order);
      break;
    default:
      hipLaunchKernelGGL((rescore_kernel<R, 1, 3>), grid, block, 0, s, xp, ldp, rn, n, cand, cval, Kc, k1, skip2,
                         knn_idx, knn_val, order);
  }
}

hipError_t launch_rescore(const float* xp, int64_t ldp, int d, const float* rn, int n, const int32_t* cand,
                          const float* cval, int Kc, int k1, float skip2, int32_t* knn_idx, float* knn_val,
                          int32_t* scratch, hipStream_t s) {
  (void)d;
  if (Kc < k1 || Kc > 256 || (ldp & 3)) return hipErrorInvalidValue;
  const int32_t* order = nullptr;
  if (scratch) {  // cluster order of the rows by their candidates, then order[n]
    int32_t* ord = scratch + cluster_order_ints(n, n);
    hipError_t e = launch_cluster_order(cand, n, Kc, n, scratch, ord, s);
    if (e != hipSuccess) return e;
    order = ord;
  }
  dim3 grid((n + 3) / 4), block(256);
  if (Kc <= 64)
    launch_rescore_r<1>(grid, block, s, xp, ldp, rn, n, cand, cval, Kc, k1, skip2, knn_idx, knn_val, order);
  else if (Kc <= 128)
    launch_rescore_r<2>(grid, block, s, xp, ldp, rn, n, cand, cval, Kc, k1, skip2, knn_idx, knn_val, order);
  else
    launch_rescore_r<4>(grid, block, s, xp, ldp, rn, n, cand, cval, Kc, k1, skip2, knn_idx, knn_val, order);
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
__global__ __launch_bounds__(256) void fill_zero_kernel(float* __restrict__ p, int64_t count) {
  fill_item(p, count, blockIdx.x);
}

hipError_t launch_fill_zero(float* buf, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int64_t items = (count + FILL_ITEM - 1) / FILL_ITEM;
  if (items > 0x7FFFFFFF || ((uintptr_t)buf & 15)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)items), dim3(256), 0, s, buf, count);
  return hipGetLastError();
}

__global__ void astar_scatter_kernel(const int32_t* __restrict__ knn, int n, int k1, float* __restrict__ H,
                                     int64_t ldH, int32_t* __restrict__ cnt, int sym) {
  scatter_pair(knn, n, k1, H, ldH, cnt, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, sym != 0);
}

hipError_t launch_astar_scatter(const int32_t* knn_idx, int n, int k1, float* H, int64_t ldH, int32_t* cnt,
                                bool sym, hipStream_t s) {
  const int64_t total = (int64_t)n * k1;
  hipLaunchKernelGGL(astar_scatter_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, knn_idx, n, k1, H,
                     ldH, cnt, (int)sym);
  return hipGetLastError();
}

__global__ void astar_sigma_kernel(const int32_t* __restrict__ cnt, int n, int k1, float* __restrict__ sigma,
                                   int sym) {
  astar_sigma_row(cnt, n, k1, sigma, blockIdx.x * blockDim.x + threadIdx.x, sym != 0);
}

hipError_t launch_astar_sigma(const int32_t* cnt, int n, int k1, float* sigma, bool sym, hipStream_t s) {
  hipLaunchKernelGGL(astar_sigma_kernel, dim3((n + 255) / 256), dim3(256), 0, s, cnt, n, k1, sigma, (int)sym);
  return hipGetLastError();
}

// ---------------------------------------------------------------- a5 + a6
__global__ __launch_bounds__(256) void propagate_kernel(const float* __restrict__ hin, const float* __restrict__ sin,
                                                        int64_t ld, int64_t cols, const int32_t* __restrict__ knn,
                                                        const float* __restrict__ kv, int k1, int k2, int alpha,
                                                        int agg, float* __restrict__ hout, float* __restrict__ sout,
                                                        uint16_t* __restrict__ hi, uint16_t* __restrict__ lo,
                                                        const int32_t* __restrict__ order) {
  __shared__ PropShared sh;
  const int i = order ? order[xcd_linear(blockIdx.x, gridDim.x)] : (int)blockIdx.x;
  propagate_row(hin, sin, ld, cols, knn, kv, k1, k2, alpha, agg, hout, sout, hi, lo, i, sh);
}

hipError_t launch_propagate(const float* hin, const float* sin, int n, int64_t ld, int64_t cols,
                            const int32_t* knn_idx, const float* knn_val, int k1, int k2, int alpha, int agg,
                            float* hout, float* sout, uint16_t* hi, uint16_t* lo, const int32_t* order,
                            hipStream_t s) {
  if (k2 < 1 || k2 > 256 || (cols & 3) || (ld & 3)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(propagate_kernel, dim3(n), dim3(256), 0, s, hin, sin, ld, cols, knn_idx, knn_val, k1, k2, alpha,
                     agg, hout, sout, hi, lo, order);
  return hipGetLastError();
}

// ---------------------------------------------------------------- sparse first layer
__global__ void mutual_kernel(const int32_t* __restrict__ knn, int n, int k1, uint8_t* __restrict__ mflag,
                              int32_t* __restrict__ innm) {
  mutual_pair(knn, n, k1, mflag, innm, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

hipError_t launch_mutual(const int32_t* knn_idx, int n, int k1, uint8_t* mflag, int32_t* innm, hipStream_t s) {
  const int64_t total = (int64_t)n * k1;
  hipLaunchKernelGGL(mutual_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, knn_idx, n, k1, mflag,
                     innm);
  return hipGetLastError();
}

// ---------------------------------------------------------------- prefix sums
constexpr int SCAN_BLOCK = 1024;  // counts per block (4 per thread)

__device__ __forceinline__ bool scan_skipped(const int32_t* skip, int32_t skip_val) {
  return skip && *skip == skip_val;
}

__global__ __launch_bounds__(256) void scan_sums_kernel(const int32_t* __restrict__ in, int64_t n,
                                                        int32_t* __restrict__ part, const int32_t* skip,
                                                        int32_t skip_val) {
  if (scan_skipped(skip, skip_val)) return;
  __shared__ int red[4];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + tid * 4;
  int v = 0;
  for (int e = 0; e < 4; e++) v += (base + e < n) ? in[base + e] : 0;
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, kWave);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// One workgroup: part[0, nb) -> exclusive prefix in place, part[nb] = total.
__global__ __launch_bounds__(256) void scan_parts_kernel(int32_t* part, int nb, const int32_t* skip,
                                                         int32_t skip_val) {
  if (scan_skipped(skip, skip_val)) return;
  __shared__ int32_t sh[256];
  const int tid = threadIdx.x;
  const int per = (nb + 255) / 256;
  const int b = min(nb, tid * per), e = min(nb, b + per);
  int sum = 0;
  for (int k = b; k < e; k++) sum += part[k];
  sh[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int v = tid >= o ? sh[tid - o] : 0;
    __syncthreads();
    sh[tid] += v;
    __syncthreads();
  }
  int run = sh[tid] - sum;
  for (int k = b; k < e; k++) {  // read before write (in place)
    const int v = part[k];
    part[k] = run;
    run += v;
  }
  if (tid == 255) part[nb] = sh[255];
}

__global__ __launch_bounds__(256) void scan_apply_kernel(const int32_t* __restrict__ in, int64_t n,
                                                         const int32_t* __restrict__ part, int32_t* __restrict__ out,
                                                         const int32_t* skip, int32_t skip_val) {
  if (scan_skipped(skip, skip_val)) return;
  __shared__ int wsum[4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + tid * 4;
  int v[4], mine = 0;
  for (int e = 0; e < 4; e++) {
    v[e] = (base + e < n) ? in[base + e] : 0;
    mine += v[e];
  }
  int incl = mine;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int run = part[blockIdx.x] + incl - mine;
  for (int x = 0; x < w; x++) run += wsum[x];
  for (int e = 0; e < 4; e++) {
    if (base + e < n) out[base + e] = run;
    run += v[e];
  }
  if (blockIdx.x == gridDim.x - 1 && tid == 255) out[n] = part[gridDim.x];
}

hipError_t launch_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* part, hipStream_t s,
                       const int32_t* skip, int32_t skip_val) {
  if (n < 1 || !in || !out || !part) return hipErrorInvalidValue;
  const int64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
  if (nb > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(scan_sums_kernel, dim3((unsigned)nb), dim3(256), 0, s, in, n, part, skip, skip_val);
  hipLaunchKernelGGL(scan_parts_kernel, dim3(1), dim3(256), 0, s, part, (int)nb, skip, skip_val);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(256), 0, s, in, n, part, out, skip, skip_val);
  return hipGetLastError();
}

__global__ void csr_kernel(const int32_t* __restrict__ knn, int n, int k1, const uint8_t* __restrict__ mflag,
                           const int32_t* __restrict__ off, int32_t* __restrict__ cursor, int32_t* __restrict__ inl) {
  csr_pair(knn, n, k1, mflag, off, cursor, inl, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

hipError_t launch_csr(const int32_t* knn_idx, int n, int k1, const uint8_t* mflag, const int32_t* off,
                      int32_t* cursor, int32_t* inl, hipStream_t s) {
  const int64_t total = (int64_t)n * k1;
  hipLaunchKernelGGL(csr_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, knn_idx, n, k1, mflag, off,
                     cursor, inl);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void first_layer_kernel(const int32_t* __restrict__ knn, const float* __restrict__ kv,
                                                          const uint8_t* __restrict__ mflag,
                                                          const int32_t* __restrict__ off,
                                                          const int32_t* __restrict__ inl, int k1, int k2, int alpha,
                                                          int agg, int sym, int64_t ld, float* __restrict__ hout,
                                                          float* __restrict__ sout, uint16_t* __restrict__ hi,
                                                          uint16_t* __restrict__ lo, SlOut sl, int use_sl) {
  __shared__ FirstShared sh;
  first_layer_row(knn, kv, mflag, off, inl, k1, k2, alpha, agg, sym != 0, ld, hout, sout, hi, lo, blockIdx.x, sh,
                  use_sl ? &sl : nullptr);
}

hipError_t launch_first_layer(const int32_t* knn_idx, const float* knn_val, const uint8_t* mflag,
                              const int32_t* off, const int32_t* inl, int n, int k1, int k2, int alpha, int agg,
                              bool sym, int64_t ld, float* hout, float* sout, uint16_t* hi, uint16_t* lo,
                              const SlOut* sl, hipStream_t s) {
  if (k2 < 1 || k2 > 256 || (ld & 3) || agg == RERANK_AGG_MAX) return hipErrorInvalidValue;
  if (sl && (hi || !sl->rows.col || !sl->gate || !sl->prev)) return hipErrorInvalidValue;
  const SlOut none{};
  hipLaunchKernelGGL(first_layer_kernel, dim3(n), dim3(256), 0, s, knn_idx, knn_val, mflag, off, inl, k1, k2, alpha,
                     agg, (int)sym, ld, hout, sout, hi, lo, sl ? *sl : none, sl ? 1 : 0);
  return hipGetLastError();
}

// ---------------------------------------------------------------- helpers
static unsigned grid_for(int64_t n, int per_thread) {
  int64_t g = (n / per_thread + 255) / 256;
  if (g < 1) g = 1;
  if (g > 256 * 1024) g = 256 * 1024;
  return (unsigned)g;
}

__global__ void split_bf16_kernel(const float* __restrict__ h, int64_t total, uint16_t* __restrict__ hi,
                                  uint16_t* __restrict__ lo) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const float v = h[t];
    const uint16_t a = bf16_rne(v);
    hi[t] = a;
    if (lo) lo[t] = bf16_rne(v - __uint_as_float((uint32_t)a << 16));
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
