// a7, sparse form -- the final query x gallery product from the non-zeros of
// the refined features.
//
// A* rows hold O(k1) non-zeros (Eq. 9-11) and a layer of Eq. 14 widens row i
// only to the union of its k2 neighbours' supports, so after a few layers a
// row of H still has a few dozen to a few hundred non-zeros out of N and the
// dense product multiplies mostly zeros. Here (Gustavson's row-by-row sparse
// product with a dense accumulator):
//   1. every row of H is compacted into CSR (columns ascending);
//   2. the gallery rows are also laid out by column (CSC);
//   3. one workgroup per query keeps the gallery accumulators of a chunk of
//      the gallery in LDS and, for each non-zero column c of the query in
//      ascending c, adds h_q[c] * h_g[c] for every gallery row g that is
//      non-zero in c (one FMA per slot per column: the FP32 sum order depends
//      only on the data, so results are deterministic);
//   4. D[q][g] = 1 - sq * sg * acc, the dense epilogue's expression.
// The four waves of a workgroup own disjoint quarters of the accumulator
// chunk, so the column loop needs no block barrier; within a wave LDS
// accesses complete in issue order.
//
// The compacted rows live in a spare N x N feature buffer (16 bytes per
// non-zero: CSR and CSC). If they do not fit, a device flag makes every
// sparse kernel return at once and the FP32 matrix-core product, launched
// behind them and gated on the same flag, computes D. No host round trip.
#include "gemm_body.h"
#include "kernels.h"

namespace rr {

// One workgroup per row: number of non-zeros of a dense row (ld % 4 == 0).
__global__ __launch_bounds__(256) void nnz_count_kernel(const float* __restrict__ H, int64_t ld,
                                                        int32_t* __restrict__ cnt) {
  __shared__ int red[4];
  const int i = blockIdx.x, tid = threadIdx.x;
  const f32x4* row = (const f32x4*)(H + (int64_t)i * ld);
  int c = 0;
  for (int64_t k = tid; k < (ld >> 2); k += 256) {
    const f32x4 v = row[k];
    c += (v.x != 0.f) + (v.y != 0.f) + (v.z != 0.f) + (v.w != 0.f);
  }
  for (int m = 32; m > 0; m >>= 1) c += __shfl_xor(c, m, kWave);
  if ((tid & 63) == 0) red[tid >> 6] = c;
  __syncthreads();
  if (tid == 0) cnt[i] = red[0] + red[1] + red[2] + red[3];
}

// Exclusive scan of cnt[0..n) into off[0..n] (one workgroup). With a flag:
// flag[0] = 1 (and off all zero) when the total exceeds cap.
__global__ __launch_bounds__(256) void scan_gate_kernel(const int32_t* __restrict__ cnt, int n,
                                                        int32_t* __restrict__ off, int64_t cap,
                                                        int32_t* __restrict__ flag) {
  __shared__ int64_t sh[256];
  const int tid = threadIdx.x;
  const int per = (n + 255) / 256;
  const int b = min(n, tid * per), e = min(n, b + per);
  int64_t sum = 0;
  for (int k = b; k < e; k++) sum += cnt[k];
  sh[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int64_t v = tid >= o ? sh[tid - o] : 0;
    __syncthreads();
    sh[tid] += v;
    __syncthreads();
  }
  const int64_t total = sh[255];
  const bool fits = total <= cap && total <= 0x7FFFFFFF;
  int64_t run = sh[tid] - sum;
  for (int k = b; k < e; k++) {
    off[k] = fits ? (int32_t)run : 0;
    run += cnt[k];
  }
  if (tid == 0) {
    off[n] = fits ? (int32_t)total : 0;
    if (flag) flag[0] = fits ? 0 : 1;
  }
}

// One workgroup per row: write the row's non-zeros, columns ascending.
__global__ __launch_bounds__(256) void csr_fill_kernel(const float* __restrict__ H, int64_t ld,
                                                       const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ flag, int32_t* __restrict__ col,
                                                       float* __restrict__ val) {
  if (flag[0]) return;
  __shared__ int wsum[4];
  const int i = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t n4 = ld >> 2;
  const f32x4* row = (const f32x4*)(H + (int64_t)i * ld);
  int base = off[i];
  for (int64_t k0 = 0; k0 < n4; k0 += 256) {
    const int64_t k = k0 + tid;
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (k < n4) v = row[k];
    const int mine = (v.x != 0.f) + (v.y != 0.f) + (v.z != 0.f) + (v.w != 0.f);
    int incl = mine;  // inclusive prefix over the wave
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int x = 0; x < 4; x++) {
      before += (x < w) ? wsum[x] : 0;
      total += wsum[x];
    }
    int at = base + before + incl - mine;
    const float e4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; e++)
      if (e4[e] != 0.f) {
        col[at] = (int32_t)(k * 4 + e);
        val[at] = e4[e];
        at++;
      }
    base += total;
    __syncthreads();  // wsum is rewritten by the next chunk
  }
}

// CSC of the gallery rows q..n-1, one wave per row: column counts, then
// placement (the order inside a column is arbitrary; every entry of a column
// goes to a different accumulator, so it does not affect the sums).
__global__ __launch_bounds__(256) void csc_count_kernel(const int32_t* __restrict__ off, int q, int n,
                                                        const int32_t* __restrict__ col,
                                                        const int32_t* __restrict__ flag,
                                                        int32_t* __restrict__ ccnt) {
  if (flag[0]) return;
  const int lane = threadIdx.x & 63;
  for (int r = q + (int)(blockIdx.x * 4 + (threadIdx.x >> 6)); r < n; r += gridDim.x * 4)
    for (int t = off[r] + lane; t < off[r + 1]; t += 64) atomicAdd(ccnt + col[t], 1);
}

__global__ __launch_bounds__(256) void csc_fill_kernel(const int32_t* __restrict__ off, int q, int n,
                                                       const int32_t* __restrict__ col,
                                                       const float* __restrict__ val,
                                                       const int32_t* __restrict__ coff,
                                                       const int32_t* __restrict__ flag,
                                                       int32_t* __restrict__ cursor, int32_t* __restrict__ crow,
                                                       float* __restrict__ cval) {
  if (flag[0]) return;
  const int lane = threadIdx.x & 63;
  for (int r = q + (int)(blockIdx.x * 4 + (threadIdx.x >> 6)); r < n; r += gridDim.x * 4)
    for (int t = off[r] + lane; t < off[r + 1]; t += 64) {
      const int c = col[t];
      const int pos = coff[c] + atomicAdd(cursor + c, 1);
      crow[pos] = r - q;
      cval[pos] = val[t];
    }
}

constexpr int SF_GCH = 16384;  // gallery accumulators per pass (64 KiB of LDS)
constexpr int SF_QCH = 512;    // query non-zeros staged per pass
constexpr int SF_ILP = 4;      // columns whose first 64 entries are loaded together

struct SparseFinalArgs {
  const int32_t* off;  // CSR row offsets (n + 1)
  const int32_t* col;
  const float* val;
  const int32_t* coff;  // CSC column offsets (ld + 1)
  const int32_t* crow;  // gallery position of each CSC entry
  const float* cval;
  const float* sq;  // sigma of the queries
  const float* sg;  // sigma of the gallery
  int g;
  const int32_t* flag;
  float* dist;
  int64_t ldd;
};

__global__ __launch_bounds__(256) void sparse_final_kernel(SparseFinalArgs a) {
  if (a.flag[0]) return;
  __shared__ float acc[SF_GCH];
  __shared__ int cb[SF_QCH], ce[SF_QCH];
  __shared__ float qv[SF_QCH];
  const int qi = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int b = a.off[qi], nq = a.off[qi + 1] - b;
  const float sq = a.sq[qi];
  float* drow = a.dist + (int64_t)qi * a.ldd;
  for (int g0 = 0; g0 < a.g; g0 += SF_GCH) {
    if (g0) __syncthreads();  // the waves' quarters move with the chunk width
    const int gw = min(SF_GCH, a.g - g0);
    const int quarter = (gw + 3) >> 2;
    const int lo = min(gw, w * quarter), len = min(gw, lo + quarter) - lo;
    for (int k = lane; k < len; k += 64) acc[lo + k] = 0.f;
    for (int t0 = 0; t0 < nq; t0 += SF_QCH) {
      const int tn = min(SF_QCH, nq - t0);
      if (g0 == 0 || nq > SF_QCH) {  // stage the query's columns (once if they fit)
        __syncthreads();
        for (int t = tid; t < tn; t += 256) {
          const int c = a.col[b + t0 + t];
          cb[t] = a.coff[c];
          ce[t] = a.coff[c + 1];
          qv[t] = a.val[b + t0 + t];
        }
        __syncthreads();
      }
      const int base = g0 + lo;  // gallery position of acc[lo]
      for (int t = 0; t < tn; t += SF_ILP) {
        int r[SF_ILP];
        float x[SF_ILP];
#pragma unroll
        for (int u = 0; u < SF_ILP; u++) {
          r[u] = -1;
          x[u] = 0.f;
          if (t + u < tn) {
            const int s = cb[t + u] + lane;
            if (s < ce[t + u]) {
              r[u] = a.crow[s] - base;
              x[u] = a.cval[s];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < SF_ILP; u++) {
          if (t + u >= tn) break;
          const float v = qv[t + u];
          if ((unsigned)r[u] < (unsigned)len) acc[lo + r[u]] = __builtin_fmaf(v, x[u], acc[lo + r[u]]);
          for (int s = cb[t + u] + 64 + lane; s < ce[t + u]; s += 64) {  // columns longer than 64
            const int rr = a.crow[s] - base;
            if ((unsigned)rr < (unsigned)len) acc[lo + rr] = __builtin_fmaf(v, a.cval[s], acc[lo + rr]);
          }
        }
      }
    }
    for (int k = lane; k < len; k += 64) drow[g0 + lo + k] = 1.0f - sq * a.sg[g0 + lo + k] * acc[lo + k];
  }
}

// Dense fallback: the FP32 matrix-core product, run only when flag[0] != 0.
__global__ __launch_bounds__(256) void gemm_dist_gated_kernel(GemmArgs g, int tiles_n,
                                                              const int32_t* __restrict__ flag) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[GEMM_LDS_1BUF];
  if (flag[0] == 0) return;
  gemm_tile<MODE_F32, EPI_DIST>(g, (int)blockIdx.x / tiles_n, (int)blockIdx.x % tiles_n, lds);
}

hipError_t launch_sparse_final(const float* H, int n, int q, int64_t ld, const float* sigma, float* dist, void* pool,
                               int64_t pool_bytes, int32_t* ints, hipStream_t s) {
  const int g = n - q;
  if (!H || !sigma || !dist || !pool || !ints || n < 2 || q < 1 || g < 1 || ld < n || (ld & 31) || pool_bytes < 16)
    return hipErrorInvalidValue;
  if ((const char*)pool < (const char*)(H + (int64_t)n * ld) && (const char*)H < (const char*)pool + pool_bytes)
    return hipErrorInvalidValue;  // the compacted rows must not overwrite H
  int32_t* ccnt = ints;            // ld   (cleared here with cursor: 16-byte aligned, ld % 32 == 0)
  int32_t* cursor = ccnt + ld;     // ld
  int32_t* coff = cursor + ld;     // ld + 1
  int32_t* cnt = coff + ld + 1;    // n
  int32_t* off = cnt + n;          // n + 1
  int32_t* flag = off + n + 1;     // 2
  const int64_t cap = pool_bytes / 16;  // entries of each of the four arrays
  int32_t* col = (int32_t*)pool;
  float* val = (float*)((char*)pool + cap * 4);
  int32_t* crow = (int32_t*)((char*)pool + cap * 8);
  float* cval = (float*)((char*)pool + cap * 12);
  hipError_t e = launch_fill_zero((float*)ccnt, 2 * ld, s);  // ccnt and cursor
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(nnz_count_kernel, dim3(n), dim3(256), 0, s, H, ld, cnt);
  hipLaunchKernelGGL(scan_gate_kernel, dim3(1), dim3(256), 0, s, cnt, n, off, cap, flag);
  hipLaunchKernelGGL(csr_fill_kernel, dim3(n), dim3(256), 0, s, H, ld, off, flag, col, val);
  const unsigned rb = (unsigned)min((g + 3) / 4, 4096);
  hipLaunchKernelGGL(csc_count_kernel, dim3(rb), dim3(256), 0, s, off, q, n, col, flag, ccnt);
  hipLaunchKernelGGL(scan_gate_kernel, dim3(1), dim3(256), 0, s, ccnt, (int)ld, coff, cap, (int32_t*)nullptr);
  hipLaunchKernelGGL(csc_fill_kernel, dim3(rb), dim3(256), 0, s, off, q, n, col, val, coff, flag, cursor, crow, cval);
  SparseFinalArgs sa{off, col, val, coff, crow, cval, sigma, sigma + q, g, flag, dist, (int64_t)g};
  hipLaunchKernelGGL(sparse_final_kernel, dim3(q), dim3(256), 0, s, sa);
  const int tm = (q + BM - 1) / BM, tn = (g + BN - 1) / BN;
  GemmArgs ga{(const uint8_t*)H, (const uint8_t*)(H + (int64_t)q * ld), q, g, ld * 4, ld * 4, (int)(ld * 4 / BKB),
              sigma, sigma + q, dist, (int64_t)g};
  hipLaunchKernelGGL(gemm_dist_gated_kernel, dim3((unsigned)tm * tn), dim3(256), 0, s, ga, tn, flag);
  return hipGetLastError();
}

}  // namespace rr
