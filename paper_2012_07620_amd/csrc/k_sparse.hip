// a7, sparse form -- the final query x gallery product from the non-zeros of
// the refined features.
//
// A* rows hold O(k1) non-zeros (Eq. 9-11) and a layer of Eq. 14 widens row i
// only to the union of its k2 neighbours' supports, so after a few layers a
// row of H still has a few dozen to a few hundred non-zeros out of N and the
// dense product multiplies mostly zeros. Here (Gustavson's row-by-row sparse
// product with a dense accumulator):
//   1. every row of H is compacted into CSR (columns ascending);
//   2. the gallery rows are also laid out by column (CSC), in buckets of
//      (gallery chunk, quarter of the chunk, column);
//   3. one workgroup per query keeps the gallery accumulators of a chunk of
//      the gallery in LDS and, for each non-zero column c of the query in
//      ascending c, adds h_q[c] * h_g[c] for every gallery row g that is
//      non-zero in c (one product and one LDS add per slot per column: the
//      FP32 sum order depends only on the data, so results are
//      deterministic);
//   4. D[q][g] = 1 - sq * acc, the gallery values having been stored times
//      their row's sg in step 2.
// The four waves of a workgroup own disjoint quarters of the accumulator
// chunk and read only their quarter's buckets, so the column loop needs no
// block barrier; within a wave LDS accesses complete in issue order. Queries
// are walked in cluster order (queries of one cluster read the same columns).
//
// When the layers were kept as CSR rows (sparse layers) step 1 is skipped.
// Otherwise the compacted rows live in a spare N x N feature buffer (16 bytes
// per non-zero: CSR and CSC). If they do not fit, a device-side selection
// makes every sparse kernel return at once and the FP32 matrix-core product,
// launched behind them and gated on the same selection, computes D. No host
// round trip.
//
// The sparse layers themselves (slot bounds, layers >= 2 from CSR rows, the
// gated dense layer) are launched from here too; their row bodies are in
// rows_body.h.
#include "gemm_body.h"
#include "kernels.h"
#include "rows_body.h"

namespace rr {

// ================================================================ sparse layers
// Slot size of every row of layer l, and their 64-bit total into gates[l]
// (one atomic per wave).
__global__ __launch_bounds__(256) void sl_size_kernel(const int32_t* __restrict__ knn, int n, int k1, int k2,
                                                      int first, int sym, const int32_t* __restrict__ off,
                                                      const int32_t* __restrict__ cnt_prev, SlGate* gates,
                                                      int32_t* __restrict__ size) {
  if (gates[0].dense) return;  // gates[0] = layer l - 1
  const int i = blockIdx.x * 256 + threadIdx.x;
  int64_t b = 0;
  if (i < n) {
    for (int r = 0; r < k2; r++) {
      const int j = knn[(int64_t)i * k1 + r];
      b += first ? (int64_t)(k1 + (sym ? off[j + 1] - off[j] : 0)) : (int64_t)cnt_prev[j];
    }
    b = min(b, (int64_t)n);
    size[i] = (int32_t)b;
  }
  uint64_t t = (uint64_t)b;
  for (int m = 32; m > 0; m >>= 1) t += shfl_xor_u64(t, m);
  if ((threadIdx.x & 63) == 0 && t) atomicAdd(&gates[1].total, (unsigned long long)t);
}

// Gate l from the slot total: dense when the slots do not fit (or layer
// l - 1 was dense).
__global__ void sl_gate_kernel(int64_t cap, SlGate* gates, int l) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const unsigned long long total = gates[l].total;
  const bool dense = gates[l - 1].dense || total > (unsigned long long)cap || total > 0x7FFFFFFFull;
  gates[l].dense = dense ? 1 : 0;  // sparse only when the int32 slot starts are exact
}

hipError_t launch_sl_slots(const int32_t* knn_idx, int n, int k1, int k2, bool first, bool sym, const int32_t* off,
                           const int32_t* cnt_prev, const SlOut& out, int32_t* part, hipStream_t s) {
  if (k2 < 1 || k2 > k1 || (first && sym && !off) || (!first && !cnt_prev) || !out.gate || !out.prev ||
      out.gate != out.prev + 1 || !out.rows.so || !out.rows.cnt || !part)
    return hipErrorInvalidValue;
  // gates[l - 1] = out.prev, gates[l] = out.gate (gates start zeroed: total accumulates here)
  hipLaunchKernelGGL(sl_size_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, knn_idx, n, k1, k2,
                     (int)first, (int)sym, off, cnt_prev, (SlGate*)out.prev, out.rows.cnt);
  hipLaunchKernelGGL(sl_gate_kernel, dim3(1), dim3(64), 0, s, out.cap, (SlGate*)out.prev, 1);
  // slot starts (int32, exact whenever the gate is sparse); skipped after a dense layer
  hipError_t e = launch_scan(out.rows.cnt, n, out.rows.so, part, s, &out.prev->dense, 1);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void sparse_prop_kernel(SlRows in, const float* __restrict__ sin,
                                                          const int32_t* __restrict__ knn,
                                                          const float* __restrict__ kv, int k1, int k2, int alpha,
                                                          int agg, int64_t ld, float* __restrict__ hout,
                                                          float* __restrict__ sout, SlOut out) {
  if (out.prev->dense) return;
  __shared__ FirstShared sh;
  sparse_prop_row(in, sin, knn, kv, k1, k2, alpha, agg, ld, hout, sout, &out, blockIdx.x, sh);
}

hipError_t launch_sparse_prop(SlRows in, const float* sin, const int32_t* knn_idx, const float* knn_val, int n,
                              int k1, int k2, int alpha, int agg, int64_t ld, float* hout, float* sout, SlOut out,
                              hipStream_t s) {
  if (k2 < 1 || k2 > 256 || (ld & 3) || agg == RERANK_AGG_MAX || !out.rows.col || !out.gate || !out.prev)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(sparse_prop_kernel, dim3(n), dim3(256), 0, s, in, sin, knn_idx, knn_val, k1, k2, alpha, agg, ld,
                     hout, sout, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void propagate_gated_kernel(const float* __restrict__ hin,
                                                              const float* __restrict__ sin, int64_t ld,
                                                              const int32_t* __restrict__ knn,
                                                              const float* __restrict__ kv, int k1, int k2, int alpha,
                                                              int agg, float* __restrict__ hout,
                                                              float* __restrict__ sout, SlGate* gates, int l,
                                                              uint16_t* __restrict__ hi, uint16_t* __restrict__ lo) {
  if (!gates[l - 1].dense) return;
  __shared__ PropShared sh;
  propagate_row(hin, sin, ld, ld, knn, kv, k1, k2, alpha, agg, hout, sout, hi, lo, blockIdx.x, sh);
}

hipError_t launch_propagate_gated(const float* hin, const float* sin, int n, int64_t ld, const int32_t* knn_idx,
                                  const float* knn_val, int k1, int k2, int alpha, int agg, float* hout, float* sout,
                                  SlGate* gates, int l, hipStream_t s, uint16_t* hi, uint16_t* lo) {
  if (l < 1 || k2 < 1 || k2 > 256 || (ld & 3)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(propagate_gated_kernel, dim3(n), dim3(256), 0, s, hin, sin, ld, knn_idx, knn_val, k1, k2, alpha,
                     agg, hout, sout, gates, l, hi, lo);
  return hipGetLastError();
}

// Last layer of a dense final product from the CSR rows of the layer before:
// the row builder's dense writer (zeros written outside the row's support),
// so the layer costs one write of the dense rows instead of k2 dense reads
// per row.
__global__ __launch_bounds__(256) void sparse_prop_dense_kernel(SlRows in, const float* __restrict__ sin,
                                                                const int32_t* __restrict__ knn,
                                                                const float* __restrict__ kv, int k1, int k2,
                                                                int alpha, int agg, int64_t ld,
                                                                float* __restrict__ hout, float* __restrict__ sout,
                                                                uint16_t* __restrict__ hi, uint16_t* __restrict__ lo,
                                                                const SlGate* gate_in) {
  if (gate_in->dense) return;
  __shared__ FirstShared sh;
  const CsrSrc src{in};
  sparse_row_core(src, sin, knn, kv, k1, k2, alpha, agg, ld, hout, hi, lo, sout, nullptr, blockIdx.x, sh);
}

hipError_t launch_sparse_prop_dense(SlRows in, const float* sin, const int32_t* knn_idx, const float* knn_val, int n,
                                    int k1, int k2, int alpha, int agg, int64_t ld, float* hout, float* sout,
                                    uint16_t* hi, uint16_t* lo, const SlGate* gate_in, hipStream_t s) {
  if (k2 < 1 || k2 > 256 || (ld & 3) || agg == RERANK_AGG_MAX || !gate_in || !in.col || !in.so || !in.cnt)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(sparse_prop_dense_kernel, dim3(n), dim3(256), 0, s, in, sin, knn_idx, knn_val, k1, k2, alpha,
                     agg, ld, hout, sout, hi, lo, gate_in);
  return hipGetLastError();
}

// ================================================================ final product
// Which rows the final product uses, chosen on the device.
struct SparseSel {
  const int32_t* rs;  // row starts
  const int32_t* rc;  // row counts
  const int32_t* col;
  const float* val;
  int32_t* crow;  // column layout of the gallery rows
  float* cval;
  int32_t mode;  // 0: sparse-layer rows, 1: compacted rows, 2: dense product
  int32_t pad;
};

// Compaction of dense rows runs unless the last layer is already CSR.
__device__ __forceinline__ bool input_is_csr(const SlGate* lay) { return lay && !lay->dense; }

// One workgroup per row: number of non-zeros of a dense row (ld % 4 == 0).
__global__ __launch_bounds__(256) void nnz_count_kernel(const float* __restrict__ H, int64_t ld,
                                                        int32_t* __restrict__ cnt, const SlGate* lay) {
  if (input_is_csr(lay)) return;
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
// flag[0] = 1 (and off all zero) when the total exceeds cap. Skipped when
// `skip_csr` says the rows are already CSR, or `skip_dense` selects the dense
// product.
__global__ __launch_bounds__(256) void scan_gate_kernel(const int32_t* cnt, int n, int32_t* off, int64_t cap,
                                                        int32_t* __restrict__ flag, const SlGate* skip_csr,
                                                        const SparseSel* skip_dense) {
  if (input_is_csr(skip_csr) || (skip_dense && skip_dense->mode == 2)) return;
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
  for (int k = b; k < e; k++) {  // read before write: off may be cnt (in place)
    const int32_t v = cnt[k];
    off[k] = fits ? (int32_t)run : 0;
    run += v;
  }
  if (tid == 0) {
    off[n] = fits ? (int32_t)total : 0;
    if (flag) flag[0] = fits ? 0 : 1;
  }
}

// One workgroup per row: write the row's non-zeros, columns ascending.
__global__ __launch_bounds__(256) void csr_fill_kernel(const float* __restrict__ H, int64_t ld,
                                                       const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ flag, const SlGate* lay,
                                                       int32_t* __restrict__ col, float* __restrict__ val) {
  if (input_is_csr(lay) || flag[0]) return;
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

// One thread: pick the rows of the final product.
__global__ void select_kernel(const SlGate* lay, SlRows lrows, const int32_t* flag, const int32_t* off,
                              const int32_t* cnt, void* pool, int64_t pool_bytes, SparseSel* sel) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  SparseSel o{};
  if (input_is_csr(lay)) {
    const int64_t capp = pool_bytes / 8;  // column layout only
    o = SparseSel{lrows.so, lrows.cnt, lrows.col, lrows.val, (int32_t*)pool, (float*)((char*)pool + capp * 4), 0, 0};
  } else if (flag[0] == 0) {
    const int64_t cap = pool_bytes / 16;  // compacted rows + column layout
    o = SparseSel{off, cnt, (const int32_t*)pool, (const float*)((char*)pool + cap * 4),
                  (int32_t*)((char*)pool + cap * 8), (float*)((char*)pool + cap * 12), 1, 0};
  } else {
    o.mode = 2;
  }
  *sel = o;
}

// Column layout of the gallery rows q..n-1, split by gallery chunk (the
// accumulator width of one pass of the product) and by quarter of the chunk
// (the slots one wave owns): entry (g, c) goes to bucket
// (g / SF_GCH * 4 + quarter) * ld + c, so each wave of a pass reads only the
// entries it adds. One wave per row: bucket counts, then placement (the order
// inside a bucket is arbitrary; every entry of a bucket goes to a different
// accumulator, so it does not affect the sums).
constexpr int SF_GCH = kSparseChunk;  // gallery accumulators per pass (64 KiB of LDS)

__device__ __forceinline__ int64_t csc_bucket(int gp, int g) {
  const int ch = gp / SF_GCH, in = gp - ch * SF_GCH;
  const int gw = min(SF_GCH, g - ch * SF_GCH);
  const int quarter = (gw + 3) >> 2;
  return (int64_t)ch * 4 + in / quarter;
}

__global__ __launch_bounds__(256) void csc_count_kernel(const SparseSel* __restrict__ sel, int q, int n, int64_t ld,
                                                        int32_t* __restrict__ ccnt) {
  if (sel->mode == 2) return;
  const auto rs = gmem(sel->rs);
  const auto rc = gmem(sel->rc);
  const auto col = gmem(sel->col);
  const int lane = threadIdx.x & 63;
  for (int r = q + (int)(blockIdx.x * 4 + (threadIdx.x >> 6)); r < n; r += gridDim.x * 4) {
    const int b = rs[r], e = b + rc[r];
    int32_t* cb = ccnt + csc_bucket(r - q, n - q) * ld;
    for (int t = b + lane; t < e; t += 64) atomicAdd(cb + col[t], 1);
  }
}

// The gallery values are stored times their row's sigma (sg), so the product
// ends with D = 1 - sq * acc and reads no per-column scale.
__global__ __launch_bounds__(256) void csc_fill_kernel(const SparseSel* __restrict__ sel, int q, int n, int64_t ld,
                                                       const int32_t* __restrict__ coff, const float* __restrict__ sg,
                                                       int32_t* __restrict__ cursor) {
  if (sel->mode == 2) return;
  const auto rs = gmem(sel->rs);
  const auto rc = gmem(sel->rc);
  const auto col = gmem(sel->col);
  const auto val = gmem(sel->val);
  const auto crow = gmem(sel->crow);
  const auto cval = gmem(sel->cval);
  const int lane = threadIdx.x & 63;
  for (int r = q + (int)(blockIdx.x * 4 + (threadIdx.x >> 6)); r < n; r += gridDim.x * 4) {
    const int b = rs[r], e = b + rc[r];
    const int64_t cb = csc_bucket(r - q, n - q) * ld;
    const float sr = sg[r - q];
    for (int t = b + lane; t < e; t += 64) {
      const int64_t c = cb + col[t];
      const int pos = coff[c] + atomicAdd(cursor + c, 1);
      crow[pos] = r - q;
      cval[pos] = val[t] * sr;
    }
  }
}

constexpr int SF_QCH = 256;  // query non-zeros staged per pass
constexpr int SF_ILP = 16;   // columns whose first 64 entries are loaded together

// D[q][g] = 1 - sq * sum_c u_q[c] (sg u_g[c]). One workgroup per query, the
// queries in cluster order with consecutive ones on one XCD (they read the
// same gallery columns). Wave w owns quarter w of each gallery chunk and reads
// only that quarter's buckets.
__global__ __launch_bounds__(256) void sparse_final_kernel(const SparseSel* __restrict__ sel,
                                                           const int32_t* __restrict__ coff, int64_t ld,
                                                           const int32_t* __restrict__ qorder,
                                                           const float* __restrict__ sq, int g,
                                                           float* __restrict__ dist, int64_t ldd) {
  if (sel->mode == 2) return;
  __shared__ float acc[SF_GCH];
  __shared__ int cb[4][SF_QCH], ce[4][SF_QCH];
  __shared__ float qv[SF_QCH];
  const auto col = gmem(sel->col);
  const auto val = gmem(sel->val);
  const auto crow = gmem(sel->crow);
  const auto cval = gmem(sel->cval);
  const int qi = qorder[xcd_linear(blockIdx.x, gridDim.x)], tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int b = gmem(sel->rs)[qi], nq = gmem(sel->rc)[qi];
  const float sqq = sq[qi];
  float* drow = dist + (int64_t)qi * ldd;
  for (int g0 = 0; g0 < g; g0 += SF_GCH) {
    if (g0) __syncthreads();  // the quarters move with the chunk width: previous write-outs first
    const int gw = min(SF_GCH, g - g0);
    const int quarter = (gw + 3) >> 2;
    const int lo = min(gw, w * quarter), len = min(gw, lo + quarter) - lo;
    for (int k = lane; k < len; k += 64) acc[lo + k] = 0.f;  // own quarter
    const int32_t* cof = coff + (int64_t)(g0 / SF_GCH) * 4 * ld;  // this chunk's buckets
    const int base = g0 + lo;  // gallery position of acc[lo]
    for (int t0 = 0; t0 < nq; t0 += SF_QCH) {
      const int tn = min(SF_QCH, nq - t0);
      __syncthreads();  // every wave is done with the previous staging
      for (int t = tid; t < tn; t += 256) {
        const int c = col[b + t0 + t];
        qv[t] = val[b + t0 + t];
#pragma unroll
        for (int x = 0; x < 4; x++) {
          cb[x][t] = cof[x * ld + c];
          ce[x][t] = cof[x * ld + c + 1];
        }
      }
      __syncthreads();
      for (int t = 0; t < tn; t += SF_ILP) {
        // bucket bounds of SF_ILP columns, then their first 64 entries: loads
        // without branches (a load inside a divergent block is waited for at
        // the block's end), invalid lanes read entry 0 and drop it
        int bb[SF_ILP], be[SF_ILP];
#pragma unroll
        for (int u = 0; u < SF_ILP; u++) {
          const int tt = min(t + u, tn - 1);
          bb[u] = cb[w][tt];
          be[u] = (t + u < tn) ? ce[w][tt] : bb[u];
        }
        int r[SF_ILP];
        float xv[SF_ILP];
#pragma unroll
        for (int u = 0; u < SF_ILP; u++) {
          const int s = bb[u] + lane;
          const bool ok = s < be[u];
          const int si = ok ? s : 0;
          const int rv = crow[si];
          xv[u] = cval[si];
          r[u] = ok ? rv - base : -1;
        }
        // one LDS add per entry (no return value, so nothing waits); a
        // wave's LDS operations run in issue order, so every slot gets its
        // columns' terms in ascending column order
#pragma unroll
        for (int u = 0; u < SF_ILP; u++) {
          if (t + u >= tn) break;
          const float v = qv[t + u];
          if ((unsigned)r[u] < (unsigned)len) atomicAdd(&acc[lo + r[u]], v * xv[u]);
          for (int s = bb[u] + 64 + lane; s < be[u]; s += 64) {  // buckets longer than 64
            const int rr = crow[s] - base;
            if ((unsigned)rr < (unsigned)len) atomicAdd(&acc[lo + rr], v * cval[s]);
          }
        }
      }
    }
    for (int k = lane; k < len; k += 64) drow[g0 + lo + k] = 1.0f - sqq * acc[lo + k];
  }
}

// Dense fallback: the FP32 matrix-core product, run only in mode 2.
__global__ __launch_bounds__(256) void gemm_dist_gated_kernel(GemmArgs g, int tiles_n,
                                                              const SparseSel* __restrict__ sel) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[GEMM_LDS_1BUF];
  if (sel->mode != 2) return;
  gemm_tile<MODE_F32, EPI_DIST>(g, (int)blockIdx.x / tiles_n, (int)blockIdx.x % tiles_n, lds);
}

hipError_t launch_sparse_final(const float* H, int n, int q, int64_t ld, const float* sigma, float* dist, void* pool,
                               int64_t pool_bytes, int32_t* ints, const SlGate* lay_gate, const SlRows* lay,
                               const int32_t* knn, int k1, hipStream_t s) {
  const int g = n - q;
  if (!H || !sigma || !dist || !pool || !ints || n < 2 || q < 1 || g < 1 || ld < n || (ld & 31) || pool_bytes < 16)
    return hipErrorInvalidValue;
  if ((lay_gate == nullptr) != (lay == nullptr)) return hipErrorInvalidValue;
  // the pool must not overlap the rows: the last layer's buffer is H (dense n x ld, or CSR in the same bytes)
  if ((const char*)pool < (const char*)(H + (int64_t)n * ld) && (const char*)H < (const char*)pool + pool_bytes)
    return hipErrorInvalidValue;
  if (lay && pool_bytes < (int64_t)n * ld * 4) return hipErrorInvalidValue;  // column layout of up to n*ld/2 entries
  const int64_t nbm = sparse_buckets(n, ld);  // layout size (buckets of any gallery of this n)
  const int64_t nb = (int64_t)((g + SF_GCH - 1) / SF_GCH) * 4 * ld;  // buckets in use
  int32_t* ccnt = ints;            // nbm (cleared here with cursor: 16-byte aligned, ld % 32 == 0)
  int32_t* cursor = ccnt + nbm;    // nbm
  int32_t* coff = cursor + nbm;    // nbm + 1
  int32_t* cnt = coff + nbm + 1;   // n
  int32_t* off = cnt + n;             // n + 1
  int32_t* flag = off + n + 1;        // 2
  SparseSel* sel = (SparseSel*)(flag + 2);  // 8-byte aligned: 3 nbm + 2 n + 4 ints precede it
  int32_t* part = (int32_t*)sel + 16;       // scan block sums
  int32_t* oscr = ints + sparse_final_head(n, ld);
  int32_t* qorder = oscr + cluster_order_ints(n, n);  // queries in cluster order
  static_assert(sizeof(SparseSel) <= 16 * 4, "selection record");
  const int64_t cap = pool_bytes / 16;  // compacted entries (CSR and CSC, 16 bytes each)
  if (scan_parts(nb) > sparse_scan_parts(n, ld)) return hipErrorInvalidValue;
  if (!knn || k1 < 1) return hipErrorInvalidValue;
  hipError_t e = launch_cluster_order(knn, q, k1, n, oscr, qorder, s);
  if (e != hipSuccess) return e;
  e = launch_fill_zero((float*)ccnt, nb, s);  // the buckets in use
  if (e != hipSuccess) return e;
  e = launch_fill_zero((float*)cursor, nb, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(nnz_count_kernel, dim3(n), dim3(256), 0, s, H, ld, cnt, lay_gate);
  hipLaunchKernelGGL(scan_gate_kernel, dim3(1), dim3(256), 0, s, cnt, n, off, cap, flag, lay_gate,
                     (const SparseSel*)nullptr);
  hipLaunchKernelGGL(csr_fill_kernel, dim3(n), dim3(256), 0, s, H, ld, off, flag, lay_gate, (int32_t*)pool,
                     (float*)((char*)pool + cap * 4));
  const SlRows none{};
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(64), 0, s, lay_gate, lay ? *lay : none, flag, off, cnt, pool,
                     pool_bytes, sel);
  const unsigned rb = (unsigned)min((g + 3) / 4, 4096);
  hipLaunchKernelGGL(csc_count_kernel, dim3(rb), dim3(256), 0, s, sel, q, n, ld, ccnt);
  e = launch_scan(ccnt, nb, coff, part, s, &sel->mode, 2);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(csc_fill_kernel, dim3(rb), dim3(256), 0, s, sel, q, n, ld, coff, sigma + q, cursor);
  hipLaunchKernelGGL(sparse_final_kernel, dim3(q), dim3(256), 0, s, sel, coff, ld, qorder, sigma, g, dist, (int64_t)g);
  const int tm = (q + BM - 1) / BM, tn = (g + BN - 1) / BN;
  GemmArgs ga{(const uint8_t*)H, (const uint8_t*)(H + (int64_t)q * ld), q, g, ld * 4, ld * 4, (int)(ld * 4 / BKB),
              sigma, sigma + q, dist, (int64_t)g};
  hipLaunchKernelGGL(gemm_dist_gated_kernel, dim3((unsigned)tm * tn), dim3(256), 0, s, ga, tn, sel);
  return hipGetLastError();
}

}  // namespace rr
