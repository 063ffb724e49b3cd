// Retrieval metrics of Section 4.1 (Evaluation Metrics) over identity labels.
// The ranking list of a query is its gallery positions by ascending distance,
// ties to the lower position (Algorithm 1's list L); its true matches are the
// gallery positions carrying the query's label. AP is the trapezoid area under
// the query's precision-recall curve: the i-th true match (0-based) at list
// position r adds (1/P) * (p_before + p_at) / 2 with p_at = (i+1)/(r+1) and
// p_before = i/r (1 at r = 0); mAP and Recall@K average over the queries that
// have a true match.
#include <limits.h>

#include "common.h"
#include "eval.h"

namespace rr {

constexpr int EV_PPT = 4;              // true matches owned by one thread in a pass
constexpr int EV_PASS = 256 * EV_PPT;  // true matches ranked per pass over the row
constexpr int EV_TILE = 4096;          // distances staged in LDS at a time

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}
__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m, kWave));
  return v;
}

// One workgroup per query; no sort. A true match j is ranked by counting,
// while the row streams through LDS, r_j = #{g : (D_g, g) < (D_j, j)} (its list
// position) and i_j = the same count over true matches (its order among
// them); the thread owning j counts both. Distances must be finite.
__global__ __launch_bounds__(256) void eval_query_kernel(const float* __restrict__ dist, int g, int64_t ld,
                                                         const int32_t* __restrict__ qlab,
                                                         const int32_t* __restrict__ glab, double* __restrict__ ap,
                                                         int32_t* __restrict__ first) {
  __shared__ float dv[EV_TILE];
  __shared__ uint32_t mbits[EV_TILE / 32];
  __shared__ int mpos[EV_PASS];
  __shared__ float mval[EV_PASS];
  __shared__ double term[EV_PASS];
  __shared__ int red[4];
  __shared__ int wcnt[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int qi = blockIdx.x;
  const float* row = dist + (int64_t)qi * ld;
  const int lab = qlab[qi];

  int c0 = 0;
  for (int j = tid; j < g; j += 256) c0 += glab[j] == lab;
  c0 = wave_sum_i32(c0);
  if (lane == 0) red[wave] = c0;
  __syncthreads();
  const int P = red[0] + red[1] + red[2] + red[3];
  if (P == 0) {  // the whole workgroup leaves together
    if (tid == 0) {
      ap[qi] = 0.0;
      first[qi] = -1;
    }
    return;
  }
  const double inv_p = 1.0 / P;
  double apsum = 0.0;  // thread 0: the terms in gallery order of the matches
  int fmin = INT_MAX;
  for (int base = 0; base < P; base += EV_PASS) {
    const int npass = min(EV_PASS, P - base);
    // matches base .. base + npass - 1 (in gallery order) into mpos / mval
    int seen = 0;  // matches in earlier 256-position chunks (uniform)
    for (int c = 0; c < g; c += 256) {
      const int j = c + tid;
      const bool m = j < g && glab[min(j, g - 1)] == lab;
      const uint64_t bal = __ballot(m);
      if (lane == 0) wcnt[wave] = __popcll(bal);
      __syncthreads();
      int before = seen + __popcll(bal & ((1ull << lane) - 1));
      for (int w = 0; w < wave; w++) before += wcnt[w];
      if (m && before >= base && before < base + npass) {
        mpos[before - base] = j;
        mval[before - base] = row[j];
      }
      seen += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
      __syncthreads();
      if (seen >= base + npass) break;
    }
    float mv[EV_PPT];
    int mp[EV_PPT], r[EV_PPT], im[EV_PPT];
    const int mine = min(max(npass - tid * EV_PPT, 0), EV_PPT);
#pragma unroll
    for (int k = 0; k < EV_PPT; k++) {
      mv[k] = k < mine ? mval[tid * EV_PPT + k] : -INFINITY;  // -inf: never preceded by a finite distance
      mp[k] = k < mine ? mpos[tid * EV_PPT + k] : -1;
      r[k] = 0;
      im[k] = 0;
    }
    const bool busy = npass > wave * 64 * EV_PPT;  // this wave owns matches (uniform)
    for (int t0 = 0; t0 < g; t0 += EV_TILE) {
      const int len = min(EV_TILE, g - t0);
      __syncthreads();  // the previous tile is no longer read
      for (int e = tid; e < EV_TILE; e += 256) {
        const bool in = e < len;
        const int ge = t0 + min(e, len - 1);  // clamped: loads stay in the row
        dv[e] = in ? row[ge] : 0.f;
        const uint64_t b = __ballot(in && glab[ge] == lab);  // 64 consecutive positions per wave
        if (lane == 0) {
          mbits[e >> 5] = (uint32_t)b;
          mbits[(e >> 5) + 1] = (uint32_t)(b >> 32);
        }
      }
      __syncthreads();
      if (busy) {
        for (int w = 0; w < (len + 31) / 32; w++) {
          const uint32_t bits = mbits[w];
          const int lim = min(32, len - w * 32);
          for (int u = 0; u < lim; u++) {
            const int e = w * 32 + u;
            const float v = dv[e];
            const int gp = t0 + e;
            const int ism = (bits >> u) & 1;
#pragma unroll
            for (int k = 0; k < EV_PPT; k++) {
              const int pre = (v < mv[k]) | ((v == mv[k]) & (gp < mp[k]));
              r[k] += pre;
              im[k] += pre & ism;
            }
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < EV_PPT; k++)
      if (k < mine) {
        const double pb = r[k] == 0 ? 1.0 : (double)im[k] / (double)r[k];
        const double pa = (double)(im[k] + 1) / (double)(r[k] + 1);
        term[tid * EV_PPT + k] = inv_p * (pb + pa) * 0.5;
        fmin = min(fmin, r[k]);
      }
    __syncthreads();
    if (tid == 0)
      for (int s = 0; s < npass; s++) apsum += term[s];
  }
  fmin = wave_min_i32(fmin);
  __syncthreads();
  if (lane == 0) red[wave] = fmin;
  __syncthreads();
  if (tid == 0) {
    ap[qi] = apsum;
    first[qi] = min(min(red[0], red[1]), min(red[2], red[3]));
  }
}

struct EvalKs {
  int32_t k[kEvalMaxK];
};

// mAP and Recall@K over the queries with a true match: per-thread partials
// over a fixed stride, then summed by one thread in thread order
// (deterministic).
__global__ __launch_bounds__(256) void eval_summary_kernel(const double* __restrict__ ap,
                                                           const int32_t* __restrict__ first, int q, EvalKs ks, int nk,
                                                           double* __restrict__ out) {
  __shared__ double s_ap[256];
  __shared__ int s_n[256];
  __shared__ int s_hit[kEvalMaxK][256];
  const int tid = threadIdx.x;
  double a = 0.0;
  int n = 0;
  int hit[kEvalMaxK];
#pragma unroll
  for (int j = 0; j < kEvalMaxK; j++) hit[j] = 0;
  for (int i = tid; i < q; i += 256) {
    const int f = first[i];
    if (f < 0) continue;
    a += ap[i];
    n++;
#pragma unroll
    for (int j = 0; j < kEvalMaxK; j++) hit[j] += (j < nk) & (f < ks.k[j]);
  }
  s_ap[tid] = a;
  s_n[tid] = n;
#pragma unroll
  for (int j = 0; j < kEvalMaxK; j++) s_hit[j][tid] = hit[j];
  __syncthreads();
  if (tid == 0) {
    double sa = 0.0;
    long long sn = 0;
    for (int t = 0; t < 256; t++) {
      sa += s_ap[t];
      sn += s_n[t];
    }
    out[0] = sn ? sa / (double)sn : 0.0;
    for (int j = 0; j < nk; j++) {
      long long h = 0;
      for (int t = 0; t < 256; t++) h += s_hit[j][t];
      out[1 + j] = sn ? (double)h / (double)sn : 0.0;
    }
    out[nk + 1] = (double)sn;
  }
}

hipError_t launch_evaluate(const float* dist, int q, int g, int64_t ld, const int32_t* qlab, const int32_t* glab,
                           const int32_t* ks, int nk, double* ap, int32_t* first, double* summary, hipStream_t s) {
  if (q < 1 || g < 1 || ld < g || nk < 1 || nk > kEvalMaxK) return hipErrorInvalidValue;
  EvalKs k{};
  for (int j = 0; j < nk; j++) k.k[j] = ks[j];
  hipLaunchKernelGGL(eval_query_kernel, dim3((unsigned)q), dim3(256), 0, s, dist, g, ld, qlab, glab, ap, first);
  hipLaunchKernelGGL(eval_summary_kernel, dim3(1), dim3(256), 0, s, (const double*)ap, (const int32_t*)first, q, k, nk,
                     summary);
  return hipGetLastError();
}

}  // namespace rr
