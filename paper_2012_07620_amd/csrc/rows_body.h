// Per-work-item bodies of the row-parallel kernels (a1, a3, a3b, a4, a6),
// shared by the direct launches and the persistent grouped launches.
#pragma once
#include "../../include/rerank.h"
#include "common.h"
#include "kernels.h"

// Every multiply-add below is written out (explicit FMA or separate
// operations) so that the direct and grouped launches, and the dense and
// sparse first layer, round identically.
#pragma clang fp contract(off)

namespace rr {

// ============================================================== a1: prep
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

// One wavefront per row: exact FP32 copy (zero-padded to ldp), 1/|x_i| from a
// compensated sum of squares with correctly rounded sqrt and division, and the
// low-precision copy with its row scale.
template <SimPrec P, bool IN_BF16>
__device__ __forceinline__ void prep_row(const void* __restrict__ x, int i, int d, float* __restrict__ xp,
                                         int64_t ldp, float* __restrict__ rn, void* __restrict__ xl, int64_t ldl,
                                         float* __restrict__ sl) {
  const int lane = threadIdx.x & 63;
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

// ============================================================== a3: top-k
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
// ASC (the ranking list of Algorithm 1): the K smallest values of the row,
// ties to the lower column, no forced self member; oval may be null.
template <int R, bool ASC = false>
__device__ __forceinline__ void topk_row(const float* __restrict__ S, int64_t ldS, int N, int i, int K,
                                         int32_t* __restrict__ oidx, float* __restrict__ oval, int ldo,
                                         uint64_t* ring) {
  const int lane = threadIdx.x & 63;
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
      if (!ASC) {  // S rows: 256-byte aligned, padded to a multiple of 64 columns
        v[u] = (col < N) ? *(const f32x4*)(srow + col) : f32x4{0.f, 0.f, 0.f, 0.f};
      } else {  // caller's distance rows: any stride, no padding
#pragma unroll
        for (int e = 0; e < 4; e++) v[u][e] = (col + e < N) ? srow[col + e] : 0.f;
      }
    }
    uint64_t lm = 0;
    if (c0 == 0) {
#pragma unroll
      for (int u = 0; u < U; u++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int col = u * 256 + lane * 4 + e;
          if (col < N)
            lm = umax64(lm, ASC ? sel_key(-v[u][e], (uint32_t)col)
                                : (col == i ? self_key(i) : sel_key(v[u][e], (uint32_t)col)));
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
        if (col < N)
          key = ASC ? sel_key(-v[u][e], (uint32_t)col) : ((col == i) ? self_key(i) : sel_key(v[u][e], (uint32_t)col));
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
      if (ASC) {
        if (oval) oval[(int64_t)i * ldo + e] = -key_val(best[r]);
      } else {
        oval[(int64_t)i * ldo + e] = (j == (uint32_t)i) ? 1.0f : key_val(best[r]);
      }
    }
  }
}

// ============================================================== a3b: re-score
// Candidates of row i re-scored as cos(x_i, x_j) with a compensated FP32 dot
// product (error about one rounding of the result, far below the spacing of
// distinct similarities the tie rule has to resolve), then sorted under
// (similarity desc, column asc) with the row itself first; the first k1 are
// N(i, k1) of Eq. 8. One wavefront per row; 16 lanes per candidate, four
// candidates at a time.
template <int R>
__device__ __forceinline__ void rescore_row(const float* __restrict__ xp, int64_t ldp, const float* __restrict__ rn,
                                            int i, const int32_t* __restrict__ cand, int Kc, int k1,
                                            int32_t* __restrict__ kidx, float* __restrict__ kval) {
  const int lane = threadIdx.x & 63;
  const int sub = lane >> 4, sl = lane & 15;
  const float* xi = xp + (int64_t)i * ldp;
  const float rni = rn[i];
  uint64_t keys[R];
#pragma unroll
  for (int r = 0; r < R; r++) keys[r] = 0;
  for (int c0 = 0; c0 < Kc; c0 += 4) {
    const int c = c0 + sub;
    const int j = (c < Kc) ? cand[(int64_t)i * Kc + c] : i;
    DF acc{0.f, 0.f};
    if (j != i) {
      const float* xj = xp + (int64_t)j * ldp;
      for (int k = sl * 4; k < ldp; k += 64) {
        const f32x4 a = *(const f32x4*)(xi + k);
        const f32x4 b = *(const f32x4*)(xj + k);
        dot2_acc(acc, a.x, b.x);
        dot2_acc(acc, a.y, b.y);
        dot2_acc(acc, a.z, b.z);
        dot2_acc(acc, a.w, b.w);
      }
    }
#pragma unroll
    for (int m = 8; m > 0; m >>= 1) {
      DF o{__shfl_xor(acc.hi, m, kWave), __shfl_xor(acc.lo, m, kWave)};
      acc = df_add(acc, o);
    }
    const float dot = acc.hi + acc.lo;
    const uint64_t key = (j == i) ? self_key((uint32_t)i) : sel_key((dot * rni) * rn[j], (uint32_t)j);
    // candidate c0 + s is held by lane (c0 + s) % 64 of slot (c0 + s) / 64
#pragma unroll
    for (int s = 0; s < 4; s++) {
      const uint64_t ks = shfl_u64(key, s * 16);
      const int cs = c0 + s;
      if (cs < Kc) {
#pragma unroll
        for (int r = 0; r < R; r++)
          if ((cs >> 6) == r && lane == (cs & 63)) keys[r] = ks;
      }
    }
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

// ============================================================== a4: A*
// Zero a float range: 8 float4 per thread per item (one item = 8192 floats).
constexpr int FILL_ITEM = 256 * 4 * 8;
__device__ __forceinline__ void fill_item(float* __restrict__ p, int64_t count, int64_t item) {
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
  const int64_t base = item * FILL_ITEM;
#pragma unroll
  for (int u = 0; u < 8; u++) {
    const int64_t at = base + (int64_t)(u * 256 + threadIdx.x) * 4;
    if (at + 3 < count) {
      *(f32x4*)(p + at) = z;
    } else {
      for (int e = 0; e < 4; e++)
        if (at + e < count) p[at + e] = 0.f;
    }
  }
}

// H[i][j] = H[j][i] = A*_ij for every j in N(i, k1): 1 when i is also in
// N(j, k1), else 1/2 (Eq. 10). When both directions exist both writers store
// the same value, so plain stores suffice. cnt[0..n) counts in-degrees,
// cnt[n..2n) mutual pairs per row.
// sym = false (vertex features = rows of A, Eq. 8): H[i][j] = 1 only.
__device__ __forceinline__ void scatter_pair(const int32_t* __restrict__ knn, int n, int k1, float* __restrict__ H,
                                             int64_t ldH, int32_t* __restrict__ cnt, int64_t t, bool sym = true) {
  if (t >= (int64_t)n * k1) return;
  const int i = (int)(t / k1);
  const int j = knn[t];
  if (!sym) {
    H[(int64_t)i * ldH + j] = 1.0f;
    return;
  }
  const int32_t* lj = knn + (int64_t)j * k1;
  bool mut = false;
  for (int s = 0; s < k1; s++) mut |= (lj[s] == i);
  const float v = mut ? 1.0f : 0.5f;
  H[(int64_t)i * ldH + j] = v;
  H[(int64_t)j * ldH + i] = v;
  atomicAdd(cnt + j, 1);
  if (mut) atomicAdd(cnt + n + i, 1);
}

// |A*_i|^2 = (#mutual) * 1 + (#one-way) * 1/4, one-way = out-only + in-only.
// sym = false: every A row holds k1 ones, |A_i| = sqrt(k1).
__device__ __forceinline__ void astar_sigma_row(const int32_t* __restrict__ cnt, int n, int k1, float* __restrict__ sigma,
                                                int i, bool sym = true) {
  if (i >= n) return;
  if (!sym) {
    sigma[i] = __fdiv_rn(1.0f, __fsqrt_rn((float)k1));
    return;
  }
  const int m = cnt[n + i];
  const float sq = (float)m + 0.25f * (float)(k1 - m + cnt[i] - m);
  sigma[i] = __fdiv_rn(1.0f, __fsqrt_rn(sq));
}

// ============================================================== a5 + a6
// One workgroup per output row: gather the row itself and its k2 - 1 other
// edge rows (Eq. 12: the first k2 members of N(i, k1), member 0 = i), sum
// with weights (Eq. 14, sum aggregator), reduce the squared norm. Rows are
// kept unnormalised and the norm is carried as sigma = 1/|u| (the next layer
// and the final product fold it in), so each layer is one streaming pass.
struct PropShared {
  int nb[256];
  float cf[256];   // per-member coefficient (sum/mean: residual folded into member 0; max: message only)
  float res;       // max aggregator: residual coefficient of the row itself
  float red[4];
};

__device__ __forceinline__ float sq_acc4(float ss, f32x4 a) {
  ss = __builtin_fmaf(a.x, a.x, ss);
  ss = __builtin_fmaf(a.y, a.y, ss);
  ss = __builtin_fmaf(a.z, a.z, ss);
  return __builtin_fmaf(a.w, a.w, ss);
}

__device__ __forceinline__ void split_store4(uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int64_t at,
                                             f32x4 acc) {
  uint16_t h4[4], l4[4];
#pragma unroll
  for (int e = 0; e < 4; e++) {
    h4[e] = bf16_rne(acc[e]);
    l4[e] = bf16_rne(acc[e] - __uint_as_float((uint32_t)h4[e] << 16));
  }
  *(uint2*)(hi + at) = make_uint2(h4[0] | ((uint32_t)h4[1] << 16), h4[2] | ((uint32_t)h4[3] << 16));
  *(uint2*)(lo + at) = make_uint2(l4[0] | ((uint32_t)l4[1] << 16), l4[2] | ((uint32_t)l4[3] << 16));
}

// Coefficients of row i. Message r is e_ir^alpha h_{j_r} (member 0 is the row
// itself with e_ii = 1), each times the carried 1/|u_j| of its input row.
// sum: member 0 also takes the residual h_i; mean: messages scaled by 1/k2,
// residual added to member 0; max: messages kept apart, residual in res.
__device__ __forceinline__ void load_coefs(const float* __restrict__ sin, const int32_t* __restrict__ knn,
                                           const float* __restrict__ kv, int k1, int k2, int alpha, int agg, int i,
                                           PropShared& sh) {
  const int tid = threadIdx.x;
  if (tid < k2) {
    const int j = knn[(int64_t)i * k1 + tid];
    float w = 1.0f;
    if (tid > 0) {
      const float e = kv[(int64_t)i * k1 + tid];
      for (int a = 0; a < alpha; a++) w *= e;
    }
    const float sj = sin ? sin[j] : 1.0f;
    const float msg = w * sj;
    float c = msg;
    if (agg == RERANK_AGG_MEAN) c = msg / (float)k2;
    if (tid == 0) {
      if (agg == RERANK_AGG_MAX)
        sh.res = sj;
      else
        c = sj + c;  // residual + own message (sum: exactly 2 * sj)
    }
    sh.cf[tid] = c;
    sh.nb[tid] = j;
  }
  __syncthreads();
}

__device__ __forceinline__ void finish_norm(float ss, float* __restrict__ sout, int i, PropShared& sh) {
  const int tid = threadIdx.x;
  ss = wave_sum_f32(ss);
  if ((tid & 63) == 0) sh.red[tid >> 6] = ss;
  __syncthreads();
  if (tid == 0) {
    const float t = (sh.red[0] + sh.red[1]) + (sh.red[2] + sh.red[3]);
    sout[i] = __fdiv_rn(1.0f, __fsqrt_rn(t));
  }
  __syncthreads();  // sh is reused by the next row of a persistent workgroup
}

// One workgroup per output row: gather the row itself and its k2 - 1 other
// edge rows (Eq. 12: the first k2 members of N(i, k1), member 0 = i), sum
// with weights (Eq. 14, sum aggregator), reduce the squared norm. Rows are
// kept unnormalised and the norm is carried as sigma = 1/|u| (the next layer
// and the final product fold it in), so each layer is one streaming pass.
// Thread t owns float4 columns t, t + 256, ... (the sparse first layer below
// uses the same order, so both give identical sums).
__device__ __forceinline__ void propagate_row(const float* __restrict__ hin, const float* __restrict__ sin,
                                              int64_t ld, int64_t cols, const int32_t* __restrict__ knn,
                                              const float* __restrict__ kv, int k1, int k2, int alpha, int agg,
                                              float* __restrict__ hout, float* __restrict__ sout,
                                              uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int i,
                                              PropShared& sh) {
  const int tid = threadIdx.x;
  load_coefs(sin, knn, kv, k1, k2, alpha, agg, i, sh);
  float ss = 0.f;
  const int64_t c4 = cols >> 2;
  for (int64_t c = tid; c < c4; c += 256) {
    const f32x4 v0 = ((const f32x4*)(hin + (int64_t)sh.nb[0] * ld))[c];
    const float c0 = sh.cf[0];
    f32x4 acc = {c0 * v0.x, c0 * v0.y, c0 * v0.z, c0 * v0.w};
    if (agg == RERANK_AGG_MAX) {
      for (int r = 1; r < k2; r++) {
        const f32x4 v = ((const f32x4*)(hin + (int64_t)sh.nb[r] * ld))[c];
        const float w = sh.cf[r];
        acc = f32x4{fmaxf(acc.x, w * v.x), fmaxf(acc.y, w * v.y), fmaxf(acc.z, w * v.z), fmaxf(acc.w, w * v.w)};
      }
      const float rs = sh.res;
      acc = f32x4{__builtin_fmaf(rs, v0.x, acc.x), __builtin_fmaf(rs, v0.y, acc.y), __builtin_fmaf(rs, v0.z, acc.z),
                  __builtin_fmaf(rs, v0.w, acc.w)};
    } else {
      for (int r = 1; r < k2; r++) {
        const f32x4 v = ((const f32x4*)(hin + (int64_t)sh.nb[r] * ld))[c];
        const float w = sh.cf[r];
        acc = f32x4{__builtin_fmaf(w, v.x, acc.x), __builtin_fmaf(w, v.y, acc.y), __builtin_fmaf(w, v.z, acc.z),
                    __builtin_fmaf(w, v.w, acc.w)};
      }
    }
    if (hi)
      split_store4(hi, lo, (int64_t)i * ld + c * 4, acc);
    else
      ((f32x4*)(hout + (int64_t)i * ld))[c] = acc;
    ss = sq_acc4(ss, acc);
  }
  finish_norm(ss, sout, i, sh);
}

// ---------------------------------------------------------------- sparse A*
// A* row j has its out-list N(j, k1) (value 1 when mutual, else 1/2) and its
// non-mutual in-edges (rows m with j in N(m, k1) but m not in N(j, k1), value
// 1/2). mflag[m][r] marks whether the pair (m, N(m,k1)[r]) is mutual; the
// non-mutual in-edges of every row are gathered into a CSR transpose.

// Mutual flag of pair t = (m, r), and the non-mutual in-degree count.
__device__ __forceinline__ void mutual_pair(const int32_t* __restrict__ knn, int n, int k1, uint8_t* __restrict__ mflag,
                                            int32_t* __restrict__ innm, int64_t t) {
  if (t >= (int64_t)n * k1) return;
  const int m = (int)(t / k1);
  const int j = knn[t];
  const int32_t* lj = knn + (int64_t)j * k1;
  bool mut = false;
  for (int s = 0; s < k1; s++) mut |= (lj[s] == m);
  mflag[t] = mut ? 1 : 0;
  if (!mut) atomicAdd(innm + j, 1);
}

// Exclusive prefix sum of innm[0..n) into off[0..n], one 256-thread workgroup.
__device__ __forceinline__ void scan_offsets(const int32_t* __restrict__ innm, int n, int32_t* __restrict__ off,
                                             int32_t* sh /* 256 ints */) {
  const int tid = threadIdx.x;
  const int per = (n + 255) / 256;
  const int b = tid * per, e = min(n, b + per);
  int sum = 0;
  for (int k = b; k < e; k++) sum += innm[k];
  sh[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int v = tid >= o ? sh[tid - o] : 0;
    __syncthreads();
    sh[tid] += v;
    __syncthreads();
  }
  int run = sh[tid] - sum;
  for (int k = b; k < e; k++) {
    off[k] = run;
    run += innm[k];
  }
  if (tid == 255) off[n] = sh[255];
  __syncthreads();
}

// Place the non-mutual in-edge (m -> j) of pair t into j's CSR segment.
__device__ __forceinline__ void csr_pair(const int32_t* __restrict__ knn, int n, int k1,
                                         const uint8_t* __restrict__ mflag, const int32_t* __restrict__ off,
                                         int32_t* __restrict__ cursor, int32_t* __restrict__ inl, int64_t t) {
  if (t >= (int64_t)n * k1 || mflag[t]) return;
  const int j = knn[t];
  const int pos = atomicAdd(cursor + j, 1);
  inl[off[j] + pos] = (int)(t / k1);
}

// First layer without a dense h^(0): u_i = sum_r c_r A*_{j_r}, built in LDS
// one column chunk at a time from the sparse A* rows, in member order r, with
// the same FMA sequence and per-thread column order as propagate_row on a
// dense A* (so the result is identical), then written once.
constexpr int FIRST_CHUNK = 8192;  // floats of the output row held in LDS
constexpr int FIRST_ENTRIES = 2048; // sparse A* entries of one row staged in LDS
struct FirstShared {
  PropShared p;
  float row[FIRST_CHUNK];
  int col[FIRST_ENTRIES];
  float val[FIRST_ENTRIES];
  int start[257];  // entries of member r are [start[r], start[r+1])
  int wsum[4];     // per-wave counts of a CSR store step
  int obase;       // first entry of the row's CSR slot
};

// ---------------------------------------------------------------- CSR rows
// Sparse-layer output: decide dense or CSR for this layer (the same answer in
// every workgroup: it reads only gates written by earlier launches), mark the
// gate from workgroup 0, and take this row's slot of min(n, bound) entries.
// Returns true for CSR output; *pos is the slot's first entry.
__device__ __forceinline__ bool sl_begin(const SlOut* o, int bound, int i, FirstShared& sh, int* pos) {
  if (!o) return false;
  const unsigned long long total = o->gate->total;
  const bool dense = o->prev->dense != 0 || total > (unsigned long long)o->cap || total > 0x7FFFFFFFull;
  if (threadIdx.x == 0) {
    if (i == 0) o->gate->dense = dense ? 1 : 0;
    if (!dense) sh.obase = atomicAdd(&o->gate->cursor, min(bound, o->n));
  }
  __syncthreads();
  *pos = sh.obase;
  return !dense;
}

// Append the non-zeros of the LDS chunk row[0, width) (columns c0 + k) to the
// row's CSR slot at *pos, columns ascending, and add their squares to ss in
// the same per-thread order as the dense store (thread t owns float4 columns
// t, t + 256, ...). Every thread ends with the same *pos.
__device__ __forceinline__ void store_chunk_csr(const float* row, int width, int64_t c0, const SlRows& out, int* pos,
                                                FirstShared& sh, float* ss) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int w4 = width >> 2;
  for (int cb = 0; cb < w4; cb += 256) {
    const int c = cb + tid;
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (c < w4) {
      v = ((const f32x4*)row)[c];
      *ss = sq_acc4(*ss, v);
    }
    const int mine = (v.x != 0.f) + (v.y != 0.f) + (v.z != 0.f) + (v.w != 0.f);
    int incl = mine;  // inclusive prefix over the wave
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, kWave);
      if (lane >= o) incl += t;
    }
    if (lane == 63) sh.wsum[w] = incl;
    __syncthreads();
    int before = 0, total = 0;
    for (int x = 0; x < 4; x++) {
      before += (x < w) ? sh.wsum[x] : 0;
      total += sh.wsum[x];
    }
    int at = *pos + before + incl - mine;
    const float e4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; e++)
      if (e4[e] != 0.f) {
        out.col[at] = (int32_t)(c0 + (int64_t)c * 4 + e);
        out.val[at] = e4[e];
        at++;
      }
    *pos += total;
    __syncthreads();  // wsum is rewritten by the next step
  }
}

// sym = false: h^(0) = rows of A (out-list entries only, value 1). The
// aggregator is sum or mean (max runs the dense layer).
__device__ __forceinline__ void first_layer_row(const int32_t* __restrict__ knn, const float* __restrict__ kv,
                                                const uint8_t* __restrict__ mflag, const int32_t* __restrict__ off,
                                                const int32_t* __restrict__ inl, int k1, int k2, int alpha, int agg,
                                                bool sym, int64_t ld, float* __restrict__ hout,
                                                float* __restrict__ sout, uint16_t* __restrict__ hi,
                                                uint16_t* __restrict__ lo, int i, FirstShared& sh,
                                                const SlOut* sl = nullptr) {
  const int tid = threadIdx.x;
  load_coefs(nullptr, knn, kv, k1, k2, alpha, agg, i, sh.p);
  // entry counts per member: out-list (k1) + non-mutual in-list (A* only)
  if (tid == 0) {
    int acc = 0;
    for (int r = 0; r < k2; r++) {
      sh.start[r] = acc;
      const int j = sh.p.nb[r];
      acc += k1 + (sym ? off[j + 1] - off[j] : 0);
    }
    sh.start[k2] = acc;
  }
  __syncthreads();
  const bool staged = sh.start[k2] <= FIRST_ENTRIES;
  if (staged) {
    for (int r = 0; r < k2; r++) {
      const int j = sh.p.nb[r];
      const int base = sh.start[r];
      const int32_t* lj = knn + (int64_t)j * k1;
      const uint8_t* fj = sym ? mflag + (int64_t)j * k1 : nullptr;
      for (int s = tid; s < k1; s += 256) {
        sh.col[base + s] = lj[s];
        sh.val[base + s] = (!sym || fj[s]) ? 1.0f : 0.5f;
      }
      const int b = sym ? off[j] : 0, n_in = sym ? off[j + 1] - b : 0;
      for (int s = tid; s < n_in; s += 256) {
        sh.col[base + k1 + s] = inl[b + s];
        sh.val[base + k1 + s] = 0.5f;
      }
    }
  }
  __syncthreads();
  int pos = 0;
  const bool csr = sl_begin(sl, sh.start[k2], i, sh, &pos);
  const int pos0 = pos;
  float ss = 0.f;
  for (int64_t c0 = 0; c0 < ld; c0 += FIRST_CHUNK) {
    const int width = (int)min((int64_t)FIRST_CHUNK, ld - c0);
    for (int k = tid; k < FIRST_CHUNK; k += 256) sh.row[k] = 0.f;
    __syncthreads();
    for (int r = 0; r < k2; r++) {
      const float c = sh.p.cf[r];
      if (staged) {
        for (int s = sh.start[r] + tid; s < sh.start[r + 1]; s += 256) {
          const int64_t m = sh.col[s] - c0;
          if (m >= 0 && m < width) sh.row[m] = __builtin_fmaf(c, sh.val[s], sh.row[m]);
        }
      } else {  // very large in-degree: read the entries from memory
        const int j = sh.p.nb[r];
        const int32_t* lj = knn + (int64_t)j * k1;
        const uint8_t* fj = sym ? mflag + (int64_t)j * k1 : nullptr;
        for (int s = tid; s < k1; s += 256) {
          const int64_t m = lj[s] - c0;
          if (m >= 0 && m < width) sh.row[m] = __builtin_fmaf(c, (!sym || fj[s]) ? 1.0f : 0.5f, sh.row[m]);
        }
        const int b = sym ? off[j] : 0, e = sym ? off[j + 1] : 0;
        for (int s = b + tid; s < e; s += 256) {
          const int64_t m = inl[s] - c0;
          if (m >= 0 && m < width) sh.row[m] = __builtin_fmaf(c, 0.5f, sh.row[m]);
        }
      }
      __syncthreads();
    }
    if (csr) {
      store_chunk_csr(sh.row, width, c0, sl->rows, &pos, sh, &ss);
    } else {
      const int w4 = width >> 2;
      for (int c = tid; c < w4; c += 256) {
        const f32x4 acc = ((const f32x4*)sh.row)[c];
        if (hi)
          split_store4(hi, lo, (int64_t)i * ld + c0 + c * 4, acc);
        else
          ((f32x4*)(hout + (int64_t)i * ld + c0))[c] = acc;
        ss = sq_acc4(ss, acc);
      }
    }
    __syncthreads();
  }
  if (csr && tid == 0) {
    sl->rows.so[i] = pos0;
    sl->rows.cnt[i] = pos - pos0;
  }
  finish_norm(ss, sout, i, sh.p);
}

// Layer l >= 2 of the sparse layers: u_i = sum_r c_r h_{j_r} from the CSR
// rows of layer l - 1 (coefficients from load_coefs with their carried
// 1/|u_j|), built in LDS column chunks in member order r with one FMA per
// entry: the same sums, rounding for rounding, as propagate_row on the dense
// rows (a zero entry there is an FMA that leaves the sum unchanged).
// Sum and mean aggregators.
__device__ __forceinline__ void sparse_prop_row(const SlRows& in, const float* __restrict__ sin,
                                                const int32_t* __restrict__ knn, const float* __restrict__ kv,
                                                int k1, int k2, int alpha, int agg, int64_t ld,
                                                float* __restrict__ hout, float* __restrict__ sout, const SlOut* sl,
                                                int i, FirstShared& sh) {
  const int tid = threadIdx.x;
  load_coefs(sin, knn, kv, k1, k2, alpha, agg, i, sh.p);
  if (tid == 0) {
    int acc = 0;
    for (int r = 0; r < k2; r++) {
      sh.start[r] = acc;
      acc += in.cnt[sh.p.nb[r]];
    }
    sh.start[k2] = acc;
  }
  __syncthreads();
  const bool staged = sh.start[k2] <= FIRST_ENTRIES;
  if (staged) {
    for (int r = 0; r < k2; r++) {
      const int j = sh.p.nb[r];
      const int b = in.so[j], base = sh.start[r], len = sh.start[r + 1] - base;
      for (int s = tid; s < len; s += 256) {
        sh.col[base + s] = in.col[b + s];
        sh.val[base + s] = in.val[b + s];
      }
    }
  }
  __syncthreads();
  int pos = 0;
  const bool csr = sl_begin(sl, sh.start[k2], i, sh, &pos);
  const int pos0 = pos;
  float ss = 0.f;
  for (int64_t c0 = 0; c0 < ld; c0 += FIRST_CHUNK) {
    const int width = (int)min((int64_t)FIRST_CHUNK, ld - c0);
    for (int k = tid; k < FIRST_CHUNK; k += 256) sh.row[k] = 0.f;
    __syncthreads();
    for (int r = 0; r < k2; r++) {
      const float c = sh.p.cf[r];
      if (staged) {
        for (int s = sh.start[r] + tid; s < sh.start[r + 1]; s += 256) {
          const int64_t m = sh.col[s] - c0;
          if (m >= 0 && m < width) sh.row[m] = __builtin_fmaf(c, sh.val[s], sh.row[m]);
        }
      } else {
        const int j = sh.p.nb[r];
        const int b = in.so[j], e = b + in.cnt[j];
        for (int s = b + tid; s < e; s += 256) {
          const int64_t m = in.col[s] - c0;
          if (m >= 0 && m < width) sh.row[m] = __builtin_fmaf(c, in.val[s], sh.row[m]);
        }
      }
      __syncthreads();
    }
    if (csr) {
      store_chunk_csr(sh.row, width, c0, sl->rows, &pos, sh, &ss);
    } else {
      const int w4 = width >> 2;
      for (int c = tid; c < w4; c += 256) {
        const f32x4 acc = ((const f32x4*)sh.row)[c];
        ((f32x4*)(hout + (int64_t)i * ld + c0))[c] = acc;
        ss = sq_acc4(ss, acc);
      }
    }
    __syncthreads();
  }
  if (csr && tid == 0) {
    sl->rows.so[i] = pos0;
    sl->rows.cnt[i] = pos - pos0;
  }
  finish_norm(ss, sout, i, sh.p);
}

}  // namespace rr
