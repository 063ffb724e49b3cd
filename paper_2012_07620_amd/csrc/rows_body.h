// Per-work-item bodies of the row-parallel kernels (a1, a3, a3b, a4, a6),
// shared by the direct launches and the persistent grouped launches.
#pragma once
#include <type_traits>
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

// One wavefront per row: exact FP32 copy (zero-padded to ldp; not written
// when xp is null, where the caller's FP32 rows are used in place), 1/|x_i|
// from a compensated sum of squares with correctly rounded sqrt and division,
// and the low-precision copy with its row scale. A row of a multiple of 4
// elements on an aligned input moves 4 elements per lane and access (16-byte
// FP32, 8-byte bf16 loads); any other row one element. The choice depends
// only on d and the input address, so every launch of a problem makes the
// same one.
template <SimPrec P, bool IN_BF16>
__device__ __forceinline__ void prep_row(const void* __restrict__ x, int i, int d, float* __restrict__ xp,
                                         int64_t ldp, float* __restrict__ rn, void* __restrict__ xl, int64_t ldl,
                                         float* __restrict__ sl) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  const int lane = threadIdx.x & 63;
  const int64_t src = (int64_t)i * d;
  const float* xf = (const float*)x + src;
  const uint16_t* xh = (const uint16_t*)x + src;
  float* xr = xp ? xp + (int64_t)i * ldp : nullptr;
  const bool vec = (d & 3) == 0 && ((uintptr_t)x & (IN_BF16 ? 7u : 15u)) == 0;
  auto in1 = [&](int k) -> float { return IN_BF16 ? __uint_as_float((uint32_t)xh[k] << 16) : xf[k]; };
  auto in4 = [&](int k) -> f32x4 {  // elements k .. k + 3, k < d, d a multiple of 4
    if (IN_BF16) {
      const u32x2 b = *(const u32x2*)(xh + k);
      return f32x4{__uint_as_float(b.x << 16), __uint_as_float(b.x & 0xFFFF0000u), __uint_as_float(b.y << 16),
                   __uint_as_float(b.y & 0xFFFF0000u)};
    }
    return *(const f32x4*)(xf + k);
  };
  DF acc{0.f, 0.f};
  float amax = 0.f;
  uint16_t* xb = P == SimPrec::BF16 ? (uint16_t*)xl + (int64_t)i * ldl : nullptr;
  uint8_t* xq = P == SimPrec::FP8 ? (uint8_t*)xl + (int64_t)i * ldl : nullptr;
  // FP8 quantises after the row maximum is known, so it reads the row twice;
  // its first KEEP steps stay in registers (d <= 2048 without a second read)
  constexpr int KEEP = P == SimPrec::FP8 ? 8 : 1;
  f32x4 keep[KEEP];
  if (vec) {
    // one step of the first pass: copy, sum of squares, maximum, and the
    // bfloat16 copy (its rows are padded like the FP32 ones)
    auto step = [&](int k) -> f32x4 {
      const f32x4 v = k < d ? in4(k) : f32x4{0.f, 0.f, 0.f, 0.f};
      if (k < ldp) {
        if (xr) *(f32x4*)(xr + k) = v;
#pragma unroll
        for (int e = 0; e < 4; e++) {
          dot2_acc(acc, v[e], v[e]);
          amax = fmaxf(amax, fabsf(v[e]));
        }
      }
      if (P == SimPrec::BF16 && k < ldl) {
        u32x2 o = {0u, 0u};
        if (k < d) {
          if (IN_BF16) {
            o = *(const u32x2*)(xh + k);
          } else {
            o.x = (uint32_t)bf16_rne(v[0]) | ((uint32_t)bf16_rne(v[1]) << 16);
            o.y = (uint32_t)bf16_rne(v[2]) | ((uint32_t)bf16_rne(v[3]) << 16);
          }
        }
        *(u32x2*)(xb + k) = o;
      }
      return v;
    };
    const int kend = ldp > ldl ? (int)ldp : (int)ldl;
#pragma unroll
    for (int j = 0; j < KEEP; j++) keep[j] = step(4 * lane + 256 * j);
    for (int k = 4 * lane + 256 * KEEP; k < kend; k += 256) step(k);
  } else {
    for (int k = lane; k < ldp; k += 64) {
      const float v = k < d ? in1(k) : 0.f;
      if (xr) xr[k] = v;
      dot2_acc(acc, v, v);
      amax = fmaxf(amax, fabsf(v));
    }
    if (P == SimPrec::BF16)
      for (int k = lane; k < ldl; k += 64) xb[k] = k < d ? (IN_BF16 ? xh[k] : bf16_rne(xf[k])) : (uint16_t)0;
  }
  acc = wave_sum_df(acc);
  const float n2 = acc.hi + acc.lo;
  const float r = __fdiv_rn(1.0f, __fsqrt_rn(n2));
  if (P == SimPrec::BF16) {
    if (lane == 0) sl[i] = r;
  } else if (P == SimPrec::FP8) {
    amax = wave_max_f32(amax);
    const float scale = amax > 0.f ? amax / 448.0f : 1.0f;
    const float inv = amax > 0.f ? 448.0f / amax : 1.0f;
    if (vec) {
      auto put = [&](int k, const f32x4& v) {
        if (k < ldl) {
          uint32_t o = 0u;
#pragma unroll
          for (int e = 0; e < 4; e++) o |= e4m3_rne_sat(v[e] * inv) << (8 * e);  // v = 0 past d: code 0
          *(uint32_t*)(xq + k) = o;
        }
      };
#pragma unroll
      for (int j = 0; j < KEEP; j++) put(4 * lane + 256 * j, keep[j]);
      for (int k = 4 * lane + 256 * KEEP; k < ldl; k += 256) put(k, k < d ? in4(k) : f32x4{0.f, 0.f, 0.f, 0.f});
    } else {
      for (int k = lane; k < ldl; k += 64) xq[k] = (uint8_t)(k < d ? e4m3_rne_sat(in1(k) * inv) : 0u);
    }
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
template <int R, bool ASC = false, typename T = float>
__device__ __forceinline__ void topk_row(const T* __restrict__ S, int64_t ldS, int N, int i, int K,
                                         int32_t* __restrict__ oidx, float* __restrict__ oval, int ldo,
                                         uint64_t* ring) {
  static_assert(!ASC || sizeof(T) == 4, "distance rows are FP32");
  const int lane = threadIdx.x & 63;
  const T* srow = S + (int64_t)i * ldS;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;

  uint64_t best[R];
#pragma unroll
  for (int r = 0; r < R; r++) best[r] = 0;
  uint64_t tau = 0;
  float tf = -INFINITY;  // value of tau's key (all values pass while tau is 0)
  int head = 0, cnt = 0;

  constexpr int U = 4;
  constexpr int CH = 64 * 4 * U;
  // chunk c0 into registers (zeros past N); the next chunk is loaded while
  // the current one is processed
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  typedef typename std::conditional<!ASC && sizeof(T) == 2, h4, f32x4>::type raw4;
  auto load = [&](int c0, raw4 (&r)[U]) {
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int col = c0 + u * 256 + lane * 4;
      if constexpr (!ASC) {  // S rows (FP32 or binary16): 256-byte aligned, padded to a multiple of 64 columns
        r[u] = (col < N) ? *(const raw4*)(srow + col) : raw4{0, 0, 0, 0};
      } else {  // caller's distance rows: any stride, no padding
#pragma unroll
        for (int e = 0; e < 4; e++) r[u][e] = (col + e < N) ? srow[col + e] : 0.f;
      }
    }
  };
  raw4 nxt[U];
  load(0, nxt);
  for (int c0 = 0; c0 < N; c0 += CH) {
    f32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      if constexpr (!ASC && sizeof(T) == 2) {
        v[u] = f32x4{(float)nxt[u].x, (float)nxt[u].y, (float)nxt[u].z, (float)nxt[u].w};
      } else {
        v[u] = nxt[u];
      }
    }
    if (c0 + CH < N) load(c0 + CH, nxt);
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
      tf = tau ? key_val(tau) : -INFINITY;
    }
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int col = c0 + u * 256 + lane * 4 + e;
        // a key above tau has a value of at least tau's (or is the row's own
        // column): full keys are built only when some lane has such a value.
        // Written as "not below" so that a NaN, which the key orders by its
        // bits, still reaches the key comparison and a row of NaN values
        // fills its K slots.
        const float sv = ASC ? -v[u][e] : v[u][e];
        const bool cand = col < N && (!(sv < tf) || (!ASC && col == i));
        if (!__ballot(cand)) continue;
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
            tf = tau ? key_val(tau) : -INFINITY;
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

// a3 with block maxima. bmrow[b] holds the largest stored similarity of row
// i in column block b (128 columns; the launch stages the four rows of a
// workgroup in LDS from bm[b * ldbm + i]). The row itself ranks first, so
// K - 1 other members are needed; blocks are disjoint, so any K - 1 blocks'
// maxima are K - 1 distinct elements of the row, and the (K - 1)-th largest of
// any set of non-diagonal block maxima is at or below the value of the row's
// K-th member. The wave takes that bound t0 over each lane's largest
// non-diagonal block maximum (a 64-entry sort), lists the blocks whose
// maximum reaches t0 (and the diagonal block) in LDS, and reads only those,
// four at a time; keys with a value of at least t0 that beat the K-th best so
// far go through an LDS ring into the sorted list (as topk_row). Every member
// lies in a listed block, so the lists are exactly topk_row's. With more than
// 65 candidates (K - 1 > 64) every block is read. A row that ends with fewer
// than K keys (only possible when S and the block maxima disagree, as with
// non-finite inputs, whose NaN values pass no bound) writes -1 as its first
// index and nothing else; the launcher then selects such rows again over the
// whole row (topk_redo_kernel), so every list holds K columns of the row. The
// whole-row selection is not inlined here: it needs about twice the registers
// of this function and would halve its occupancy.
template <int R, typename T>
__device__ __forceinline__ void topk_pruned_row(const T* __restrict__ S, int64_t ldS, int N, int i, int K,
                                                const float* bmrow, int32_t* __restrict__ oidx,
                                                float* __restrict__ oval, int ldo, uint64_t* ring, int* list) {
  constexpr int NB = 8;  // up to 512 blocks: lane l holds blocks l, l + 64, ...
  constexpr int Q = 4;   // blocks read per step
  constexpr float NEG = -__builtin_inff();
  const int lane = threadIdx.x & 63;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int TB = (N + 127) / 128, dblk = i / 128;
  const T* srow = S + (int64_t)i * ldS;
  float bx[NB];
#pragma unroll
  for (int b = 0; b < NB; b++) {
    const int t = b * 64 + lane;
    bx[b] = t < TB ? bmrow[t] : NEG;
  }
  float t0 = NEG;
  if (K == 1) {
    t0 = __builtin_inff();
  } else if (K - 1 <= 64) {
    float lm = NEG;
#pragma unroll
    for (int b = 0; b < NB; b++)
      if (b * 64 + lane != dblk) lm = fmaxf(lm, bx[b]);
    uint64_t k[1] = {((uint64_t)ord_f32(lm) << 32) | (uint64_t)lane};
    wave_sort_desc<1>(k);
    const uint64_t kk = wave_rank_key<1>(k, K - 2);
    t0 = unord_f32((uint32_t)(kk >> 32));  // -inf when fewer than K - 1 blocks exist
  }
  // the listed blocks, in block order
  int nl = 0;
#pragma unroll
  for (int b = 0; b < NB; b++) {
    const int t = b * 64 + lane;
    const bool sel = t < TB && (bx[b] >= t0 || t == dblk);
    const uint64_t m = __ballot(sel);
    if (sel) list[nl + __popcll(m & below)] = t;
    nl += __popcll(m);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  uint64_t best[R];
#pragma unroll
  for (int r = 0; r < R; r++) best[r] = (r == 0 && lane == 0) ? self_key((uint32_t)i) : 0ull;
  uint64_t tau = K == 1 ? self_key((uint32_t)i) : 0ull;  // the K-th best key so far
  int head = 0, cnt = 0;
  for (int l0 = 0; l0 < nl; l0 += Q) {
    float v[Q][2];
    int c[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) {
      c[q] = l0 + q < nl ? list[l0 + q] * 128 : N;
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const int col = c[q] + h * 64 + lane;
        v[q][h] = col < N ? (float)srow[col] : 0.f;
      }
    }
#pragma unroll
    for (int q = 0; q < Q; q++)
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const int col = c[q] + h * 64 + lane;
        const bool pass = col < N && col != i && v[q][h] >= t0 && sel_key(v[q][h], (uint32_t)col) > tau;
        const uint64_t m = __ballot(pass);
        if (!m) continue;
        if (pass) ring[(head + cnt + __popcll(m & below)) & 127] = sel_key(v[q][h], (uint32_t)col);
        cnt += __popcll(m);
        if (cnt >= 64) {
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          const uint64_t bk = ring[(head + lane) & 127];
          head = (head + 64) & 127;
          cnt -= 64;
          wave_merge_batch<R>(best, bk);
          tau = wave_rank_key<R>(best, K - 1);
        }
      }
  }
  if (cnt > 0) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const uint64_t bk = lane < cnt ? ring[(head + lane) & 127] : 0ull;
    wave_merge_batch<R>(best, bk);
  }
  int have = 0;  // keys held (key 0 = empty)
#pragma unroll
  for (int r = 0; r < R; r++) have += __popcll(__ballot(r * 64 + lane < K && best[r] != 0ull));
  if (have < K) {
    if (lane == 0) oidx[(int64_t)i * ldo] = -1;  // selected again over the whole row
    return;
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

// ============================================================== a3b: re-score
// Candidates of row i re-scored as cos(x_i, x_j): the FP32 products are exact
// in FP64 and summed there (the sum's error, a few units of 2^-53 of
// sum |x_ik x_jk|, is far below one FP32 rounding), scaled by the inverse
// norms in FP64 and rounded to FP32 once; then sorted under (similarity
// desc, column asc) with the row itself first; the first k1 are N(i, k1) of
// Eq. 8. FP64 FMAs run at the rate of unpacked FP32 ones on gfx950, so this is
// cheaper than a compensated FP32 sum.
//
// One wavefront per row. The row is taken in blocks of 256 U features (U
// 16-byte loads per lane, x_i's block held in registers; U from the row
// length: 8 for rows over 1024 features, down to 1 up to 256); each
// candidate's block is read by the whole wavefront, max(1, 8 / U) candidates
// per step, the next step's loads in flight while a step is multiplied, and
// the partial dot products are summed across the wavefront in a fixed order
// (the result does not depend on the launch).
__host__ __device__ constexpr int rescore_u(int64_t ldp) {
  return ldp > 1024 ? 8 : ldp > 512 ? 4 : ldp > 256 ? 2 : 1;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

template <int R, int U>
__device__ __forceinline__ void rescore_row_u(const float* __restrict__ xp, int64_t ldp,
                                              const float* __restrict__ rn, int i, const int32_t* __restrict__ cand,
                                              const float* __restrict__ cval, int Kc, int k1, float skip2,
                                              int32_t* __restrict__ kidx, float* __restrict__ kval) {
  constexpr int C = U >= 8 ? 1 : 8 / U;  // candidates per step (two steps' loads in flight)
  const int lane = threadIdx.x & 63;
  const float* xi = xp + (int64_t)i * ldp;
  const int32_t* ci = cand + (int64_t)i * Kc;
  // Candidates arrive sorted by their product values g. With skip2 = 2 delta
  // >= 0 (delta bounds |g - exact|), a candidate past position k1 can enter
  // the exact top-k1 only if g >= g[k1 - 1] - skip2: those form a prefix,
  // and only that prefix is re-scored (same lists and values as all of it).
  int cnt = Kc;
  if (skip2 >= 0.f) {
    const float thr = cval[(int64_t)i * Kc + (k1 - 1)] - skip2;
    int last = k1 - 1;
    for (int c = k1 + lane; c < Kc; c += 64)
      if (cval[(int64_t)i * Kc + c] >= thr) last = max(last, c);
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) last = max(last, __shfl_xor(last, m, kWave));
    cnt = last + 1;
  }
  double dotv[R];  // lane l, slot r: the dot product of candidate 64 r + l
#pragma unroll
  for (int r = 0; r < R; r++) dotv[r] = 0.0;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  for (int64_t k0 = 0; k0 < ldp; k0 += 256 * U) {
    f32x4 a[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t k = k0 + u * 256 + lane * 4;
      a[u] = k < ldp ? *(const f32x4*)(xi + k) : zero;
    }
    // candidates c .. c + C - 1 of block k0 into b (zeros past cnt and for the row itself)
    auto fetch = [&](f32x4 (&b)[C][U], int c) {
#pragma unroll
      for (int q = 0; q < C; q++) {
        const int j = c + q < cnt ? ci[c + q] : i;
        const float* xj = xp + (int64_t)j * ldp;
#pragma unroll
        for (int u = 0; u < U; u++) {
          const int64_t k = k0 + u * 256 + lane * 4;
          b[q][u] = (k < ldp && j != i) ? *(const f32x4*)(xj + k) : zero;
        }
      }
    };
    f32x4 nb[C][U];  // the next step's blocks, loaded while this step's are multiplied
    fetch(nb, 0);
    for (int c = 0; c < cnt; c += C) {
      f32x4 b[C][U];
#pragma unroll
      for (int q = 0; q < C; q++)
#pragma unroll
        for (int u = 0; u < U; u++) b[q][u] = nb[q][u];
      if (c + C < cnt) fetch(nb, c + C);
#pragma unroll
      for (int q = 0; q < C; q++) {
        double sq = 0.0;
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
          for (int e = 0; e < 4; e++) sq = __builtin_fma((double)a[u][e], (double)b[q][u][e], sq);
        sq = wave_sum_f64(sq);
#pragma unroll
        for (int r = 0; r < R; r++)
          if (((c + q) >> 6) == r && lane == ((c + q) & 63)) dotv[r] += sq;
      }
    }
  }
  const double rni = rn[i];
  uint64_t keys[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int c = r * 64 + lane;
    keys[r] = 0ull;
    if (c < cnt) {
      const int j = ci[c];
      keys[r] = j == i ? self_key((uint32_t)i) : sel_key((float)(dotv[r] * rni * (double)rn[j]), (uint32_t)j);
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

// The re-score of row i with the block size its row length calls for.
template <int R>
__device__ __forceinline__ void rescore_row(const float* __restrict__ xp, int64_t ldp, const float* __restrict__ rn,
                                            int i, const int32_t* __restrict__ cand, const float* __restrict__ cval,
                                            int Kc, int k1, float skip2, int32_t* __restrict__ kidx,
                                            float* __restrict__ kval) {
  switch (rescore_u(ldp)) {
    case 8:
      rescore_row_u<R, 8>(xp, ldp, rn, i, cand, cval, Kc, k1, skip2, kidx, kval);
      break;
    case 4:
      rescore_row_u<R, 4>(xp, ldp, rn, i, cand, cval, Kc, k1, skip2, kidx, kval);
      break;
    case 2:
      rescore_row_u<R, 2>(xp, ldp, rn, i, cand, cval, Kc, k1, skip2, kidx, kval);
      break;
    default:
      rescore_row_u<R, 1>(xp, ldp, rn, i, cand, cval, Kc, k1, skip2, kidx, kval);
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
#pragma unroll 8
  for (int s = 0; s < k1; s++) mut |= (lj[s] == i);  // eight loads in flight per step
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
  if (lo) *(uint2*)(lo + at) = make_uint2(l4[0] | ((uint32_t)l4[1] << 16), l4[2] | ((uint32_t)l4[3] << 16));
}

// Coefficients of row i. Message r is e_ir^alpha h_{j_r} (member 0 is the row
// itself with e_ii = 1), each times the carried 1/|u_j| of its input row.
// sum: member 0 also takes the residual h_i; mean: messages scaled by 1/k2,
// residual added to member 0; max: messages kept apart, residual in res.
// Coefficient of member r (thread r < k2); returns its row j.
__device__ __forceinline__ int coef_member(const float* __restrict__ sin, const int32_t* __restrict__ knn,
                                           const float* __restrict__ kv, int k1, int k2, int alpha, int agg, int i,
                                           int r, PropShared& sh) {
  const int j = knn[(int64_t)i * k1 + r];
  float w = 1.0f;
  if (r > 0) {
    const float e = kv[(int64_t)i * k1 + r];
    for (int a = 0; a < alpha; a++) w *= e;
  }
  const float sj = sin ? sin[j] : 1.0f;
  const float msg = w * sj;
  float c = msg;
  if (agg == RERANK_AGG_MEAN) c = msg / (float)k2;
  if (r == 0) {
    if (agg == RERANK_AGG_MAX)
      sh.res = sj;
    else
      c = sj + c;  // residual + own message (sum: exactly 2 * sj)
  }
  sh.cf[r] = c;
  sh.nb[r] = j;
  return j;
}

__device__ __forceinline__ void load_coefs(const float* __restrict__ sin, const int32_t* __restrict__ knn,
                                           const float* __restrict__ kv, int k1, int k2, int alpha, int agg, int i,
                                           PropShared& sh) {
  const int tid = threadIdx.x;
  if (tid < k2) coef_member(sin, knn, kv, k1, k2, alpha, agg, i, tid, sh);
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
#pragma unroll 8
  for (int s = 0; s < k1; s++) mut |= (lj[s] == m);  // eight loads in flight per step
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

// Rows built from sparse member rows (the first layer from A* / A, and the
// sparse layers from CSR rows), one LDS column chunk at a time.
constexpr int FIRST_CHUNK = 3072;    // floats of the output row held in LDS (fallback path; 12 KB like the rank table)
constexpr int FIRST_WORDS = FIRST_CHUNK / 32;  // touched-column bitmap of a chunk
constexpr int FIRST_ENTRIES = 1024;  // member entries of one row staged in LDS
constexpr int ROW_WORDS = 2048;      // touched-column bitmap of a whole row (rows up to 65536 columns)
struct RankTab {
  int base[ROW_WORDS];         // touched columns before each bitmap word
  float val[FIRST_ENTRIES];    // sums of the touched columns, in column order
};
struct FirstShared {
  PropShared p;
  union {
    float row[FIRST_CHUNK];  // chunked path: sums; valid only where the bitmap is set
    RankTab rk;              // ranked path
  };
  uint32_t bits[ROW_WORDS];  // touched columns (of the chunk, or of the whole row)
  int col[FIRST_ENTRIES];
  float val[FIRST_ENTRIES];
  int start[257];  // entries of member r are [start[r], start[r+1])
  int mcnt[256];   // entry count of member r
  int mbase[256];  // where member r's entries start in its source
  int wsum[4];     // per-wave counts of a CSR store
};

// ---------------------------------------------------------------- sparse rows
// Sparse-layer output: CSR unless the layer's gate (set before the layer by
// the slot layout) says dense. *pos is the first entry of row i's slot.
__device__ __forceinline__ bool sl_begin(const SlOut* o, int i, int* pos) {
  if (!o || o->gate->dense) return false;
  *pos = o->rows.so[i];
  return true;
}

// Entries of the vertex feature h^(0)_j: A* row j (sym) is its out-list
// N(j, k1) (value 1 when the pair is mutual, else 1/2) followed by its
// non-mutual in-edges (value 1/2); an A row (not sym) is its out-list, value 1.
struct FirstSrc {
  const int32_t* knn;
  const uint8_t* mflag;
  const int32_t* off;
  const int32_t* inl;
  int k1;
  bool sym;
  __device__ int count(int j) const { return k1 + (sym ? off[j + 1] - off[j] : 0); }
  __device__ int base(int j) const { return sym ? off[j] : 0; }
  __device__ void entry(int j, int mbase, int e, int* c, float* v) const {
    if (e < k1) {
      *c = knn[(int64_t)j * k1 + e];
      *v = (!sym || mflag[(int64_t)j * k1 + e]) ? 1.0f : 0.5f;
    } else {
      *c = inl[mbase + e - k1];
      *v = 0.5f;
    }
  }
};

// Entries of a CSR row of the previous sparse layer.
struct CsrSrc {
  SlRows in;
  __device__ int count(int j) const { return in.cnt[j]; }
  __device__ int base(int j) const { return in.so[j]; }
  __device__ void entry(int, int mbase, int e, int* c, float* v) const {
    *c = in.col[mbase + e];
    *v = in.val[mbase + e];
  }
};

// row[m] += c * v in member order; the first touch of a column starts from 0.
__device__ __forceinline__ void sparse_add(FirstShared& sh, int m, float c, float v) {
  const uint32_t bit = 1u << (m & 31);
  const uint32_t old = atomicOr(&sh.bits[m >> 5], bit);
  sh.row[m] = __builtin_fmaf(c, v, (old & bit) ? sh.row[m] : 0.0f);
}

// CSR rows whose staged entries fit skip the column chunks. A bitmap of the
// whole row marks every column the members touch; a prefix count over its
// words gives each touched column its rank (its position in column order),
// and the sums live in an LDS array indexed by rank, starting from 0 and
// taking one FMA per entry in member order, exactly as in the chunks. The
// ranks give the ascending column order of the output directly, and the
// bitmap gives the dense store's per-thread order for the squared norm
// (thread t owns float4 columns t, t + 256, ...).
__device__ __forceinline__ int col_rank(const FirstShared& sh, int c) {
  const uint32_t wd = sh.bits[c >> 5];
  return sh.rk.base[c >> 5] + __builtin_popcount(wd & ((1u << (c & 31)) - 1u));
}

// Sums of a staged row by column rank: whole-row bitmap of the touched
// columns, rank table, then the members' terms added member by member (the
// dense layer's order). Leaves bits, rk and wsum set for the caller.
__device__ __forceinline__ void ranked_sums(FirstShared& sh, int k2, int64_t ld) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int words = (int)(ld >> 5);
  const int total_e = sh.start[k2];
  for (int k = tid; k < words; k += 256) sh.bits[k] = 0u;
  __syncthreads();
  for (int s = tid; s < total_e; s += 256) {
    const int c = sh.col[s];
    atomicOr(&sh.bits[c >> 5], 1u << (c & 31));
  }
  __syncthreads();
  // ranks: thread t owns a contiguous run of words
  const int per = (words + 255) / 256;
  const int w0 = min(words, tid * per), w1 = min(words, w0 + per);
  int mine = 0;
  for (int x = w0; x < w1; x++) mine += __builtin_popcount(sh.bits[x]);
  int incl = mine;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += t;
  }
  if (lane == 63) sh.wsum[w] = incl;
  __syncthreads();
  int run = incl - mine;
  for (int x = 0; x < w; x++) run += sh.wsum[x];
  const int touched = sh.wsum[0] + sh.wsum[1] + sh.wsum[2] + sh.wsum[3];
  for (int x = w0; x < w1; x++) {
    sh.rk.base[x] = run;
    run += __builtin_popcount(sh.bits[x]);
  }
  for (int k = tid; k < touched; k += 256) sh.rk.val[k] = 0.f;
  __syncthreads();
  for (int r = 0; r < k2; r++) {
    const float c = sh.p.cf[r];
    for (int s = sh.start[r] + tid; s < sh.start[r + 1]; s += 256) {  // distinct columns within a member
      const int k = col_rank(sh, sh.col[s]);
      sh.rk.val[k] = __builtin_fmaf(c, sh.val[s], sh.rk.val[k]);
    }
    __syncthreads();
  }
}

// CSR output of a staged row. Returns the end of the written entries; *ss
// receives the squared norm.
__device__ __forceinline__ int ranked_row(FirstShared& sh, int k2, int64_t ld, const SlRows& out, int pos,
                                          float* ss) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int words = (int)(ld >> 5);
  ranked_sums(sh, k2, ld);
  const int per = (words + 255) / 256;
  const int w0 = min(words, tid * per), w1 = min(words, w0 + per);
  float acc = 0.f;
  const int nf = (int)(ld >> 2);
  for (int f = tid; f < nf; f += 256) {
    const uint32_t nib = (sh.bits[f >> 3] >> ((f & 7) * 4)) & 0xFu;
    if (nib) {
      const int k0 = col_rank(sh, 4 * f);  // rank of the first column of this float4
      int k = k0;
      for (int e = 0; e < 4; e++)
        if (nib & (1u << e)) {
          const float v = sh.rk.val[k++];
          acc = __builtin_fmaf(v, v, acc);
        }
    }
  }
  *ss = acc;
  // output: the same contiguous word runs, exact zeros (cancelled sums) dropped
  int keep = 0;
  for (int x = w0; x < w1; x++) {
    const int b0 = sh.rk.base[x], nb = __builtin_popcount(sh.bits[x]);
    for (int k = b0; k < b0 + nb; k++) keep += sh.rk.val[k] != 0.f;
  }
  int incl = keep;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += t;
  }
  __syncthreads();  // everyone has read wsum above
  if (lane == 63) sh.wsum[w] = incl;
  __syncthreads();
  int at = pos + incl - keep, total = 0;
  for (int x = 0; x < 4; x++) {
    at += (x < w) ? sh.wsum[x] : 0;
    total += sh.wsum[x];
  }
  for (int x = w0; x < w1; x++) {
    uint32_t wd = sh.bits[x];
    int k = sh.rk.base[x];
    while (wd) {
      const int b = __builtin_ctz(wd);
      wd &= wd - 1u;
      const float v = sh.rk.val[k++];
      if (v != 0.f) {
        out.col[at] = 32 * x + b;
        out.val[at] = v;
        at++;
      }
    }
  }
  __syncthreads();  // wsum, bits and the table are reused by the caller
  return pos + total;
}

// Dense output of a staged row (row i of hout, or of the hi / lo planes): one
// pass over the row, zeros where no column was touched; *ss receives the
// squared norm, accumulated per thread over float4 f = tid, tid + 256, ...
// like the chunked writer, so both give the same bits.
__device__ __forceinline__ void ranked_dense_row(FirstShared& sh, int k2, int64_t ld, float* __restrict__ hout,
                                                 uint16_t* __restrict__ hi, uint16_t* __restrict__ lo, int i,
                                                 float* ss) {
  const int tid = threadIdx.x;
  ranked_sums(sh, k2, ld);
  float acc = 0.f;
  const int nf = (int)(ld >> 2);
  for (int f = tid; f < nf; f += 256) {
    const uint32_t nib = (sh.bits[f >> 3] >> ((f & 7) * 4)) & 0xFu;
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (nib) {
      int k = col_rank(sh, 4 * f);  // rank of the first touched column of this float4
      for (int e = 0; e < 4; e++)
        if (nib & (1u << e)) v[e] = sh.rk.val[k++];
    }
    if (hi)
      split_store4(hi, lo, (int64_t)i * ld + 4 * f, v);
    else
      ((f32x4*)(hout + (int64_t)i * ld))[f] = v;
    acc = sq_acc4(acc, v);
  }
  *ss = acc;
  __syncthreads();  // bits and the table are reused by the caller
}

// u_i = sum_r cf_r h_{j_r} over the k2 members (coefficients already in sh.p)
// from sparse member rows, one LDS column chunk at a time, in member order r
// with one FMA per entry: the same sums, rounding for rounding, as
// propagate_row on dense rows (a zero entry there is an FMA that leaves the
// sum unchanged). Written as dense rows (hout, or bf16 hi/lo planes) or as a
// CSR row (sl); the squared norm is accumulated in the dense store's
// per-thread order (thread t owns float4 columns t, t + 256, ... of a chunk),
// so sigma is identical either way.
template <class Src>
__device__ __forceinline__ void sparse_row_core(const Src& src, const float* __restrict__ sin,
                                                const int32_t* __restrict__ knn, const float* __restrict__ kv,
                                                int k1, int k2, int alpha, int agg, int64_t ld,
                                                float* __restrict__ hout, uint16_t* __restrict__ hi,
                                                uint16_t* __restrict__ lo, float* __restrict__ sout,
                                                const SlOut* sl, int i, FirstShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int pos = 0;
  const bool csr = sl_begin(sl, i, &pos);  // issued first: independent of the members
  if (tid < k2) {  // coefficients and entry counts in one round of loads
    const int j = coef_member(sin, knn, kv, k1, k2, alpha, agg, i, tid, sh.p);
    sh.mcnt[tid] = src.count(j);
    sh.mbase[tid] = src.base(j);
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int r = 0; r < k2; r++) {
      sh.start[r] = acc;
      acc += sh.mcnt[r];
    }
    sh.start[k2] = acc;
  }
  __syncthreads();
  const int total_e = sh.start[k2];
  const bool staged = total_e <= FIRST_ENTRIES;
  if (staged) {  // all entries at once: member of entry e = last r with start[r] <= e
    for (int e = tid; e < total_e; e += 256) {
      int lo_r = 0, hi_r = k2 - 1;
      while (lo_r < hi_r) {
        const int mid = (lo_r + hi_r + 1) >> 1;
        if (sh.start[mid] <= e)
          lo_r = mid;
        else
          hi_r = mid - 1;
      }
      int c;
      float v;
      src.entry(sh.p.nb[lo_r], sh.mbase[lo_r], e - sh.start[lo_r], &c, &v);
      sh.col[e] = c;
      sh.val[e] = v;
    }
  }
  __syncthreads();
  const int pos0 = pos;
  float ss = 0.f;
  if (staged && (ld >> 5) <= ROW_WORDS) {  // whole row at once, no column chunks
    if (csr) {
      const int end = ranked_row(sh, k2, ld, sl->rows, pos, &ss);
      if (tid == 0) {
        sl->rows.so[i] = pos0;
        sl->rows.cnt[i] = end - pos0;
      }
    } else {
      ranked_dense_row(sh, k2, ld, hout, hi, lo, i, &ss);
    }
    finish_norm(ss, sout, i, sh.p);
    return;
  }
  for (int64_t c0 = 0; c0 < ld; c0 += FIRST_CHUNK) {
    const int width = (int)min((int64_t)FIRST_CHUNK, ld - c0);
    for (int k = tid; k < FIRST_WORDS; k += 256) sh.bits[k] = 0u;
    __syncthreads();
    for (int r = 0; r < k2; r++) {
      const float c = sh.p.cf[r];
      if (staged) {
        for (int s = sh.start[r] + tid; s < sh.start[r + 1]; s += 256) {
          const int64_t m = sh.col[s] - c0;
          if (m >= 0 && m < width) sparse_add(sh, (int)m, c, sh.val[s]);
        }
      } else {  // too many entries to stage: read them from memory for every chunk
        const int j = sh.p.nb[r], mb = sh.mbase[r];
        for (int e = tid; e < sh.mcnt[r]; e += 256) {
          int cc;
          float v;
          src.entry(j, mb, e, &cc, &v);
          const int64_t m = cc - c0;
          if (m >= 0 && m < width) sparse_add(sh, (int)m, c, v);
        }
      }
      __syncthreads();
    }
    const int w4 = width >> 2;
    if (!csr) {
      for (int c = tid; c < w4; c += 256) {
        const uint32_t nib = (sh.bits[c >> 3] >> ((c & 7) * 4)) & 0xFu;
        const f32x4 acc = {(nib & 1u) ? sh.row[4 * c] : 0.f, (nib & 2u) ? sh.row[4 * c + 1] : 0.f,
                           (nib & 4u) ? sh.row[4 * c + 2] : 0.f, (nib & 8u) ? sh.row[4 * c + 3] : 0.f};
        if (hi)
          split_store4(hi, lo, (int64_t)i * ld + c0 + c * 4, acc);
        else
          ((f32x4*)(hout + (int64_t)i * ld + c0))[c] = acc;
        ss = sq_acc4(ss, acc);
      }
    } else {
      for (int c = tid; c < w4; c += 256) {  // squares in the dense order (skipped zeros change nothing)
        const uint32_t nib = (sh.bits[c >> 3] >> ((c & 7) * 4)) & 0xFu;
        for (int e = 0; e < 4; e++)
          if (nib & (1u << e)) {
            const float v = sh.row[4 * c + e];
            ss = __builtin_fmaf(v, v, ss);
          }
      }
      // word t of the bitmap = columns 32t .. 32t + 31; keep the non-zero sums
      uint32_t keep = 0u;
      if (tid < (width >> 5)) {
        uint32_t wd = sh.bits[tid];
        while (wd) {
          const int b = __builtin_ctz(wd);
          wd &= wd - 1u;
          if (sh.row[32 * tid + b] != 0.f) keep |= 1u << b;
        }
      }
      const int mine = __builtin_popcount(keep);
      int incl = mine;
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, kWave);
        if (lane >= o) incl += t;
      }
      if (lane == 63) sh.wsum[w] = incl;
      __syncthreads();
      int at = pos + incl - mine, total = 0;
      for (int x = 0; x < 4; x++) {
        at += (x < w) ? sh.wsum[x] : 0;
        total += sh.wsum[x];
      }
      while (keep) {
        const int b = __builtin_ctz(keep);
        keep &= keep - 1u;
        sl->rows.col[at] = (int32_t)(c0 + 32 * tid + b);
        sl->rows.val[at] = sh.row[32 * tid + b];
        at++;
      }
      pos += total;
    }
    __syncthreads();  // bits, row and wsum are reused by the next chunk
  }
  if (csr && tid == 0) {
    sl->rows.so[i] = pos0;
    sl->rows.cnt[i] = pos - pos0;
  }
  finish_norm(ss, sout, i, sh.p);
}

// First layer without a dense h^(0): u_i = sum_r c_r h^(0)_{j_r} from the
// sparse A* (sym) or A rows. The aggregator is sum or mean (max runs the
// dense layer).
__device__ __forceinline__ void first_layer_row(const int32_t* __restrict__ knn, const float* __restrict__ kv,
                                                const uint8_t* __restrict__ mflag, const int32_t* __restrict__ off,
                                                const int32_t* __restrict__ inl, int k1, int k2, int alpha, int agg,
                                                bool sym, int64_t ld, float* __restrict__ hout,
                                                float* __restrict__ sout, uint16_t* __restrict__ hi,
                                                uint16_t* __restrict__ lo, int i, FirstShared& sh,
                                                const SlOut* sl = nullptr) {
  const FirstSrc src{knn, mflag, off, inl, k1, sym};
  sparse_row_core(src, nullptr, knn, kv, k1, k2, alpha, agg, ld, hout, hi, lo, sout, sl, i, sh);
}

// Layer l >= 2 of the sparse layers from the CSR rows of layer l - 1
// (coefficients carry the rows' 1/|u_j|). Sum and mean aggregators.
__device__ __forceinline__ void sparse_prop_row(const SlRows& in, const float* __restrict__ sin,
                                                const int32_t* __restrict__ knn, const float* __restrict__ kv,
                                                int k1, int k2, int alpha, int agg, int64_t ld,
                                                float* __restrict__ hout, float* __restrict__ sout, const SlOut* sl,
                                                int i, FirstShared& sh) {
  const CsrSrc src{in};
  sparse_row_core(src, sin, knn, kv, k1, k2, alpha, agg, ld, hout, nullptr, nullptr, sout, sl, i, sh);
}

}  // namespace rr
