// Internal helpers shared by the gfx950 kernels of the re-ranking library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rr {

// Global-memory view of a pointer the compiler cannot prove global (one read
// from memory), so its accesses become global loads and stores, counted on
// vmcnt only, instead of flat ones, which also hold up every LDS wait.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Workgroups are dealt to the 8 XCDs round-robin (each XCD has its own L2).
// Renumber them so each XCD gets a contiguous run of logical indices: work
// that is close in logical order then shares one L2.
__device__ __forceinline__ int xcd_linear(int bid, int nwg) {
  const int q = nwg >> 3, rem = nwg & 7;
  const int x = bid & 7, local = bid >> 3;
  return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + local;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Order-preserving map float -> uint32 (larger float -> larger integer);
// -0.0 is mapped like +0.0. A NaN (any sign or payload) maps to 0, below
// -inf, so an undefined similarity ranks after every number and a few
// non-finite rows do not displace the neighbours of the others; unord_f32(0)
// is a NaN again.
__device__ __forceinline__ uint32_t ord_f32(float v) {
  uint32_t b = __float_as_uint(v);
  if (b == 0x80000000u) b = 0u;
  const uint32_t o = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
  return v == v ? o : 0u;
}
__device__ __forceinline__ float unord_f32(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}
// Selection key of column j with similarity v: larger key = better rank under
// (similarity descending, column ascending). Key 0 means "empty".
__device__ __forceinline__ uint64_t sel_key(float v, uint32_t j) {
  return ((uint64_t)ord_f32(v) << 32) | (uint64_t)(~j);
}
// The row's own column always ranks first (member 0 of its own list).
__device__ __forceinline__ uint64_t self_key(uint32_t i) {
  return (0xFFFFFFFFull << 32) | (uint64_t)(~i);
}
__device__ __forceinline__ uint32_t key_col(uint64_t k) { return ~(uint32_t)k; }
__device__ __forceinline__ float key_val(uint64_t k) { return unord_f32((uint32_t)(k >> 32)); }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  int lo = __shfl_xor((int)(uint32_t)v, m, kWave);
  int hi = __shfl_xor((int)(uint32_t)(v >> 32), m, kWave);
  return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  int lo = __shfl((int)(uint32_t)v, src, kWave);
  int hi = __shfl((int)(uint32_t)(v >> 32), src, kWave);
  return ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
}
__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

// Wave-wide bitonic sort, descending, of 64*R keys: element e = r*64 + lane
// lives in v[r] of lane `lane`.
template <int R>
__device__ __forceinline__ void wave_sort_desc(uint64_t (&v)[R]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 2; k <= 64 * R; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64) {
        const int jr = j >> 6;
#pragma unroll
        for (int r = 0; r < R; r++) {
          if ((r & jr) == 0) {
            const int p = r | jr;
            const bool desc = (((r << 6) & k) == 0);
            const uint64_t a = v[r], b = v[p];
            const bool sw = desc ? (a < b) : (a > b);
            v[r] = sw ? b : a;
            v[p] = sw ? a : b;
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; r++) {
          const uint64_t o = shfl_xor_u64(v[r], j);
          const bool desc = ((((r << 6) | lane) & k) == 0);
          const bool lower = ((lane & j) == 0);
          v[r] = (desc == lower) ? umax64(v[r], o) : umin64(v[r], o);
        }
      }
    }
  }
}

// Sort a bitonic sequence of 64*R keys into descending order.
template <int R>
__device__ __forceinline__ void wave_merge_desc(uint64_t (&v)[R]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 32 * R; j > 0; j >>= 1) {
    if (j >= 64) {
      const int jr = j >> 6;
#pragma unroll
      for (int r = 0; r < R; r++) {
        if ((r & jr) == 0) {
          const int p = r | jr;
          const uint64_t a = v[r], b = v[p];
          v[r] = umax64(a, b);
          v[p] = umin64(a, b);
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < R; r++) {
        const uint64_t o = shfl_xor_u64(v[r], j);
        v[r] = ((lane & j) == 0) ? umax64(v[r], o) : umin64(v[r], o);
      }
    }
  }
}

// Merge 64 new keys (any order, one per lane) into the descending list
// `best` of 64*R keys, keeping the 64*R largest.
template <int R>
__device__ __forceinline__ void wave_merge_batch(uint64_t (&best)[R], uint64_t batch) {
  uint64_t b[1] = {batch};
  wave_sort_desc<1>(b);
  const int lane = threadIdx.x & 63;
  const uint64_t rev = shfl_u64(b[0], 63 - lane);
  best[R - 1] = umax64(best[R - 1], rev);
  wave_merge_desc<R>(best);
}

// Key at rank `rank` (wave-uniform) of a descending wave list.
template <int R>
__device__ __forceinline__ uint64_t wave_rank_key(const uint64_t (&v)[R], int rank) {
  uint64_t sel = v[0];
#pragma unroll
  for (int r = 1; r < R; r++)
    if ((rank >> 6) == r) sel = v[r];
  return shfl_u64(sel, rank & 63);
}

// ---- compensated FP32 arithmetic (Ogita, Rump and Oishi 2005: TwoSum and
// the FMA-based TwoProduct), used where FP32 must resolve near-ties.
struct DF {
  float hi, lo;
};
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float z = s - a;
  e = (a - (s - z)) + (b - z);
}
__device__ __forceinline__ void dot2_acc(DF& acc, float a, float b) {
  const float p = a * b;
  const float pe = __builtin_fmaf(a, b, -p);
  float s, e;
  two_sum(acc.hi, p, s, e);
  acc.hi = s;
  acc.lo += e + pe;
}
__device__ __forceinline__ DF df_add(DF a, DF b) {
  float s, e;
  two_sum(a.hi, b.hi, s, e);
  return DF{s, e + a.lo + b.lo};
}
__device__ __forceinline__ DF wave_sum_df(DF v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    DF o{__shfl_xor(v.hi, m, kWave), __shfl_xor(v.lo, m, kWave)};
    v = df_add(v, o);
  }
  return v;
}
__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}
__device__ __forceinline__ float wave_max_f32(float v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, kWave));
  return v;
}

}  // namespace rr
