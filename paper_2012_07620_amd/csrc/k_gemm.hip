// a2 / a7 -- "NT" products C = A * B^T on gfx950 matrix cores.
//
// Both operands are K-major rows (feature rows for the Eq. 7 similarity,
// refined feature rows for the final ranking product), so each 128 x 128
// output tile streams 128-byte K slices of 128 A rows and 128 B rows through
// LDS (double-buffered, 144-byte padded rows), and four wavefronts each own a
// 64 x 64 sub-tile of 2 x 2 MFMA 32x32 blocks.
//
// K order inside a stage: lane half h = lane/32 feeds the MFMA with bytes
// [64h, 64h+64) of its row's 128-byte slice. A and B use the same map, so
// every product pairs equal K positions; the K summation order is simply
// permuted, which a dot product allows.
//
// Element types per 128-byte stage: 32 fp32 (v_mfma 32x32x2 f32, 16 steps),
// 64 bf16 (32x32x16 bf16, 4 steps) or 128 OCP e4m3 (32x32x64 f8f6f4, unit
// block scales, 2 steps). Accumulation is FP32 in every mode.
#include "common.h"
#include "kernels.h"

namespace rr {

constexpr int BM = 128, BN = 128, BKB = 128, LDSR = BKB + 16, TILEB = BM * LDSR;

enum { MODE_F32 = 0, MODE_BF16 = 1, MODE_FP8 = 2 };
enum { EPI_SIM = 0, EPI_DIST = 1 };

struct TileMap {
  int tm, tn;
};

// Workgroups are dealt to the 8 XCDs round-robin. Renumber them so each XCD
// gets a contiguous run of logical tiles, then walk the tiles in groups of 8
// row-tiles so neighbouring workgroups on an XCD share A and B rows in its L2.
__device__ __forceinline__ TileMap map_tile(int bid, int nwg, int tiles_m, int tiles_n) {
  const int q = nwg >> 3, rem = nwg & 7;
  const int x = bid & 7, local = bid >> 3;
  const int pid = (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + local;
  constexpr int G = 8;
  const int per_group = G * tiles_n;
  const int group = pid / per_group;
  const int first_m = group * G;
  const int gsz = min(tiles_m - first_m, G);
  const int in = pid - group * per_group;
  return TileMap{first_m + in % gsz, in / gsz};
}

template <int MODE>
__device__ __forceinline__ void mfma_stage(f32x16 (&acc)[2][2], const u32x4 (&a)[2][4], const u32x4 (&b)[2][4]) {
  if constexpr (MODE == MODE_F32) {
#pragma unroll
    for (int c = 0; c < 4; c++)
#pragma unroll
      for (int e = 0; e < 4; e++)
#pragma unroll
        for (int sm = 0; sm < 2; sm++)
#pragma unroll
          for (int sn = 0; sn < 2; sn++)
            acc[sm][sn] = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a[sm][c][e]),
                                                               __uint_as_float(b[sn][c][e]), acc[sm][sn], 0, 0, 0);
  } else if constexpr (MODE == MODE_BF16) {
#pragma unroll
    for (int c = 0; c < 4; c++)
#pragma unroll
      for (int sm = 0; sm < 2; sm++)
#pragma unroll
        for (int sn = 0; sn < 2; sn++)
          acc[sm][sn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[sm][c]),
                                                                __builtin_bit_cast(bf16x8, b[sn][c]), acc[sm][sn], 0,
                                                                0, 0);
  } else {
#pragma unroll
    for (int kk = 0; kk < 2; kk++)
#pragma unroll
      for (int sm = 0; sm < 2; sm++)
#pragma unroll
        for (int sn = 0; sn < 2; sn++) {
          const u32x4 a0 = a[sm][2 * kk], a1 = a[sm][2 * kk + 1];
          const u32x4 b0 = b[sn][2 * kk], b1 = b[sn][2 * kk + 1];
          const i32x8 av = {(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3],
                            (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
          const i32x8 bv = {(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3],
                            (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
          // formats 0/0 = e4m3 for A and B; scale exponents 127 = 2^0
          acc[sm][sn] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, acc[sm][sn], 0, 0, 0, 127, 0, 127);
        }
  }
}

template <int MODE, int EPI>
__global__ __launch_bounds__(256) void gemm_nt_kernel(const uint8_t* __restrict__ A, int M, int64_t lda,
                                                      const uint8_t* __restrict__ B, int Nn, int64_t ldb, int nst,
                                                      const float* __restrict__ sa, const float* __restrict__ sb,
                                                      float* __restrict__ out, int64_t ldo, int tiles_m,
                                                      int tiles_n) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[4 * TILEB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const TileMap t = map_tile(blockIdx.x, gridDim.x, tiles_m, tiles_n);
  const int m0 = t.tm * BM, n0 = t.tn * BN;

  const uint8_t* pa[4];
  const uint8_t* pb[4];
  int ls[4];
#pragma unroll
  for (int u = 0; u < 4; u++) {
    const int f = u * 256 + tid, row = f >> 3, c = f & 7;
    pa[u] = A + (int64_t)min(m0 + row, M - 1) * lda + c * 16;
    pb[u] = B + (int64_t)min(n0 + row, Nn - 1) * ldb + c * 16;
    ls[u] = row * LDSR + c * 16;
  }
  u32x4 ra[4], rb[4];
  auto gload = [&](int st) {
#pragma unroll
    for (int u = 0; u < 4; u++) {
      ra[u] = *(const u32x4*)(pa[u] + (int64_t)st * BKB);
      rb[u] = *(const u32x4*)(pb[u] + (int64_t)st * BKB);
    }
  };
  auto lstore = [&](int buf) {
    uint8_t* base = lds + buf * 2 * TILEB;
#pragma unroll
    for (int u = 0; u < 4; u++) {
      *(u32x4*)(base + ls[u]) = ra[u];
      *(u32x4*)(base + TILEB + ls[u]) = rb[u];
    }
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int sm = 0; sm < 2; sm++)
#pragma unroll
    for (int sn = 0; sn < 2; sn++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[sm][sn][r] = 0.f;

  const int fa = (wm * 64 + (lane & 31)) * LDSR + (lane >> 5) * 64;
  const int fb = (wn * 64 + (lane & 31)) * LDSR + (lane >> 5) * 64;

  gload(0);
  lstore(0);
  __syncthreads();
  for (int st = 0; st < nst; st++) {
    const int buf = st & 1;
    if (st + 1 < nst) gload(st + 1);
    const uint8_t* la = lds + buf * 2 * TILEB;
    const uint8_t* lb = la + TILEB;
    u32x4 a[2][4], b[2][4];
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
      for (int c = 0; c < 4; c++) {
        a[s][c] = *(const u32x4*)(la + fa + s * 32 * LDSR + c * 16);
        b[s][c] = *(const u32x4*)(lb + fb + s * 32 * LDSR + c * 16);
      }
    mfma_stage<MODE>(acc, a, b);
    if (st + 1 < nst) lstore(buf ^ 1);
    __syncthreads();
  }

  // 32x32 accumulator layout: register r of lane l holds
  // row 8*(r/4) + 4*(l/32) + r%4, column l%32 of its block.
#pragma unroll
  for (int sm = 0; sm < 2; sm++)
#pragma unroll
    for (int sn = 0; sn < 2; sn++) {
      const int col = n0 + wn * 64 + sn * 32 + (lane & 31);
      if (col >= Nn) continue;
      const float scol = sb[col];
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int row = m0 + wm * 64 + sm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        if (row < M) {
          const float v = acc[sm][sn][r];
          if (EPI == EPI_SIM)
            out[(int64_t)row * ldo + col] = v * sa[row] * scol + 0.0f;
          else
            out[(int64_t)row * ldo + col] = 1.0f - sa[row] * scol * v;
        }
      }
    }
}

template <int MODE, int EPI>
static hipError_t launch_gemm_t(const void* a, int M, int64_t lda, const void* b, int Nn, int64_t ldb, int64_t kbytes,
                                const float* sa, const float* sb, float* out, int64_t ldo, hipStream_t s) {
  const int tm = (M + BM - 1) / BM, tn = (Nn + BN - 1) / BN;
  const int64_t nwg = (int64_t)tm * tn;
  if (nwg <= 0 || nwg > 0x7FFFFFFF || kbytes % BKB) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gemm_nt_kernel<MODE, EPI>), dim3((unsigned)nwg), dim3(256), 0, s, (const uint8_t*)a, M, lda,
                     (const uint8_t*)b, Nn, ldb, (int)(kbytes / BKB), sa, sb, out, ldo, tm, tn);
  return hipGetLastError();
}

hipError_t launch_gemm_sim(SimPrec prec, const void* a, int M, int64_t lda_bytes, int64_t kbytes, const float* sa,
                           float* out, int64_t ldo, hipStream_t s) {
  switch (prec) {
    case SimPrec::F32:
      return launch_gemm_t<MODE_F32, EPI_SIM>(a, M, lda_bytes, a, M, lda_bytes, kbytes, sa, sa, out, ldo, s);
    case SimPrec::BF16:
      return launch_gemm_t<MODE_BF16, EPI_SIM>(a, M, lda_bytes, a, M, lda_bytes, kbytes, sa, sa, out, ldo, s);
    case SimPrec::FP8:
      return launch_gemm_t<MODE_FP8, EPI_SIM>(a, M, lda_bytes, a, M, lda_bytes, kbytes, sa, sa, out, ldo, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_dist(const float* a, int M, const float* b, int Nn, int64_t ld_elems, int64_t kelems,
                            const float* sa, const float* sb, float* out, int64_t ldo, hipStream_t s) {
  return launch_gemm_t<MODE_F32, EPI_DIST>(a, M, ld_elems * 4, b, Nn, ld_elems * 4, kelems * 4, sa, sb, out, ldo, s);
}

}  // namespace rr

namespace rr {
hipError_t launch_gemm_dist_bf16x3(const uint16_t*, const uint16_t*, int, const uint16_t*, const uint16_t*, int,
                                   int64_t, int64_t, const float*, const float*, float*, int64_t, hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace rr
