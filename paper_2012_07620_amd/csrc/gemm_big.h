// Large-tile engine for the low-precision similarity product S = X X^T
// (Eq. 7) on gfx950 matrix cores: 256 x 256 output tiles, four wavefronts in
// 2 x 2, each owning a 128 x 128 sub-tile of 4 x 4 MFMA 32x32 blocks (256
// FP32 accumulators per lane).
//
// Why a second engine: with bf16 (32x32x16) or e4m3 (32x32x64) MFMAs a
// 64 x 64 sub-tile reads as many LDS bytes per multiply-add as the matrix
// cores consume at full rate (16 MAC per byte), so the 128 x 128 engine is
// LDS-bound; 128 x 128 per wave halves the LDS bytes per multiply-add and the
// L2 bytes per tile. One workgroup per CU: LDS holds two 128-byte K stages of
// 256 A rows and 256 B rows (144-byte padded rows, 144 KB), the next stage is
// prefetched into registers while the current one is multiplied, and one
// block barrier separates stages.
//
// K order inside a stage is the same lane-half permutation as the 128 x 128
// engine (lane half h feeds bytes [64h, 64h + 64) of a row's 128-byte slice),
// applied to both operands.
#pragma once
#include "gemm_body.h"

namespace rr {

constexpr int BT = 256;                      // output tile edge
constexpr int BIG_BUF = 2 * BT * LDSR;       // one stage: A and B, 73728 bytes
constexpr int BIG_LDS_BYTES = 2 * BIG_BUF;   // two stages, 147456 bytes
constexpr int BIG_TSTRIDE = 129;             // transposed staging row stride (floats)
static_assert(2 * 128 * BIG_TSTRIDE * 4 <= BIG_LDS_BYTES, "mirror staging must fit");

// One 256 x 256 tile (tm, tn) of S = v * sa[row] * sb[col]; with `mirror`
// also the transposed tile at (tn, tm). MODE is MODE_BF16 or MODE_FP8.
template <int MODE>
__device__ __forceinline__ void gemm_tile_big(const GemmArgs& g, int tm, int tn, bool mirror, uint8_t* lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = tm * BT, n0 = tn * BT;

  // global -> register staging: 2048 16-byte chunks per operand per stage
  const uint8_t* pa[8];
  const uint8_t* pb[8];
  int ls[8];
#pragma unroll
  for (int u = 0; u < 8; u++) {
    const int f = u * 256 + tid, row = f >> 3, c = f & 7;
    pa[u] = g.A + (int64_t)min(m0 + row, g.M - 1) * g.lda + c * 16;
    pb[u] = g.B + (int64_t)min(n0 + row, g.Nn - 1) * g.ldb + c * 16;
    ls[u] = row * LDSR + c * 16;
  }
  u32x4 ra[8], rb[8];
  auto gload = [&](int st) {
#pragma unroll
    for (int u = 0; u < 8; u++) {
      ra[u] = *(const u32x4*)(pa[u] + (int64_t)st * BKB);
      rb[u] = *(const u32x4*)(pb[u] + (int64_t)st * BKB);
    }
  };
  auto lstore = [&](int buf) {
    uint8_t* base = lds + buf * BIG_BUF;
#pragma unroll
    for (int u = 0; u < 8; u++) {
      *(u32x4*)(base + ls[u]) = ra[u];
      *(u32x4*)(base + BT * LDSR + ls[u]) = rb[u];
    }
  };

  f32x16 acc[4][4];
#pragma unroll
  for (int sm = 0; sm < 4; sm++)
#pragma unroll
    for (int sn = 0; sn < 4; sn++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[sm][sn][r] = 0.f;

  const int fa = (wm * 128 + (lane & 31)) * LDSR + (lane >> 5) * 64;
  const int fb = (wn * 128 + (lane & 31)) * LDSR + (lane >> 5) * 64;

  gload(0);
  lstore(0);
  if (g.nst > 1) gload(1);
  __syncthreads();
  for (int st = 0; st < g.nst; st++) {
    const uint8_t* la = lds + (st & 1) * BIG_BUF;
    const uint8_t* lb = la + BT * LDSR;
    if constexpr (MODE == MODE_BF16) {
#pragma unroll
      for (int c = 0; c < 4; c++) {  // k-step c: 16 bf16 of K
        u32x4 a[4], b[4];
#pragma unroll
        for (int s = 0; s < 4; s++) {
          a[s] = *(const u32x4*)(la + fa + s * 32 * LDSR + c * 16);
          b[s] = *(const u32x4*)(lb + fb + s * 32 * LDSR + c * 16);
        }
#pragma unroll
        for (int sm = 0; sm < 4; sm++)
#pragma unroll
          for (int sn = 0; sn < 4; sn++)
            acc[sm][sn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, a[sm]), __builtin_bit_cast(bf16x8, b[sn]), acc[sm][sn], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < 2; kk++) {  // k-step kk: 64 e4m3 of K
        i32x8 a[4], b[4];
#pragma unroll
        for (int s = 0; s < 4; s++) {
          const u32x4 a0 = *(const u32x4*)(la + fa + s * 32 * LDSR + kk * 32);
          const u32x4 a1 = *(const u32x4*)(la + fa + s * 32 * LDSR + kk * 32 + 16);
          const u32x4 b0 = *(const u32x4*)(lb + fb + s * 32 * LDSR + kk * 32);
          const u32x4 b1 = *(const u32x4*)(lb + fb + s * 32 * LDSR + kk * 32 + 16);
          a[s] = i32x8{(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3], (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
          b[s] = i32x8{(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3], (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
        }
#pragma unroll
        for (int sm = 0; sm < 4; sm++)
#pragma unroll
          for (int sn = 0; sn < 4; sn++)
            // formats 0/0 = e4m3 for A and B; scale exponents 127 = 2^0
            acc[sm][sn] =
                __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a[sm], b[sn], acc[sm][sn], 0, 0, 0, 127, 0, 127);
      }
    }
    if (st + 1 < g.nst) {
      lstore((st + 1) & 1);  // that buffer was last read before the previous barrier
      if (st + 2 < g.nst) gload(st + 2);
    }
    __syncthreads();
  }

  // 32x32 accumulator layout: register r of lane l holds
  // row 8*(r/4) + 4*(l/32) + r%4, column l%32 of its block.
#pragma unroll
  for (int sm = 0; sm < 4; sm++)
#pragma unroll
    for (int sn = 0; sn < 4; sn++) {
      const int col = n0 + wn * 128 + sn * 32 + (lane & 31);
      const float scol = (col < g.Nn) ? g.sb[col] : 0.f;
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int row = m0 + wm * 128 + sm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        if (row < g.M && col < g.Nn) g.out[(int64_t)row * g.ldo + col] = acc[sm][sn][r] * g.sa[row] * scol + 0.0f;
      }
    }
  if (mirror) {
    // C^T through LDS, one row of waves (wm = p) at a time: wave (p, wn)
    // stages its 128 x 128 block transposed in region wn, then all threads
    // write rows n0 + wn*128 + lc, columns m0 + p*128 + lr.
    float* tr = (float*)lds;
#pragma unroll
    for (int p = 0; p < 2; p++) {
      if (wm == p) {
        float* reg = tr + wn * 128 * BIG_TSTRIDE;
#pragma unroll
        for (int sm = 0; sm < 4; sm++)
#pragma unroll
          for (int sn = 0; sn < 4; sn++) {
            const int lc = sn * 32 + (lane & 31);
            const int col = n0 + wn * 128 + lc;
            const float scol = (col < g.Nn) ? g.sb[col] : 0.f;
#pragma unroll
            for (int r = 0; r < 16; r++) {
              const int lr = sm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
              const int row = m0 + p * 128 + lr;
              reg[lc * BIG_TSTRIDE + lr] = (row < g.M && col < g.Nn) ? acc[sm][sn][r] * g.sa[row] * scol + 0.0f : 0.f;
            }
          }
      }
      __syncthreads();
      const int c = tid & 127;
      for (int rr = tid >> 7; rr < 256; rr += 2) {  // rr = wn * 128 + lc
        const int row = n0 + rr, col = m0 + p * 128 + c;
        if (row < g.Nn && col < g.M) g.out[(int64_t)row * g.ldo + col] = tr[rr * BIG_TSTRIDE + c];
      }
      __syncthreads();
    }
  }
}

}  // namespace rr
