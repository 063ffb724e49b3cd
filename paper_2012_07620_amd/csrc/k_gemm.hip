// a2 / a7 -- direct launches of the matrix-core products (one 128 x 128 tile
// per workgroup); the tile engine is in gemm_body.h.
#include "gemm_body.h"
#include "kernels.h"

namespace rr {

struct TileMap {
  int tm, tn;
};

// Tiles are renumbered per XCD (xcd_linear), then walked in groups of 8
// row-tiles so neighbouring workgroups on an XCD share A and B rows in its L2.

__device__ __forceinline__ TileMap grouped_order(int pid, int tiles_m, int tiles_n) {
  constexpr int G = 8;
  const int per_group = G * tiles_n;
  const int group = pid / per_group;
  const int first_m = group * G;
  const int gsz = min(tiles_m - first_m, G);
  const int in = pid - group * per_group;
  return TileMap{first_m + in % gsz, in / gsz};
}

// 128-byte K slices per LDS stage. The final product's K (the padded N x N
// row stride) is whole 256-byte stages: two slices halve its barrier pairs
// (15.6 -> 15.2 ms at N = 19281). The similarity keeps one (two measured no
// faster: its 2048-element K leaves few stages per tile).
constexpr int DIST_KS = 2;
constexpr int SIM_KS = 1;

// FP8 similarity tiles are held to three waves per SIMD (168 registers; the
// binary16 staging leaves LDS for three workgroups per CU): 0.64 -> 0.55 ms at
// N = 19281. So is the BF16 final product (one 36 KB stage buffer; 172 -> 160
// registers, no spills): 2.45 -> 2.38 ms (four waves spill and take 4.5 ms).
// The others keep the compiler's allocation (the BF16 similarity already fits).
template <int MODE, int EPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    (MODE == MODE_FP8 && EPI == EPI_SIM_SYM16) || (MODE == MODE_BF16 && EPI == EPI_DIST) ? 3 : 1)))
void gemm_nt_kernel(GemmArgs g, int tiles_m, int tiles_n) {
  constexpr bool SYM = EPI == EPI_SIM_SYM || EPI == EPI_SIM_SYM16;
  constexpr int KS = (EPI == EPI_DIST && MODE == MODE_F32) ? DIST_KS : SYM ? SIM_KS : 1;
  __shared__ __attribute__((aligned(16))) uint8_t lds[SYM ? sim_lds_bytes(EPI) : gemm_stage_lds(KS)];
  const int pid = xcd_linear(blockIdx.x, gridDim.x);
  int tm, tn;
  if (SYM) {
    upper_tile(pid, tiles_m, tm, tn);
  } else {
    const TileMap t = grouped_order(pid, tiles_m, tiles_n);
    tm = t.tm;
    tn = t.tn;
  }
  gemm_tile<MODE, EPI, 1, KS>(g, tm, tn, lds);
}

// K ranges per tile (at most max_parts) of a partly filled last round of
// `tiles` tiles on `slots` resident workgroups: the fewest partial rounds per
// tile, needing a saving of at least a fifth of a round, at least 8 K stages
// per range and room for the partial tiles in ws_bytes; 1 = no split. *rem
// receives the number of tail tiles.
static int tail_parts(int64_t tiles, int slots, int nst, int64_t tile_bytes, int64_t ws_bytes, int max_parts,
                      int64_t* rem) {
  *rem = 0;
  if (slots <= 0 || tiles <= slots) return 1;
  *rem = tiles % slots;
  int parts = 1;
  double best = 1.0;
  for (int p = 2; p <= max_parts; p++) {
    const double cost = (double)((*rem * p + slots - 1) / slots) / p;
    if (cost < best - 1e-9 && nst >= 8 * p && *rem * p * tile_bytes <= ws_bytes) {
      best = cost;
      parts = p;
    }
  }
  return (best > 0.8 || *rem == 0) ? 1 : parts;
}

template <int MODE, int EPI>
static hipError_t launch_gemm_t(const void* a, int M, int64_t lda, const void* b, int Nn, int64_t ldb, int64_t kbytes,
                                const float* sa, const float* sb, float* out, int64_t ldo, hipStream_t s,
                                float* bm = nullptr, int64_t ldbm = 0) {
  const int tm = (M + BM - 1) / BM, tn = (Nn + BN - 1) / BN;
  const int64_t nwg = (EPI == EPI_SIM_SYM || EPI == EPI_SIM_SYM16) ? (int64_t)tm * (tm + 1) / 2 : (int64_t)tm * tn;
  constexpr int KS = (EPI == EPI_DIST && MODE == MODE_F32) ? DIST_KS
                     : (EPI == EPI_SIM_SYM || EPI == EPI_SIM_SYM16) ? SIM_KS
                                                                   : 1;
  if (nwg <= 0 || nwg > 0x7FFFFFFF || kbytes % (BKB * KS) || kbytes <= 0) return hipErrorInvalidValue;
  GemmArgs g{(const uint8_t*)a, (const uint8_t*)b, M, Nn, lda, ldb, (int)(kbytes / BKB), sa, sb, out, ldo, bm, ldbm};
  hipLaunchKernelGGL((gemm_nt_kernel<MODE, EPI>), dim3((unsigned)nwg), dim3(256), 0, s, g, tm, tn);
  return hipGetLastError();
}

// Tail of a similarity product split along K, as for the final product:
// partial tiles of the last round's upper-triangle tiles (logical tiles
// first..), summed in range order by sim_fix_kernel, which applies the
// similarity epilogue (tile and mirror).
template <int MODE>
__global__ __launch_bounds__(256) void sim_part_kernel(GemmArgs g, int tiles, int first, int parts,
                                                       float* __restrict__ ws) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[gemm_stage_lds(SIM_KS)];
  const int w = xcd_linear(blockIdx.x, gridDim.x);
  const int k = w % parts;
  int tm, tn;
  upper_tile(first + w / parts, tiles, tm, tn);
  GemmArgs gp = g;
  gp.out = ws + (int64_t)w * BM * BN;
  const int64_t nsk = g.nst / SIM_KS;
  gemm_tile<MODE, EPI_PART, 1, SIM_KS>(gp, tm, tn, lds, (int)(k * nsk / parts * SIM_KS),
                                       (int)((k + 1) * nsk / parts * SIM_KS));
}

template <int EPI>
__global__ __launch_bounds__(256) void sim_fix_kernel(GemmArgs g, int tiles, int first, int parts,
                                                      const float* __restrict__ ws) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[sim_lds_bytes(EPI)];
  int tm, tn;
  upper_tile(first + (int)blockIdx.x, tiles, tm, tn);
  gemm_sim_fix_tile<EPI>(g, tm, tn, ws + (int64_t)blockIdx.x * parts * BM * BN, parts, lds);
}

// Resident workgroups of a similarity kernel (per instantiation, queried once
// per process on the current device; thread-safe initialisation).
template <int MODE, int EPI>
static int sim_slots() {
  static const int slots = [] {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)gemm_nt_kernel<MODE, EPI>, 256, 0) !=
            hipSuccess)
      return 0;
    return cus * per;
  }();
  return slots;
}

template <int MODE, int EPI>
static hipError_t launch_sim_t(const void* a, int M, int64_t lda, int64_t kbytes, const float* sa, float* out,
                               int64_t ldo, float* ws, int64_t ws_bytes, hipStream_t s, float* bm, int64_t ldbm) {
  const int T = (M + BM - 1) / BM;
  const int64_t nwg = (int64_t)T * (T + 1) / 2;
  if (nwg <= 0 || nwg > 0x7FFFFFFF || kbytes % (BKB * SIM_KS) || kbytes <= 0) return hipErrorInvalidValue;
  const int nst = (int)(kbytes / BKB);
  int64_t rem = 0;
  // at most two ranges: a similarity tile is short, so summing more partials
  // in the fix-up costs more than the finer split saves
  const int parts =
      ws ? tail_parts(nwg, sim_slots<MODE, EPI>(), nst / SIM_KS, (int64_t)BM * BN * 4, ws_bytes, 2, &rem) : 1;
  if (parts == 1)
    return launch_gemm_t<MODE, EPI>(a, M, lda, a, M, lda, kbytes, sa, sa, out, ldo, s, bm, ldbm);
  const int64_t first = nwg - rem;
  GemmArgs g{(const uint8_t*)a, (const uint8_t*)a, M, M, lda, lda, nst, sa, sa, out, ldo, bm, ldbm};
  hipLaunchKernelGGL((gemm_nt_kernel<MODE, EPI>), dim3((unsigned)first), dim3(256), 0, s, g, T, T);
  hipLaunchKernelGGL((sim_part_kernel<MODE>), dim3((unsigned)(rem * parts)), dim3(256), 0, s, g, T, (int)first, parts,
                     ws);
  hipLaunchKernelGGL((sim_fix_kernel<EPI>), dim3((unsigned)rem), dim3(256), 0, s, g, T, (int)first, parts,
                     (const float*)ws);
  return hipGetLastError();
}

hipError_t launch_gemm_sim(SimPrec prec, const void* a, int M, int64_t lda_bytes, int64_t kbytes, const float* sa,
                           void* out, int64_t ldo, bool half_out, float* ws, int64_t ws_bytes, hipStream_t s,
                           float* bm, int64_t ldbm) {
  float* o = (float*)out;
  if (half_out && prec == SimPrec::F32) return hipErrorInvalidValue;  // the FP32 path keeps S exact
  switch (prec) {
    case SimPrec::F32:
      return launch_sim_t<MODE_F32, EPI_SIM_SYM>(a, M, lda_bytes, kbytes, sa, o, ldo, ws, ws_bytes, s, bm, ldbm);
    case SimPrec::BF16:
      return half_out
                 ? launch_sim_t<MODE_BF16, EPI_SIM_SYM16>(a, M, lda_bytes, kbytes, sa, o, ldo, ws, ws_bytes, s, bm, ldbm)
                 : launch_sim_t<MODE_BF16, EPI_SIM_SYM>(a, M, lda_bytes, kbytes, sa, o, ldo, ws, ws_bytes, s, bm, ldbm);
    case SimPrec::FP8:
      return half_out
                 ? launch_sim_t<MODE_FP8, EPI_SIM_SYM16>(a, M, lda_bytes, kbytes, sa, o, ldo, ws, ws_bytes, s, bm, ldbm)
                 : launch_sim_t<MODE_FP8, EPI_SIM_SYM>(a, M, lda_bytes, kbytes, sa, o, ldo, ws, ws_bytes, s, bm, ldbm);
  }
  return hipErrorInvalidValue;
}

// Tail of the FP32 final product split along K. Tiles run in rounds of
// `slots` resident workgroups; when the last round is partly empty, its tiles
// (logical tiles first..tiles-1) are computed as `parts` K ranges each
// (gemm_part_kernel, partial tiles in `ws`) and summed in range order by
// gemm_fix_kernel, which applies the epilogue. Fixed ranges and order: the
// result is deterministic.
__global__ __launch_bounds__(256) void gemm_part_kernel(GemmArgs g, int tiles_m, int tiles_n, int first, int parts,
                                                        float* __restrict__ ws) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[gemm_stage_lds(DIST_KS)];
  const int w = xcd_linear(blockIdx.x, gridDim.x);
  const int k = w % parts;
  const TileMap t = grouped_order(first + w / parts, tiles_m, tiles_n);
  GemmArgs gp = g;
  gp.out = ws + (int64_t)((w / parts) * parts + k) * BM * BN;
  const int64_t nsk = g.nst / DIST_KS;  // whole LDS stages
  gemm_tile<MODE_F32, EPI_PART, 1, DIST_KS>(gp, t.tm, t.tn, lds, (int)(k * nsk / parts * DIST_KS),
                                            (int)((k + 1) * nsk / parts * DIST_KS));
}

__global__ __launch_bounds__(256) void gemm_fix_kernel(GemmArgs g, int tiles_m, int tiles_n, int first, int parts,
                                                       const float* __restrict__ ws) {
  const int w = blockIdx.x;
  const TileMap t = grouped_order(first + w, tiles_m, tiles_n);
  gemm_fix_tile(g, t.tm, t.tn, ws + (int64_t)w * parts * BM * BN, parts);
}


// Resident workgroups of the FP32 final product (queried once per process,
// on the device current at the first call; thread-safe initialisation).
static int dist_slots() {
  static const int slots = [] {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)gemm_nt_kernel<MODE_F32, EPI_DIST>, 256,
                                                     0) != hipSuccess)
      return 0;
    return cus * per;
  }();
  return slots;
}

hipError_t launch_gemm_dist(const float* a, int M, const float* b, int Nn, int64_t ld_elems, int64_t kelems,
                            const float* sa, const float* sb, float* out, int64_t ldo, float* ws, int64_t ws_bytes,
                            hipStream_t s) {
  const int tm = (M + BM - 1) / BM, tn = (Nn + BN - 1) / BN;
  const int64_t tiles = (int64_t)tm * tn;
  const int slots = ws ? dist_slots() : 0;
  const int nst = (int)(kelems * 4 / BKB);
  if (nst % DIST_KS) return hipErrorInvalidValue;  // K is padded to whole LDS stages
  int64_t rem = 0;
  const int parts =
      (kelems * 4 % BKB == 0) ? tail_parts(tiles, slots, nst, (int64_t)BM * BN * 4, ws_bytes, 8, &rem) : 1;
  if (parts == 1)
    return launch_gemm_t<MODE_F32, EPI_DIST>(a, M, ld_elems * 4, b, Nn, ld_elems * 4, kelems * 4, sa, sb, out, ldo, s);
  if (tiles > 0x7FFFFFFF || rem * parts > 0x7FFFFFFF) return hipErrorInvalidValue;
  const int64_t first = tiles - rem;
  GemmArgs g{(const uint8_t*)a, (const uint8_t*)b, M, Nn, ld_elems * 4, ld_elems * 4, nst, sa, sb, out, ldo};
  hipLaunchKernelGGL((gemm_nt_kernel<MODE_F32, EPI_DIST>), dim3((unsigned)first), dim3(256), 0, s, g, tm, tn);
  hipLaunchKernelGGL(gemm_part_kernel, dim3((unsigned)(rem * parts)), dim3(256), 0, s, g, tm, tn, (int)first, parts, ws);
  hipLaunchKernelGGL(gemm_fix_kernel, dim3((unsigned)rem), dim3(256), 0, s, g, tm, tn, (int)first, parts,
                     (const float*)ws);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void gemm_x3_kernel(GemmX3Args g, int tiles_m, int tiles_n) {
  extern __shared__ __attribute__((aligned(16))) uint8_t lds_x3[];
  const TileMap t = grouped_order(xcd_linear(blockIdx.x, gridDim.x), tiles_m, tiles_n);
  gemm_tile_x3(g, t.tm, t.tn, lds_x3);
}

hipError_t launch_gemm_dist_bf16(const uint16_t* a, int M, const uint16_t* b, int Nn, int64_t ld_elems,
                                 int64_t kelems, const float* sa, const float* sb, float* out, int64_t ldo,
                                 hipStream_t s) {
  if (kelems % 64 || ld_elems % 64) return hipErrorInvalidValue;  // whole 128-byte bf16 slices
  return launch_gemm_t<MODE_BF16, EPI_DIST>(a, M, ld_elems * 2, b, Nn, ld_elems * 2, kelems * 2, sa, sb, out, ldo, s);
}

// Raises the dynamic-LDS limit of gemm_x3_kernel once per process
// (thread-safe initialisation); the status of that call.
static hipError_t x3_attr() {
  static const hipError_t e = hipFuncSetAttribute((const void*)gemm_x3_kernel,
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, X3_LDS_BYTES);
  return e;
}

hipError_t launch_gemm_dist_bf16x3(const uint16_t* a_hi, const uint16_t* a_lo, int M, const uint16_t* b_hi,
                                   const uint16_t* b_lo, int Nn, int64_t ld_elems, int64_t kelems, const float* sa,
                                   const float* sb, float* out, int64_t ldo, hipStream_t s) {
  const hipError_t e = x3_attr();
  if (e != hipSuccess) return e;
  const int tm = (M + BM - 1) / BM, tn = (Nn + BN - 1) / BN;
  const int64_t nwg = (int64_t)tm * tn;
  if (nwg <= 0 || nwg > 0x7FFFFFFF || kelems % 64 || kelems <= 0 || ld_elems % 64) return hipErrorInvalidValue;
  GemmX3Args g{a_hi, a_lo, b_hi, b_lo, M, Nn, ld_elems, (int)(kelems / 64), sa, sb, out, ldo};
  hipLaunchKernelGGL(gemm_x3_kernel, dim3((unsigned)nwg), dim3(256), X3_LDS_BYTES, s, g, tm, tn);
  return hipGetLastError();
}

}  // namespace rr
