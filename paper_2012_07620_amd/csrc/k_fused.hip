// a2 + a3 fused: the Eq. 7 similarity product with the Eq. 8 candidate
// selection, so the N x N similarity S is never written.
//
// Eq. 8 keeps, per row i, the K columns of largest S_ij (ties: smaller j
// first), i.e. the K largest selection keys. Any set of columns that contains
// those K gives the same answer, so the path works in three steps:
//  1. sample: the tiles of P evenly spread column panels are computed for
//     every row and stored (M x 128P values); from them each row gets tau_i,
//     a similarity value at or below its K-th best;
//  2. emit: the upper-triangle tiles of the other panels are computed once
//     each, and every element S_ij of a tile is offered to row i and, off the
//     diagonal, to row j (S is symmetric); the stored sample tiles are offered
//     the same way. A value at or above its row's tau is appended, as its
//     selection key, to the row's candidate buffer (one atomic per row and
//     tile reserves the slots);
//  3. select: the K best keys of each buffer, in rank order.
// Every ordered pair (i, j) is offered exactly once, so a row's buffer holds
// every key at or above its K-th best. A buffer that would overflow marks its
// row panel, which the row-panel kernel (running per-range lists merged in
// the epilogue, every tile of the panel's row computed) then recomputes. All
// values come from the same tile engine and the same rounding as the unfused
// similarity (sim_value), so the selected lists are the ones the unfused
// path selects on the same bits.
#include "gemm_body.h"
#include "kernels.h"

namespace rr {

static_assert(KNN_LIST == KNN_LIST_MAX, "one merging wave holds the largest K the host admits");

// ---------------------------------------------------------------- geometry

struct FusedGeo {
  int T, P, sp, so;
  int64_t m;  // stored sample columns per row
  __device__ __forceinline__ int sample(int t) const { return so + t * sp; }
  __device__ __forceinline__ bool is_sample(int x) const {
    return x >= so && (x - so) % sp == 0 && (x - so) / sp < P;
  }
  __device__ __forceinline__ int count_le(int x) const {  // sample panels <= x
    return x < so ? 0 : min(P, (x - so) / sp + 1);
  }
  // the x-th panel that is not a sample panel: the least fixed point of
  // y = x + count_le(y), reached from below
  __device__ __forceinline__ int other(int x) const {
    int y = x;
    for (;;) {
      const int z = x + count_le(y);
      if (z == y) return y;
      y = z;
    }
  }
};

static FusedGeo geo_of(const FusedLayout& L) { return FusedGeo{L.T, L.P, L.sp, L.so, L.m}; }

// Stored similarity type of a mode. Kernels take it as a template parameter
// of its own (not as SimT<MODE> in their signatures): a type that depends on
// an unnamed enumerator is mangled differently by the host and device passes,
// so the host could not find such a kernel.
template <int MODE>
using SimT = typename std::conditional<MODE == MODE_F32, float, _Float16>::type;

// ---------------------------------------------------------------- 1. sample

// Tile (tm, sample panel t) of the product, stored as S stores it, at
// samp[row][t * 128 + c] (zeros outside the matrix). Groups of 8 row panels
// x all sample panels keep the sample rows in each XCD's L2.
template <int MODE, typename OT>
__global__ __launch_bounds__(256) void knn_sample_kernel(GemmArgs g, FusedGeo f, OT* __restrict__ samp) {
  static_assert(std::is_same<OT, SimT<MODE>>::value, "stored type of the mode");
  __shared__ __attribute__((aligned(16))) uint8_t lds[gemm_stage_lds(1)];
  const int pid = xcd_linear(blockIdx.x, gridDim.x);
  constexpr int G = 8;
  const int per = G * f.P, grp = pid / per, in = pid - grp * per;
  const int gsz = min(f.T - grp * G, G);
  const int tm = grp * G + in % gsz, t = in / gsz;
  const int tn = f.sample(t);
  f32x16 acc[2][2];
  gemm_tile_acc<MODE, 1, 1>(g, tm, tn, lds, acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int sm = 0; sm < 2; sm++)
#pragma unroll
    for (int sn = 0; sn < 2; sn++) {
      const int lc = wn * 64 + sn * 32 + (lane & 31);
      const int col = tn * BN + lc;
      const float scol = col < g.Nn ? g.sb[min(col, g.Nn - 1)] : 0.f;
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int row = tm * BM + wm * 64 + sm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        const float srow = g.sa[min(row, g.M - 1)];  // loaded outside the bounds check
        if (row < g.M)
          samp[(int64_t)row * f.m + t * BN + lc] = col < g.Nn ? sim_value<OT>(acc[sm][sn][r], srow, scol) : (OT)0.f;
      }
    }
}

// One wavefront per row i: tau_i, a similarity value at or below the row's
// K-th best: the (K-1)-th largest of its sample values, not counting its own
// column (the row itself takes rank 0), over the union of each lane's four
// largest -- a sub-multiset of the sample, whose order statistics can only be
// lower. -inf when fewer such values exist; +inf for K = 1 (only the row
// itself). Also clears the row's candidate count and, for i < T, panel i's
// overflow mark.
template <typename OT>
__global__ __launch_bounds__(256) void knn_tau_kernel(const OT* __restrict__ samp, FusedGeo f, int n, int K,
                                                      float* __restrict__ tau, int* __restrict__ cnt,
                                                      int* __restrict__ flag) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  constexpr float NEG = -__builtin_inff();
  float l0 = NEG, l1 = NEG, l2 = NEG, l3 = NEG;  // this lane's four largest, descending
  const OT* row = samp + (int64_t)i * f.m;
  auto put = [&](float v) {
    l3 = fmaxf(l3, fminf(l2, v));
    l2 = fmaxf(l2, fminf(l1, v));
    l1 = fmaxf(l1, fminf(l0, v));
    l0 = fmaxf(l0, v);
  };
  for (int64_t b = 0; b < f.m; b += 256) {
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int t = (int)b + u * 64 + lane;
      const int j = f.sample(t / BN) * BN + t % BN;
      const float s = t < f.m ? (float)row[t] : NEG;
      v[u] = (t < f.m && j < n && j != i && s == s) ? s : NEG;  // a NaN ranks last, as in the keys
    }
#pragma unroll
    for (int u = 0; u < 4; u++) put(v[u]);
  }
  float t = __builtin_inff();
  if (K > 1) {
    uint64_t k[4] = {(uint64_t)ord_f32(l0) << 32, (uint64_t)ord_f32(l1) << 32, (uint64_t)ord_f32(l2) << 32,
                     (uint64_t)ord_f32(l3) << 32};
    wave_sort_desc<4>(k);
    t = unord_f32((uint32_t)(wave_rank_key<4>(k, K - 2) >> 32));
  }
  if (lane == 0) {
    tau[i] = t;
    cnt[i] = 0;
    if (i < f.T) flag[i] = 0;
  }
}

// ---------------------------------------------------------------- 2. emit

struct EmitArgs {
  const float* tau;
  int* cnt;
  uint64_t* cand;
  int64_t C;
  int n;
};

template <int MODE>
__host__ __device__ constexpr int emit_ts() {  // staged tile row stride (elements): conflict-free columns
  return MODE == MODE_F32 ? BN + 1 : BN + 2;
}
template <int MODE>
__host__ __device__ constexpr int emit_tile_bytes() {
  return BM * emit_ts<MODE>() * (MODE == MODE_F32 ? 4 : 2);
}
template <int MODE>
__host__ __device__ constexpr int emit_lds_bytes() {
  return emit_tile_bytes<MODE>() + 256 * 4 > gemm_stage_lds(1) ? emit_tile_bytes<MODE>() + 256 * 4
                                                                 : gemm_stage_lds(1);
}

// Offer the staged tile (rows of panel tm x columns of panel tn) to its rows
// (row side) and, when col_side, to its columns' rows (column side). Lane
// half 0 of wave w collects for tile row 32w + l, half 1 for tile column
// 32w + l: one pass marks the elements whose similarity reaches the row's
// tau in a 128-bit mask, one atomic reserves that many slots, then the marked
// keys are stored. Every key at or above the row's K-th best is marked (some
// equal to tau but ranked below it may be too; the selection drops them).
// Column-side lanes walk the elements from a 32-element offset, so the two
// halves read different LDS banks. vt: thresholds of the tile rows (0..127)
// and of the tile columns' rows (128..255).
template <typename OT>
__device__ __forceinline__ void emit_tile(const OT* T, int TS, const float* vt, int tm, int tn, bool col_side,
                                          const EmitArgs& e) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool colh = lane >= 32;
  const int x = wave * 32 + (lane & 31);
  const int m0 = tm * BM, n0 = tn * BN;
  const int self = colh ? n0 + x : m0 + x;  // the matrix row this lane collects for
  const int other0 = colh ? m0 : n0;        // element c lies in matrix column other0 + c
  const int step = colh ? TS : 1;
  const int off = colh ? 32 : 0;
  const bool active = self < e.n && (!colh || col_side);
  const bool full = m0 + BM <= e.n && n0 + BN <= e.n;
  const bool diag = tm == tn;  // then col_side is false: the row's own column is element x
  const OT th = (OT)vt[colh ? BM + x : x];  // exact: tau is a stored value or +-inf
  const OT* src = T + (colh ? x : x * TS);
  uint32_t bits[4] = {0u, 0u, 0u, 0u};
  if (active) {
    if (full) {
#pragma unroll
      for (int k = 0; k < BN; k++) {
        const int c = (k + off) & (BN - 1);
        bits[k >> 5] |= (uint32_t)(src[c * step] >= th) << (k & 31);
      }
    } else {
#pragma unroll 8
      for (int k = 0; k < BN; k++) {
        const int c = (k + off) & (BN - 1);
        bits[k >> 5] |= (uint32_t)(src[c * step] >= th && other0 + c < e.n) << (k & 31);
      }
    }
    if (diag) bits[x >> 5] |= 1u << (x & 31);  // off = 0 on the row side
  }
  const int cnt = __popc(bits[0]) + __popc(bits[1]) + __popc(bits[2]) + __popc(bits[3]);
  if (cnt == 0) return;
  int pos = atomicAdd(e.cnt + self, cnt);
  uint64_t* dst = e.cand + (int64_t)self * e.C;
#pragma unroll
  for (int w = 0; w < 4; w++) {
    uint32_t b = bits[w];
    while (b) {
      const int k = w * 32 + __builtin_ctz(b);
      b &= b - 1;
      const int c = (k + off) & (BN - 1);
      const int o = other0 + c;
      if (pos < e.C) dst[pos] = o == self ? self_key((uint32_t)self) : sel_key((float)src[c * step], (uint32_t)o);
      pos++;
    }
  }
}

// Workgroups [0, nsym): upper-triangle tiles of the non-sample panels,
// computed on the matrix cores; [nsym, nsym + T * P): the stored sample
// tiles (row panel q / P, sample panel q % P), offered to their column side
// only when the row panel is not itself a sample panel (else the mirrored
// pair is a stored sample tile of its own).
// FP8 tiles are held to three waves per SIMD, as the FP8 similarity kernel.
template <int MODE, typename OT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == MODE_FP8 ? 3 : 1)))
void knn_emit_kernel(GemmArgs g, FusedGeo f, const OT* __restrict__ samp, EmitArgs e, int nsym) {
  static_assert(std::is_same<OT, SimT<MODE>>::value, "stored type of the mode");
  constexpr int TS = emit_ts<MODE>();
  __shared__ __attribute__((aligned(16))) uint8_t lds[emit_lds_bytes<MODE>()];
  OT* T = (OT*)lds;
  float* vt = (float*)(lds + emit_tile_bytes<MODE>());
  const int tid = threadIdx.x;
  const int bid = blockIdx.x;
  int tm, tn;
  bool col_side;
  if (bid < nsym) {
    int a, b;
    upper_tile(xcd_linear(bid, nsym), f.T - f.P, a, b);
    tm = f.other(a);
    tn = f.other(b);
    col_side = tm != tn;
    f32x16 acc[2][2];
    gemm_tile_acc<MODE, 1, 1>(g, tm, tn, lds, acc);
    const int lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
#pragma unroll
    for (int sm = 0; sm < 2; sm++)
#pragma unroll
      for (int sn = 0; sn < 2; sn++) {
        const int lc = wn * 64 + sn * 32 + (lane & 31);
        const int col = tn * BN + lc;
        const float scol = col < g.Nn ? g.sb[min(col, g.Nn - 1)] : 0.f;
#pragma unroll
        for (int r = 0; r < 16; r++) {
          const int lr = wm * 64 + sm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
          const int row = tm * BM + lr;
          const float srow = g.sa[min(row, g.M - 1)];  // loaded outside the bounds check
          T[lr * TS + lc] = (row < g.M && col < g.Nn) ? sim_value<OT>(acc[sm][sn][r], srow, scol) : (OT)0.f;
        }
      }
  } else {
    const int q = bid - nsym;
    tm = q / f.P;
    const int t = q % f.P;
    tn = f.sample(t);
    col_side = !f.is_sample(tm);
    constexpr int V = 16 / (int)sizeof(OT);  // elements per 16-byte load
    typedef OT ov __attribute__((ext_vector_type(V)));
    for (int x = tid; x < BM * BN / V; x += 256) {
      const int lr = x / (BN / V), c = x % (BN / V) * V;
      const int row = tm * BM + lr;
      ov v = {};
      if (row < e.n) v = *(const ov*)(samp + (int64_t)row * f.m + t * BN + c);
#pragma unroll
      for (int u = 0; u < V; u++) T[lr * TS + c + u] = v[u];
    }
  }
  {
    const int r = tid < BM ? tm * BM + tid : tn * BN + (tid - BM);
    vt[tid] = r < e.n ? e.tau[r] : __builtin_inff();
  }
  __syncthreads();
  emit_tile<OT>(T, TS, vt, tm, tn, col_side, e);
}

// ---------------------------------------------------------------- 3. select

// One wavefront per row: the K best keys of its candidate buffer, written as
// the candidate list (column, similarity; the row itself first with 1). A
// buffer that overflowed marks the row's panel for the row-panel kernel.
__global__ __launch_bounds__(256) void knn_select_kernel(const uint64_t* __restrict__ cand,
                                                         const int* __restrict__ cnt, int n, int64_t C, int K,
                                                         int* __restrict__ flag, int32_t* __restrict__ idx,
                                                         float* __restrict__ val) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int c = cnt[i];
  // an overflowed buffer, or fewer than K kept values (possible only when the
  // bound and the values disagree, as with non-finite inputs): the row panel
  // is recomputed in full
  if (c > C || c < K) {
    if (lane == 0) flag[i / BM] = 1;
    return;
  }
  const uint64_t* src = cand + (int64_t)i * C;
  uint64_t best[1] = {0ull};
  uint64_t kth = 0ull;
  for (int b = 0; b < c; b += 256) {
    uint64_t x[4];
#pragma unroll
    for (int u = 0; u < 4; u++) x[u] = b + u * 64 + lane < c ? src[b + u * 64 + lane] : 0ull;
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint64_t y = x[u] > kth ? x[u] : 0ull;
      if (!__ballot(y != 0ull)) continue;
      wave_merge_batch<1>(best, y);
      kth = wave_rank_key<1>(best, K - 1);
    }
  }
  if (lane < K) {
    const uint32_t j = key_col(best[0]);
    idx[(int64_t)i * K + lane] = (int32_t)j;
    val[(int64_t)i * K + lane] = (j == (uint32_t)i) ? 1.0f : key_val(best[0]);
  }
}

// ---------------------------------------------------------------- fallback

// Row-panel kernel: each workgroup owns a panel of 128 rows and one range of
// column tiles; it computes those tiles one after another and merges each
// into the K best keys of each of its rows (knn_epilogue: lists in the
// workgroup's slice of the per-range list buffer, thresholds in LDS); a second
// kernel merges the per-range lists of every row. Every tile of the panel's
// row is computed. Only panels marked in `gate` run.
template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void knn_panel_kernel(GemmArgs g, int tiles_m, int tiles_n, int ranges, int tpr, int K, uint64_t* __restrict__ part,
                      const int* __restrict__ gate) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[knn_lds_bytes(MODE)];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tm = (int)blockIdx.x / ranges, rg = (int)blockIdx.x % ranges;
  if (!gate[tm]) return;
  KnnShared& ks = *(KnnShared*)(lds + knn_stage_bytes(MODE));
  if (tid < BM) {
    ks.tau[tid] = 0ull;
    ks.have[tid] = 0;
  }
  if (tid == 0) {
    ks.lists = part;
    ks.K = K;
    ks.range = rg;
  }
  __syncthreads();
  const int t0 = rg * tpr, t1 = min(tiles_n, t0 + tpr);
  for (int tn = t0; tn < t1; tn++) {
    if (tid == 0) ks.first = tn == t0;  // read after the tile's first barrier
    gemm_tile<MODE, EPI_KNN, 1, 1>(g, tm, tn, lds);
  }
  for (int lr = wave * 32; lr < wave * 32 + 32; lr++) {  // empty entries of lists shorter than K
    const int i = tm * BM + lr;
    if (i >= g.M) break;
    if (lane >= ks.have[lr] && lane < K) part[((int64_t)rg * g.M + i) * K + lane] = 0ull;
  }
}

// One wavefront per row of a marked panel: the K best of its per-range lists.
__global__ __launch_bounds__(256) void knn_merge_kernel(const uint64_t* __restrict__ part, int n, int ranges, int K,
                                                        const int* __restrict__ gate, int32_t* __restrict__ idx,
                                                        float* __restrict__ val) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n || !gate[i / BM]) return;
  uint64_t best[1] = {0ull};
  for (int r = 0; r < ranges; r++) {
    const uint64_t b = lane < K ? part[((int64_t)r * n + i) * K + lane] : 0ull;
    wave_merge_batch<1>(best, b);
  }
  if (lane < K) {
    const uint32_t j = key_col(best[0]);
    idx[(int64_t)i * K + lane] = (int32_t)j;
    val[(int64_t)i * K + lane] = (j == (uint32_t)i) ? 1.0f : key_val(best[0]);
  }
}

// ---------------------------------------------------------------- launch

template <int MODE>
static hipError_t launch_fused_t(const void* a, int M, int64_t lda, int64_t kbytes, const float* sa, int K, void* ws,
                                 int32_t* idx, float* val, hipStream_t s) {
  using OT = SimT<MODE>;
  const FusedLayout L = fused_layout(M, K, (int)sizeof(OT));
  const FusedGeo f = geo_of(L);
  char* base = (char*)ws;
  OT* samp = (OT*)(base + L.o_samp);
  uint64_t* cand = (uint64_t*)(base + L.o_cand);
  float* tau = (float*)(base + L.o_tau);
  int* cnt = (int*)(base + L.o_cnt);
  int* flag = (int*)(base + L.o_flag);
  const GemmArgs g{(const uint8_t*)a, (const uint8_t*)a, M, M, lda, lda, (int)(kbytes / BKB), sa, sa, nullptr, 0};
  const int rows4 = (M + 3) / 4;
  hipLaunchKernelGGL((knn_sample_kernel<MODE, OT>), dim3((unsigned)(L.T * L.P)), dim3(256), 0, s, g, f, samp);
  hipLaunchKernelGGL(knn_tau_kernel<OT>, dim3((unsigned)rows4), dim3(256), 0, s, (const OT*)samp, f, M, K, tau, cnt,
                     flag);
  const int To = L.T - L.P;
  const int64_t nsym = (int64_t)To * (To + 1) / 2;
  const int64_t nwg = nsym + (int64_t)L.T * L.P;
  if (nwg > 0x7FFFFFFF) return hipErrorInvalidValue;
  const EmitArgs e{tau, cnt, cand, L.C, M};
  hipLaunchKernelGGL((knn_emit_kernel<MODE, OT>), dim3((unsigned)nwg), dim3(256), 0, s, g, f, (const OT*)samp, e,
                     (int)nsym);
  hipLaunchKernelGGL(knn_select_kernel, dim3((unsigned)rows4), dim3(256), 0, s, (const uint64_t*)cand,
                     (const int*)cnt, M, L.C, K, flag, idx, val);
  // rows whose buffer overflowed: their panels recomputed row-panel-wise, the
  // per-range lists in the candidate buffer (ranges * M * K <= M * C)
  int ranges = (int)(L.C / K);
  if (ranges > kKnnMaxRanges) ranges = kKnnMaxRanges;
  if (ranges > L.T) ranges = L.T;
  const int tpr = (L.T + ranges - 1) / ranges;
  hipLaunchKernelGGL(knn_panel_kernel<MODE>, dim3((unsigned)(L.T * ranges)), dim3(256), 0, s, g, L.T, L.T, ranges,
                     tpr, K, cand, (const int*)flag);
  hipLaunchKernelGGL(knn_merge_kernel, dim3((unsigned)rows4), dim3(256), 0, s, (const uint64_t*)cand, M, ranges, K,
                     (const int*)flag, idx, val);
  return hipGetLastError();
}

hipError_t launch_knn_fused(SimPrec prec, const void* a, int M, int64_t lda_bytes, int64_t kbytes, const float* sa,
                            int K, void* ws, int32_t* idx, float* val, hipStream_t s) {
  if (M < 1 || K < 1 || K > KNN_LIST || K > M || kbytes % BKB || lda_bytes < kbytes || lda_bytes % 16)
    return hipErrorInvalidValue;
  switch (prec) {
    case SimPrec::F32:
      return launch_fused_t<MODE_F32>(a, M, lda_bytes, kbytes, sa, K, ws, idx, val, s);
    case SimPrec::BF16:
      return launch_fused_t<MODE_BF16>(a, M, lda_bytes, kbytes, sa, K, ws, idx, val, s);
    case SimPrec::FP8:
      return launch_fused_t<MODE_FP8>(a, M, lda_bytes, kbytes, sa, K, ws, idx, val, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace rr
