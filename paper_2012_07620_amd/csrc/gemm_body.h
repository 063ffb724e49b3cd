// Tile engine of the "NT" products C = A * B^T on gfx950 matrix cores,
// shared by the direct launches (one tile per workgroup) and the persistent
// grouped launches of the serving path (workgroups loop over tiles).
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
#pragma once
#include <type_traits>

#include "common.h"

namespace rr {

constexpr int BM = 128, BN = 128, BKB = 128, LDSR = BKB + 16, TILEB = BM * LDSR;
constexpr int GEMM_LDS_BYTES = 4 * TILEB;  // 73728: two stage buffers, or one + the mirror-tile staging
constexpr int GEMM_LDS_1BUF = 2 * TILEB;   // 36864: one stage buffer (EPI_DIST)

enum { MODE_F32 = 0, MODE_BF16 = 1, MODE_FP8 = 2 };
// EPI_SIM_SYM16: EPI_SIM_SYM storing S as IEEE binary16 (the low-precision
// paths, whose S only ranks candidates that are then re-scored in FP32).
// EPI_PART: no epilogue; the raw accumulators of a K range go to a 128 x 128
// partial tile (g.out, tile-local layout) for a later fixed-order sum.
// EPI_KNN: the similarity tile is not stored; its values are merged into the
// running top-K lists of the tile's rows (knn_epilogue).
enum { EPI_DIST = 1, EPI_SIM_SYM = 2, EPI_SIM_SYM16 = 3, EPI_PART = 4, EPI_KNN = 5 };
// LDS of a similarity tile (one stage buffer, reused for staging the output
// tile): FP32 S needs 128 x 132 floats, binary16 S fits in the stage buffer.
__host__ __device__ constexpr int sim_lds_bytes(int epi) {
  return epi == EPI_SIM_SYM16 ? GEMM_LDS_1BUF : GEMM_LDS_BYTES;
}
// Layout of that LDS in the epilogue: the staged tile (128 rows of 128 + one
// 16-byte run of padding, in the output type), the column-maximum join (256
// floats), then the tile's scales (256 floats: rows m0 .., columns n0 ..).
__host__ __device__ constexpr int sim_stage_bytes(int epi) {
  return epi == EPI_SIM_SYM16 ? BM * (BN + 8) * 2 : BM * (BN + 4) * 4;
}
__host__ __device__ constexpr int sim_join_off(int epi) { return (sim_stage_bytes(epi) + 15) & ~15; }
__host__ __device__ constexpr int sim_scale_off(int epi) { return sim_join_off(epi) + 256 * 4; }
static_assert(sim_scale_off(EPI_SIM_SYM) + 256 * 4 <= sim_lds_bytes(EPI_SIM_SYM), "FP32 epilogue LDS");
static_assert(sim_scale_off(EPI_SIM_SYM16) + 256 * 4 <= sim_lds_bytes(EPI_SIM_SYM16), "binary16 epilogue LDS");

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

// Stored similarity of an accumulator value with its row and column inverse
// norms: FP32, or binary16 rounded to nearest even in the low-precision
// paths; -0 becomes +0. Every kernel that writes or keys on S uses this one
// expression, so all of them see the same bits.
template <typename OT>
__device__ __forceinline__ OT sim_value(float acc, float sa, float sb) {
  return (OT)(acc * sa * sb + 0.0f);
}

struct GemmArgs {
  const uint8_t* A;
  const uint8_t* B;
  int M, Nn;
  int64_t lda, ldb;  // bytes
  int nst;           // 128-byte K stages
  const float* sa;
  const float* sb;
  float* out;
  int64_t ldo;  // floats
  // similarity epilogues: when set, bm[b * ldbm + i] = the largest stored
  // similarity of row i over column block b (columns 128 b .. 128 b + 127);
  // block-major, so a tile's rows write one contiguous run
  float* bm = nullptr;
  int64_t ldbm = 0;
};

// This thread's share of tile (tm, tn)'s scales: the row scale of row
// m0 + t (threads t < 128), else the column scale of column n0 + t - 128;
// 0 outside the matrix. Fetched before the tile's K loop, so its latency
// hides behind the products, and put in LDS for the epilogue.
__device__ __forceinline__ float sim_scale_fetch(const GemmArgs& g, int tm, int tn) {
  const int t = threadIdx.x;
  if (t < BM) {
    const int r = tm * BM + t;
    return r < g.M ? g.sa[r] : 0.f;
  }
  const int c = tn * BN + t - BM;
  return c < g.Nn ? g.sb[c] : 0.f;
}
template <int EPI>
__device__ __forceinline__ void sim_scale_put(uint8_t* lds, float v) {
  ((float*)(lds + sim_scale_off(EPI)))[threadIdx.x] = v;
  __syncthreads();
}

// Similarity epilogue of tile (tm, tn) from its accumulators (EPI_SIM_SYM or
// EPI_SIM_SYM16); uses `lds` (sim_lds_bytes(EPI)), which holds the tile's
// scales (sim_scale_put) on entry, and block barriers.
template <int EPI>
__device__ __forceinline__ void sim_epilogue(const GemmArgs& g, int tm, int tn, const f32x16 (&acc)[2][2],
                                             uint8_t* lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = tm * BM, n0 = tn * BN;
  // Similarity: the scaled tile is staged row-major in LDS (free after the
  // loop's last barrier) in the output type (binary16 values are rounded
  // here, once, as a direct store would), then written with 16-byte stores
  // per lane: rows of the tile at (tm, tn) and, off the diagonal, rows of
  // its transpose at (tn, tm) (lanes along the tile's columns, each
  // gathering one 16-byte run of a transposed row). Zeros stand in outside
  // M x Nn and are not stored.
  constexpr bool H16 = (EPI == EPI_SIM_SYM16);
  using OT = typename std::conditional<H16, _Float16, float>::type;
  constexpr int V = 16 / (int)sizeof(OT);  // elements per 16-byte store
  constexpr int TS = BN + V;               // staged row stride (16-byte aligned rows)
  static_assert(BM * TS * (int)sizeof(OT) == sim_stage_bytes(EPI), "staged tile layout");
  typedef OT ov __attribute__((ext_vector_type(V)));
  OT* T = (OT*)lds;
  // Scales are 0 outside the matrix, so those entries stage as +0 with no
  // branch (they are neither stored nor counted in a maximum).
  const float* sc = (const float*)(lds + sim_scale_off(EPI));
#pragma unroll
  for (int sm = 0; sm < 2; sm++) {
    f32x4 rs[4];  // row scales of this lane's rows 8 j + 4 (lane / 32) + e of the sub-block
#pragma unroll
    for (int j = 0; j < 4; j++) rs[j] = *(const f32x4*)(sc + wm * 64 + sm * 32 + j * 8 + (lane >> 5) * 4);
#pragma unroll
    for (int sn = 0; sn < 2; sn++) {
      const int lc = wn * 64 + sn * 32 + (lane & 31);
      const float scol = sc[BM + lc];
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int lr = wm * 64 + sm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        T[lr * TS + lc] = sim_value<OT>(acc[sm][sn][r], rs[r >> 2][r & 3], scol);
      }
    }
  }
  __syncthreads();
  constexpr int CPR = BN / V;           // 16-byte chunks per tile row
  constexpr int RPP = 256 / CPR;        // tile rows per pass
  OT* out = (OT*)g.out;                 // ldo counts elements of the output type
  const bool vec = (((uintptr_t)g.out & 15) == 0) && (g.ldo % V == 0);
  auto put = [&](int64_t row, int col0, int lim, const ov& v) {  // V values at (row, col0..), cols < lim
    if (vec && col0 + V <= lim) {
      *(ov*)(out + row * g.ldo + col0) = v;
    } else {
#pragma unroll
      for (int e = 0; e < V; e++)
        if (col0 + e < lim) out[row * g.ldo + col0 + e] = v[e];
    }
  };
  // the tile: lanes along a row (CPR consecutive lanes of one wavefront per
  // row; a group of CPR lanes takes rows grp, grp + RPP, ..., NP of them)
  constexpr int NP = BM / RPP;
  static_assert(NP == CPR / 2, "each lane pair of a group ends with one row's maximum");
  const int grp = tid / CPR, ch = tid % CPR;
  float rm[NP];  // this lane's maximum over its V columns of each of its rows
#pragma unroll
  for (int k = 0; k < NP; k++) {
    const int lr = grp + k * RPP;
    const int row = m0 + lr;
    const ov v = *(const ov*)(T + lr * TS + ch * V);
    if (row < g.M) put(row, n0 + ch * V, g.Nn, v);
    rm[k] = -__builtin_inff();
#pragma unroll
    for (int e = 0; e < V; e++)
      if (n0 + ch * V + e < g.Nn) rm[k] = fmaxf(rm[k], (float)v[e]);
  }
  if (g.bm) {
    // each row's maximum over this column block, by a reduce-scatter over the
    // group's lanes: at step m the lane with bit m set keeps the upper half of
    // the rows it still holds and takes its partner's values for them; the
    // pair (2j, 2j + 1) ends holding one row, whose index is read off the bits
    int k = 0;
#pragma unroll
    for (int m = CPR / 2; m >= 2; m >>= 1) {
      const int h = NP * m / CPR;  // rows still held per lane after this step
      const bool up = (ch & m) != 0;
#pragma unroll
      for (int j = 0; j < NP / 2; j++) {
        if (j < h) {
          const float send = up ? rm[j] : rm[j + h];
          const float keep = up ? rm[j + h] : rm[j];
          rm[j] = fmaxf(keep, __shfl_xor(send, m, kWave));
        }
      }
      if (up) k += h;
    }
    rm[0] = fmaxf(rm[0], __shfl_xor(rm[0], 1, kWave));
    const int row = m0 + grp + k * RPP;
    if ((ch & 1) == 0 && row < g.M) g.bm[(int64_t)tn * g.ldbm + row] = rm[0];
  }
  if (tm != tn) {  // the transpose: lane = tile column, one V-run of tile rows each
    const int lc = tid & 127;
    const int row = n0 + lc;
    float cmx = -__builtin_inff();
    for (int ch = tid >> 7; ch < BM / V; ch += 2) {
      ov v;
#pragma unroll
      for (int e = 0; e < V; e++) v[e] = T[(ch * V + e) * TS + lc];
      if (row < g.Nn) put(row, m0 + ch * V, g.M, v);
#pragma unroll
      for (int e = 0; e < V; e++)
        if (m0 + ch * V + e < g.M) cmx = fmaxf(cmx, (float)v[e]);
    }
    if (g.bm) {  // row n0 + lc's maximum over column block tm: two halves, joined in LDS after the tile
      float* cm = (float*)(lds + sim_join_off(EPI));
      cm[tid] = cmx;
      __syncthreads();
      if (tid < BN && row < g.Nn) g.bm[(int64_t)tm * g.ldbm + row] = fmaxf(cm[tid], cm[tid + BN]);
    }
  }
}

// ---------------------------------------------------------------- fused top-k
// The fused similarity + top-K workgroup keeps, per tile row, its list of the
// K best selection keys so far (descending, key 0 = empty) in its own slice
// of the per-range list buffer in global memory (read and written only by the
// wave that owns the row), and in LDS after the stage buffers (which also
// stage each tile) the row's K-th key and list length, then K, the list
// buffer's base and the range index.
struct KnnShared {
  uint64_t tau[BM];  // K-th key of each tile row's list (0 while shorter than K)
  int have[BM];      // entries in each tile row's list
  uint64_t* lists;   // per-range lists, [range][M][K]
  int K, range;
  int first;         // the current tile is the first of the range (lists empty)
};
__host__ __device__ constexpr int knn_stage_bytes(int mode) {
  return mode == MODE_F32 ? GEMM_LDS_BYTES : GEMM_LDS_1BUF;  // FP32 or binary16 tile staging
}
__host__ __device__ constexpr int knn_lds_bytes(int mode) { return knn_stage_bytes(mode) + (int)sizeof(KnnShared); }
constexpr int KNN_LIST = 64;  // largest K: one key per lane of the merging wave
constexpr int KNN_RC = 8;     // rows whose filter and list loads are issued together

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// Selection key of staged tile element (lr, c) for row i (0 outside the matrix).
template <typename OT>
__device__ __forceinline__ uint64_t knn_key(const OT* T, int TS, int lr, int i, int c, int n0, const GemmArgs& g) {
  const int col = n0 + c;
  if (i >= g.M || col >= g.Nn) return 0ull;
  return col == i ? self_key((uint32_t)i) : sel_key((float)T[lr * TS + c], (uint32_t)col);
}

__device__ __forceinline__ uint64_t* knn_list(const KnnShared& ks, int i, int M) {
  return ks.lists + ((int64_t)ks.range * M + i) * ks.K;
}

__device__ __forceinline__ void knn_set_row(KnnShared& ks, int lr, int n_new, uint64_t kth) {
  if ((threadIdx.x & 63) == 0) {
    ks.tau[lr] = n_new == ks.K ? kth : 0ull;
    ks.have[lr] = n_new;
  }
}

// First tile of a range: row lr's list is the K best of the tile's 128 keys.
template <typename OT>
__device__ __forceinline__ void knn_first_row(const OT* T, int TS, KnnShared& ks, int lr, int i, int n0,
                                              const GemmArgs& g) {
  const int lane = threadIdx.x & 63;
  const int K = ks.K;
  uint64_t v[2] = {knn_key(T, TS, lr, i, lane, n0, g), knn_key(T, TS, lr, i, 64 + lane, n0, g)};
  const int cnt = __popcll(__ballot(v[0] != 0ull)) + __popcll(__ballot(v[1] != 0ull));
  wave_sort_desc<2>(v);
  if (lane < K) knn_list(ks, i, g.M)[lane] = v[0];
  knn_set_row(ks, lr, min(K, cnt), readlane_u64(v[0], K - 1));
}

// Later tiles: the keys of row lr that beat its K-th key merged into its list
// L (lane e holds entry e). Keys are distinct, so an element's place in the
// merged list is the number of elements of both sets above it: found with one
// pass over the new keys, then every element is stored once.
template <typename OT>
__device__ __forceinline__ void knn_rank_merge(const OT* T, int TS, KnnShared& ks, int lr, int i, int n0,
                                               const GemmArgs& g, uint64_t L) {
  const int lane = threadIdx.x & 63;
  const int K = ks.K;
  uint64_t* gl = knn_list(ks, i, g.M);
  const uint64_t tau = ks.tau[lr];
  const uint64_t k0 = knn_key(T, TS, lr, i, lane, n0, g), k1 = knn_key(T, TS, lr, i, 64 + lane, n0, g);
  const bool s0 = k0 > tau, s1 = k1 > tau;
  const uint64_t p0 = __ballot(s0), p1 = __ballot(s1);
  int up = 0, r0 = 0, r1 = 0, a0 = 0, a1 = 0;
#pragma unroll
  for (int h = 0; h < 2; h++) {
    uint64_t pend = h ? p1 : p0;
    while (pend) {
      const int l = __ffsll((unsigned long long)pend) - 1;
      pend &= pend - 1;
      const uint64_t x = readlane_u64(h ? k1 : k0, l);
      up += x > L;
      r0 += x > k0;
      r1 += x > k1;
      const int above = __popcll(__ballot(L > x));
      if (lane == l) {
        if (h) a1 = above;
        else a0 = above;
      }
    }
  }
  const int dL = lane + up, d0 = r0 + a0, d1 = r1 + a1;
  if (L != 0ull && dL < K) gl[dL] = L;
  if (s0 && d0 < K) gl[d0] = k0;
  if (s1 && d1 < K) gl[d1] = k1;
  // the entry that lands at K - 1 is the new K-th key
  const uint64_t mL = __ballot(L != 0ull && dL == K - 1), m0 = __ballot(s0 && d0 == K - 1),
                 m1 = __ballot(s1 && d1 == K - 1);
  const uint64_t kth = mL   ? readlane_u64(L, __ffsll((unsigned long long)mL) - 1)
                       : m0 ? readlane_u64(k0, __ffsll((unsigned long long)m0) - 1)
                       : m1 ? readlane_u64(k1, __ffsll((unsigned long long)m1) - 1)
                            : 0ull;
  knn_set_row(ks, lr, min(K, ks.have[lr] + __popcll(p0) + __popcll(p1)), kth);
}

// Similarity tile (tm, tn), scaled exactly as the stored similarity (binary16
// rounding in the low-precision modes, as their S), merged into the K best
// keys of each tile row under (similarity desc, column asc), the row's own
// column first. Wave w owns tile rows 32w .. 32w + 31; after the first tile it
// finds, eight rows at a time, the rows with a key beating their K-th key,
// loads those rows' lists and merges them.
template <int MODE>
__device__ __forceinline__ void knn_epilogue(const GemmArgs& g, int tm, int tn, const f32x16 (&acc)[2][2],
                                             uint8_t* lds) {
  using OT = typename std::conditional<MODE == MODE_F32, float, _Float16>::type;
  constexpr int TS = BN + 16 / (int)sizeof(OT);
  static_assert(BM * TS * (int)sizeof(OT) <= knn_stage_bytes(MODE), "staged tile must fit the stage buffers");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = tm * BM, n0 = tn * BN;
  OT* T = (OT*)lds;
  KnnShared& ks = *(KnnShared*)(lds + knn_stage_bytes(MODE));
#pragma unroll
  for (int sm = 0; sm < 2; sm++)
#pragma unroll
    for (int sn = 0; sn < 2; sn++) {
      const int lc = wn * 64 + sn * 32 + (lane & 31);
      const int col = n0 + lc;
      const float scol = (col < g.Nn) ? g.sb[min(col, g.Nn - 1)] : 0.f;
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int lr = wm * 64 + sm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        const int row = m0 + lr;
        const float srow = g.sa[min(row, g.M - 1)];  // loaded outside the bounds check
        T[lr * TS + lc] = (row < g.M && col < g.Nn) ? sim_value<OT>(acc[sm][sn][r], srow, scol) : (OT)0.f;
      }
    }
  __syncthreads();
  if (ks.first) {
    for (int lr = wave * 32; lr < wave * 32 + 32 && m0 + lr < g.M; lr++) knn_first_row(T, TS, ks, lr, m0 + lr, n0, g);
    return;
  }
  __threadfence_block();  // the lists stored by this wave's merges of earlier tiles
  for (int r0 = wave * 32; r0 < wave * 32 + 32; r0 += KNN_RC) {
    uint32_t todo = 0;
#pragma unroll
    for (int u = 0; u < KNN_RC; u++) {
      const int lr = r0 + u, i = m0 + lr;
      const uint64_t tau = ks.tau[lr];
      const bool any = knn_key(T, TS, lr, i, lane, n0, g) > tau || knn_key(T, TS, lr, i, 64 + lane, n0, g) > tau;
      if (__ballot(any)) todo |= 1u << u;
    }
    if (!todo) continue;
    uint64_t L[KNN_RC];
#pragma unroll
    for (int u = 0; u < KNN_RC; u++) {
      const int lr = r0 + u;
      L[u] = ((todo >> u) & 1) && lane < ks.have[lr] ? knn_list(ks, m0 + lr, g.M)[lane] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < KNN_RC; u++)
      if ((todo >> u) & 1) knn_rank_merge(T, TS, ks, r0 + u, m0 + r0 + u, n0, g, L[u]);
  }
}

// LDS bytes of one stage buffer pair (A and B) holding KS 128-byte K slices.
__host__ __device__ constexpr int gemm_stage_lds(int ks) { return 2 * BM * (ks * BKB + 16); }

// One 128 x 128 output tile (tm, tn). Uses `lds` (gemm_stage_lds(KS) bytes for
// NBUF = 1 with EPI_DIST / EPI_PART, else GEMM_LDS_BYTES) and block barriers:
// every thread of the workgroup must call it with the same tile. NBUF = 1
// keeps one LDS stage and prefetches the next into registers (more workgroups
// per CU; measured faster than NBUF = 2 double buffering on the 19281-row
// problem). KS 128-byte K slices share one LDS stage (one barrier pair per
// KS slices; the similarity's mirror staging fits in the same LDS); the K
// range [st0, st1), counted in slices, must then be whole stages. EPI_SIM_SYM / EPI_SIM_SYM16 (A == B, tm <= tn): also stores the
// mirrored tile C^T, so only the upper triangle of tiles is computed.
// gemm_tile_acc: the products of tile (tm, tn) over K slices [st0, st1) into
// `acc` (FP32, the 32x32 MFMA layout), no epilogue; LDS is free again when it
// returns. gemm_tile: the same followed by the EPI epilogue.
template <int MODE, int NBUF = 1, int KS = 1>
__device__ __forceinline__ void gemm_tile_acc(const GemmArgs& g, int tm, int tn, uint8_t* lds, f32x16 (&acc)[2][2],
                                              int st0 = 0, int st1 = -1) {
  static_assert(KS == 1 || (NBUF == 1 && gemm_stage_lds(KS) <= GEMM_LDS_BYTES), "wide stages: one buffer");
  constexpr int SB = KS * BKB;      // bytes per row per LDS stage
  constexpr int LR = SB + 16;       // padded LDS row
  constexpr int TB = BM * LR;       // one operand's stage
  constexpr int CH = SB / 16;       // 16-byte chunks per row per stage
  constexpr int NL = BM * CH / 256; // 16-byte loads per thread per operand
  if (st1 < 0) st1 = g.nst;  // K slices [st0, st1)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = tm * BM, n0 = tn * BN;

  const uint8_t* pa[NL];
  const uint8_t* pb[NL];
  int ls[NL];
#pragma unroll
  for (int u = 0; u < NL; u++) {
    const int f = u * 256 + tid, row = f / CH, c = f % CH;
    pa[u] = g.A + (int64_t)min(m0 + row, g.M - 1) * g.lda + c * 16;
    pb[u] = g.B + (int64_t)min(n0 + row, g.Nn - 1) * g.ldb + c * 16;
    ls[u] = row * LR + c * 16;
  }
  u32x4 ra[NL], rb[NL];
  auto gload = [&](int st) {
#pragma unroll
    for (int u = 0; u < NL; u++) {
      ra[u] = *(const u32x4*)(pa[u] + (int64_t)st * BKB);
      rb[u] = *(const u32x4*)(pb[u] + (int64_t)st * BKB);
    }
  };
  auto lstore = [&](int buf) {
    uint8_t* base = lds + buf * 2 * TB;
#pragma unroll
    for (int u = 0; u < NL; u++) {
      *(u32x4*)(base + ls[u]) = ra[u];
      *(u32x4*)(base + TB + ls[u]) = rb[u];
    }
  };

#pragma unroll
  for (int sm = 0; sm < 2; sm++)
#pragma unroll
    for (int sn = 0; sn < 2; sn++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[sm][sn][r] = 0.f;

  const int fa = (wm * 64 + (lane & 31)) * LR + (lane >> 5) * 64;
  const int fb = (wn * 64 + (lane & 31)) * LR + (lane >> 5) * 64;

  if (NBUF == 2) {
    gload(st0);
    lstore(0);
    __syncthreads();
    for (int st = st0; st < st1; st++) {
      const int buf = (st - st0) & 1;
      if (st + 1 < st1) gload(st + 1);
      const uint8_t* la = lds + buf * 2 * TB;
      const uint8_t* lb = la + TB;
      u32x4 a[2][4], b[2][4];
#pragma unroll
      for (int s = 0; s < 2; s++)
#pragma unroll
        for (int c = 0; c < 4; c++) {
          a[s][c] = *(const u32x4*)(la + fa + s * 32 * LR + c * 16);
          b[s][c] = *(const u32x4*)(lb + fb + s * 32 * LR + c * 16);
        }
      mfma_stage<MODE>(acc, a, b);
      if (st + 1 < st1) lstore(buf ^ 1);
      __syncthreads();
    }
  } else {
    // one stage buffer, next stage prefetched into registers
    gload(st0);
    for (int st = st0; st < st1; st += KS) {
      if (st > st0) __syncthreads();
      lstore(0);
      __syncthreads();
      if (st + KS < st1) gload(st + KS);
      const uint8_t* la = lds;
      const uint8_t* lb = la + TB;
#pragma unroll
      for (int q = 0; q < KS; q++) {
        u32x4 a[2][4], b[2][4];
#pragma unroll
        for (int s = 0; s < 2; s++)
#pragma unroll
          for (int c = 0; c < 4; c++) {
            a[s][c] = *(const u32x4*)(la + fa + s * 32 * LR + q * BKB + c * 16);
            b[s][c] = *(const u32x4*)(lb + fb + s * 32 * LR + q * BKB + c * 16);
          }
        mfma_stage<MODE>(acc, a, b);
      }
    }
    __syncthreads();
  }
}

template <int MODE, int EPI, int NBUF = 1, int KS = 1>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int tm, int tn, uint8_t* lds, int st0 = 0,
                                          int st1 = -1) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = tm * BM, n0 = tn * BN;
  constexpr bool SIM = EPI == EPI_SIM_SYM || EPI == EPI_SIM_SYM16;
  float scale = 0.f;
  if constexpr (SIM || EPI == EPI_DIST) scale = sim_scale_fetch(g, tm, tn);
  f32x16 acc[2][2];
  gemm_tile_acc<MODE, NBUF, KS>(g, tm, tn, lds, acc, st0, st1);
  // 32x32 accumulator layout: register r of lane l holds
  // row 8*(r/4) + 4*(l/32) + r%4, column l%32 of its block.
  if constexpr (EPI == EPI_PART) {
#pragma unroll
    for (int sm = 0; sm < 2; sm++)
#pragma unroll
      for (int sn = 0; sn < 2; sn++)
#pragma unroll
        for (int r = 0; r < 16; r++) g.out[((sm * 2 + sn) * 16 + r) * 256 + tid] = acc[sm][sn][r];
    __syncthreads();
  } else if constexpr (EPI == EPI_DIST) {
    // the tile's scales through LDS (free after the K loop), read as float4
    // runs of this lane's rows, so no load waits inside the bounds checks
    float* sc = (float*)lds;
    sc[tid] = scale;
    __syncthreads();
#pragma unroll
    for (int sm = 0; sm < 2; sm++) {
      f32x4 rs[4];
#pragma unroll
      for (int j = 0; j < 4; j++) rs[j] = *(const f32x4*)(sc + wm * 64 + sm * 32 + j * 8 + (lane >> 5) * 4);
#pragma unroll
      for (int sn = 0; sn < 2; sn++) {
        const int col = n0 + wn * 64 + sn * 32 + (lane & 31);
        const float scol = sc[BM + wn * 64 + sn * 32 + (lane & 31)];
#pragma unroll
        for (int r = 0; r < 16; r++) {
          const int row = m0 + wm * 64 + sm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
          if (row < g.M && col < g.Nn)
            g.out[(int64_t)row * g.ldo + col] = 1.0f - rs[r >> 2][r & 3] * scol * acc[sm][sn][r];
        }
      }
    }
    __syncthreads();  // LDS is reused by the next tile of a persistent workgroup
  } else if constexpr (EPI == EPI_KNN) {
    knn_epilogue<MODE>(g, tm, tn, acc, lds);
    __syncthreads();  // the staged tile is overwritten by the next tile's stages
  } else {
    static_assert(SIM, "similarity epilogues");
    sim_scale_put<EPI>(lds, scale);
    sim_epilogue<EPI>(g, tm, tn, acc, lds);
    __syncthreads();  // LDS is reused by the next tile of a persistent workgroup
  }
}

// Sum of the `parts` partial tiles of one K-split tile, in range order
// (part 0 + part 1 + ...), for this thread's 64 accumulator positions. Each
// range is one pass of 64 independent loads, so the passes wait on memory
// once each rather than once per element.
__device__ __forceinline__ void fix_sum(const float* __restrict__ part, int parts, float (&v)[4][16]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int s = 0; s < 4; s++)
#pragma unroll
    for (int r = 0; r < 16; r++) v[s][r] = part[(s * 16 + r) * 256 + tid];
  for (int k = 1; k < parts; k++) {
    const float* pk = part + (int64_t)k * BM * BN;
#pragma unroll
    for (int s = 0; s < 4; s++)
#pragma unroll
      for (int r = 0; r < 16; r++) v[s][r] += pk[(s * 16 + r) * 256 + tid];
  }
}

// Tail tile (tm, tn) of EPI_DIST computed as `parts` K ranges: sum the EPI_PART
// partial tiles in range order, then the EPI_DIST epilogue.
__device__ __forceinline__ void gemm_fix_tile(const GemmArgs& g, int tm, int tn, const float* __restrict__ part,
                                              int parts) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = tm * BM, n0 = tn * BN;
  float v[4][16];
  fix_sum(part, parts, v);
#pragma unroll
  for (int sm = 0; sm < 2; sm++)
#pragma unroll
    for (int sn = 0; sn < 2; sn++) {
      const int col = n0 + wn * 64 + sn * 32 + (lane & 31);
      const float scol = (col < g.Nn) ? g.sb[min(col, g.Nn - 1)] : 0.f;
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int row = m0 + wm * 64 + sm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        const float srow = g.sa[min(row, g.M - 1)];  // loaded outside the bounds check
        if (row < g.M && col < g.Nn) g.out[(int64_t)row * g.ldo + col] = 1.0f - srow * scol * v[sm * 2 + sn][r];
      }
    }
}

// Tail tile (tm, tn) of a similarity product computed as `parts` K ranges:
// the partial tiles summed in range order, then the similarity epilogue.
template <int EPI>
__device__ __forceinline__ void gemm_sim_fix_tile(const GemmArgs& g, int tm, int tn, const float* __restrict__ part,
                                                  int parts, uint8_t* lds) {
  const float scale = sim_scale_fetch(g, tm, tn);
  float v[4][16];
  fix_sum(part, parts, v);
  f32x16 acc[2][2];
#pragma unroll
  for (int sm = 0; sm < 2; sm++)
#pragma unroll
    for (int sn = 0; sn < 2; sn++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[sm][sn][r] = v[sm * 2 + sn][r];
  sim_scale_put<EPI>(lds, scale);
  sim_epilogue<EPI>(g, tm, tn, acc, lds);
}

// ---------------------------------------------------------------- bf16x3
// FP32-accurate product on bfloat16 matrix cores: each FP32 operand x is held
// as hi = bf16(x) and lo = bf16(x - hi) (both round-to-nearest-even), and
// a.b is accumulated in FP32 as hi.hi + hi.lo + lo.hi (Henry, Tang and
// Heinecke 2019, "bf16x3"); the dropped lo.lo term is below 2^-16 of |a||b|.
// Operands: four K-major bf16 planes (A hi/lo, B hi/lo), row stride ld
// elements; 64 K-elements (128 bytes per plane row) per stage. One LDS stage
// buffer (4 planes, 72 KB, so two workgroups share a CU) with the next stage
// prefetched into registers while the current one is multiplied.
constexpr int X3_LDS_BYTES = 4 * TILEB;  // 73728

struct GemmX3Args {
  const uint16_t* ahi;
  const uint16_t* alo;
  const uint16_t* bhi;
  const uint16_t* blo;
  int M, Nn;
  int64_t ld;  // elements
  int nst;     // 64-element stages
  const float* sa;
  const float* sb;
  float* out;
  int64_t ldo;
};

__device__ __forceinline__ void gemm_tile_x3(const GemmX3Args& g, int tm, int tn, uint8_t* lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = tm * BM, n0 = tn * BN;
  const int64_t ldb = g.ld * 2;  // bytes
  const uint8_t* src[4] = {(const uint8_t*)g.ahi, (const uint8_t*)g.alo, (const uint8_t*)g.bhi,
                           (const uint8_t*)g.blo};
  int64_t roff[4][2];  // [u][A or B] row byte offsets of this thread's chunks
  int ls[4];
#pragma unroll
  for (int u = 0; u < 4; u++) {
    const int f = u * 256 + tid, row = f >> 3, c = f & 7;
    roff[u][0] = (int64_t)min(m0 + row, g.M - 1) * ldb + c * 16;
    roff[u][1] = (int64_t)min(n0 + row, g.Nn - 1) * ldb + c * 16;
    ls[u] = row * LDSR + c * 16;
  }
  u32x4 rg[4][4];  // [plane][u]
  auto gload = [&](int st) {
#pragma unroll
    for (int pl = 0; pl < 4; pl++)
#pragma unroll
      for (int u = 0; u < 4; u++) rg[pl][u] = *(const u32x4*)(src[pl] + roff[u][pl >> 1] + (int64_t)st * BKB);
  };
  auto lstore = [&](int buf) {
    uint8_t* base = lds + buf * 4 * TILEB;  // buf is always 0: single stage buffer
#pragma unroll
    for (int pl = 0; pl < 4; pl++)
#pragma unroll
      for (int u = 0; u < 4; u++) *(u32x4*)(base + pl * TILEB + ls[u]) = rg[pl][u];
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
  for (int st = 0; st < g.nst; st++) {
    __syncthreads();  // every wave is done with the previous stage
    lstore(0);
    __syncthreads();
    if (st + 1 < g.nst) gload(st + 1);  // in flight during the products below
    const uint8_t* base = lds;
#pragma unroll
    for (int c = 0; c < 4; c++) {
      bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
      for (int s = 0; s < 2; s++) {
        ah[s] = __builtin_bit_cast(bf16x8, *(const u32x4*)(base + 0 * TILEB + fa + s * 32 * LDSR + c * 16));
        al[s] = __builtin_bit_cast(bf16x8, *(const u32x4*)(base + 1 * TILEB + fa + s * 32 * LDSR + c * 16));
        bh[s] = __builtin_bit_cast(bf16x8, *(const u32x4*)(base + 2 * TILEB + fb + s * 32 * LDSR + c * 16));
        bl[s] = __builtin_bit_cast(bf16x8, *(const u32x4*)(base + 3 * TILEB + fb + s * 32 * LDSR + c * 16));
      }
#pragma unroll
      for (int sm = 0; sm < 2; sm++)
#pragma unroll
        for (int sn = 0; sn < 2; sn++) {
          acc[sm][sn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[sm], bh[sn], acc[sm][sn], 0, 0, 0);
          acc[sm][sn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[sm], bl[sn], acc[sm][sn], 0, 0, 0);
          acc[sm][sn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[sm], bh[sn], acc[sm][sn], 0, 0, 0);
        }
    }
  }
#pragma unroll
  for (int sm = 0; sm < 2; sm++)
#pragma unroll
    for (int sn = 0; sn < 2; sn++) {
      const int col = n0 + wn * 64 + sn * 32 + (lane & 31);
      if (col >= g.Nn) continue;
      const float scol = g.sb[col];
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int row = m0 + wm * 64 + sm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        const float srow = g.sa[min(row, g.M - 1)];  // loaded outside the bounds check
        if (row < g.M) g.out[(int64_t)row * g.ldo + col] = 1.0f - srow * scol * acc[sm][sn][r];
      }
    }
  __syncthreads();
}

// Upper-triangle tile t (0 <= t < T(T+1)/2) of a T x T tile grid. Tile rows
// are taken in bands of 8; a band's tiles are listed column by column
// (tn ascending, the band's rows with tm <= tn inside a column), so the
// workgroups resident on one XCD at a time cover a few columns of one band and
// share its 8 row blocks and their column blocks in that XCD's L2.
__device__ __forceinline__ void upper_tile(int t, int T, int& tm, int& tn) {
  constexpr int G = 8;
  for (int r0 = 0;; r0 += G) {
    const int gs = min(G, T - r0), r1 = r0 + gs;
    const int head = gs * (gs + 1) / 2;  // columns r0..r1-1: the band's own triangle
    const int cnt = head + gs * (T - r1);
    if (t < cnt || r1 >= T) {
      if (t < head) {
        int j = 0;
        while ((j + 1) * (j + 2) / 2 <= t) j++;
        tm = r0 + (t - j * (j + 1) / 2);
        tn = r0 + j;
      } else {
        const int u = t - head;
        tn = r1 + u / gs;
        tm = r0 + u % gs;
      }
      return;
    }
    t -= cnt;
  }
}

}  // namespace rr
