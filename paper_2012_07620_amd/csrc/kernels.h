// Launchers of the gfx950 kernels (host side). Every launcher enqueues on
// `s` and returns the launch status; shapes are validated by the caller.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

namespace rr {

enum class SimPrec : int { F32 = 0, BF16 = 1, FP8 = 2 };
enum class FinalPrec : int { F32 = 0, BF16X3 = 1, SPARSE = 2, BF16 = 3 };

// Sparse layers (used with the sparse final product): every propagated row is
// stored as CSR entries (columns ascending) in a slot of the layer's output
// buffer. Row i's slot holds min(n, sum of its k2 members' entry counts)
// entries; the slots are laid out by a prefix sum before the layer runs. One
// gate per layer l (gate 0 = h^(0), always sparse):
//   total  the sum of the slot sizes;
//   dense  1 when layer l is written as dense rows instead (the slots would
//          not fit in the buffer, or an earlier layer was dense).
struct SlGate {
  unsigned long long total;
  int32_t dense;
  int32_t pad;
};
// CSR rows of one layer: entries of row i are col/val[so[i] .. so[i] + cnt[i]).
struct SlRows {
  int32_t* col;
  float* val;
  int32_t* so;
  int32_t* cnt;
};
// Output side of a sparse layer: where the rows go and which gates apply.
struct SlOut {
  SlRows rows;
  SlGate* gate;        // gates[l]
  const SlGate* prev;  // gates[l - 1]
  int64_t cap;         // entries the buffer holds
  int n;               // columns of a row (bounds are capped at n)
};

// Block sums needed by launch_scan over n counts (1024 counts per block, plus the total).
inline int64_t scan_parts(int64_t n) { return (n + 1023) / 1024 + 1; }

// Row stride (elements) of the padded K-major copies the GEMMs read: every
// row is a whole number of 128-byte K slices.
inline int64_t pad_k_elems(int64_t d, int bytes_per_elem) {
  const int64_t per = 128 / bytes_per_elem;
  return (d + per - 1) / per * per;
}
// Row stride of the N x N similarity / feature buffers (256-byte rows).
inline int64_t pad_n(int64_t n) { return (n + 63) / 64 * 64; }

// a1: feature preparation. Reads X (f32 or bf16 bits), writes
//   xp  N x ldp float32 copy, zero-padded; null when the caller's FP32 rows
//       are used in place (feature_rows)
//   rn  1 / |x_i| (compensated sum of squares, correctly rounded sqrt/div)
//   xl  low-precision copy (bf16 or fp8 e4m3, ldl elements) when prec != F32
//   sl  per-row scale of the low-precision product (rn_i, or rn_i * s_i)
hipError_t launch_prep(const void* x, int in_bf16, int n, int d, float* xp, int64_t ldp, float* rn,
                       SimPrec prec, void* xl, int64_t ldl, float* sl, hipStream_t s);

// a2 / a7: C = A * B^T on matrix cores. A: M rows, B: Nn rows, K-major,
// row strides in bytes (multiples of 128), kbytes = K extent in bytes.
// Similarity epilogue: out[i][j] = acc * sa[i] * sb[j] (-0 -> +0), ldo
// elements: FP32, or binary16 (round to nearest even) with half_out, which
// the low-precision paths use (their S only ranks candidates that are then
// re-scored in FP32; binary16 rounding, at most 2^-11 relative, is below the
// error of the BF16 / FP8 product itself) to halve S's bytes. ws (ws_bytes,
// may be null): scratch for splitting the last, partly filled round of tiles
// along K (fixed ranges summed in order: deterministic).
// bm (may be null): also the largest stored similarity of each row over each
// block of 128 columns, bm[b * ldbm + i] (ldbm >= M).
hipError_t launch_gemm_sim(SimPrec prec, const void* a, int M, int64_t lda_bytes, int64_t kbytes,
                           const float* sa, void* out, int64_t ldo, bool half_out, float* ws, int64_t ws_bytes,
                           hipStream_t s, float* bm = nullptr, int64_t ldbm = 0);

// a2 + a3 fused (S never written): the K best candidates of each of the M
// rows of A (the Eq. 7 similarity of A with itself, scaled by sa and rounded
// as launch_gemm_sim rounds it for prec), written as launch_topk writes them
// (idx / val, M x K, the row itself first). K <= 64 and K <= M. ws: the
// scratch described by fused_layout(M, K, prec).
//
// Method: a sample of the columns (P whole column panels of 128, evenly
// spread) is multiplied first and stored; from it each row gets tau_i, a
// similarity value at or below its K-th best. The upper-triangle tiles of the
// other panels are then computed once each and every element of a tile is
// offered to both of its rows (i, j) and (j, i), the stored sample tiles
// likewise; an element is appended to its row's candidate buffer only if its
// value is at least that row's tau. A superset of each row's K best is kept,
// so the K best of the buffer are exact. A row whose buffer overflows (more
// than C values at or above its tau) is recomputed, with its whole row panel,
// by the row-panel kernel that merges running lists.
//
// Sizes: for a uniformly drawn sample of m of the M columns, the number of
// keys at or above the K-th best of the sample has mean about K M / m and
// relative standard deviation about 1 / sqrt(K); C allows f = 1 + 6 / sqrt(K)
// times the mean, plus 128. m balances the stored sample (M m sbytes) against
// the candidate slots (8 M C): m = sqrt(8 f K M / sbytes), rounded up to
// whole panels, at least 8 panels (all of them for M <= 1024). The scratch
// grows as M^1.5: for M = 19281 and K = 34 (FP32) it is about 0.4 GB against
// 1.5 GB for S.
constexpr int kKnnMaxRanges = 32;  // column ranges of the row-panel kernel
constexpr int KNN_LIST_MAX = 64;
struct FusedLayout {
  int T;          // row / column panels of 128
  int P, sp, so;  // sample panels: so + t * sp for t < P
  int64_t m;      // stored sample columns per row (P * 128)
  int64_t C;      // candidate slots per row
  size_t o_samp, o_cand, o_tau, o_cnt, o_flag, bytes;
};
// sbytes: bytes per stored similarity (4 for FP32, 2 for binary16).
inline FusedLayout fused_layout(int64_t n, int K, int sbytes) {
  FusedLayout L{};
  L.T = (int)((n + 127) / 128);
  const double f = 1.0 + 6.0 / std::sqrt((double)K);
  const double mopt = std::sqrt(8.0 * f * K * (double)n / sbytes);
  int64_t P = (int64_t)std::ceil(mopt / 128.0);
  if (P < 8) P = 8;
  if (P > L.T) P = L.T;
  L.P = (int)P;
  L.sp = L.T / L.P;
  L.so = L.sp / 2;
  L.m = (int64_t)L.P * 128;
  const int64_t mv = L.m < n ? L.m : n;
  const int64_t c = (int64_t)std::ceil(f * K * (double)n / (double)mv) + 128;
  L.C = c < n ? c : n;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t at = off;
    off += (b + 255) & ~(size_t)255;
    return at;
  };
  L.o_samp = take((size_t)n * L.m * sbytes);
  L.o_cand = take((size_t)n * L.C * 8);
  L.o_tau = take((size_t)n * 4);
  L.o_cnt = take((size_t)n * 4);
  L.o_flag = take((size_t)L.T * 4);
  L.bytes = off;
  return L;
}
inline FusedLayout fused_layout(int64_t n, int K, SimPrec prec) {
  return fused_layout(n, K, prec == SimPrec::F32 ? 4 : 2);
}
hipError_t launch_knn_fused(SimPrec prec, const void* a, int M, int64_t lda_bytes, int64_t kbytes, const float* sa,
                            int K, void* ws, int32_t* idx, float* val, hipStream_t s);
// Final epilogue: out[q][g] = 1 - sa[q] * sb[g] * acc, ldo floats.
// Final product, D = 1 - sa[i] * sb[j] * acc. ws (ws_bytes, may be null):
// scratch for splitting the last, partly filled round of tiles along K.
hipError_t launch_gemm_dist(const float* a, int M, const float* b, int Nn, int64_t ld_elems, int64_t kelems,
                            const float* sa, const float* sb, float* out, int64_t ldo, float* ws, int64_t ws_bytes,
                            hipStream_t s);
// Final product on bfloat16 operands (rows rounded to bf16, row stride
// ld_elems, K = kelems): D = 1 - sa[i] * sb[j] * acc, FP32 accumulation.
hipError_t launch_gemm_dist_bf16(const uint16_t* a, int M, const uint16_t* b, int Nn, int64_t ld_elems,
                                 int64_t kelems, const float* sa, const float* sb, float* out, int64_t ldo,
                                 hipStream_t s);
hipError_t launch_gemm_dist_bf16x3(const uint16_t* a_hi, const uint16_t* a_lo, int M, const uint16_t* b_hi,
                                   const uint16_t* b_lo, int Nn, int64_t ld_elems, int64_t kelems,
                                   const float* sa, const float* sb, float* out, int64_t ldo, hipStream_t s);

// a3: per-row top-K (K <= 256) of rows [0, rows) of S (FP32, or binary16
// with half; row stride ldS elements, N valid columns) under (value desc,
// column asc), the row's own column first.
hipError_t launch_topk(const void* S, bool half, int64_t ldS, int N, int rows, int K, int32_t* idx, float* val,
                       int ldo, hipStream_t s);
// The same lists from S and its block maxima bm (as launch_gemm_sim writes
// them): only the column blocks whose maximum reaches a lower bound on the
// row's K-th best value are read. N <= kPrunedMaxN (at most 512 blocks per
// row) and K <= kPrunedMaxK (pruning needs 4 (K - 1) <= blocks <= 512, so
// larger K never prunes); bm 16-byte aligned with ldbm a multiple of 4 and at
// least rows rounded up to 4 (four rows' maxima are read as one vector).
constexpr int kPrunedMaxN = 512 * 128;
constexpr int kPrunedMaxK = 128;
hipError_t launch_topk_pruned(const void* S, bool half, int64_t ldS, int N, int rows, int K, const float* bm,
                              int64_t ldbm, int32_t* idx, float* val, int ldo, hipStream_t s);

// Cluster order of rows [0, rows) of `lists` (row width w, entries < n):
// the rows sorted by the key min(i, entries of row i), rows of one key in
// arbitrary order. scratch: cluster_order_ints(rows, n) int32, 16-byte
// aligned. Writes order[0, rows).
inline int64_t cluster_order_ints(int64_t rows, int64_t n) { return (3 * n + rows + 1 + scan_parts(n) + 3) / 4 * 4; }
hipError_t launch_cluster_order(const int32_t* lists, int rows, int w, int n, int32_t* scratch, int32_t* order,
                                hipStream_t s);
// 2 delta for the candidate skip of the re-score, for similarity products
// whose low-precision copy has lbytes bytes per element (0: FP32), over at most
// K terms; delta bounds |product value - re-scored value|.
//  * FP32: (K + 8) u / (1 - (K + 8) u) of |x_i| |x_j| by Cauchy-Schwarz,
//    u = 2^-24, scaled by the two inverse norms; here doubled for margin.
//  * BF16: both operands rounded to bfloat16 (relative error <= 2^-9 each,
//    so the summed product error is <= (2^-8 + 2^-18) |x_i| |x_j|), FP32
//    accumulation (<= (K + 8) 2^-24 of the same), scaling by the inverse norms
//    (< 1e-6) and binary16 storage (<= 2^-11 for |S| <= 1), plus 1e-6 for the
//    re-score's own error.
//  * FP8: e4m3 rounds to 2^-4, too coarse to skip anything: -1 (re-score
//    every candidate).
__host__ __device__ inline float rescore_skip2(int lbytes, int64_t K) {
  const double ku = (double)(K + 8) * 0x1p-24;
  if (lbytes == 0) return (float)(2.0 * 2.0 * ku / (1.0 - ku));
  if (lbytes == 2) return (float)(2.0 * (0x1p-8 + 0x1p-18 + 2.0 * ku + 0x1p-11 + 2e-6));
  return -1.f;
}

// a3b: re-score of Kc candidates per row (FP32 products summed in FP64), then the k1 cut.
// cval: the candidates' product values (sorted descending, as top-k writes
// them); skip2 = rescore_skip2(...) skips candidates that cannot reach the
// top k1 (-1: re-score all). scratch (cluster_order_ints(n, n) + n int32,
// 16-byte aligned) or nullptr: rows are re-scored in an order that keeps rows
// with shared candidates on one XCD (the results do not depend on the order).
hipError_t launch_rescore(const float* xp, int64_t ldp, int d, const float* rn, int n, const int32_t* cand,
                          const float* cval, int Kc, int k1, float skip2, int32_t* knn_idx, float* knn_val,
                          int32_t* scratch, hipStream_t s);
// Copy the first k1 of Kc candidates (no re-score).
hipError_t launch_take_prefix(const int32_t* cand_idx, const float* cand_val, int n, int Kc, int k1,
                              int32_t* knn_idx, float* knn_val, hipStream_t s);

// a4: zero a float range (fill kernel, usable under graph capture).
hipError_t launch_fill_zero(float* buf, int64_t count, hipStream_t s);
// a4: scatter A* = (A + A^T)/2 into a zeroed N x ldH buffer; cnt[0..n) counts
// in-degrees and cnt[n..2n) mutual pairs (both zeroed beforehand).
// sym = false scatters the rows of A instead (H[i][j] = 1, no counts).
hipError_t launch_astar_scatter(const int32_t* knn_idx, int n, int k1, float* H, int64_t ldH, int32_t* cnt,
                                bool sym, hipStream_t s);
// sigma_i = 1 / |h^(0)_i| from the counts (A*) or sqrt(k1) (A): zero-layer final product.
hipError_t launch_astar_sigma(const int32_t* cnt, int n, int k1, float* sigma, bool sym, hipStream_t s);

// a5 + a6: one propagation layer (Eq. 14, sum aggregator) with lazy
// normalisation: hout_i = sin_i*hin_i + sum_{r<k2} w_ir * sin_{j_r} * hin_{j_r},
// w_i0 = 1 for the row itself, w_ir = val_ir^alpha; sout_i = 1/|hout_i|.
// sin == nullptr means all ones. When hi/lo are non-null the row is written
// as bf16 high/low parts (final bf16x3 product) instead of FP32.
// agg: rerank_aggregator of Eq. 13. order (n rows, or nullptr for index
// order): rows are computed in this order, consecutive ones on one XCD, so
// the neighbour rows a cluster shares are read from that XCD's L2.
hipError_t launch_propagate(const float* hin, const float* sin, int n, int64_t ld, int64_t cols,
                            const int32_t* knn_idx, const float* knn_val, int k1, int k2, int alpha, int agg,
                            float* hout, float* sout, uint16_t* hi, uint16_t* lo, const int32_t* order,
                            hipStream_t s);
// Sparse first layer (A* never stored densely when layers >= 1):
// mutual flags of every (i, r) pair and non-mutual in-degree counts ...
hipError_t launch_mutual(const int32_t* knn_idx, int n, int k1, uint8_t* mflag, int32_t* innm, hipStream_t s);
// ... exclusive prefix sum of the counts (off has n + 1 entries) ...
// Exclusive prefix sum of in[0, n) into out[0, n], out[n] = the total, in
// three launches (block sums, a scan of the block sums, block scans). part
// holds scan_parts(n) int32. With `skip`, nothing runs when *skip == skip_val
// (read on the device). The total must fit in int32.
hipError_t launch_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* part, hipStream_t s,
                       const int32_t* skip = nullptr, int32_t skip_val = 0);
// ... CSR transpose of the non-mutual edges (cursor zeroed beforehand) ...
hipError_t launch_csr(const int32_t* knn_idx, int n, int k1, const uint8_t* mflag, const int32_t* off,
                      int32_t* cursor, int32_t* inl, hipStream_t s);
// ... and layer 1 built from the sparse A* rows (same result as the dense layer).
// (sym = false: rows of A; agg: sum or mean)
// sl != nullptr: CSR output (sparse layers) unless the layer's gate says
// dense, in which case the dense rows go to hout as without sl.
hipError_t launch_first_layer(const int32_t* knn_idx, const float* knn_val, const uint8_t* mflag,
                              const int32_t* off, const int32_t* inl, int n, int k1, int k2, int alpha, int agg,
                              bool sym, int64_t ld, float* hout, float* sout, uint16_t* hi, uint16_t* lo,
                              const SlOut* sl, hipStream_t s);
// Sparse layers. Slot sizes of layer l (first: members' A* / A entry counts
// from the kNN lists and the in-edge offsets `off` (A* only); otherwise the
// previous layer's row counts) into out.cnt, their prefix sum into out.so,
// and gates[l] (dense when the total exceeds out.cap or gates[l - 1] is
// dense). The layer then overwrites out.cnt with the rows' actual counts.
// out.rows.so must hold n + 1 entries; part holds scan_parts(n) int32.
hipError_t launch_sl_slots(const int32_t* knn_idx, int n, int k1, int k2, bool first, bool sym, const int32_t* off,
                           const int32_t* cnt_prev, const SlOut& out, int32_t* part, hipStream_t s);
// Layer l >= 2 from the CSR rows of layer l - 1 (runs when gates[l - 1] is
// sparse): CSR out, or dense rows into hout when gates[l] turns dense.
hipError_t launch_sparse_prop(SlRows in, const float* sin, const int32_t* knn_idx, const float* knn_val, int n,
                              int k1, int k2, int alpha, int agg, int64_t ld, float* hout, float* sout, SlOut out,
                              hipStream_t s);
// The dense layer, run only when gates[l - 1] is dense.
hipError_t launch_propagate_gated(const float* hin, const float* sin, int n, int64_t ld, const int32_t* knn_idx,
                                  const float* knn_val, int k1, int k2, int alpha, int agg, float* hout, float* sout,
                                  SlGate* gates, int l, hipStream_t s, uint16_t* hi = nullptr, uint16_t* lo = nullptr);
// Layer l + 1 written as dense rows (hout, or the bf16 hi / lo planes of a
// last layer) from the CSR rows `in` of layer l, unless gates[l] says layer l
// was dense (then launch_propagate_gated for layer l + 1 computes it). The
// same sums and norms as the dense layer, bit for bit.
hipError_t launch_sparse_prop_dense(SlRows in, const float* sin, const int32_t* knn_idx, const float* knn_val, int n,
                                    int k1, int k2, int alpha, int agg, int64_t ld, float* hout, float* sout,
                                    uint16_t* hi, uint16_t* lo, const SlGate* gate_in, hipStream_t s);
// Ranking list: per row of D (q rows, stride g), the r smallest positions in
// ascending order, ties to the lower position (r <= 256).
hipError_t launch_rank(const float* D, int q, int g, int r, int32_t* out, hipStream_t s);
// a7, sparse form: D[q][g] = 1 - sq[q] * <h_q, sg[g] h_{Q+g}> from the
// non-zeros of H (n rows, row stride ld, columns < ld; sigma = sq then sg).
// `pool` (pool_bytes, must not overlap H) holds the compacted rows and the
// gallery's column layout; `ints` holds sparse_final_ints(n, ld) int32 of
// counters, offsets and the queries' cluster order (from knn, n x k1). When
// the compacted rows exceed pool_bytes / 16 the FP32 matrix-core product
// computes D instead (decided on the device). D is q x (n - q), row stride
// n - q. With `lay` (the gate and rows of the last sparse layer, H then being
// that layer's buffer): when the gate is sparse the CSR rows are used as they
// are and only the column layout goes into `pool`.
constexpr int kSparseChunk = 16384;  // gallery accumulators per pass of the sparse product
inline int64_t sparse_chunks(int64_t n) { return (n + kSparseChunk - 1) / kSparseChunk; }
// column buckets: (gallery chunk, quarter of the chunk, column)
inline int64_t sparse_buckets(int64_t n, int64_t ld) { return sparse_chunks(n) * 4 * ld; }
inline int64_t sparse_scan_parts(int64_t n, int64_t ld) { return scan_parts(sparse_buckets(n, ld)); }
inline int64_t sparse_final_head(int64_t n, int64_t ld) {
  return (3 * sparse_buckets(n, ld) + 2 * n + 4 + 16 + sparse_scan_parts(n, ld) + 3) / 4 * 4;
}
inline int64_t sparse_final_ints(int64_t n, int64_t ld) {
  return sparse_final_head(n, ld) + cluster_order_ints(n, n) + n;  // + the queries' cluster order
}
hipError_t launch_sparse_final(const float* H, int n, int q, int64_t ld, const float* sigma, float* dist, void* pool,
                               int64_t pool_bytes, int32_t* ints, const SlGate* lay_gate, const SlRows* lay,
                               const int32_t* knn, int k1, hipStream_t s);
// Split rows of an FP32 matrix into bf16 high/low parts (for L = 0 or raw).
hipError_t launch_split_bf16(const float* h, int n, int64_t ld, uint16_t* hi, uint16_t* lo, hipStream_t s);

// Copy helpers.
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int64_t count, hipStream_t s);
hipError_t launch_copy_f32(const float* src, float* dst, int64_t count, hipStream_t s);

}  // namespace rr
