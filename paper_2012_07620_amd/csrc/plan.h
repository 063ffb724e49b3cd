// Parameter validation and device working-set layout of one problem.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/rerank.h"
#include "kernels.h"

namespace rr {

constexpr int kMaxCand = 256;   // k1 + extra candidates held by one wavefront
constexpr int kMaxLayers = 256; // Table 2 goes up to 256 layers
constexpr int kMaxAlpha = 8;
// Problems up to this size are batched by the serving path's grouped launches;
// the direct path computes them with the same tile work (no split tail), so a
// request's result does not depend on which path ran it.
constexpr int kGroupedMaxN = 8192;

struct Plan {
  int n = 0, q = 0, g = 0, d = 0, k1 = 0, k2 = 0, layers = 0, alpha = 0, kc = 0;
  SimPrec prec = SimPrec::F32;
  FinalPrec fprec = FinalPrec::F32;
  bool rescore = false;
  int node = RERANK_NODE_ADJ_SYM;
  int agg = RERANK_AGG_SUM;
  int64_t ldp = 0;  // fp32 feature copy row stride (elements)
  int64_t ldl = 0;  // low-precision copy row stride (elements)
  int lbytes = 0;   // bytes per low-precision element
  int64_t ldN = 0;  // similarity / A* row stride
  int64_t ldH = 0;  // propagated feature row stride (ldN, or ldp in raw mode)
  int64_t tb = 0;   // column blocks of 128 per S row (the block maxima's row stride)
  // byte offsets into the working set
  size_t o_xp = 0, o_xl = 0, o_rn = 0, o_sl = 0, o_a = 0, o_b = 0, o_ci = 0, o_cv = 0, o_ki = 0, o_kv = 0,
         o_sa = 0, o_sb = 0, o_cnt = 0, o_hi = 0, o_lo = 0, o_mflag = 0, o_off = 0, o_inl = 0, o_sp = 0,
         o_slg = 0, o_slr = 0, o_part = 0,
         o_ord = 0,
         o_fk = 0,   // scratch of the fused similarity + top-k (fused_layout)
         o_bm = 0,   // block maxima of S for the pruned top-k (n x tb floats), 0 = none
         o_rsc = 0;  // re-score scratch (the dead S buffer, or its own block without one)
  bool sparse_first = false;   // layer 1 built from the sparse A* / A rows (layers >= 1, sum or mean)
  bool sparse_layers = false;  // layers kept as CSR rows for the sparse final product
  bool sparse_mid = false;     // dense final products, layers >= 2: layers 1..L-1 as CSR rows, the last dense
  bool fused = false;          // similarity and top-k fused: S is never written
  bool has_s = true;           // the N x N buffer A exists (knn-only fused plans have none)
  size_t total = 0;
};

// Returns RERANK_OK or an error with a reason in *why.
rerank_status validate_params(const rerank_params* p, std::string* why);
// Fills the layout for valid parameters. knn_only skips propagation buffers;
// dense_layers keeps the layers dense under the sparse final product; fused
// selects the fused similarity + top-k (a knn-only plan then holds no N x N
// buffer).
void make_plan(const rerank_params* p, bool knn_only, Plan* out, bool dense_layers = false, bool fused = false);

}  // namespace rr
