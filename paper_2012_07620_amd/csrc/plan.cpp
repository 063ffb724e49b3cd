// Parameter validation and working-set layout (pure host code).
#include "plan.h"

namespace rr {

static rerank_status bad(std::string* why, const std::string& msg, rerank_status st = RERANK_E_INVALID) {
  if (why) *why = msg;
  return st;
}

rerank_status validate_params(const rerank_params* p, std::string* why) {
  if (!p) return bad(why, "params is NULL");
  if (p->n < 2) return bad(why, "n must be >= 2");
  if (p->n_query < 1 || p->n_query > p->n - 1) return bad(why, "n_query must be in [1, n-1]");
  if (p->dim < 1) return bad(why, "dim must be >= 1");
  if (p->k1 < 1 || p->k1 > p->n) return bad(why, "k1 must be in [1, n]");
  if (p->k2 < 1 || p->k2 > p->k1) return bad(why, "k2 must be in [1, k1]");
  if (p->layers < 0 || p->layers > kMaxLayers) return bad(why, "layers must be in [0, 256]");
  if (p->alpha < 0 || p->alpha > kMaxAlpha) return bad(why, "alpha must be an integer in [0, 8]");
  if (p->sim_prec < RERANK_SIM_F32 || p->sim_prec > RERANK_SIM_FP8_E4M3) return bad(why, "unknown sim_prec");
  if (p->node != RERANK_NODE_ADJ_SYM && p->node != RERANK_NODE_RAW && p->node != RERANK_NODE_ADJ)
    return bad(why, "unknown node mode");
  if (p->aggregator < RERANK_AGG_SUM || p->aggregator > RERANK_AGG_MAX) return bad(why, "unknown aggregator");
  if (p->final_prec < RERANK_FINAL_F32 || p->final_prec > RERANK_FINAL_BF16) return bad(why, "unknown final_prec");
  if (p->final_prec == RERANK_FINAL_SPARSE && p->node == RERANK_NODE_RAW)
    return bad(why, "the sparse final product needs adjacency node features (node != RAW)");
  if (p->extra_cand < -1) return bad(why, "extra_cand must be >= -1");
  if (p->extra_cand == 0 && p->sim_prec != RERANK_SIM_F32)
    return bad(why, "low-precision similarity needs FP32 re-scoring (extra_cand != 0)");
  if (p->k1 > kMaxCand) return bad(why, "k1 above 256 is outside this library's limits", RERANK_E_UNSUPPORTED);
  // 32-bit row indices and per-launch tile counts
  if ((int64_t)p->n * (int64_t)p->n / (128 * 128) > 0x7FFFFFFF) return bad(why, "n too large", RERANK_E_UNSUPPORTED);
  return RERANK_OK;
}

static size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }

void make_plan(const rerank_params* p, bool knn_only, Plan* o, bool dense_layers, bool fused) {
  Plan& P = *o;
  P = Plan{};
  P.n = p->n;
  P.q = p->n_query;
  P.g = p->n - p->n_query;
  P.d = p->dim;
  P.k1 = p->k1;
  P.k2 = p->k2;
  P.layers = p->layers;
  P.alpha = p->alpha;
  P.prec = (SimPrec)p->sim_prec;
  P.fprec = (FinalPrec)p->final_prec;
  P.node = p->node;
  P.agg = p->aggregator;
  int extra = p->extra_cand;
  if (extra < 0) extra = (P.prec == SimPrec::F32) ? 8 : (P.prec == SimPrec::BF16 ? 16 : 32);
  int64_t kc = (int64_t)p->k1 + extra;
  if (kc > p->n) kc = p->n;
  if (kc > kMaxCand) kc = kMaxCand;
  P.kc = (int)kc;
  P.rescore = extra > 0;
  P.ldp = (P.d + 63) / 64 * 64;  // 256-byte rows: whole f32 stages and whole bf16x3 stages in raw mode
  P.lbytes = (P.prec == SimPrec::BF16) ? 2 : (P.prec == SimPrec::FP8 ? 1 : 0);
  P.ldl = P.lbytes ? pad_k_elems(P.d, P.lbytes) : 0;
  P.ldN = pad_n(P.n);
  P.ldH = (P.node == RERANK_NODE_RAW) ? P.ldp : P.ldN;
  const size_t n = (size_t)P.n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += up256(bytes);
    return at;
  };
  P.o_xp = take(n * P.ldp * 4);
  P.o_xl = P.lbytes ? take(n * P.ldl * P.lbytes) : 0;
  P.o_rn = take(n * 4);
  P.o_sl = take(n * 4);
  const size_t hrow = (size_t)(P.ldN > P.ldH ? P.ldN : P.ldH);
  P.fused = fused;
  P.has_s = !(fused && knn_only);
  if (P.has_s) {
    P.o_a = take(n * hrow * 4);
    P.o_rsc = P.o_a;  // S is dead once the candidates are selected
  } else {
    P.o_rsc = take((size_t)(cluster_order_ints(P.n, P.n) + P.n) * 4);
  }
  if (fused) P.o_fk = take(fused_layout(P.n, P.kc, P.prec).bytes);
  // The pruned selection reads about one 128-column block per member of a
  // row; it pays when those are a small part of the row (measured at
  // N = 19281: 34 candidates 0.28 -> 0.12 ms, while 42 and 58 ran faster
  // streaming whole rows), hence blocks >= 4 (candidates - 1).
  const int64_t tb = (P.n + 127) / 128;
  if (!fused && P.n <= kPrunedMaxN && P.kc <= kPrunedMaxK && 4 * (int64_t)(P.kc - 1) <= tb) {
    P.tb = tb;
    P.o_bm = take((size_t)P.tb * P.ldN * 4);  // block-major, row stride ldN (16-byte loads of 4 rows)
  }
  P.o_ci = take(n * P.kc * 4);
  P.o_cv = take(n * P.kc * 4);
  P.o_ki = take(n * P.k1 * 4);
  P.o_kv = take(n * P.k1 * 4);
  if (!knn_only) {
    // the sparse final product compacts into the feature buffer the last layer did not write
    if (P.layers > 0 || P.fprec == FinalPrec::SPARSE) P.o_b = take(n * P.ldH * 4);
    P.o_sa = take(n * 4);
    P.o_sb = take(n * 4);
    P.o_cnt = take(n * 8);  // in-degree and mutual counts (or in-degree and cursor), 2n int32
    P.o_part = take((size_t)scan_parts(P.n) * 4);  // block sums of the prefix sums over rows
    // cluster order of the rows for the dense layers (+ its scratch)
    if (P.layers > 0) P.o_ord = take((size_t)(cluster_order_ints(P.n, P.n) + P.n) * 4);
    P.sparse_first = (P.node != RERANK_NODE_RAW && P.layers > 0 && P.agg != RERANK_AGG_MAX);
    if (P.sparse_first && P.node == RERANK_NODE_ADJ_SYM) {
      P.o_mflag = take(n * P.k1);
      P.o_off = take((n + 1) * 4);
      P.o_inl = take(n * P.k1 * 4);
    }
    if (P.fprec == FinalPrec::SPARSE) P.o_sp = take(sparse_final_ints(P.n, P.ldN) * 4);
    P.sparse_layers = P.fprec == FinalPrec::SPARSE && P.sparse_first && !dense_layers;
    P.sparse_mid = P.fprec != FinalPrec::SPARSE && P.sparse_first && P.layers >= 2 && !dense_layers;
    if (P.sparse_layers || P.sparse_mid) {
      P.o_slg = take((size_t)(P.layers + 1) * sizeof(SlGate));
      P.o_slr = take(2 * (2 * n + 4) * 4);  // row starts (n + 1) and counts (n) of two layers
    }
    if (P.fprec == FinalPrec::BF16X3 || P.fprec == FinalPrec::BF16) P.o_hi = take(n * P.ldH * 2);
    if (P.fprec == FinalPrec::BF16X3) P.o_lo = take(n * P.ldH * 2);
  }
  P.total = off;
}

}  // namespace rr
