// Stream-ordered pipeline of one re-ranking problem (Algorithm 1):
// prep -> similarity (Eq. 7) -> top-(k1+m) -> FP32 re-score -> k1 lists
// (Eq. 8) -> A* (Eq. 9-11) -> L propagation layers (Eq. 12-14) -> final
// query x gallery product. Every step is a kernel of this library.
#include "pipeline.h"

namespace rr {

#define RR_TRY(call)                      \
  do {                                    \
    hipError_t e_ = (call);               \
    if (e_ != hipSuccess) {               \
      if (where) *where = #call;          \
      return e_;                          \
    }                                     \
  } while (0)

#define RR_STAGE(st, edge)                              \
  do {                                                  \
    if (clk) RR_TRY(clk->mark((st), (edge), s));        \
  } while (0)

hipError_t StageClock::init() {
  for (auto& st : sets)
    for (auto& pr : st.ev)
      for (auto& e : pr) {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
      }
  return hipSuccess;
}

void StageClock::destroy() {
  for (auto& st : sets)
    for (auto& pr : st.ev)
      for (auto& e : pr)
        if (e) hipEventDestroy(e), e = nullptr;
}

hipError_t StageClock::harvest(Set& st) {
  if (!st.pending) return hipSuccess;
  for (int k = 0; k < RERANK_STAGE_COUNT; k++) {
    if (!st.ran[k]) continue;
    hipError_t r = hipEventSynchronize(st.ev[k][1]);
    if (r != hipSuccess) return r;
    float ms = 0.f;
    r = hipEventElapsedTime(&ms, st.ev[k][0], st.ev[k][1]);
    if (r != hipSuccess) return r;
    sum_ms[k] += ms;
    runs[k] += 1;
    st.ran[k] = false;
  }
  st.pending = false;
  return hipSuccess;
}

hipError_t StageClock::begin_call() {
  cur = &sets[next];
  next = (next + 1) % kSets;
  return harvest(*cur);
}

hipError_t StageClock::totals(double* mean_ms) {
  for (auto& st : sets) {
    hipError_t r = harvest(st);
    if (r != hipSuccess) return r;
  }
  for (int k = 0; k < RERANK_STAGE_COUNT; k++) {
    mean_ms[k] = runs[k] ? sum_ms[k] / runs[k] : 0.0;
    sum_ms[k] = 0.0;
    runs[k] = 0;
  }
  return hipSuccess;
}

template <typename T>
static T* at(void* ws, size_t off) {
  return (T*)((char*)ws + off);
}

hipError_t enqueue_knn(const Plan& P, void* ws, const void* x, int in_bf16, hipStream_t s, const char** where,
                       StageClock* clk) {
  const float* xp = feature_rows(P, ws, x, in_bf16);
  float* rn = at<float>(ws, P.o_rn);
  float* sl = at<float>(ws, P.o_sl);
  void* xl = P.lbytes ? at<void>(ws, P.o_xl) : nullptr;
  float* S = P.has_s ? at<float>(ws, P.o_a) : nullptr;
  int32_t* ci = at<int32_t>(ws, P.o_ci);
  float* cv = at<float>(ws, P.o_cv);
  int32_t* ki = at<int32_t>(ws, P.o_ki);
  float* kv = at<float>(ws, P.o_kv);
  RR_STAGE(RERANK_STAGE_PREP, 0);
  RR_TRY(launch_prep(x, in_bf16, P.n, P.d, features_in_place(P, x, in_bf16) ? nullptr : at<float>(ws, P.o_xp), P.ldp,
                     rn, P.prec, xl, P.ldl, sl, s));
  RR_STAGE(RERANK_STAGE_PREP, 1);
  RR_STAGE(RERANK_STAGE_SIMILARITY, 0);
  if (P.fused) {  // S never written: the similarity stage also selects the candidates
    const void* a = P.prec == SimPrec::F32 ? (const void*)xp : xl;
    const int64_t row_bytes = P.prec == SimPrec::F32 ? P.ldp * 4 : P.ldl * P.lbytes;
    RR_TRY(launch_knn_fused(P.prec, a, P.n, row_bytes, row_bytes, P.prec == SimPrec::F32 ? rn : sl, P.kc,
                            at<void>(ws, P.o_fk), ci, cv, s));
    RR_STAGE(RERANK_STAGE_SIMILARITY, 1);
  } else {
    // the feature buffer B (not yet in use) holds the partial tiles of a K-split
    // last round; none for problems the serving path batches (as for the final)
    float* sws = (P.o_b && P.n > kGroupedMaxN) ? at<float>(ws, P.o_b) : nullptr;
    const int64_t sws_bytes = sws ? (int64_t)P.n * P.ldH * 4 : 0;
    // the product also records each row's largest similarity per block of
    // 128 columns, so the selection reads only the blocks that can hold a member
    float* bm = P.o_bm ? at<float>(ws, P.o_bm) : nullptr;
    if (P.prec == SimPrec::F32)
      RR_TRY(launch_gemm_sim(SimPrec::F32, xp, P.n, P.ldp * 4, P.ldp * 4, rn, S, P.ldN, false, sws, sws_bytes, s, bm,
                             P.ldN));
    else
      RR_TRY(launch_gemm_sim(P.prec, xl, P.n, P.ldl * P.lbytes, P.ldl * P.lbytes, sl, S, P.ldN, true, sws, sws_bytes,
                             s, bm, P.ldN));
    RR_STAGE(RERANK_STAGE_SIMILARITY, 1);
    RR_STAGE(RERANK_STAGE_TOPK, 0);
    if (bm)
      RR_TRY(launch_topk_pruned(S, P.prec != SimPrec::F32, P.ldN, P.n, P.n, P.kc, bm, P.ldN, ci, cv, P.kc, s));
    else
      RR_TRY(launch_topk(S, P.prec != SimPrec::F32, P.ldN, P.n, P.n, P.kc, ci, cv, P.kc, s));
    RR_STAGE(RERANK_STAGE_TOPK, 1);
  }
  RR_STAGE(RERANK_STAGE_RESCORE, 0);
  if (P.rescore)
    RR_TRY(launch_rescore(xp, P.ldp, P.d, rn, P.n, ci, cv, P.kc, P.k1, rescore_skip2(P.lbytes, P.ldp),
                          ki, kv, at<int32_t>(ws, P.o_rsc), s));
  else
    RR_TRY(launch_take_prefix(ci, cv, P.n, P.kc, P.k1, ki, kv, s));
  RR_STAGE(RERANK_STAGE_RESCORE, 1);
  return hipSuccess;
}

// CSR rows of sparse layer l (1..L) in its output buffer `buf` (the N x ldN
// feature buffer it writes: column indices, then values, n * ldN / 2 entries
// each) and the gates of l and l - 1. Row starts (n + 1) and counts (n)
// alternate between two sets by the parity of l.
static SlOut sl_out(const Plan& P, void* ws, float* buf, int l) {
  SlGate* gates = at<SlGate>(ws, P.o_slg);
  int32_t* sets = at<int32_t>(ws, P.o_slr);
  const int64_t cap = (int64_t)P.n * P.ldN / 2;
  int32_t* so = sets + (size_t)(l & 1) * (2 * P.n + 4);
  SlOut o{};
  o.rows = SlRows{(int32_t*)buf, (float*)((char*)buf + cap * 4), so, so + P.n + 1};
  o.gate = gates + l;
  o.prev = gates + (l - 1);
  o.cap = cap;
  o.n = P.n;
  return o;
}

hipError_t enqueue_rerank(const Plan& P, void* ws, const void* x, int in_bf16, float* dist, hipStream_t s,
                          const char** where, StageClock* clk) {
  hipError_t e = enqueue_knn(P, ws, x, in_bf16, s, where, clk);
  if (e != hipSuccess) return e;
  const float* xp = feature_rows(P, ws, x, in_bf16);
  float* rn = at<float>(ws, P.o_rn);
  float* A = at<float>(ws, P.o_a);
  float* B = (P.layers > 0 || P.fprec == FinalPrec::SPARSE) ? at<float>(ws, P.o_b) : nullptr;
  int32_t* ki = at<int32_t>(ws, P.o_ki);
  float* kv = at<float>(ws, P.o_kv);
  float* sa = at<float>(ws, P.o_sa);
  float* sb = at<float>(ws, P.o_sb);
  uint16_t* hi = (P.fprec == FinalPrec::BF16X3 || P.fprec == FinalPrec::BF16) ? at<uint16_t>(ws, P.o_hi) : nullptr;
  uint16_t* lo = P.fprec == FinalPrec::BF16X3 ? at<uint16_t>(ws, P.o_lo) : nullptr;

  const float* cur;
  const float* csig;
  RR_STAGE(RERANK_STAGE_ADJACENCY, 0);
  int first = 0;  // layers already done
  if (P.node != RERANK_NODE_RAW) {
    const bool sym = (P.node == RERANK_NODE_ADJ_SYM);
    int32_t* cnt = at<int32_t>(ws, P.o_cnt);
    RR_TRY(launch_fill_zero((float*)cnt, (int64_t)P.n * 2, s));
    if (P.sparse_first) {
      uint8_t* mflag = sym ? at<uint8_t>(ws, P.o_mflag) : nullptr;
      int32_t* off = sym ? at<int32_t>(ws, P.o_off) : nullptr;
      int32_t* inl = sym ? at<int32_t>(ws, P.o_inl) : nullptr;
      if (sym) {
        RR_TRY(launch_mutual(ki, P.n, P.k1, mflag, cnt, s));
        RR_TRY(launch_scan(cnt, P.n, off, at<int32_t>(ws, P.o_part), s));
        RR_TRY(launch_csr(ki, P.n, P.k1, mflag, off, cnt + P.n, inl, s));
      }
      RR_STAGE(RERANK_STAGE_ADJACENCY, 1);
      RR_STAGE(RERANK_STAGE_PROPAGATE, 0);
      const bool last = (P.layers == 1);
      if (P.sparse_layers || P.sparse_mid) {  // layer 1 as CSR rows
        SlGate* gates = at<SlGate>(ws, P.o_slg);
        RR_TRY(launch_fill_zero((float*)gates, (int64_t)(P.layers + 1) * (sizeof(SlGate) / 4), s));
        const SlOut o = sl_out(P, ws, B, 1);
        RR_TRY(launch_sl_slots(ki, P.n, P.k1, P.k2, true, sym, off, nullptr, o, at<int32_t>(ws, P.o_part), s));
        RR_TRY(launch_first_layer(ki, kv, mflag, off, inl, P.n, P.k1, P.k2, P.alpha, P.agg, sym, P.ldN, B, sa,
                                  nullptr, nullptr, &o, s));
      } else {
        RR_TRY(launch_first_layer(ki, kv, mflag, off, inl, P.n, P.k1, P.k2, P.alpha, P.agg, sym, P.ldN, B, sa,
                                  last ? hi : nullptr, last ? lo : nullptr, nullptr, s));
      }
      cur = B;
      csig = sa;
      first = 1;
    } else {  // dense h^(0): zero layers, or the max aggregator
      RR_TRY(launch_fill_zero(A, (int64_t)P.n * P.ldN, s));
      RR_TRY(launch_astar_scatter(ki, P.n, P.k1, A, P.ldN, cnt, sym, s));
      cur = A;
      csig = nullptr;  // h^(0) is not normalised
      if (P.layers == 0) {
        RR_TRY(launch_astar_sigma(cnt, P.n, P.k1, sa, sym, s));
        csig = sa;
      }
      RR_STAGE(RERANK_STAGE_ADJACENCY, 1);
      RR_STAGE(RERANK_STAGE_PROPAGATE, 0);
    }
  } else {
    cur = xp;  // raw features, zero-padded to ldp
    csig = (P.layers == 0) ? rn : nullptr;
    RR_STAGE(RERANK_STAGE_ADJACENCY, 1);
    RR_STAGE(RERANK_STAGE_PROPAGATE, 0);
  }
  const int32_t* order = nullptr;  // dense layers walk rows in cluster order
  if (first < P.layers && !P.sparse_layers && !P.sparse_mid) {
    int32_t* oscr = at<int32_t>(ws, P.o_ord);
    int32_t* ord = oscr + cluster_order_ints(P.n, P.n);
    RR_TRY(launch_cluster_order(ki, P.n, P.k1, P.n, oscr, ord, s));
    order = ord;
  }
  for (int l = first; l < P.layers; l++) {
    float* out = (cur == A) ? B : A;
    float* osig = (csig == sa) ? sb : sa;
    const bool last = (l == P.layers - 1);
    if (P.sparse_mid && last) {
      // the last layer of a dense final product: dense rows from the CSR rows of
      // layer l, or the dense layer when layer l had to be written densely
      SlGate* gates = at<SlGate>(ws, P.o_slg);
      const SlOut prev = sl_out(P, ws, (float*)cur, l);
      RR_TRY(launch_sparse_prop_dense(prev.rows, csig, ki, kv, P.n, P.k1, P.k2, P.alpha, P.agg, P.ldH, out, osig, hi,
                                      lo, prev.gate, s));
      RR_TRY(launch_propagate_gated(cur, csig, P.n, P.ldH, ki, kv, P.k1, P.k2, P.alpha, P.agg, out, osig, gates, l + 1,
                                    s, hi, lo));
    } else if (P.sparse_layers || P.sparse_mid) {
      // layer l + 1 from the CSR rows of layer l (or dense once a layer turned dense)
      SlGate* gates = at<SlGate>(ws, P.o_slg);
      const SlOut prev = sl_out(P, ws, (float*)cur, l);
      const SlOut next = sl_out(P, ws, out, l + 1);
      RR_TRY(launch_sl_slots(ki, P.n, P.k1, P.k2, false, false, nullptr, prev.rows.cnt, next,
                             at<int32_t>(ws, P.o_part), s));
      RR_TRY(launch_sparse_prop(prev.rows, csig, ki, kv, P.n, P.k1, P.k2, P.alpha, P.agg, P.ldH, out, osig, next,
                                s));
      RR_TRY(launch_propagate_gated(cur, csig, P.n, P.ldH, ki, kv, P.k1, P.k2, P.alpha, P.agg, out, osig, gates, l + 1,
                                    s));
    } else {
      RR_TRY(launch_propagate(cur, csig, P.n, P.ldH, P.ldH, ki, kv, P.k1, P.k2, P.alpha, P.agg, out, osig,
                              last ? hi : nullptr, last ? lo : nullptr, order, s));
    }
    cur = out;
    csig = osig;
  }
  RR_STAGE(RERANK_STAGE_PROPAGATE, 1);
  RR_STAGE(RERANK_STAGE_FINAL, 0);
  const float* hq = cur;
  const float* hg = cur + (size_t)P.q * P.ldH;
  if (P.fprec == FinalPrec::F32) {
    // scratch for the tail split: whichever N x N buffer does not hold the last
    // layer; none (no split) for problems the serving path batches
    float* spare = P.n <= kGroupedMaxN ? nullptr : (cur != A) ? A : B;
    const int64_t spare_bytes = !spare ? 0
                                : (spare == A) ? (int64_t)P.n * (P.ldN > P.ldH ? P.ldN : P.ldH) * 4
                                               : (int64_t)P.n * P.ldH * 4;
    RR_TRY(launch_gemm_dist(hq, P.q, hg, P.g, P.ldH, P.ldH, csig, csig + P.q, dist, P.g, spare, spare_bytes, s));
  } else if (P.fprec == FinalPrec::SPARSE) {  // adjacency features: cur is A or B, the other one is free
    float* pool = (cur == A) ? B : A;
    if (P.sparse_layers) {
      const SlOut last = sl_out(P, ws, (float*)cur, P.layers);
      RR_TRY(launch_sparse_final(cur, P.n, P.q, P.ldH, csig, dist, pool, (int64_t)P.n * P.ldH * 4,
                                 at<int32_t>(ws, P.o_sp), last.gate, &last.rows, ki, P.k1, s));
    } else {
      RR_TRY(launch_sparse_final(cur, P.n, P.q, P.ldH, csig, dist, pool, (int64_t)P.n * P.ldH * 4,
                                 at<int32_t>(ws, P.o_sp), nullptr, nullptr, ki, P.k1, s));
    }
  } else if (P.fprec == FinalPrec::BF16) {  // the last layer wrote the rows rounded to bfloat16
    if (P.layers == 0) RR_TRY(launch_split_bf16(cur, P.n, P.ldH, hi, nullptr, s));
    RR_TRY(launch_gemm_dist_bf16(hi, P.q, hi + (size_t)P.q * P.ldH, P.g, P.ldH, P.ldH, csig, csig + P.q, dist, P.g, s));
  } else {
    if (P.layers == 0) RR_TRY(launch_split_bf16(cur, P.n, P.ldH, hi, lo, s));
    RR_TRY(launch_gemm_dist_bf16x3(hi, lo, P.q, hi + (size_t)P.q * P.ldH, lo + (size_t)P.q * P.ldH, P.g, P.ldH,
                                   P.ldH, csig, csig + P.q, dist, P.g, s));
  }
  RR_STAGE(RERANK_STAGE_FINAL, 1);
  return hipSuccess;
}

}  // namespace rr
