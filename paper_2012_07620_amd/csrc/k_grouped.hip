// Persistent grouped launches of the serving path: one launch per stage for
// a whole batch of small problems. Workgroups stride over the work items of
// all problems (the per-problem item ranges come from the batch table), and
// each item runs the same body as the direct launch, so a problem's result
// does not depend on what it was batched with.
#include "batch.h"
#include "gemm_body.h"
#include "rows_body.h"

#pragma clang fp contract(off)

namespace rr {

constexpr int kGroupedRowWGs = 2048;
constexpr int kGroupedGemmWGs = 512;  // two workgroups per CU

__device__ __forceinline__ int find_prob(const BatchTable* __restrict__ t, int stage, int item) {
  int p = 0;
  while (p + 1 < t->count && t->start[stage][p + 1] <= item) p++;
  return p;
}

#define FOR_ITEMS(stage)                                                     \
  const int total_ = t->start[stage][t->count];                              \
  for (int item = blockIdx.x; item < total_; item += gridDim.x)

template <SimPrec P>
__global__ __launch_bounds__(256) void g_prep(const BatchTable* __restrict__ t) {
  FOR_ITEMS(GS_PREP) {
    const int p = find_prob(t, GS_PREP, item);
    const ProbDesc& D = t->p[p];
    const int i = (item - t->start[GS_PREP][p]) * 4 + (threadIdx.x >> 6);
    if (i < D.n) {
      if (D.in_bf16)
        prep_row<P, true>(D.x, i, D.d, D.xp, D.ldp, D.rn, D.xl, D.ldl, D.sl);
      else
        prep_row<P, false>(D.x, i, D.d, D.xp, D.ldp, D.rn, D.xl, D.ldl, D.sl);
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void g_sim(const BatchTable* __restrict__ t) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[GEMM_LDS_BYTES];
  FOR_ITEMS(GS_SIM) {
    const int p = find_prob(t, GS_SIM, item);
    const ProbDesc& D = t->p[p];
    const uint8_t* a = (MODE == MODE_F32) ? (const uint8_t*)D.xp : (const uint8_t*)D.xl;
    const int64_t lda = (MODE == MODE_F32) ? D.ldp * 4 : D.ldl * D.lbytes;
    const float* sc = (MODE == MODE_F32) ? D.rn : D.sl;
    const GemmArgs g{a, a, D.n, D.n, lda, lda, (int)(lda / BKB), sc, sc, D.A, D.ldN};
    const int T = (D.n + BM - 1) / BM;
    int tm, tn;
    upper_tile(item - t->start[GS_SIM][p], T, tm, tn);
    gemm_tile<MODE, MODE == MODE_F32 ? EPI_SIM_SYM : EPI_SIM_SYM16>(g, tm, tn, lds);  // as the direct path
  }
}

template <int R, typename T>
__global__ __launch_bounds__(256) void g_topk(const BatchTable* __restrict__ t) {
  __shared__ uint64_t ring_all[4][128];
  FOR_ITEMS(GS_TOPK) {
    const int p = find_prob(t, GS_TOPK, item);
    const ProbDesc& D = t->p[p];
    const int i = (item - t->start[GS_TOPK][p]) * 4 + (threadIdx.x >> 6);
    if (i < D.n)
      topk_row<R, false, T>((const T*)D.A, D.ldN, D.n, i, D.kc, D.ci, D.cv, D.kc, ring_all[threadIdx.x >> 6]);
  }
}

template <int R>
__global__ __launch_bounds__(256) void g_rescore(const BatchTable* __restrict__ t) {
  FOR_ITEMS(GS_RESCORE) {
    const int p = find_prob(t, GS_RESCORE, item);
    const ProbDesc& D = t->p[p];
    const int i = (item - t->start[GS_RESCORE][p]) * 4 + (threadIdx.x >> 6);
    if (i < D.n)
      rescore_row<R>(D.xp, D.ldp, D.rn, i, D.ci, D.cv, D.kc, D.k1, rescore_skip2(D.lbytes, D.ldp), D.ki, D.kv);
  }
}

__global__ __launch_bounds__(256) void g_fill(const BatchTable* __restrict__ t) {
  FOR_ITEMS(GS_FILL) {
    const int p = find_prob(t, GS_FILL, item);
    const ProbDesc& D = t->p[p];
    const int64_t local = item - t->start[GS_FILL][p];
    if (local < D.fill_items_a)
      fill_item(D.A, (int64_t)D.n * D.ldN, local);
    else
      fill_item((float*)D.cnt, (int64_t)D.n * 2, local - D.fill_items_a);
  }
}

__global__ __launch_bounds__(256) void g_scatter(const BatchTable* __restrict__ t) {
  FOR_ITEMS(GS_SCATTER) {
    const int p = find_prob(t, GS_SCATTER, item);
    const ProbDesc& D = t->p[p];
    const int64_t pair = (int64_t)(item - t->start[GS_SCATTER][p]) * 256 + threadIdx.x;
    scatter_pair(D.ki, D.n, D.k1, D.A, D.ldN, D.cnt, pair, D.node == RERANK_NODE_ADJ_SYM);
  }
}

__global__ __launch_bounds__(256) void g_mutual(const BatchTable* __restrict__ t) {
  FOR_ITEMS(GS_MUTUAL) {
    const int p = find_prob(t, GS_MUTUAL, item);
    const ProbDesc& D = t->p[p];
    mutual_pair(D.ki, D.n, D.k1, D.mflag, D.cnt, (int64_t)(item - t->start[GS_MUTUAL][p]) * 256 + threadIdx.x);
  }
}

__global__ __launch_bounds__(256) void g_scan(const BatchTable* __restrict__ t) {
  __shared__ int32_t sh[256];
  FOR_ITEMS(GS_SCAN) {
    const ProbDesc& D = t->p[find_prob(t, GS_SCAN, item)];
    scan_offsets(D.cnt, D.n, D.off, sh);
  }
}

__global__ __launch_bounds__(256) void g_csr(const BatchTable* __restrict__ t) {
  FOR_ITEMS(GS_CSR) {
    const int p = find_prob(t, GS_CSR, item);
    const ProbDesc& D = t->p[p];
    csr_pair(D.ki, D.n, D.k1, D.mflag, D.off, D.cnt + D.n, D.inl,
             (int64_t)(item - t->start[GS_CSR][p]) * 256 + threadIdx.x);
  }
}

__global__ __launch_bounds__(256) void g_first(const BatchTable* __restrict__ t) {
  __shared__ FirstShared sh;
  FOR_ITEMS(GS_PROP) {
    const int p = find_prob(t, GS_PROP, item);
    const ProbDesc& D = t->p[p];
    first_layer_row(D.ki, D.kv, D.mflag, D.off, D.inl, D.k1, D.k2, D.alpha, D.agg, D.node == RERANK_NODE_ADJ_SYM,
                    D.ldN, D.B, D.sa, nullptr, nullptr, item - t->start[GS_PROP][p], sh);
  }
}

__global__ __launch_bounds__(256) void g_sigma(const BatchTable* __restrict__ t) {
  FOR_ITEMS(GS_SIGMA) {
    const int p = find_prob(t, GS_SIGMA, item);
    const ProbDesc& D = t->p[p];
    astar_sigma_row(D.cnt, D.n, D.k1, D.sa, (item - t->start[GS_SIGMA][p]) * 256 + threadIdx.x,
                    D.node == RERANK_NODE_ADJ_SYM);
  }
}

// Buffers of layer l, matching the direct pipeline: the layer input is h^(0)
// (A* rows in A, or the raw copy xp) for l = 0, then the outputs alternate
// between the two spare buffers; the carried norms alternate sa, sb.
__device__ __forceinline__ void layer_bufs(const ProbDesc& D, int l, const float*& hin, const float*& sin,
                                           float*& hout, float*& sout) {
  const bool adj = (D.node != RERANK_NODE_RAW);
  float* h0 = adj ? D.A : D.xp;
  float* o1 = adj ? D.B : D.A;
  float* o2 = adj ? D.A : D.B;
  hout = (l % 2 == 0) ? o1 : o2;
  sout = (l % 2 == 0) ? D.sa : D.sb;
  hin = (l == 0) ? h0 : ((l % 2 == 1) ? o1 : o2);
  sin = (l == 0) ? nullptr : ((l % 2 == 1) ? D.sa : D.sb);
}

__global__ __launch_bounds__(256) void g_prop(const BatchTable* __restrict__ t, int l) {
  __shared__ PropShared sh;
  FOR_ITEMS(GS_PROP) {
    const int p = find_prob(t, GS_PROP, item);
    const ProbDesc& D = t->p[p];
    const float* hin;
    const float* sin;
    float* hout;
    float* sout;
    layer_bufs(D, l, hin, sin, hout, sout);
    propagate_row(hin, sin, D.ldH, D.ldH, D.ki, D.kv, D.k1, D.k2, D.alpha, D.agg, hout, sout, nullptr, nullptr,
                  item - t->start[GS_PROP][p], sh);
  }
}

__global__ __launch_bounds__(256) void g_final(const BatchTable* __restrict__ t) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[GEMM_LDS_1BUF];
  const int L = t->layers;
  FOR_ITEMS(GS_FINAL) {
    const int p = find_prob(t, GS_FINAL, item);
    const ProbDesc& D = t->p[p];
    const float* h;
    const float* sg;
    if (L == 0) {
      const bool adj = (D.node != RERANK_NODE_RAW);
      h = adj ? D.A : D.xp;
      sg = adj ? D.sa : D.rn;
    } else {
      const float* hin;
      const float* sin;
      float* hout;
      float* sout;
      layer_bufs(D, L - 1, hin, sin, hout, sout);
      h = hout;
      sg = sout;
    }
    const GemmArgs g{(const uint8_t*)h, (const uint8_t*)(h + (int64_t)D.q * D.ldH), D.q, D.g, D.ldH * 4, D.ldH * 4,
                     (int)(D.ldH * 4 / BKB), sg, sg + D.q, D.dist, D.g};
    const int local = item - t->start[GS_FINAL][p];
    gemm_tile<MODE_F32, EPI_DIST>(g, local % D.tiles_fin_m, local / D.tiles_fin_m, lds);
  }
}

template <typename K, typename... Args>
static hipError_t go(K kernel, int wgs, hipStream_t s, Args... args) {
  hipLaunchKernelGGL(kernel, dim3(wgs), dim3(256), 0, s, args...);
  return hipGetLastError();
}

#define GTRY(call)                      \
  do {                                  \
    hipError_t e_ = (call);             \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

hipError_t enqueue_grouped(const BatchKey& key, const BatchTable* d_tab, hipStream_t s) {
  const SimPrec prec = (SimPrec)key.prec;
  switch (prec) {
    case SimPrec::F32:
      GTRY(go(g_prep<SimPrec::F32>, kGroupedRowWGs, s, d_tab));
      GTRY(go(g_sim<MODE_F32>, kGroupedGemmWGs, s, d_tab));
      break;
    case SimPrec::BF16:
      GTRY(go(g_prep<SimPrec::BF16>, kGroupedRowWGs, s, d_tab));
      GTRY(go(g_sim<MODE_BF16>, kGroupedGemmWGs, s, d_tab));
      break;
    case SimPrec::FP8:
      GTRY(go(g_prep<SimPrec::FP8>, kGroupedRowWGs, s, d_tab));
      GTRY(go(g_sim<MODE_FP8>, kGroupedGemmWGs, s, d_tab));
      break;
  }
  const bool half = prec != SimPrec::F32;  // S in binary16, as the direct path
  switch (key.r) {
    case 1:
      GTRY(half ? go(g_topk<1, _Float16>, kGroupedRowWGs, s, d_tab) : go(g_topk<1, float>, kGroupedRowWGs, s, d_tab));
      GTRY(go(g_rescore<1>, kGroupedRowWGs, s, d_tab));
      break;
    case 2:
      GTRY(half ? go(g_topk<2, _Float16>, kGroupedRowWGs, s, d_tab) : go(g_topk<2, float>, kGroupedRowWGs, s, d_tab));
      GTRY(go(g_rescore<2>, kGroupedRowWGs, s, d_tab));
      break;
    default:
      GTRY(half ? go(g_topk<4, _Float16>, kGroupedRowWGs, s, d_tab) : go(g_topk<4, float>, kGroupedRowWGs, s, d_tab));
      GTRY(go(g_rescore<4>, kGroupedRowWGs, s, d_tab));
      break;
  }
  int first = 0;
  if (key.node != RERANK_NODE_RAW) {
    GTRY(go(g_fill, kGroupedRowWGs, s, d_tab));  // counts (and h^(0) when it is dense)
    if (key.layers == 0 || key.agg == RERANK_AGG_MAX) {
      GTRY(go(g_scatter, kGroupedRowWGs, s, d_tab));
      if (key.layers == 0) GTRY(go(g_sigma, 256, s, d_tab));
    } else {
      if (key.node == RERANK_NODE_ADJ_SYM) {
        GTRY(go(g_mutual, kGroupedRowWGs, s, d_tab));
        GTRY(go(g_scan, kMaxBatch, s, d_tab));
        GTRY(go(g_csr, kGroupedRowWGs, s, d_tab));
      }
      GTRY(go(g_first, kGroupedRowWGs, s, d_tab));
      first = 1;
    }
  }
  for (int l = first; l < key.layers; l++) GTRY(go(g_prop, kGroupedRowWGs, s, d_tab, l));
  GTRY(go(g_final, kGroupedGemmWGs, s, d_tab));
  return hipSuccess;
}

}  // namespace rr
