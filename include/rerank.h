/*
 * rerank.h -- C ABI of the MI355X (gfx950) GNN re-ranking library.
 *
 * One re-ranking problem (Zhang et al., "Understanding Image Retrieval
 * Re-Ranking: A Graph Neural Network Perspective", Section 3.1 problem
 * definition and Section 3.3) is a set of N = Q + G feature vectors, the
 * queries first (rows 0..Q-1) and the gallery after (rows Q..N-1), the union
 * X_u of Eq. 7. Algorithm 1 turns it into query x gallery distances:
 *
 *   Eq. 7     S = cosine similarity of all rows (N x N)
 *   Eq. 8     N(i, k1): the k1 most similar rows of row i (row i itself is
 *             member 0 with similarity exactly 1; ties go to the lower index)
 *   Eq. 9-11  h_i^(0) = row i of A* = (A + A^T) / 2
 *   Eq. 12    edges e_ij = S_ij, j in N(i, k2) = the first k2 members of N(i, k1)
 *   Eq. 14    h_i <- h_i + sum_j e_ij^alpha h_j, then h_i <- h_i / |h_i|,
 *             repeated `layers` times (aggregator: sum)
 *   final     D[q][g] = 1 - cos(h_q, h_{Q+g})
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are device pointers on the context's HIP device,
 *     owned by the caller, row-major and contiguous. They must stay valid,
 *     and inputs unchanged, until the work that uses them has completed
 *     (stream order for the stream-ordered calls, until rerank_wait/
 *     rerank_poll report completion for submitted requests): FP32 features
 *     whose rows are already 256-byte multiples on a 256-byte aligned address
 *     are read in place by every stage rather than copied.
 *   - Functions return a rerank_status and never abort. Parameters are
 *     validated before any work is enqueued; on error nothing is enqueued
 *     and rerank_last_error() gives a readable reason.
 *   - Inputs must be finite and no feature row may be all zero; the values of
 *     the result are unspecified otherwise. Even then, every neighbour list
 *     holds K distinct columns of the problem (row i first), so no stage reads
 *     outside its buffers: a NaN similarity ranks after every number, and a
 *     selection whose pruning bound admits fewer than K values (a NaN passes
 *     no comparison) re-selects over the whole row.
 *   - All library-owned device memory (similarity matrix, neighbour lists,
 *     feature buffers) comes from a pool bounded by the context's budget.
 */
#ifndef RERANK_H
#define RERANK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rerank_ctx rerank_ctx; /* opaque; created and owned by the library */

typedef enum {
  RERANK_OK = 0,
  RERANK_E_INVALID = 1,   /* bad parameter or pointer */
  RERANK_E_NOMEM = 2,     /* working set exceeds the context budget, or device allocation failed */
  RERANK_E_HIP = 3,       /* a HIP runtime call or kernel launch failed */
  RERANK_E_BUSY = 4,      /* request still running (rerank_poll/cancel) */
  RERANK_E_TIMEOUT = 5,   /* rerank_wait timed out; the request keeps running */
  RERANK_E_CANCELLED = 6, /* request was cancelled before it started */
  RERANK_E_UNSUPPORTED = 7/* valid in the paper's terms but outside this library's limits */
} rerank_status;

/* Storage type of the caller's feature matrix. */
typedef enum { RERANK_IN_F32 = 0, RERANK_IN_BF16 = 1 } rerank_in_dtype;

/* Arithmetic of the Eq. 7 similarity product. F32 is the plain method.
 * BF16 and FP8_E4M3 (per-row scales) compute S on low-precision matrix cores
 * with FP32 accumulation, keep k1 + extra_cand candidates per row and
 * re-score those in FP32 before the final k1 cut. Everything after the
 * neighbour lists is FP32 in every mode. */
typedef enum { RERANK_SIM_F32 = 0, RERANK_SIM_BF16 = 1, RERANK_SIM_FP8_E4M3 = 2 } rerank_sim_prec;

/* Vertex feature h^(0) (Table 1 ablation columns): A* rows as in Eq. 11, the
 * raw features x_i (with zero layers this reproduces the initial cosine
 * ranking), or the rows of the non-symmetrised A of Eq. 8. */
typedef enum { RERANK_NODE_ADJ_SYM = 0, RERANK_NODE_RAW = 1, RERANK_NODE_ADJ = 2 } rerank_node;

/* Aggregator of Eq. 13 (the paper uses sum). mean divides the sum of the k2
 * messages e_ij^alpha h_j by k2; max takes their element-wise maximum. The
 * residual h_i is added in every case. */
typedef enum { RERANK_AGG_SUM = 0, RERANK_AGG_MEAN = 1, RERANK_AGG_MAX = 2 } rerank_aggregator;

/* Arithmetic of the final query x gallery product. F32 is plain FP32 matrix
 * cores; BF16 rounds the refined features to bfloat16 (nearest even) and
 * multiplies them on bfloat16 matrix cores with FP32 accumulation, scaled by
 * the FP32 inverse norms (cosine error below 2^-7: a low-precision mode, for
 * the low-precision similarity paths); BF16X3 splits each FP32 operand into a high and a low bfloat16 part
 * and sums the three leading partial products on bfloat16 matrix cores with
 * FP32 accumulation (relative error of each product about 2^-16). SPARSE
 * multiplies only the non-zeros of the refined features: A* rows hold O(k1)
 * non-zeros (Eq. 9-11) and each layer of Eq. 14 widens a row only to its k2
 * neighbours' supports, so query q's distances are an FP32 sum over q's
 * non-zero columns c, in ascending c, of h_q[c] times column c of the
 * gallery features. Not available with RERANK_NODE_RAW (dense features).
 * With the sum or mean aggregator and layers >= 1 the layers themselves are
 * kept as CSR rows (each row in a slot sized by its members' entry counts),
 * so no dense N x N row is written; a layer whose slots would not fit in an
 * N x N buffer is written densely instead. Dense last layers are compacted
 * before the product; when the compacted rows would exceed the spare N x N
 * buffer (average row density above 1/4) the FP32 matrix-core product runs
 * instead. All of these choices are made on the device. */
typedef enum {
  RERANK_FINAL_F32 = 0,
  RERANK_FINAL_BF16X3 = 1,
  RERANK_FINAL_SPARSE = 2,
  RERANK_FINAL_BF16 = 3
} rerank_final_prec;

typedef struct {
  int32_t n;          /* N = Q + G rows of X_u, N >= 2 */
  int32_t n_query;    /* Q, 1 <= Q <= N - 1 */
  int32_t dim;        /* feature dimension d >= 1 */
  int32_t k1;         /* Eq. 8 list length, 1 <= k1 <= N */
  int32_t k2;         /* Eq. 12 edges per vertex, 1 <= k2 <= k1 */
  int32_t layers;     /* propagation steps of Eq. 14, 0 <= layers <= 256 */
  int32_t alpha;      /* Eq. 14 weight exponent, integer 0..8 (the paper uses 2) */
  int32_t sim_prec;   /* rerank_sim_prec */
  int32_t extra_cand; /* candidates beyond k1 re-scored in FP32; -1 = default
                         (8 for F32, 16 for BF16, 32 for FP8); 0 disables
                         re-scoring (F32 only). k1 + extra_cand is capped at N
                         and at 256. */
  int32_t node;       /* rerank_node */
  int32_t final_prec; /* rerank_final_prec */
  int32_t aggregator; /* rerank_aggregator */
} rerank_params;

/* Fill *p with the paper's settings (alpha 2, sum aggregator, A* features,
 * two layers, FP32) for a problem of n rows, q queries, d dimensions and the
 * given k1/k2. Pure host function. */
void rerank_default_params(rerank_params* p, int32_t n, int32_t q, int32_t d, int32_t k1, int32_t k2);

/* Check *p against the limits above. Pure host function (no device access). */
rerank_status rerank_validate(const rerank_params* p);

/* Bytes of library-owned device memory one problem with parameters *p needs.
 * Pure host function; used for admission. */
rerank_status rerank_workspace_bytes(const rerank_params* p, size_t* bytes);

/* Context flags. STAGE_TIMING records a HIP event pair around every stage of
 * the direct calls (on the call's stream) so rerank_stage_times can report
 * per-stage device time; it adds no synchronisation. */
#define RERANK_CTX_STAGE_TIMING 1u
/* DENSE_LAYERS: write every propagation layer as dense N x N rows. By default
 * (sum or mean aggregator, A* or A features, layers >= 1) the layers are kept
 * as CSR rows wherever that is possible: all of them for RERANK_FINAL_SPARSE
 * (see rerank_final_prec), and all but the last for the other final products,
 * whose last layer is then written densely from the CSR rows before it. The
 * distances are the same either way, bit for bit. */
#define RERANK_CTX_DENSE_LAYERS 2u
/* FUSED_KNN (the similarity product fused with the candidate selection of
 * Eq. 8): rerank_knn and rerank_run select each row's k1 + extra_cand
 * candidates from the product's tiles, so the N x N similarity S is never
 * written; rerank_knn then needs no N x N buffer at all. A sample of whole
 * column panels is multiplied first to give each row a lower bound on its
 * (k1 + extra_cand)-th best similarity; then every upper-triangle tile of
 * the rest is computed once and its values at or above a row's bound are kept
 * for that row (S is symmetric: each tile serves its rows and its columns).
 * The selected lists follow the same order and tie rule as the unfused
 * path's and are the same lists on the same bits. Working set: the feature
 * copies, the stored sample and the candidate slots, which together grow as
 * N^1.5 (about 0.3 GB at N = 19281, k1 = 26, FP32, against 1.5 GB for S).
 * Requires k1 + extra_cand <= 64 (else RERANK_E_UNSUPPORTED). The serving
 * calls (rerank_submit) ignore it. */
#define RERANK_CTX_FUSED_KNN 4u

/* Bytes of library-owned device memory rerank_knn needs for *p in a context
 * created with `flags` (the Eq. 7-8 k-NN graph alone). Without
 * RERANK_CTX_FUSED_KNN this includes the N x N similarity buffer; with it
 * there is none (feature copies, the stored column sample and the candidate
 * slots).
 * Pure host function. RERANK_E_INVALID for invalid parameters, unknown flags or
 * a NULL `bytes`; RERANK_E_UNSUPPORTED when the fused path cannot take
 * k1 + extra_cand. */
rerank_status rerank_knn_workspace_bytes(const rerank_params* p, uint32_t flags, size_t* bytes);

/* Create a context on HIP device `hip_device`. The context never holds more
 * than `hbm_budget_bytes` of device memory (0 = 90% of the device's free
 * memory at creation). flags: 0 or an OR of RERANK_CTX_STAGE_TIMING,
 * RERANK_CTX_DENSE_LAYERS and RERANK_CTX_FUSED_KNN. */
rerank_status rerank_create(rerank_ctx** out, int hip_device, size_t hbm_budget_bytes, uint32_t flags);

/* Wait for all work of the context, stop its scheduler, free its memory. */
rerank_status rerank_destroy(rerank_ctx* ctx);

/* Full method (Algorithm 1), stream-ordered on `hip_stream` (a hipStream_t;
 * NULL = the null stream); the host does not wait.
 *   d_x     N x dim features, float32 or bfloat16 bit patterns (in_dtype)
 *   d_dist  out: Q x G float32, D[q][g] = 1 - cos(h_q, h_{Q+g})
 *   d_knn_idx, d_knn_val  optional out (NULL to skip): N x k1 int32 list of
 *           N(i, k1) in rank order and the matching float32 similarities
 * Calls on one context are serialised on the device in call order (they
 * share the context's working memory), whatever streams they use. */
rerank_status rerank_run(rerank_ctx* ctx, const rerank_params* p, const void* d_x, int32_t in_dtype,
                         float* d_dist, int32_t* d_knn_idx, float* d_knn_val, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * computation, kernels and results as rerank_run, with the problem's working
 * set in a static device array of RERANK_STATIC_BYTES that every GPU holds
 * from the library's first use on it until the process ends. The call makes
 * no device or host allocation and no stage timing. Arguments as for
 * rerank_run; ctx supplies the device and its DENSE_LAYERS / FUSED_KNN flags.
 * RERANK_E_NOMEM (nothing enqueued) when rerank_workspace_bytes(p) exceeds
 * RERANK_STATIC_BYTES (for example N = 5000, d = 512, FP32, one layer fits).
 * All calls on one GPU share its array and find the previous call's contents
 * there: calls whose work overlaps on the device (unordered streams, several
 * host threads) race and give undefined results; order them, e.g. on one
 * stream. The array is separate from the context's own working set, so
 * rerank_run and rerank_run_static do not interfere. */
#define RERANK_STATIC_BYTES ((size_t)256 << 20)
rerank_status rerank_run_static(rerank_ctx* ctx, const rerank_params* p, const void* d_x, int32_t in_dtype,
                                float* d_dist, int32_t* d_knn_idx, float* d_knn_val, void* hip_stream);

/* Phase 1 only (Eq. 7-8, the k-NN graph): the N x k1 neighbour lists and
 * their similarities, same argument meaning as rerank_run. */
rerank_status rerank_knn(rerank_ctx* ctx, const rerank_params* p, const void* d_x, int32_t in_dtype,
                         int32_t* d_knn_idx, float* d_knn_val, void* hip_stream);

/* Eq. 7 only: d_s (N rows, row stride ld_s >= N floats) receives S computed
 * with p->sim_prec arithmetic (low-precision modes return their
 * low-precision S). Stream-ordered like rerank_run. */
rerank_status rerank_similarity(rerank_ctx* ctx, const rerank_params* p, const void* d_x, int32_t in_dtype,
                                float* d_s, int64_t ld_s, void* hip_stream);

/* The first r entries of the ranking list L that Algorithm 1 returns: for
 * each of the q rows of d_dist (row stride g floats, as rerank_run writes
 * it), the positions of the r smallest distances in ascending order, ties to
 * the lower position. d_rank: q x r int32 (gallery position 0 = row Q of the
 * problem). 1 <= r <= min(g, 256). Stream-ordered; ctx supplies the device. */
rerank_status rerank_rank(rerank_ctx* ctx, const float* d_dist, int32_t q, int32_t g, int32_t r, int32_t* d_rank,
                          void* hip_stream);

/* Retrieval quality of a distance matrix under identity labels, the
 * evaluation metrics of Section 4.1 (mean average precision and Recall@K).
 * Each query's ranking list is its gallery positions by ascending distance,
 * ties to the lower position (as rerank_rank); its true matches are the
 * gallery positions whose label equals the query's.
 *   d_dist      q rows of g float32 distances, row stride ld_dist >= g
 *               (rerank_run writes ld_dist = g); finite values
 *   d_q_labels  q int32 labels; d_g_labels  g int32 labels
 *   ks, n_ks    HOST array of 1 <= n_ks <= 16 cut-offs, each K >= 1
 *   d_ap        out: q float64, the query's average precision = the
 *               trapezoid area under its precision-recall curve (from
 *               recall 0 at precision 1, one point per list position); 0
 *               for a query without a true match
 *   d_first     out: q int32, list position of the first true match, -1
 *               without one
 *   d_summary   out: n_ks + 2 float64: [mAP, Recall@ks[0], ...,
 *               Recall@ks[n_ks-1], number of queries with a true match];
 *               the means are over the queries with a true match (0 if none)
 * All d_ pointers are device memory owned by the caller (d_ap, d_summary
 * 8-byte aligned, the rest 4-byte aligned). Stream-ordered on hip_stream;
 * the host does not wait. RERANK_E_INVALID for NULL or misaligned pointers
 * or sizes out of range. */
rerank_status rerank_evaluate(rerank_ctx* ctx, const float* d_dist, int32_t q, int32_t g, int64_t ld_dist,
                              const int32_t* d_q_labels, const int32_t* d_g_labels, const int32_t* ks, int32_t n_ks,
                              double* d_ap, int32_t* d_first, double* d_summary, void* hip_stream);

/* ---- serving: asynchronous requests with admission and continuous batching
 * A submitted request is admitted once its working set (rerank_workspace_bytes)
 * fits in the free part of the context budget; admitted requests run
 * concurrently on the context's streams. Each request's result is the same as
 * rerank_run on the same input. The caller keeps d_x and d_dist valid until
 * the request is reported done. Tickets are unique per context.
 *   hip_stream  the stream (hipStream_t, NULL = the null stream) on which the
 *               caller produced d_x: an event is recorded on it at submit and
 *               the request's kernels start only after the work enqueued on
 *               it before the call; it must belong to the context's device
 *               (RERANK_E_HIP otherwise).
 * The memory of the direct calls (rerank_run, rerank_knn, rerank_similarity)
 * and of the serving requests comes from the one budget: a request that does
 * not fit next to the direct calls' working set while no request runs gets
 * that working set back (after its kernels finish; the next direct call
 * allocates it again), and a direct call that does not fit gets the blocks the
 * serving pool keeps cached. */
rerank_status rerank_submit(rerank_ctx* ctx, const rerank_params* p, const void* d_x, int32_t in_dtype,
                            float* d_dist, void* hip_stream, uint64_t* ticket);

/* *done = 1 once the request finished (successfully or not), else 0. */
rerank_status rerank_poll(rerank_ctx* ctx, uint64_t ticket, int* done);

/* Block until the request is done or `timeout_us` passes (negative = no
 * limit). Returns the request's own status (RERANK_OK, an error it met, or
 * RERANK_E_CANCELLED), or RERANK_E_TIMEOUT. *latency_ms (optional) receives
 * submit-to-completion time. A finished ticket is forgotten after a
 * successful wait. */
rerank_status rerank_wait(rerank_ctx* ctx, uint64_t ticket, int64_t timeout_us, double* latency_ms);

/* Cancel a request that has not started; RERANK_E_BUSY if it already runs. */
rerank_status rerank_cancel(rerank_ctx* ctx, uint64_t ticket);

/* Stages of one problem, in pipeline order (Phase 1 of the paper's Table 3 is
 * PREP..ADJACENCY, Phase 2 is PROPAGATE..FINAL). */
typedef enum {
  RERANK_STAGE_PREP = 0,       /* norms, padded / low-precision feature copies */
  RERANK_STAGE_SIMILARITY = 1, /* Eq. 7 product */
  RERANK_STAGE_TOPK = 2,       /* top-(k1 + extra) per row */
  RERANK_STAGE_RESCORE = 3,    /* FP32 re-score and k1 cut (Eq. 8) */
  RERANK_STAGE_ADJACENCY = 4,  /* A* rows, Eq. 9-11 */
  RERANK_STAGE_PROPAGATE = 5,  /* all layers of Eq. 14 */
  RERANK_STAGE_FINAL = 6,      /* query x gallery product and distances */
  RERANK_STAGE_COUNT = 7
} rerank_stage;

/* Mean device milliseconds per direct call of each stage, over the direct
 * calls since the previous rerank_stage_times on this context (waits for
 * them to finish, then restarts the averages). Needs a context created with
 * RERANK_CTX_STAGE_TIMING. ms_out receives RERANK_STAGE_COUNT values; stages
 * that did not run read 0. RERANK_E_INVALID if timing is off. */
rerank_status rerank_stage_times(rerank_ctx* ctx, double* ms_out);

/* Static name of a stage ("prep", "similarity", ...), NULL if out of range. */
const char* rerank_stage_name(int32_t stage);

/* Static string for a status code. */
const char* rerank_status_str(rerank_status s);

/* Detail of the last error raised on this thread (any context), "" if none. */
const char* rerank_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RERANK_H */
