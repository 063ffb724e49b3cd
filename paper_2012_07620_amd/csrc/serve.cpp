// Serving: asynchronous requests with admission by working-set bytes and
// continuous batching.
//
// A scheduler thread owns kSlots execution slots, each with its own HIP
// stream (default priority). Pending requests are admitted in arrival order
// as soon as a slot is idle and the request's working set fits in the
// context budget, so requests that arrive while others run start as slots
// and memory free up, and their kernels overlap on the device.
//
// Small problems (N <= kGroupedMaxN) are gathered into batches of up to kMaxBatch
// requests with the same batch key and run as one persistent grouped launch
// per stage. Each slot captures that launch sequence (table copy from pinned
// host memory + one launch per stage) into a hipGraph per key once, and a
// batch then costs one graph launch. Larger problems run the direct pipeline
// on the slot's stream. Working sets come from a caching pool bounded by the
// budget; features, lists and feature buffers stay in HBM for the whole
// request. A request's kernels start after the work its caller had enqueued
// on the stream named at submit time (an event recorded there).
#include "serve.h"

#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <vector>

#include "batch.h"
#include "pipeline.h"

namespace rr {

constexpr int kSlots = 4;

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  rerank_params params{};
  Plan plan;
  const void* x = nullptr;
  int in_bf16 = 0;
  float* dist = nullptr;
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submit
  bool small = false;
  BatchKey key{};
  void* ws = nullptr;
  size_t ws_bytes = 0;
  Clock::time_point t_submit, t_done;
  enum State { PENDING, RUNNING, DONE } state = PENDING;
  rerank_status status = RERANK_OK;
  std::string error;
};

// Budget-bounded caching pool of device working sets.
class Pool {
 public:
  Pool(size_t budget, std::atomic<size_t>* reserved) : budget_(budget), reserved_(reserved) {
    if (const char* f = std::getenv("RERANK_FAULT")) {
      if (std::strncmp(f, "alloc:", 6) == 0) fail_at_ = std::atoll(f + 6);
    }
  }
  ~Pool() { release_cache(); }

  // Returns a block of >= bytes, nullptr when the budget is exhausted right
  // now (*fatal = false, caller waits) or when the allocation failed
  // (*fatal = true).
  void* alloc(size_t bytes, bool* fatal) {
    *fatal = false;
    calls_++;
    if (fail_at_ > 0 && calls_ == fail_at_) {
      *fatal = true;
      return nullptr;
    }
    // best fit among cached blocks no larger than 1.5x the request
    auto best = free_.end();
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes && it->second <= bytes + bytes / 2 && (best == free_.end() || it->second < best->second))
        best = it;
    if (best != free_.end()) {
      void* p = best->first;
      size_t sz = best->second;
      free_.erase(best);
      live_[p] = sz;
      return p;
    }
    // make room: drop cached blocks while the budget does not allow a new one
    bool ok = try_reserve(*reserved_, budget_, bytes);
    while (!ok && !free_.empty()) {
      auto it = free_.begin();
      hipFree(it->first);
      *reserved_ -= it->second;
      free_.erase(it);
      ok = try_reserve(*reserved_, budget_, bytes);
    }
    if (!ok) return nullptr;
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      *reserved_ -= bytes;
      *fatal = true;
      return nullptr;
    }
    live_[p] = bytes;
    return p;
  }
  void release(void* p) {
    auto it = live_.find(p);
    if (it == live_.end()) return;
    free_[p] = it->second;
    live_.erase(it);
  }
  void release_cache() {
    for (auto& kv : free_) {
      hipFree(kv.first);
      *reserved_ -= kv.second;
    }
    free_.clear();
  }

 private:
  size_t budget_;
  std::atomic<size_t>* reserved_;
  std::map<void*, size_t> free_, live_;
  long long calls_ = 0, fail_at_ = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  BatchTable* h_tab = nullptr;  // pinned
  BatchTable* d_tab = nullptr;
  std::map<BatchKey, hipGraphExec_t> graphs;
  std::vector<std::shared_ptr<Request>> reqs;
  bool busy = false;
};

class Server {
 public:
  explicit Server(rerank_ctx* ctx) : ctx_(ctx), pool_(ctx->budget, &ctx->reserved) {}

  rerank_status start() {
    hipError_t e = hipSetDevice(ctx_->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    for (auto& s : slots_) {
      if ((e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreate");
      if ((e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "hipEventCreate");
      if ((e = hipHostMalloc((void**)&s.h_tab, sizeof(BatchTable), hipHostMallocDefault)) != hipSuccess)
        return hip_fail(e, "hipHostMalloc");
      if ((e = hipMalloc((void**)&s.d_tab, sizeof(BatchTable))) != hipSuccess) return hip_fail(e, "hipMalloc");
      std::memset(s.h_tab, 0, sizeof(BatchTable));
    }
    thread_ = std::thread([this] { loop(); });
    return RERANK_OK;
  }

  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stopping_ = true;
    }
    cv_work_.notify_all();
    if (thread_.joinable()) thread_.join();
    hipSetDevice(ctx_->device);
    for (auto& s : slots_) {
      if (s.stream) hipStreamSynchronize(s.stream);
      for (auto& g : s.graphs) hipGraphExecDestroy(g.second);
      if (s.done) hipEventDestroy(s.done);
      if (s.stream) hipStreamDestroy(s.stream);
      if (s.h_tab) hipHostFree(s.h_tab);
      if (s.d_tab) hipFree(s.d_tab);
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (auto& s : slots_)
        for (auto& r : s.reqs) pool_.release(r->ws);
      pool_.release_cache();
      for (hipEvent_t ev : events_) hipEventDestroy(ev);
      events_.clear();
    }
  }

  void release_cache() {
    std::lock_guard<std::mutex> lk(mu_);
    pool_.release_cache();
  }

  rerank_status submit(const rerank_params* p, const void* x, int in_bf16, float* dist, hipStream_t stream,
                       uint64_t* ticket) {
    auto r = std::make_shared<Request>();
    r->params = *p;
    make_plan(p, false, &r->plan, (ctx_->flags & RERANK_CTX_DENSE_LAYERS) != 0);
    if (r->plan.total > ctx_->budget) {
      set_error("request working set exceeds the context budget");
      return RERANK_E_NOMEM;
    }
    r->x = x;
    r->in_bf16 = in_bf16;
    r->dist = dist;
    r->ws_bytes = r->plan.total;
    r->small = p->n <= kGroupedMaxN && r->plan.rescore && r->plan.fprec == FinalPrec::F32;
    r->key = BatchKey{(int)r->plan.prec, r->plan.kc <= 64 ? 1 : (r->plan.kc <= 128 ? 2 : 4), p->layers, p->node,
                      p->aggregator};
    // the request's kernels wait for what the caller enqueued on `stream` so far
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (!events_.empty()) {
        r->ready = events_.back();
        events_.pop_back();
      }
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(ctx_->device);
    if (e == hipSuccess && !r->ready) e = hipEventCreateWithFlags(&r->ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(r->ready, stream);
    if (prev >= 0 && prev != ctx_->device) (void)hipSetDevice(prev);
    if (e != hipSuccess) {
      std::lock_guard<std::mutex> lk(mu_);
      if (r->ready) events_.push_back(r->ready);
      return hip_fail(e, "recording the request's ready event on hip_stream");
    }
    r->t_submit = Clock::now();
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (stopping_) {
        events_.push_back(r->ready);
        set_error("context is being destroyed");
        return RERANK_E_INVALID;
      }
      r->ticket = next_ticket_++;
      tickets_[r->ticket] = r;
      pending_.push_back(r);
    }
    cv_work_.notify_all();
    *ticket = r->ticket;
    return RERANK_OK;
  }

  rerank_status poll(uint64_t t, int* done) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = tickets_.find(t);
    if (it == tickets_.end()) {
      set_error("unknown ticket");
      return RERANK_E_INVALID;
    }
    *done = it->second->state == Request::DONE;
    return RERANK_OK;
  }

  rerank_status wait(uint64_t t, int64_t timeout_us, double* latency_ms) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = tickets_.find(t);
    if (it == tickets_.end()) {
      set_error("unknown ticket");
      return RERANK_E_INVALID;
    }
    std::shared_ptr<Request> r = it->second;
    auto pred = [&] { return r->state == Request::DONE; };
    if (timeout_us < 0)
      cv_done_.wait(lk, pred);
    else if (!cv_done_.wait_for(lk, std::chrono::microseconds(timeout_us), pred))
      return RERANK_E_TIMEOUT;
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    tickets_.erase(t);
    if (r->status != RERANK_OK) set_error(r->error);
    return r->status;
  }

  rerank_status cancel(uint64_t t) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = tickets_.find(t);
    if (it == tickets_.end()) {
      set_error("unknown ticket");
      return RERANK_E_INVALID;
    }
    auto r = it->second;
    if (r->state == Request::RUNNING) return RERANK_E_BUSY;
    if (r->state == Request::PENDING) {
      for (auto q = pending_.begin(); q != pending_.end(); ++q)
        if (*q == r) {
          pending_.erase(q);
          break;
        }
      finish(r, RERANK_E_CANCELLED, "cancelled before it started");
      cv_done_.notify_all();
    }
    return RERANK_OK;
  }

 private:
  void finish(const std::shared_ptr<Request>& r, rerank_status st, const std::string& err) {
    if (r->ready) {
      events_.push_back(r->ready);
      r->ready = nullptr;
    }
    r->status = st;
    r->error = err;
    r->state = Request::DONE;
    r->t_done = Clock::now();
  }

  // Build (or reuse) the slot's graph for `key`: table copy + grouped pipeline.
  hipError_t graph_for(Slot& s, const BatchKey& key, hipGraphExec_t* out) {
    auto it = s.graphs.find(key);
    if (it != s.graphs.end()) {
      *out = it->second;
      return hipSuccess;
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t e1 = hipMemcpyAsync(s.d_tab, s.h_tab, sizeof(BatchTable), hipMemcpyHostToDevice, s.stream);
    hipError_t e2 = (e1 == hipSuccess) ? enqueue_grouped(key, s.d_tab, s.stream) : e1;
    e = hipStreamEndCapture(s.stream, &g);
    if (e2 != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return e2;
    }
    if (e != hipSuccess) return e;
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    s.graphs[key] = ex;
    *out = ex;
    return hipSuccess;
  }

  static void fill_desc(const Request& r, ProbDesc& D) {
    const Plan& P = r.plan;
    char* ws = (char*)r.ws;
    D = ProbDesc{};
    D.n = P.n;
    D.q = P.q;
    D.g = P.g;
    D.d = P.d;
    D.k1 = P.k1;
    D.k2 = P.k2;
    D.kc = P.kc;
    D.alpha = P.alpha;
    D.in_bf16 = r.in_bf16;
    D.lbytes = P.lbytes;
    D.node = P.node;
    D.agg = P.agg;
    D.tiles_sim = 0;
    D.tiles_fin_m = (P.q + 127) / 128;
    D.tiles_fin_n = (P.g + 127) / 128;
    D.ldp = P.ldp;
    D.ldl = P.ldl;
    D.ldN = P.ldN;
    D.ldH = P.ldH;
    D.fill_items_a = P.sparse_first ? 0 : ((int64_t)P.n * P.ldN + FILL_ITEM_HOST - 1) / FILL_ITEM_HOST;
    D.x = r.x;
    D.dist = r.dist;
    D.xp = (float*)(ws + P.o_xp);
    D.xl = P.lbytes ? (void*)(ws + P.o_xl) : nullptr;
    D.rn = (float*)(ws + P.o_rn);
    D.sl = (float*)(ws + P.o_sl);
    D.A = (float*)(ws + P.o_a);
    D.B = P.layers > 0 ? (float*)(ws + P.o_b) : nullptr;
    D.ci = (int32_t*)(ws + P.o_ci);
    D.cv = (float*)(ws + P.o_cv);
    D.ki = (int32_t*)(ws + P.o_ki);
    D.kv = (float*)(ws + P.o_kv);
    D.sa = (float*)(ws + P.o_sa);
    D.sb = (float*)(ws + P.o_sb);
    D.cnt = (int32_t*)(ws + P.o_cnt);
    const bool csr = P.sparse_first && P.node == RERANK_NODE_ADJ_SYM;
    D.mflag = csr ? (uint8_t*)(ws + P.o_mflag) : nullptr;
    D.off = csr ? (int32_t*)(ws + P.o_off) : nullptr;
    D.inl = csr ? (int32_t*)(ws + P.o_inl) : nullptr;
  }
  static constexpr int64_t FILL_ITEM_HOST = 256 * 4 * 8;

  void fill_table(Slot& s, const BatchKey& key) {
    BatchTable& T = *s.h_tab;
    T.count = (int)s.reqs.size();
    T.layers = key.layers;
    for (int st = 0; st < GS_COUNT; st++) T.start[st][0] = 0;
    for (int i = 0; i < T.count; i++) {
      ProbDesc& D = T.p[i];
      fill_desc(*s.reqs[i], D);
      const int64_t n = D.n, T1 = (n + 127) / 128;
      int64_t items[GS_COUNT];
      items[GS_PREP] = (n + 3) / 4;
      items[GS_SIM] = T1 * (T1 + 1) / 2;
      items[GS_TOPK] = (n + 3) / 4;
      items[GS_RESCORE] = (n + 3) / 4;
      items[GS_FILL] = D.fill_items_a + (2 * n + FILL_ITEM_HOST - 1) / FILL_ITEM_HOST;
      items[GS_SCATTER] = (n * D.k1 + 255) / 256;
      items[GS_SIGMA] = (n + 255) / 256;
      items[GS_PROP] = n;
      items[GS_FINAL] = (int64_t)D.tiles_fin_m * D.tiles_fin_n;
      items[GS_MUTUAL] = (n * D.k1 + 255) / 256;
      items[GS_SCAN] = 1;
      items[GS_CSR] = (n * D.k1 + 255) / 256;
      for (int st = 0; st < GS_COUNT; st++) T.start[st][i + 1] = T.start[st][i] + (int32_t)items[st];
    }
  }

  // Launch the requests of slot s (all admitted). Returns false on failure,
  // after failing its requests.
  void launch(Slot& s) {
    hipError_t e = hipSuccess;
    const char* where = "hipStreamWaitEvent";
    for (auto& r : s.reqs)
      if (e == hipSuccess) e = hipStreamWaitEvent(s.stream, r->ready, 0);
    if (e == hipSuccess && s.reqs.size() == 1 && !s.reqs[0]->small) {
      Request& r = *s.reqs[0];
      where = "launch";
      e = enqueue_rerank(r.plan, r.ws, r.x, r.in_bf16, r.dist, s.stream, &where, nullptr);
    } else if (e == hipSuccess) {
      const BatchKey key = s.reqs[0]->key;
      fill_table(s, key);
      hipGraphExec_t ex = nullptr;
      e = graph_for(s, key, &ex);
      where = "graph capture";
      if (e == hipSuccess) {
        e = hipGraphLaunch(ex, s.stream);
        where = "hipGraphLaunch";
      }
    }
    if (e == hipSuccess) {
      e = hipEventRecord(s.done, s.stream);
      where = "hipEventRecord";
    }
    if (e != hipSuccess) {
      const std::string msg = std::string(where) + ": " + hipGetErrorString(e);
      // work enqueued before the failure may still run on the slot's stream:
      // let it drain before the working sets can go to other requests
      (void)hipStreamSynchronize(s.stream);
      (void)hipGetLastError();
      for (auto& r : s.reqs) {
        pool_.release(r->ws);
        r->ws = nullptr;
        finish(r, RERANK_E_HIP, msg);
      }
      s.reqs.clear();
      cv_done_.notify_all();
      return;
    }
    for (auto& r : s.reqs) r->state = Request::RUNNING;
    s.busy = true;
  }

  bool any_busy() const {
    for (auto& s : slots_)
      if (s.busy) return true;
    return false;
  }

  // The direct calls' working set is kept for their next call. When the head
  // request does not fit next to it and no serving request holds memory, give
  // it back (once its kernels have finished; a direct call in progress keeps
  // it and is waited for). Called with mu_ held; only tries the context lock.
  bool reclaim_direct_ws() {
    std::unique_lock<std::mutex> lk(ctx_->mu, std::try_to_lock);
    if (!lk.owns_lock() || !ctx_->ws) return false;
    if (hipEventQuery(ctx_->ws_free) != hipSuccess) return false;
    if (hipFree(ctx_->ws) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    ctx_->reserved -= ctx_->ws_bytes;
    ctx_->ws = nullptr;
    ctx_->ws_bytes = 0;
    return true;
  }

  // Admit pending requests into idle slots (called with mu_ held).
  void dispatch() {
    while (!pending_.empty()) {
      Slot* s = nullptr;
      for (auto& sl : slots_)
        if (!sl.busy) {
          s = &sl;
          break;
        }
      if (!s) return;
      auto head = pending_.front();
      bool fatal = false;
      void* ws = pool_.alloc(head->ws_bytes, &fatal);
      if (!ws) {
        if (!fatal) {
          // the pool has already dropped its cached blocks; with no request
          // running, only the direct calls' working set can be in the way
          if (!any_busy() && reclaim_direct_ws()) continue;
          return;  // wait for memory to free up (arrival order is kept)
        }
        pending_.pop_front();
        finish(head, RERANK_E_NOMEM, "device allocation of the working set failed");
        cv_done_.notify_all();
        continue;
      }
      pending_.pop_front();
      head->ws = ws;
      s->reqs.assign(1, head);
      if (head->small) {
        // gather later small requests with the same key, in arrival order
        for (auto q = pending_.begin(); q != pending_.end() && (int)s->reqs.size() < kMaxBatch;) {
          if (!(*q)->small || (*q)->key < head->key || head->key < (*q)->key) {
            ++q;
            continue;
          }
          bool f2 = false;
          void* w2 = pool_.alloc((*q)->ws_bytes, &f2);
          if (!w2) {
            if (f2) {
              finish(*q, RERANK_E_NOMEM, "device allocation of the working set failed");
              q = pending_.erase(q);
              cv_done_.notify_all();
              continue;
            }
            break;
          }
          (*q)->ws = w2;
          s->reqs.push_back(*q);
          q = pending_.erase(q);
        }
      }
      launch(*s);
    }
  }

  void complete_finished() {
    for (auto& s : slots_) {
      if (!s.busy) continue;
      hipError_t q = hipEventQuery(s.done);
      if (q == hipErrorNotReady) continue;
      const rerank_status st = (q == hipSuccess) ? RERANK_OK : RERANK_E_HIP;
      const std::string msg = (q == hipSuccess) ? "" : std::string("request failed: ") + hipGetErrorString(q);
      for (auto& r : s.reqs) {
        pool_.release(r->ws);
        r->ws = nullptr;
        finish(r, st, msg);
      }
      s.reqs.clear();
      s.busy = false;
      cv_done_.notify_all();
    }
  }

  void loop() {
    hipSetDevice(ctx_->device);
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
      complete_finished();
      if (stopping_) {
        bool any = false;
        for (auto& s : slots_) any |= s.busy;
        if (!any) break;
      } else {
        dispatch();
      }
      if (any_busy()) {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      } else if (!stopping_) {
        if (pending_.empty())
          cv_work_.wait(lk, [&] { return stopping_ || !pending_.empty(); });
        else  // the head waits for memory a direct call still uses: retry shortly
          cv_work_.wait_for(lk, std::chrono::microseconds(200));
      }
    }
    // fail whatever is still pending at shutdown
    for (auto& r : pending_) finish(r, RERANK_E_CANCELLED, "context destroyed");
    pending_.clear();
    cv_done_.notify_all();
  }

  rerank_ctx* ctx_;
  Pool pool_;
  Slot slots_[kSlots];
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<std::shared_ptr<Request>> pending_;
  std::vector<hipEvent_t> events_;  // ready events of finished requests, for reuse
  std::map<uint64_t, std::shared_ptr<Request>> tickets_;
  uint64_t next_ticket_ = 1;
  bool stopping_ = false;
  std::thread thread_;
};

void server_stop(Server* s) {
  if (!s) return;
  s->stop();
  delete s;
}

// The context's server if one was started (read under the lock that creates it).
static Server* server_of(rerank_ctx* ctx) {
  std::lock_guard<std::mutex> lk(ctx->server_mu);
  return ctx->server;
}

void server_release_cache(rerank_ctx* ctx) {
  if (Server* s = server_of(ctx)) s->release_cache();
}

static rerank_status get_server(rerank_ctx* ctx, Server** out) {
  std::lock_guard<std::mutex> lk(ctx->server_mu);
  if (!ctx->server) {
    Server* s = new Server(ctx);
    rerank_status st = s->start();
    if (st != RERANK_OK) {
      s->stop();
      delete s;
      return st;
    }
    ctx->server = s;
  }
  *out = ctx->server;
  return RERANK_OK;
}

}  // namespace rr

using namespace rr;

extern "C" {

rerank_status rerank_submit(rerank_ctx* ctx, const rerank_params* p, const void* d_x, int32_t in_dtype, float* d_dist,
                            void* hip_stream, uint64_t* ticket) {
  if (!ctx || !ticket) {
    set_error("ctx or ticket is NULL");
    return RERANK_E_INVALID;
  }
  std::string why;
  rerank_status st = validate_params(p, &why);
  if (st != RERANK_OK) {
    set_error(why);
    return st;
  }
  if (in_dtype != RERANK_IN_F32 && in_dtype != RERANK_IN_BF16) {
    set_error("unknown in_dtype");
    return RERANK_E_INVALID;
  }
  if (!d_x || !d_dist || ((uintptr_t)d_dist & 3) || ((uintptr_t)d_x & (in_dtype == RERANK_IN_F32 ? 3 : 1))) {
    set_error("d_x / d_dist NULL or misaligned");
    return RERANK_E_INVALID;
  }
  Server* s = nullptr;
  st = get_server(ctx, &s);
  if (st != RERANK_OK) return st;
  return s->submit(p, d_x, in_dtype == RERANK_IN_BF16, d_dist, (hipStream_t)hip_stream, ticket);
}

rerank_status rerank_poll(rerank_ctx* ctx, uint64_t ticket, int* done) {
  Server* srv = ctx ? server_of(ctx) : nullptr;
  if (!done || !srv) {
    set_error("ctx/done NULL or nothing submitted");
    return RERANK_E_INVALID;
  }
  return srv->poll(ticket, done);
}

rerank_status rerank_wait(rerank_ctx* ctx, uint64_t ticket, int64_t timeout_us, double* latency_ms) {
  Server* srv = ctx ? server_of(ctx) : nullptr;
  if (!srv) {
    set_error("ctx NULL or nothing submitted");
    return RERANK_E_INVALID;
  }
  return srv->wait(ticket, timeout_us, latency_ms);
}

rerank_status rerank_cancel(rerank_ctx* ctx, uint64_t ticket) {
  Server* srv = ctx ? server_of(ctx) : nullptr;
  if (!srv) {
    set_error("ctx NULL or nothing submitted");
    return RERANK_E_INVALID;
  }
  return srv->cancel(ticket);
}

}  // extern "C"
