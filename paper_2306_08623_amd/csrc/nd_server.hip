// nd_server.hip -- request loop with continuous batching on one GPU.
//
// Host runtime around the batch path: `workers` pipelines, each a context
// with a stream of its own, share one FIFO of requests. A pipeline that is
// free takes every admissible request at the head of the FIFO (up to
// max_batch) and decomposes them as one batch; requests arriving meanwhile
// wait for the next free pipeline, so batches form continuously from what
// has arrived. The pipelines run on the device at the same time: each
// one's persistent (grid-barrier) kernels take 1/workers of the device, so
// that all of them fit at once, and the ordinary kernels of one pipeline
// fill whatever the others leave free. The device intervals of every batch
// are taken from HIP events, so the overlap is measured, not assumed.
// Admission uses the footprint estimate of nd_estimate_footprint:
// a pipeline's batch stays within its workspace share, and the results held
// on the device (until the client releases them) stay within the result
// share. Results live in stream-ordered device allocations, so releasing
// them never waits for the other pipelines.
#include "nd_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

namespace {

constexpr uint64_t kBatchConstBytes = 4ull << 20;   // per-batch fixed workspace
constexpr size_t kMaxIntervals = 1u << 16;          // batch device intervals kept

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  uint32_t n = 0, r = 0, s = 0;
  uint64_t nnz = 0;
  std::vector<uint64_t> rp;
  std::vector<uint32_t> col;
  uint64_t ws = 0, res_est = 0;
  nd_request_info info{};
  bool running = false, cancelled = false;
  // device results (one allocation)
  void *dres = nullptr;
  uint64_t dres_bytes = 0;
  uint32_t *d_rcl = nullptr, *d_cnt = nullptr, *d_core = nullptr, *d_level = nullptr;
  uint64_t *d_parent = nullptr;
};


// workspace / result bytes of one graph (see nucleus.h); host CSR
void estimate(uint32_t n, uint64_t nnz, const uint64_t *rp, const uint32_t *col, uint32_t r,
              uint32_t s, uint64_t *ws, uint64_t *res) {
  const uint64_t m = nnz / 2;
  uint64_t tri = 0;
  if (s >= 3) {
    uint64_t sum = 0;   // sum over edges of min(deg) - 1, each triangle counted 3 times
    for (uint32_t u = 0; u < n; u++) {
      const uint64_t du = rp[u + 1] - rp[u];
      for (uint64_t x = rp[u]; x < rp[u + 1]; x++) {
        const uint32_t v = col[x];
        if (v <= u || v >= n) continue;
        const uint64_t dv = rp[v + 1] - rp[v];
        const uint64_t mn = du < dv ? du : dv;
        if (mn > 1) sum += mn - 1;
      }
    }
    tri = sum / 3;
  }
  if (s >= 5) {
    // s = 5..7 keep their s-cliques: k-cliques are bounded by
    // sum_v C(deg v, k - 1) / k (each k-clique is k vertices with k - 1
    // common neighbours); the tables hold every level up to s, the sorted
    // r- and s-tuples, the r-clique table and its sort, and 8 C(s,r) bytes
    // per s-clique
    const double cap = 4.0e18;
    double nk[8] = {0, (double)n, (double)m, 0, 0, 0, 0, 0};
    for (uint32_t k = 3; k <= s; k++) {
      double t = 0;
      for (uint32_t v = 0; v < n; v++) {
        const double d = (double)(rp[v + 1] - rp[v]);
        double b = 1;   // C(d, k - 1)
        for (uint32_t i = 0; i < k - 1; i++) b = b * (d - i) / (i + 1);
        if (b > 0) t += b;
      }
      nk[k] = t / k < cap ? t / k : cap;
    }
    double C = 1;
    for (uint32_t i = 0; i < r; i++) C = C * (s - i) / (i + 1);
    double w = 56.0 * (n + 1) + 32.0 * m + (153.0 + 8.0 * r) * nk[r] + 64;
    for (uint32_t k = 2; k <= s; k++) w += (4.0 * k + 12.0) * nk[k];
    w += (8.0 * r + 24.0) * nk[r] + 4.0 * s * nk[s] + 8.0 * C * nk[s] + 8.0 * nk[r];
    const double res_b = nk[r] * (4.0 * r + 28.0) + 256;
    if (ws) *ws = w < cap ? (uint64_t)w : (uint64_t)cap;
    if (res) *res = res_b < cap ? (uint64_t)res_b : (uint64_t)cap;
    return;
  }
  const uint64_t n_r = r == 1 ? n : (r == 2 ? m : tri);
  uint64_t w = 56ull * (n + 1) + 32ull * m + (153ull + 8ull * r) * n_r + 64;
  if (s >= 3) w += 24ull * (m + 1) + 36ull * tri;
  if (r == 2 && s == 4) w += 48ull * tri;   // probe parts, lengths, running sums
  if (r == 3 && s == 4) w += 32ull * tri;   // the peel's per-frontier-slot list ranges
  if (r == 2 && s == 3) w += 32ull * m;     // the same for (2,3)
  if (r == 1 && s >= 3) w += 24ull * (m + 1);   // per-slot triangle counts and sums
  if (r == 1 && s == 4) w += 48ull * tri;       // per-triangle-probe parts and sums
  if (ws) *ws = w;
  if (res) *res = n_r * (4ull * r + 28ull) + 256;
}

}  // namespace

struct nd_server {
  int device = 0;
  uint32_t workers = 2, max_batch = 512;
  int validate = 1;
  uint64_t ws_share = 0, res_share = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::unordered_map<uint64_t, Request *> reqs;
  uint64_t next_ticket = 1;
  uint64_t res_in_use = 0;   // results held + reserved by admitted requests
  uint32_t busy = 0;         // pipelines running a batch
  bool stop = false;
  std::vector<std::thread> threads;
  std::vector<nd_ctx *> ctxs;
  std::vector<hipStream_t> streams;
  hipStream_t io = nullptr;  // copies out and frees
  // device time of every batch: events recorded on the pipeline's stream
  // around its device work, read against one reference event
  hipEvent_t ev_ref = nullptr;
  std::vector<hipEvent_t> ev_begin, ev_end;
  std::vector<std::pair<float, float>> intervals;   // ms after ev_ref, last kMaxIntervals
  Clock::time_point t0;
  nd_server_stats stats{};
  std::string last_error;
  std::mutex io_mu;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }
};

namespace {

nd_status srv_fail(nd_server *S, nd_status st, const std::string &msg) {
  std::lock_guard<std::mutex> lk(S->mu);
  S->last_error = msg;
  return st;
}

// Decompose one batch on pipeline w; fills every request's info and results.
// The host half (checks, union packing) runs outside the device lock, so one
// pipeline prepares its batch while another's runs on the device.
void run_batch(nd_server *S, uint32_t w, std::vector<Request *> &batch) {
  nd_ctx *c = S->ctxs[w];
  const uint32_t G = (uint32_t)batch.size();
  std::vector<nd_graph_desc> descs(G);
  std::vector<nd_graph_result> results(G);
  for (uint32_t i = 0; i < G; i++) {
    Request *q = batch[i];
    descs[i] = nd_graph_desc{q->n, q->r, q->s, q->nnz, q->rp.data(),
                             q->col.empty() ? nullptr : q->col.data()};
  }
  BatchState *plan = nullptr;
  std::string err;
  nd_status st = nd_batch_plan(G, descs.data(), ND_MEM_HOST, results.data(), &plan, &err);
  const bool timed = S->ev_begin[w] && S->ev_end[w];
  if (timed) (void)hipEventRecord(S->ev_begin[w], c->stream);
  if (st == ND_OK) {
    st = nd_batch_execute(c, plan, descs.data(), results.data());
    err = c->last_error;
  }
  if (st != ND_OK && G > 1) {
    // one member's error (a bad graph, or an estimate too small for the
    // union) fails the whole union: run the members one by one so that only
    // the faulty one fails
    for (uint32_t i = 0; i < G; i++) {
      std::vector<Request *> one{batch[i]};
      run_batch(S, w, one);
    }
    return;
  }
  if (st != ND_OK) {
    for (Request *q : batch) q->info.status = st;
    std::lock_guard<std::mutex> lk(S->mu);
    S->last_error = err;
    return;
  }
  for (uint32_t i = 0; i < G; i++) {
    Request *q = batch[i];
    const nd_graph_result &R = results[i];
    q->info.k = R.k;
    q->info.n_r = R.n_r;
    q->info.n_s = R.n_s;
    q->info.n_int = R.n_int;
    const uint64_t b_rcl = R.n_r * q->r * 4, b_cnt = R.n_r * 4, b_par = (R.n_r + R.n_int) * 8,
                   b_lev = R.n_int * 4;
    auto al = [](uint64_t x) { return (x + 255) & ~255ull; };
    const uint64_t bytes = al(b_rcl) + 2 * al(b_cnt) + al(b_par) + al(b_lev) + 256;
    void *p = nullptr;
    if (hipMallocAsync(&p, bytes, c->stream) != hipSuccess) {
      (void)hipGetLastError();
      q->info.status = ND_E_OOM;
      continue;
    }
    char *b = (char *)p;
    q->dres = p;
    q->dres_bytes = bytes;
    q->d_rcl = (uint32_t *)b;
    b += al(b_rcl);
    q->d_cnt = (uint32_t *)b;
    b += al(b_cnt);
    q->d_core = (uint32_t *)b;
    b += al(b_cnt);
    q->d_parent = (uint64_t *)b;
    b += al(b_par);
    q->d_level = (uint32_t *)b;
    q->info.status = nd_batch_get(c, i, q->d_rcl, q->d_cnt, q->d_core, q->d_parent, q->d_level,
                                  ND_MEM_DEVICE);
    q->info.result_bytes = bytes;
  }
  if (timed) {
    float a = 0, b = 0;
    if (hipEventRecord(S->ev_end[w], c->stream) == hipSuccess &&
        hipEventSynchronize(S->ev_end[w]) == hipSuccess &&
        hipEventElapsedTime(&a, S->ev_ref, S->ev_begin[w]) == hipSuccess &&
        hipEventElapsedTime(&b, S->ev_ref, S->ev_end[w]) == hipSuccess) {
      std::lock_guard<std::mutex> lk(S->mu);
      if (S->intervals.size() >= kMaxIntervals) S->intervals.erase(S->intervals.begin());
      S->intervals.emplace_back(a, b);
    } else {
      (void)hipGetLastError();
    }
  }
}

// Device time covered by at least one batch, by at least two, and in total
// (ms), from the recorded intervals.
void device_overlap(const std::vector<std::pair<float, float>> &iv, double *any, double *two,
                    double *sum) {
  std::vector<std::pair<double, int>> ev;
  *sum = 0;
  for (const auto &x : iv) {
    if (x.second <= x.first) continue;
    ev.emplace_back(x.first, +1);
    ev.emplace_back(x.second, -1);
    *sum += x.second - x.first;
  }
  std::sort(ev.begin(), ev.end());
  *any = *two = 0;
  int depth = 0;
  double last = 0;
  for (const auto &e : ev) {
    if (depth >= 1) *any += e.first - last;
    if (depth >= 2) *two += e.first - last;
    depth += e.second;
    last = e.first;
  }
}

void worker_loop(nd_server *S, uint32_t w) {
  (void)hipSetDevice(S->device);
  for (;;) {
    std::vector<Request *> batch;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] {
        return S->stop || (!S->queue.empty() &&
                           S->res_in_use + S->queue.front()->res_est <= S->res_share);
      });
      if (S->stop) return;
      uint64_t ws_sum = kBatchConstBytes;
      while (!S->queue.empty() && batch.size() < S->max_batch) {
        Request *q = S->queue.front();
        if (ws_sum + q->ws > S->ws_share) break;
        if (S->res_in_use + q->res_est > S->res_share) break;
        S->queue.pop_front();
        q->running = true;
        ws_sum += q->ws;
        S->res_in_use += q->res_est;
        batch.push_back(q);
      }
      if (batch.empty()) continue;
      const double t = S->now_ms();
      if (S->busy > 0) S->stats.overlapped += batch.size();
      S->busy++;
      S->stats.batches++;
      S->stats.max_batch_seen = std::max<uint64_t>(S->stats.max_batch_seen, batch.size());
      S->stats.waiting -= batch.size();
      S->stats.running += batch.size();
      for (Request *q : batch) {
        q->info.t_start_ms = t;
        q->info.batch_size = (uint32_t)batch.size();
        q->info.worker = w;
      }
    }
    run_batch(S, w, batch);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      const double t = S->now_ms();
      S->busy--;
      for (Request *q : batch) {
        q->running = false;
        q->rp.clear();
        q->rp.shrink_to_fit();
        q->col.clear();
        q->col.shrink_to_fit();
        S->res_in_use -= q->res_est;
        if (q->cancelled && q->info.status == ND_OK) q->info.status = ND_E_CANCELLED;
        if (q->info.status == ND_OK) {
          S->res_in_use += q->dres_bytes;
          S->stats.result_bytes += q->dres_bytes;
          S->stats.completed++;
        } else {
          if (q->dres) (void)hipFreeAsync(q->dres, S->ctxs[w]->stream);
          q->dres = nullptr;
          q->dres_bytes = 0;
          if (q->info.status == ND_E_CANCELLED) S->stats.cancelled++;
          else S->stats.failed++;
        }
        q->info.t_done_ms = t;
        q->info.done = 1;
        S->stats.running--;
      }
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

Request *find(nd_server *S, uint64_t ticket) {
  auto it = S->reqs.find(ticket);
  return it == S->reqs.end() ? nullptr : it->second;
}

}  // namespace

extern "C" {

nd_status nd_estimate_footprint(const nd_graph_desc *g, nd_mem where, uint64_t *workspace,
                                uint64_t *result) {
  if (!g || !g->row_ptr || (g->nnz && !g->col) || g->r < 1 || g->s <= g->r)
    return ND_E_INVALID_ARG;
  if (where == ND_MEM_HOST) {
    estimate(g->n, g->nnz, g->row_ptr, g->col, g->r, g->s, workspace, result);
    return ND_OK;
  }
  if (where != ND_MEM_DEVICE) return ND_E_INVALID_ARG;
  std::vector<uint64_t> rp(g->n + 1ull);
  std::vector<uint32_t> col(std::max<uint64_t>(g->nnz, 1));
  if (hipMemcpy(rp.data(), g->row_ptr, rp.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      (g->nnz &&
       hipMemcpy(col.data(), g->col, g->nnz * 4, hipMemcpyDeviceToHost) != hipSuccess)) {
    (void)hipGetLastError();
    return ND_E_DEVICE;
  }
  estimate(g->n, g->nnz, rp.data(), col.data(), g->r, g->s, workspace, result);
  return ND_OK;
}

nd_status nd_server_create(nd_server **out, const nd_server_options *opt) {
  if (!out) return ND_E_INVALID_ARG;
  *out = nullptr;
  nd_server *S = new (std::nothrow) nd_server();
  if (!S) return ND_E_OOM;
  uint64_t budget = 0;
  if (opt) {
    S->device = opt->device;
    if (opt->workers) S->workers = opt->workers;
    if (opt->max_batch) S->max_batch = opt->max_batch;
    budget = opt->mem_budget;
    S->validate = opt->validate;
  }
  if (S->workers > 16) S->workers = 16;
  if (hipSetDevice(S->device) != hipSuccess) {
    (void)hipGetLastError();
    delete S;
    return ND_E_DEVICE;
  }
  int pools = 0;
  if (hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, S->device) !=
          hipSuccess ||
      !pools) {
    (void)hipGetLastError();
    delete S;
    return ND_E_UNSUPPORTED;
  }
  if (!budget) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      delete S;
      return ND_E_DEVICE;
    }
    budget = fr / 2;
  }
  // three quarters for the pipelines' workspaces, one quarter for results
  S->ws_share = budget / 4 * 3 / S->workers;
  S->res_share = budget / 4;
  S->stats.workspace_share = S->ws_share;
  S->stats.result_share = S->res_share;
  S->t0 = Clock::now();
  if (hipStreamCreateWithFlags(&S->io, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    delete S;
    return ND_E_DEVICE;
  }
  S->ev_begin.assign(S->workers, nullptr);
  S->ev_end.assign(S->workers, nullptr);
  if (hipEventCreate(&S->ev_ref) != hipSuccess || hipEventRecord(S->ev_ref, S->io) != hipSuccess ||
      hipEventSynchronize(S->ev_ref) != hipSuccess) {
    (void)hipGetLastError();
    nd_server_destroy(S);
    return ND_E_DEVICE;
  }
  for (uint32_t w = 0; w < S->workers; w++)
    if (hipEventCreate(&S->ev_begin[w]) != hipSuccess ||
        hipEventCreate(&S->ev_end[w]) != hipSuccess) {
      (void)hipGetLastError();
      nd_server_destroy(S);
      return ND_E_DEVICE;
    }
  for (uint32_t w = 0; w < S->workers; w++) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      nd_server_destroy(S);
      return ND_E_DEVICE;
    }
    S->streams.push_back(st);
    nd_options o{};
    o.device = S->device;
    o.hip_stream = st;
    o.validate = S->validate;
    o.mem_limit = 0;   // admission bounds the work; see the header
    nd_ctx *c = nullptr;
    nd_status rc = nd_create(&c, &o);
    if (rc != ND_OK) {
      nd_server_destroy(S);
      return rc;
    }
    c->grid_div = S->workers;   // every pipeline's persistent grids fit at once
    S->ctxs.push_back(c);
  }
  for (uint32_t w = 0; w < S->workers; w++) S->threads.emplace_back(worker_loop, S, w);
  *out = S;
  return ND_OK;
}

void nd_server_destroy(nd_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto &t : S->threads) t.join();
  (void)hipSetDevice(S->device);
  for (auto &kv : S->reqs) {
    if (kv.second->dres) (void)hipFreeAsync(kv.second->dres, S->io);
    delete kv.second;
  }
  if (S->io) (void)hipStreamSynchronize(S->io);
  for (nd_ctx *c : S->ctxs) nd_destroy(c);
  for (hipEvent_t e : S->ev_begin)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : S->ev_end)
    if (e) (void)hipEventDestroy(e);
  if (S->ev_ref) (void)hipEventDestroy(S->ev_ref);
  for (hipStream_t st : S->streams) (void)hipStreamDestroy(st);
  if (S->io) (void)hipStreamDestroy(S->io);
  delete S;
}

nd_status nd_server_submit(nd_server *S, const nd_graph_desc *d, nd_mem where,
                           uint64_t *ticket) {
  if (!S || !d || !ticket) return ND_E_INVALID_ARG;
  if (d->r < 1 || d->s <= d->r) return srv_fail(S, ND_E_INVALID_ARG, "need 1 <= r < s");
  if (!nd_rs_supported(d->r, d->s)) return srv_fail(S, ND_E_UNSUPPORTED, "this (r,s) pair is not built");
  if (!d->row_ptr || (d->nnz && !d->col)) return srv_fail(S, ND_E_INVALID_ARG, "NULL CSR");
  if (where != ND_MEM_HOST && where != ND_MEM_DEVICE)
    return srv_fail(S, ND_E_INVALID_ARG, "bad memory kind");
  if (d->nnz & 1) return srv_fail(S, ND_E_BAD_GRAPH, "nnz is odd");
  if (d->n == 0xFFFFFFFFu) return srv_fail(S, ND_E_UNSUPPORTED, "n must be below 2^32-1");
  Request *q = new (std::nothrow) Request();
  if (!q) return ND_E_OOM;
  q->n = d->n;
  q->r = d->r;
  q->s = d->s;
  q->nnz = d->nnz;
  q->rp.resize(d->n + 1ull);
  q->col.resize(d->nnz);
  if (where == ND_MEM_HOST) {
    memcpy(q->rp.data(), d->row_ptr, q->rp.size() * 8);
    if (d->nnz) memcpy(q->col.data(), d->col, d->nnz * 4);
  } else {
    std::lock_guard<std::mutex> lk(S->io_mu);
    (void)hipSetDevice(S->device);
    if (hipMemcpyAsync(q->rp.data(), d->row_ptr, q->rp.size() * 8, hipMemcpyDeviceToHost,
                       S->io) != hipSuccess ||
        (d->nnz && hipMemcpyAsync(q->col.data(), d->col, d->nnz * 4, hipMemcpyDeviceToHost,
                                  S->io) != hipSuccess) ||
        hipStreamSynchronize(S->io) != hipSuccess) {
      (void)hipGetLastError();
      delete q;
      return srv_fail(S, ND_E_DEVICE, "copy of a device request failed");
    }
  }
  if (q->rp[0] != 0 || q->rp[d->n] != d->nnz) {
    delete q;
    return srv_fail(S, ND_E_BAD_GRAPH, "row_ptr[0] must be 0 and row_ptr[n] must be nnz");
  }
  for (uint32_t u = 0; u < d->n; u++)
    if (q->rp[u + 1] < q->rp[u]) {
      delete q;
      return srv_fail(S, ND_E_BAD_GRAPH, "row_ptr decreases");
    }
  estimate(q->n, q->nnz, q->rp.data(), q->col.data(), q->r, q->s, &q->ws, &q->res_est);
  q->info.workspace = q->ws;
  if (q->ws + kBatchConstBytes > S->ws_share || q->res_est > S->res_share) {
    const std::string msg = "request needs about " + std::to_string(q->ws) +
                            " workspace bytes and " + std::to_string(q->res_est) +
                            " result bytes; the server's shares are " +
                            std::to_string(S->ws_share) + " and " +
                            std::to_string(S->res_share);
    delete q;
    return srv_fail(S, ND_E_OOM, msg);
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
      delete q;
      return ND_E_STATE;
    }
    q->ticket = S->next_ticket++;
    q->info.status = ND_OK;
    q->info.t_submit_ms = S->now_ms();
    S->reqs[q->ticket] = q;
    S->queue.push_back(q);
    S->stats.submitted++;
    S->stats.waiting++;
    *ticket = q->ticket;
  }
  S->cv_work.notify_one();
  return ND_OK;
}

nd_status nd_server_poll(nd_server *S, uint64_t ticket, nd_request_info *info) {
  if (!S || !info) return ND_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  Request *q = find(S, ticket);
  if (!q) return ND_E_INVALID_ARG;
  *info = q->info;
  return ND_OK;
}

nd_status nd_server_wait(nd_server *S, uint64_t ticket, double timeout_ms,
                         nd_request_info *info) {
  if (!S) return ND_E_INVALID_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  Request *q = find(S, ticket);
  if (!q) return ND_E_INVALID_ARG;
  auto done = [&] { return q->info.done != 0; };
  if (timeout_ms < 0) {
    S->cv_done.wait(lk, done);
  } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms),
                                  done)) {
    if (info) *info = q->info;
    return ND_E_STATE;
  }
  if (info) *info = q->info;
  return ND_OK;
}

nd_status nd_server_get(nd_server *S, uint64_t ticket, uint32_t *rcliques, uint32_t *counts,
                        uint32_t *coreness, uint64_t *parent, uint32_t *level, nd_mem where) {
  if (!S) return ND_E_INVALID_ARG;
  if (where != ND_MEM_HOST && where != ND_MEM_DEVICE) return ND_E_INVALID_ARG;
  Request *q;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    q = find(S, ticket);
    if (!q) return ND_E_INVALID_ARG;
    if (!q->info.done || q->info.status != ND_OK || !q->dres) {
      S->last_error = "the request has no results (not done, failed or cancelled)";
      return ND_E_STATE;
    }
  }
  // a finished request is only changed by release, which the caller orders
  const hipMemcpyKind kind = where == ND_MEM_HOST ? hipMemcpyDeviceToHost
                                                  : hipMemcpyDeviceToDevice;
  const uint64_t n_r = q->info.n_r, n_int = q->info.n_int;
  std::lock_guard<std::mutex> lk(S->io_mu);
  (void)hipSetDevice(S->device);
  struct Part {
    void *dst;
    const void *src;
    uint64_t bytes;
  } parts[] = {{rcliques, q->d_rcl, n_r * q->r * 4},
               {counts, q->d_cnt, n_r * 4},
               {coreness, q->d_core, n_r * 4},
               {parent, q->d_parent, (n_r + n_int) * 8},
               {level, q->d_level, n_int * 4}};
  for (const Part &p : parts) {
    if (!p.dst || !p.bytes) continue;
    if (hipMemcpyAsync(p.dst, p.src, p.bytes, kind, S->io) != hipSuccess) {
      (void)hipGetLastError();
      return srv_fail(S, ND_E_DEVICE, "result copy failed");
    }
  }
  if (hipStreamSynchronize(S->io) != hipSuccess) {
    (void)hipGetLastError();
    return srv_fail(S, ND_E_DEVICE, "result copy failed");
  }
  return ND_OK;
}

nd_status nd_server_release(nd_server *S, uint64_t ticket) {
  if (!S) return ND_E_INVALID_ARG;
  Request *q;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    q = find(S, ticket);
    if (!q) return ND_E_INVALID_ARG;
    if (!q->info.done) {
      S->last_error = "release of a request that has not ended";
      return ND_E_STATE;
    }
    S->reqs.erase(ticket);
    if (q->info.status == ND_OK) {
      S->res_in_use -= q->dres_bytes;
      S->stats.result_bytes -= q->dres_bytes;
    }
  }
  if (q->dres) {
    std::lock_guard<std::mutex> lk(S->io_mu);
    (void)hipSetDevice(S->device);
    (void)hipFreeAsync(q->dres, S->io);
  }
  delete q;
  S->cv_work.notify_all();
  return ND_OK;
}

nd_status nd_server_cancel(nd_server *S, uint64_t ticket) {
  if (!S) return ND_E_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    Request *q = find(S, ticket);
    if (!q) return ND_E_INVALID_ARG;
    if (q->info.done) return ND_OK;
    q->cancelled = true;
    if (!q->running) {
      auto it = std::find(S->queue.begin(), S->queue.end(), q);
      if (it != S->queue.end()) S->queue.erase(it);
      q->rp.clear();
      q->col.clear();
      q->info.status = ND_E_CANCELLED;
      q->info.done = 1;
      q->info.t_done_ms = S->now_ms();
      S->stats.waiting--;
      S->stats.cancelled++;
    }
  }
  S->cv_done.notify_all();
  S->cv_work.notify_all();
  return ND_OK;
}

nd_status nd_server_get_stats(nd_server *S, nd_server_stats *out) {
  if (!S || !out) return ND_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  *out = S->stats;
  device_overlap(S->intervals, &out->device_busy_ms, &out->device_overlap_ms,
                 &out->device_batch_ms);
  return ND_OK;
}

const char *nd_server_last_error(const nd_server *S) {
  return S ? S->last_error.c_str() : "";
}

}  // extern "C"
