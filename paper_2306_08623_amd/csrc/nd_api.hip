// nd_api.hip -- the C ABI declared in include/nucleus.h: context, device
// workspace, the decomposition pipeline and the result getters.
#include "nd_internal.h"

#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <thread>

#include <algorithm>
#include <cstring>
#include <new>

nd_status nd_validate_loaded(nd_ctx *c);

nd_status nd_fail(nd_ctx *c, nd_status st, const std::string &msg) {
  if (c) c->last_error = msg;
  return st;
}

nd_status nd_hip(nd_ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return ND_OK;
  if (e == hipErrorOutOfMemory)
    return nd_fail(c, ND_E_OOM, std::string(what) + ": " + hipGetErrorString(e));
  return nd_fail(c, ND_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device memory of a context: its arena, the caller's callbacks, or
// hipMalloc / hipFree.
static void *dev_alloc(nd_ctx *c, size_t bytes) {
  if (c->arena) {
    const uint64_t at = (c->arena_used + 255) & ~255ull;
    if (at > c->arena_cap || bytes > c->arena_cap - at) return nullptr;
    c->arena_used = at + bytes;
    return c->arena + at;
  }
  if (c->alloc_fn) return c->alloc_fn(bytes, (void *)c->stream, c->alloc_user);
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

static void dev_free(nd_ctx *c, void *p, size_t bytes) {
  if (!p || c->arena) return;   // arena memory is reused after nd_arena_reset
  if (c->free_fn) c->free_fn(p, bytes, (void *)c->stream, c->alloc_user);
  else (void)hipFree(p);
}

void nd_arena_reset(nd_ctx *c) {
  for (auto &b : c->bufs) {
    b.p = nullptr;
    b.bytes = 0;
  }
  c->arena_used = 0;
  c->bytes_held = 0;
  c->bytes_peak = 0;
}

void *nd_buf(nd_ctx *c, int id, size_t bytes, nd_status *st) {
  *st = ND_OK;
  if ((int)c->bufs.size() <= id) c->bufs.resize(std::max(id + 1, (int)B_COUNT));
  DevBuf &b = c->bufs[id];
  if (bytes == 0) bytes = 8;
  if (b.p && b.bytes >= bytes) return b.p;
  // grow with slack, except in an arena, where every byte counts
  size_t want = c->arena ? bytes : std::max<size_t>(bytes, b.bytes + b.bytes / 4);
  uint64_t held_after = c->bytes_held - b.bytes + want;
  if (c->mem_limit && held_after > c->mem_limit) {
    want = bytes;
    held_after = c->bytes_held - b.bytes + want;
    if (held_after > c->mem_limit) {
      *st = nd_fail(c, ND_E_OOM, "device workspace limit reached (" + std::to_string(held_after) +
                                     " > " + std::to_string(c->mem_limit) + " bytes)");
      return nullptr;
    }
  }
  if (b.p) {
    if (!c->arena) {
      // the old buffer may still be read by queued kernels
      hipError_t e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) {
        *st = nd_hip(c, e, "sync before realloc");
        return nullptr;
      }
    }
    dev_free(c, b.p, b.bytes);
    c->bytes_held -= b.bytes;
    b.p = nullptr;
    b.bytes = 0;
  }
  void *p = dev_alloc(c, want);
  if (!p) {
    if (c->arena)
      *st = nd_fail(c, ND_E_OOM,
                    "the fixed scratch of " + std::to_string(c->arena_cap) +
                        " bytes is too small for this graph (" + std::to_string(want) +
                        " more bytes needed at offset " + std::to_string(c->arena_used) + ")");
    else
      *st = nd_fail(c, ND_E_OOM,
                    std::string(c->alloc_fn ? "allocator callback" : "hipMalloc") + " of " +
                        std::to_string(want) + " bytes failed");
    return nullptr;
  }
  b.p = p;
  b.bytes = want;
  c->bytes_held += want;
  c->bytes_peak = std::max(c->bytes_peak, c->bytes_held);
  return p;
}

void nd_report(nd_ctx *c, const char *fmt, ...) {
  if (!(c->flags & ND_FLAG_PROGRESS)) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[nd] %s\n", buf);
  std::fflush(stderr);
}

void nd_report_while_running(nd_ctx *c, const char *phase, const uint32_t *progress) {
  const auto t0 = std::chrono::steady_clock::now();
  auto last = t0;
  for (;;) {
    const hipError_t q = hipStreamQuery(c->stream);
    if (q != hipErrorNotReady) {
      if (q != hipSuccess) (void)hipGetLastError();   // reported by the next sync
      return;
    }
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
    const auto now = std::chrono::steady_clock::now();
    if (now - last >= std::chrono::seconds(10)) {
      last = now;
      const volatile uint32_t *p = progress;
      nd_report(c, "%s running %.0f s: round %u, level %u, frontier %u", phase,
                std::chrono::duration<double>(now - t0).count(), p[0], p[1], p[2]);
    }
  }
}

nd_status nd_persistent_launch(nd_ctx *c, const void *kern, uint32_t *nb, uint32_t *nb_arg,
                         dim3 block, void **args, hipEvent_t before, hipEvent_t after,
                         const char *what) {
  DevScalars *sc = (DevScalars *)c->bufs[B_SCAL].p;
  for (;;) {
    *nb_arg = *nb;
    nd_status st = nd_hip(c, hipMemsetAsync(sc->bar, 0, sizeof(sc->bar), c->stream), "barrier reset");
    if (st != ND_OK) return st;
    if (before) (void)hipEventRecord(before, c->stream);
    // a plain launch: the kernel's own residency gate checks that all of
    // its workgroups run at once (see nd_internal.h)
    st = nd_hip(c, hipLaunchKernel(kern, dim3(*nb), block, args, 0, c->stream), what);
    if (after) (void)hipEventRecord(after, c->stream);
    if (st != ND_OK) return st;
    if (c->report_phase && c->progress) nd_report_while_running(c, c->report_phase, c->progress);
    uint32_t status = 0;
    if ((st = nd_hip(c, hipMemcpyAsync(&status, &sc->status, 4, hipMemcpyDeviceToHost,
                                       c->stream), what)) != ND_OK ||
        (st = nd_hip(c, hipStreamSynchronize(c->stream), what)) != ND_OK)
      return st;
    if (!(status & ND_DERR_RESIDENCY)) {
      if (c->info.grid_retries) {   // remember what fitted, for later launches
        bool found = false;
        for (auto &e : c->resident_cap)
          if (e.first == kern) { e.second = std::min(e.second, *nb); found = true; }
        if (!found) c->resident_cap.emplace_back(kern, *nb);
      }
      return ND_OK;
    }
    // not resident: no workgroup got past the gate's barrier, so nothing
    // was written; clear the status and shrink
    c->info.grid_retries++;
    nd_report(c, "%s: grid of %u workgroups not resident, retrying smaller", what, *nb);
    const uint32_t zero = 0;
    if ((st = nd_hip(c, hipMemcpyAsync(&sc->status, &zero, 4, hipMemcpyHostToDevice, c->stream),
                     "status reset")) != ND_OK ||
        (st = nd_hip(c, hipStreamSynchronize(c->stream), "status reset")) != ND_OK)
      return st;
    if (*nb <= 1) return nd_fail(c, ND_E_DEVICE, std::string(what) + ": no resident grid");
    *nb = std::max<uint32_t>(1, *nb / 4 * 3);
  }
}

static nd_status set_dev(nd_ctx *c) {
  return nd_hip(c, hipSetDevice(c->device), "hipSetDevice");
}

extern "C" {

const char *nd_status_str(nd_status st) {
  switch (st) {
    case ND_OK: return "ok";
    case ND_E_INVALID_ARG: return "invalid argument";
    case ND_E_BAD_GRAPH: return "input is not a simple undirected CSR graph";
    case ND_E_UNSUPPORTED: return "unsupported";
    case ND_E_OOM: return "out of device memory";
    case ND_E_OVERFLOW: return "32-bit overflow";
    case ND_E_DEVICE: return "HIP runtime error";
    case ND_E_WATCHDOG: return "device watchdog";
    case ND_E_STATE: return "call out of order";
    case ND_E_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

// message of the last failed nd_create or nd_decompose_noalloc on this
// thread (no context of the caller's exists)
static thread_local std::string g_create_error;

}  // extern "C"

void nd_thread_error(const char *msg) { g_create_error = msg; }

extern "C" {

const char *nd_last_error(const nd_ctx *c) {
  return c ? c->last_error.c_str() : g_create_error.c_str();
}

static nd_status create_fail(nd_ctx *c, nd_status st, const std::string &msg) {
  g_create_error = msg;
  delete c;
  return st;
}

nd_status nd_create(nd_ctx **out, const nd_options *opt) {
  if (!out) return ND_E_INVALID_ARG;
  *out = nullptr;
  nd_ctx *c = new (std::nothrow) nd_ctx();
  if (!c) return ND_E_OOM;
  if (opt) {
    c->device = opt->device;
    c->stream = (hipStream_t)opt->hip_stream;
    c->validate = opt->validate;
    c->mem_limit = opt->mem_limit;
    c->peel_blocks = opt->peel_blocks;
    c->work_chunk = opt->work_chunk;
    c->watchdog = opt->watchdog;
    c->flags = opt->flags;
    if ((opt->alloc == nullptr) != (opt->free == nullptr)) {
      g_create_error = "nd_options.alloc and nd_options.free must be given together";
      delete c;
      return ND_E_INVALID_ARG;
    }
    c->alloc_fn = opt->alloc;
    c->free_fn = opt->free;
    c->alloc_user = opt->alloc_user;
  }
  g_create_error.clear();
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return create_fail(c, ND_E_DEVICE,
                       std::string("hipGetDeviceCount: ") + hipGetErrorString(e) +
                           " (devices: " + std::to_string(ndev) + ")");
  }
  if (c->device < 0 || c->device >= ndev)
    return create_fail(c, ND_E_INVALID_ARG, "device ordinal out of range");
  if ((e = hipSetDevice(c->device)) != hipSuccess)
    return create_fail(c, ND_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
  if ((e = hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount,
                                 c->device)) != hipSuccess ||
      c->cu_count <= 0)
    return create_fail(c, ND_E_DEVICE,
                       std::string("compute unit count: ") + hipGetErrorString(e));
  c->bufs.resize(B_COUNT);
  if (c->flags & ND_FLAG_PROGRESS) {
    if (hipHostMalloc((void **)&c->progress, 16, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      c->progress = nullptr;
      return create_fail(c, ND_E_OOM, "pinned progress words");
    }
    memset(c->progress, 0, 16);
  }
  c->events_ok = true;
  for (int i = 0; i < 10; i++)
    if (hipEventCreate(&c->ev[i]) != hipSuccess) c->events_ok = false;
  nd_status st;
  if (!nd_buf(c, B_SCAL, sizeof(DevScalars), &st)) {
    nd_destroy(c);
    return st;
  }
  *out = c;
  return ND_OK;
}

void nd_destroy(nd_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  nd_batch_release(c);
  for (auto &b : c->bufs)
    if (b.p) dev_free(c, b.p, b.bytes);
  for (int i = 0; i < 10; i++)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  if (c->progress) (void)hipHostFree(c->progress);
  delete c;
}

nd_status nd_load_csr(nd_ctx *c, uint32_t n, uint64_t nnz, const uint64_t *row_ptr,
                      const uint32_t *col, nd_mem where) {
  if (!c) return ND_E_INVALID_ARG;
  nd_status st = set_dev(c);
  if (st != ND_OK) return st;
  c->have_graph = false;
  c->decomposed = false;
  c->cut_valid = false;
  c->info_valid = false;
  if (!row_ptr || (nnz && !col)) return nd_fail(c, ND_E_INVALID_ARG, "NULL row_ptr or col");
  if (where != ND_MEM_HOST && where != ND_MEM_DEVICE)
    return nd_fail(c, ND_E_INVALID_ARG, "bad memory kind");
  if (n == 0xFFFFFFFFu) return nd_fail(c, ND_E_UNSUPPORTED, "n must be below 2^32-1");
  if (nnz & 1) return nd_fail(c, ND_E_BAD_GRAPH, "nnz is odd: the CSR cannot be symmetric");
  if (nnz / 2 >= 0xFFFFFFFFull) return nd_fail(c, ND_E_UNSUPPORTED, "edge ids exceed 32 bits");
  if (where == ND_MEM_HOST && c->validate) {
    if (row_ptr[0] != 0 || row_ptr[n] != nnz)
      return nd_fail(c, ND_E_BAD_GRAPH, "row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
    for (uint32_t u = 0; u < n; u++)
      if (row_ptr[u + 1] < row_ptr[u]) return nd_fail(c, ND_E_BAD_GRAPH, "row_ptr decreases");
  }
  uint64_t *rp = (uint64_t *)nd_buf(c, B_RP, (n + 1ull) * 8, &st);
  if (!rp) return st;
  uint32_t *dcol = (uint32_t *)nd_buf(c, B_COL, std::max<uint64_t>(nnz, 1) * 4, &st);
  if (!dcol) return st;
  hipMemcpyKind kind = where == ND_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  if ((st = nd_hip(c, hipMemcpyAsync(rp, row_ptr, (n + 1ull) * 8, kind, c->stream), "copy row_ptr")) !=
      ND_OK)
    return st;
  if (nnz &&
      (st = nd_hip(c, hipMemcpyAsync(dcol, col, nnz * 4, kind, c->stream), "copy col")) != ND_OK)
    return st;
  c->n = n;
  c->nnz = nnz;
  c->m = nnz / 2;
  if (c->validate) {
    st = nd_validate_loaded(c);
    if (st != ND_OK) return st;
  }
  c->have_graph = true;
  return ND_OK;
}

nd_status nd_set_approx(nd_ctx *c, double delta) {
  if (!c) return ND_E_INVALID_ARG;
  if (!(delta >= 0.0 && delta <= 64.0))
    return nd_fail(c, ND_E_INVALID_ARG, "delta must be in [0, 64]");
  c->approx_delta = delta;   // applies to the next decomposition; results stay readable
  return ND_OK;
}

nd_status nd_set_schedule(nd_ctx *c, const nd_schedule *table, uint32_t n) {
  if (!c) return ND_E_INVALID_ARG;
  if (n && !table) return nd_fail(c, ND_E_INVALID_ARG, "NULL schedule table");
  for (uint32_t i = 0; i < n; i++)
    if (table[i].r < 1 || table[i].s <= table[i].r || table[i].s > kMaxS ||
        table[i].kind > ND_SCHED_BATCH)
      return nd_fail(c, ND_E_INVALID_ARG, "schedule entry with an invalid (r,s) or kind");
  c->sched.assign(table, table + n);
  return ND_OK;
}

nd_status nd_set_rs(nd_ctx *c, uint32_t r, uint32_t s) {
  if (!c) return ND_E_INVALID_ARG;
  if (r < 1 || s <= r) return nd_fail(c, ND_E_INVALID_ARG, "need 1 <= r < s");
  if (!nd_rs_supported(r, s)) return nd_fail(c, ND_E_UNSUPPORTED, "this (r,s) pair is not built");
  c->r = r;
  c->s = s;
  c->decomposed = false;
  c->info_valid = false;
  return ND_OK;
}

static nd_status check_device_status(nd_ctx *c, DevScalars *host) {
  DevScalars *sc = (DevScalars *)c->bufs[B_SCAL].p;
  nd_status st = nd_hip(
      c, hipMemcpyAsync(host, sc, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream),
      "scalars readback");
  if (st != ND_OK) return st;
  st = nd_hip(c, hipStreamSynchronize(c->stream), "stream sync");
  if (st != ND_OK) return st;
  if (host->status & ND_DERR_WATCHDOG)
    return nd_fail(c, ND_E_WATCHDOG, "a device loop exceeded its bound");
  if (host->status & ND_DERR_LINKQ)
    return nd_fail(c, ND_E_OOM, "link spill queue overflowed");
  if (host->status & ND_DERR_OVERFLOW)
    return nd_fail(c, ND_E_UNSUPPORTED,
                   "a listing buffer or a 32-bit work range was exceeded (an oriented "
                   "out-neighbourhood, or the (2,4) probe range of one edge)");
  if (host->status & ND_DERR_BADGRAPH) return nd_fail(c, ND_E_BAD_GRAPH, "bad graph");
  return ND_OK;
}

}  // extern "C"

// The whole pipeline on the graph held in B_RP / B_COL (n, nnz, r, s set).
nd_status nd_run_pipeline(nd_ctx *c) {
  nd_status st;
  c->decomposed = false;
  c->cut_valid = false;
  c->info_valid = false;
  memset(&c->info, 0, sizeof(c->info));
  c->bytes_peak = c->bytes_held;
  DevScalars *sc = (DevScalars *)c->bufs[B_SCAL].p;
  if ((st = nd_hip(c, hipMemsetAsync(sc, 0, sizeof(DevScalars), c->stream), "scalars")) != ND_OK)
    return st;
  if (c->events_ok) (void)hipEventRecord(c->ev[0], c->stream);
  GraphView gv;
  memset(&gv, 0, sizeof(gv));
  if ((st = nd_stage_prep(c, &gv)) != ND_OK) return st;
  if (c->events_ok) (void)hipEventRecord(c->ev[1], c->stream);
  nd_report(c, "prep queued: n=%u m=%llu (r,s)=(%u,%u) n_r=%llu", c->n,
            (unsigned long long)c->m, c->r, c->s, (unsigned long long)c->n_r);
  if ((st = nd_stage_count(c, gv)) != ND_OK) return st;
  if (c->events_ok) (void)hipEventRecord(c->ev[2], c->stream);
  DevScalars hs;
  if ((st = check_device_status(c, &hs)) != ND_OK) return st;
  c->info.n_s = hs.n_s;
  c->info.max_outdeg = hs.max_outdeg;
  nd_report(c, "count done: n_s=%llu", (unsigned long long)hs.n_s);
  if ((st = nd_stage_peel(c, gv)) != ND_OK) return st;
  if (c->events_ok) (void)hipEventRecord(c->ev[3], c->stream);
  if ((st = check_device_status(c, &hs)) != ND_OK) return st;
  nd_report(c, "peel done: %u rounds, k=%u", hs.rounds, hs.k);
  if ((st = nd_stage_tree(c, gv)) != ND_OK) return st;
  if (c->events_ok) (void)hipEventRecord(c->ev[4], c->stream);
  if ((st = check_device_status(c, &hs)) != ND_OK) return st;
  nd_report(c, "tree done: %llu nodes", (unsigned long long)c->n_int);
  c->gv = gv;
  nd_info &I = c->info;
  I.n = c->n;
  I.r = c->r;
  I.s = c->s;
  I.m = c->m;
  I.n_r = c->n_r;
  I.k = c->n_r ? hs.k : 0;
  I.rounds = hs.rounds;
  I.n_int = c->n_int;
  I.visits = hs.visits;
  I.decrements = hs.decrements;
  I.links = hs.links;
  I.link_calls = hs.link_calls;
  I.unites = hs.unites;
  I.bucket_scans = hs.bucket_scans;
  I.hier_visits = hs.hier_visits;
  I.orient_rounds = hs.orient_round;
  I.device_bytes = c->bytes_held;
  I.device_peak = c->bytes_peak;
  I.approx_delta = c->approx_delta;
  if (c->approx_delta <= 0) I.round_cap = 0;
  I.cas_retries = hs.cas_retries;
  I.cascades = (!I.hier_te && hs.links > hs.link_calls) ? hs.links - hs.link_calls : 0;
  if (c->events_ok) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) I.ms_prep = ms;
    if (hipEventElapsedTime(&ms, c->ev[1], c->ev[2]) == hipSuccess) I.ms_count = ms;
    if (hipEventElapsedTime(&ms, c->ev[2], c->ev[3]) == hipSuccess) I.ms_peel = ms;
    if (hipEventElapsedTime(&ms, c->ev[3], c->ev[4]) == hipSuccess) I.ms_tree = ms;
    if (c->n_r && hipEventElapsedTime(&ms, c->ev[5], c->ev[6]) == hipSuccess)
      I.ms_peel_kernel = ms;
    if (c->s > 2 && c->m && hipEventElapsedTime(&ms, c->ev[7], c->ev[8]) == hipSuccess)
      I.ms_count_kernel = ms;
    if (I.hier_te && c->n_r && hipEventElapsedTime(&ms, c->ev[6], c->ev[9]) == hipSuccess)
      I.ms_hier = ms;
    (void)hipGetLastError();
  }
  c->decomposed = true;
  c->info_valid = true;
  return ND_OK;
}

extern "C" {

nd_status nd_decompose(nd_ctx *c) {
  if (!c) return ND_E_INVALID_ARG;
  nd_status st = set_dev(c);
  if (st != ND_OK) return st;
  if (!c->have_graph) return nd_fail(c, ND_E_STATE, "no graph loaded");
  if (!c->r) return nd_fail(c, ND_E_STATE, "r and s not set");
  c->last_error.clear();
  return nd_run_pipeline(c);
}

nd_status nd_sync(nd_ctx *c) {
  if (!c) return ND_E_INVALID_ARG;
  nd_status st = set_dev(c);
  if (st != ND_OK) return st;
  DevScalars hs;
  return check_device_status(c, &hs);
}

nd_status nd_get_info(nd_ctx *c, nd_info *out) {
  if (!c || !out) return ND_E_INVALID_ARG;
  if (!c->info_valid) return nd_fail(c, ND_E_STATE, "no decomposition result");
  *out = c->info;
  return ND_OK;
}

static nd_status copy_out(nd_ctx *c, void *dst, const void *src, size_t bytes, nd_mem where) {
  if (bytes == 0) return ND_OK;
  if (where != ND_MEM_HOST && where != ND_MEM_DEVICE)
    return nd_fail(c, ND_E_INVALID_ARG, "bad memory kind");
  hipMemcpyKind kind = where == ND_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  nd_status st = nd_hip(c, hipMemcpyAsync(dst, src, bytes, kind, c->stream), "copy out");
  if (st != ND_OK) return st;
  return nd_hip(c, hipStreamSynchronize(c->stream), "copy out sync");
}

nd_status nd_get_rcliques(nd_ctx *c, uint32_t *out, nd_mem where) {
  if (!c || (!out && c->n_r)) return ND_E_INVALID_ARG;
  nd_status st = set_dev(c);
  if (st != ND_OK) return st;
  if (!c->decomposed) return nd_fail(c, ND_E_STATE, "no decomposition result");
  const size_t bytes = c->n_r * c->r * 4ull;
  if (bytes == 0) return ND_OK;
  if (where == ND_MEM_DEVICE) {
    if ((st = nd_write_rcliques(c, c->gv, out)) != ND_OK) return st;
    return nd_hip(c, hipStreamSynchronize(c->stream), "rcliques sync");
  }
  uint32_t *tmp = (uint32_t *)nd_buf(c, B_RCL, bytes, &st);
  if (!tmp) return st;
  if ((st = nd_write_rcliques(c, c->gv, tmp)) != ND_OK) return st;
  return copy_out(c, out, tmp, bytes, where);
}

nd_status nd_get_counts(nd_ctx *c, uint32_t *out, nd_mem where) {
  if (!c || (!out && c->n_r)) return ND_E_INVALID_ARG;
  nd_status st = set_dev(c);
  if (st != ND_OK) return st;
  if (!c->decomposed) return nd_fail(c, ND_E_STATE, "no decomposition result");
  return copy_out(c, out, c->bufs[B_CNT0].p, c->n_r * 4ull, where);
}

nd_status nd_get_coreness(nd_ctx *c, uint32_t *out, nd_mem where) {
  if (!c || (!out && c->n_r)) return ND_E_INVALID_ARG;
  nd_status st = set_dev(c);
  if (st != ND_OK) return st;
  if (!c->decomposed) return nd_fail(c, ND_E_STATE, "no decomposition result");
  return copy_out(c, out, c->bufs[B_CNT].p, c->n_r * 4ull, where);
}

nd_status nd_get_peel_rounds(nd_ctx *c, uint32_t *out, nd_mem where) {
  if (!c || (!out && c->n_r)) return ND_E_INVALID_ARG;
  nd_status st = set_dev(c);
  if (st != ND_OK) return st;
  if (!c->decomposed) return nd_fail(c, ND_E_STATE, "no decomposition result");
  return copy_out(c, out, c->bufs[B_ROUND].p, c->n_r * 4ull, where);
}

nd_status nd_get_tree(nd_ctx *c, uint64_t *parent, uint32_t *level, nd_mem where) {
  if (!c) return ND_E_INVALID_ARG;
  nd_status st = set_dev(c);
  if (st != ND_OK) return st;
  if (!c->decomposed) return nd_fail(c, ND_E_STATE, "no decomposition result");
  if (c->n_r == 0) return ND_OK;
  if (parent && (st = copy_out(c, parent, c->bufs[B_PARENT].p, (c->n_r + c->n_int) * 8ull,
                               where)) != ND_OK)
    return st;
  if (level && c->n_int &&
      (st = copy_out(c, level, c->bufs[B_LEVEL].p, c->n_int * 4ull, where)) != ND_OK)
    return st;
  return ND_OK;
}

}  // extern "C"
