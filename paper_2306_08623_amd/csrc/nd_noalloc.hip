// nd_noalloc.hip -- nd_decompose_noalloc: the whole decomposition of one
// graph without allocating device memory. Every intermediate buffer of the
// pipeline is carved, in order, from one fixed device array per GPU
// (`scratch`, ND_NOALLOC_SCRATCH_BYTES); the caller passes the CSR and the
// output arrays. The kernels are the ones nd_decompose runs.
#include "nd_internal.h"

#include <mutex>
#include <new>

namespace {

// One copy per GPU, held until the process ends. Host code never uses this
// name as an address: the device address of each GPU's copy comes from
// hipGetSymbolAddress at set-up and is kept in NoAllocDevice::scratch_ptr.
static __device__ __align__(256) unsigned char scratch[ND_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct NoAllocDevice {
  std::mutex mu;               // one call at a time per GPU
  bool ready = false;
  char *scratch_ptr = nullptr;   // this GPU's copy of `scratch`
  nd_ctx *ctx = nullptr;       // context whose buffers live in the scratch
};

NoAllocDevice g_dev[kMaxDevices];

// the message goes where nd_last_error(NULL) reads it (this thread's)
nd_status fail(nd_status st, const char *msg) {
  nd_thread_error(msg);
  return st;
}

template <typename... A>
nd_status failf(nd_status st, const char *fmt, A... args) {
  char buf[512];
  snprintf(buf, sizeof(buf), fmt, args...);
  nd_thread_error(buf);
  return st;
}

// Once per device, with that device current: the scratch address and a
// context bound to it (host objects sized once, so later calls allocate
// nothing).
nd_status setup(int device, NoAllocDevice &D) {
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return failf(ND_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      cus <= 0) {
    (void)hipGetLastError();
    return fail(ND_E_DEVICE, "compute unit count");
  }
  nd_ctx *c = new (std::nothrow) nd_ctx();
  if (!c) return fail(ND_E_OOM, "host context");
  c->device = device;
  c->validate = 1;
  c->cu_count = cus;
  c->events_ok = false;
  c->arena = (char *)p;
  c->arena_cap = ND_NOALLOC_SCRATCH_BYTES;
  c->bufs.resize(B_COUNT + kBatchGroups * kBatchFields);
  c->resident_cap.reserve(16);
  c->last_error.reserve(512);
  D.scratch_ptr = (char *)p;
  D.ctx = c;
  D.ready = true;
  return ND_OK;
}

}  // namespace

extern "C" {

nd_status nd_decompose_noalloc(int device, void *hip_stream, uint32_t n, uint64_t nnz,
                               const uint64_t *row_ptr, const uint32_t *col, uint32_t r,
                               uint32_t s, uint64_t cap, uint32_t *coreness, uint64_t *parent,
                               uint32_t *level, nd_info *info) {
  nd_thread_error("");
  if (device < 0 || device >= kMaxDevices) return fail(ND_E_INVALID_ARG, "device ordinal");
  if (!row_ptr || (nnz && !col)) return fail(ND_E_INVALID_ARG, "NULL row_ptr or col");
  if (cap && (!coreness || !parent || !level))
    return fail(ND_E_INVALID_ARG, "NULL output array");
  // the CSR copy and the per-slot edge ids alone must fit the scratch
  const uint64_t min_bytes = 8ull * (n + 1ull) + 12ull * nnz;
  if (min_bytes > ND_NOALLOC_SCRATCH_BYTES)
    return failf(ND_E_OOM,
                 "graph too large for the fixed scratch: n=%u nnz=%llu needs at least %llu of "
                 "%llu bytes",
                 n, (unsigned long long)nnz, (unsigned long long)min_bytes,
                 (unsigned long long)ND_NOALLOC_SCRATCH_BYTES);
  NoAllocDevice &D = g_dev[device];
  std::lock_guard<std::mutex> lock(D.mu);
  if (hipSetDevice(device) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ND_E_DEVICE, "hipSetDevice");
  }
  if (!D.ready) {
    nd_status st = setup(device, D);
    if (st != ND_OK) return st;
  }
  nd_ctx *c = D.ctx;
  // the previous call has finished (each call waits for its stream), so
  // the whole scratch is free again
  nd_arena_reset(c);
  c->stream = (hipStream_t)hip_stream;
  c->last_error.clear();
  nd_status st = ND_OK;
  if (!nd_buf(c, B_SCAL, sizeof(DevScalars), &st) ||
      (st = nd_load_csr(c, n, nnz, row_ptr, col, ND_MEM_DEVICE)) != ND_OK ||
      (st = nd_set_rs(c, r, s)) != ND_OK || (st = nd_decompose(c)) != ND_OK) {
    fail(st, c->last_error.c_str());
    (void)hipStreamSynchronize(c->stream);
    return st;
  }
  if (c->n_r > cap) {
    if (info) *info = c->info;
    return failf(ND_E_INVALID_ARG,
                 "outputs hold %llu r-cliques, the graph has %llu (coreness needs n_r "
                 "entries, parent 2 n_r, level n_r)",
                 (unsigned long long)cap, (unsigned long long)c->n_r);
  }
  if ((st = nd_get_coreness(c, coreness, ND_MEM_DEVICE)) != ND_OK ||
      (st = nd_get_tree(c, parent, level, ND_MEM_DEVICE)) != ND_OK) {
    fail(st, c->last_error.c_str());
    return st;
  }
  if (info) *info = c->info;
  return ND_OK;
}

}  // extern "C"
