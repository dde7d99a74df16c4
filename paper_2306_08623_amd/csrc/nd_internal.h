// nd_internal.h -- shared declarations of the gfx950 nucleus decomposition
// library: device views of the graph tables, device helpers, and the host
// context. Only the library's own .hip files include this header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <vector>

#include "nucleus.h"

#define ND_NONE 0xFFFFFFFFu          // empty r-clique id / empty L entry
#define ND_ALIVE 0xFFFFFFFFu         // peel_round of an unpeeled r-clique
#define ND_NONE64 0xFFFFFFFFFFFFFFFFull

// error codes written by kernels into the device status word
#define ND_DERR_WATCHDOG 1u
#define ND_DERR_LINKQ 2u
#define ND_DERR_BADGRAPH 4u
#define ND_DERR_OVERFLOW 8u
#define ND_DERR_RESIDENCY 16u   // a persistent grid was not fully resident

// ---------------------------------------------------------------------------
// Device views (plain pointers, passed by value to kernels)
// ---------------------------------------------------------------------------

// Undirected CSR plus per-slot edge ids and the oriented out-CSR (DG).
struct GraphView {
  uint32_t n;
  uint64_t nnz;              // 2m
  uint64_t m;
  const uint64_t *rp;        // [n+1]
  const uint32_t *col;       // [nnz], rows ascending
  const uint32_t *eid;       // [nnz] id of the undirected edge in each slot
  const uint32_t *eu;        // [m] smaller endpoint of edge id
  const uint32_t *ev;        // [m] larger endpoint
  const uint64_t *okey;      // [n] orientation key: u -> v is an out-edge iff okey[u] < okey[v]
  const uint64_t *dgp;       // [n+1] oriented out-CSR offsets
  const uint32_t *dgc;       // [m] out-neighbours, ascending vertex id
  const uint32_t *dge;       // [m] edge id of each out-slot
  // edge -> triangle lists (r = 3, and (r,s) = (2,4))
  const uint64_t *wp;        // [m+1] offsets of W(e), the common neighbours of e
  const uint32_t *wc;        // [3 n_tri] W entries (third vertex), ascending per edge
  const uint32_t *wt;        // [3 n_tri] triangle id of each W entry
  const uint32_t *te;        // [3 n_tri] (e_ab, e_ac, e_bc) of triangle (a<b<c)
  // (2,4) only, per W entry (edge e, third vertex w, triangle t): the probed
  // list part, (list << 30 | start offset) with list 0 = W(e), 1/2 = W of
  // t's other edges in te order, holding t's candidates x > w; and the
  // running sum of the parts' lengths over all entries ([3 n_tri + 1])
  const uint32_t *wsel;
  const uint64_t *wg;
  // (1,3), (1,4): running sum over CSR slots v -> w of the entries of W(vw)
  // above w (the triangles at v whose smaller other vertex is w); [2m + 1]
  const uint64_t *sg;
  // (1,4) only, per triangle probe of (1,3) (global index sg[slot] + j):
  // the probed list part for the 4th vertex y > x, as in wsel (list 0 =
  // W(vw), 1 = W(vx), 2 = W(wx)), and the running sum of the parts' lengths
  const uint32_t *tsel;
  const uint64_t *tg;
  // s = 5..7 (nd_gen.hip): the s-cliques kept in HBM. rcl: the n_r
  // lexicographic r-tuples (r >= 2); sm: the nsm = C(s,r) r-clique ids of
  // every s-clique; io / il: the s-cliques of every r-clique (CSR, [n_r + 1]
  // offsets)
  const uint32_t *rcl;
  const uint32_t *sm;
  const uint64_t *io;
  const uint32_t *il;
  uint32_t nsm;
};

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// first index x in [lo, hi) with a[x] > v (a ascending), hi if none
__device__ __forceinline__ uint64_t upper_bound_u32(const uint32_t *a, uint64_t lo, uint64_t hi,
                                                    uint32_t v) {
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (a[mid] <= v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Coherent (agent-scope) relaxed atomics. Plain loads may hit a stale line in
// another XCD's L2; these go to the coherence point. (Relaxed: no cache
// invalidation; ordering comes from fences where it is needed.)
__device__ __forceinline__ uint32_t ld_acq32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_acq64(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas32(uint32_t *p, uint32_t expect, uint32_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// First index in [lo, hi) of a sorted array whose value is >= x.
template <typename IdxT>
__device__ __forceinline__ IdxT lower_bound_u32(const uint32_t *a, IdxT lo, IdxT hi, uint32_t x) {
  while (lo < hi) {
    IdxT mid = lo + ((hi - lo) >> 1);
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Index of x in the sorted range a[lo, hi), or hi when absent.
template <typename IdxT>
__device__ __forceinline__ IdxT find_u32(const uint32_t *a, IdxT lo, IdxT hi, uint32_t x) {
  IdxT p = lower_bound_u32<IdxT>(a, lo, hi, x);
  return (p < hi && a[p] == x) ? p : hi;
}

// Indices of x in two non-empty, strictly increasing ranges a[lo1, hi1) and
// a[lo2, hi2) (hi of a range when x is absent from it). The two searches
// advance in lockstep, so their chains of dependent loads overlap; a range
// already settled keeps loading its last valid slot, so every load is in
// bounds. A present x is always tested as a midpoint (the step that brings a
// range's upper end down to x's slot tests that slot), so a range is settled
// as soon as its midpoint equals x, and no load follows the search.
template <typename IdxT>
__device__ __forceinline__ void find2_u32(const uint32_t *a, IdxT lo1, IdxT hi1, IdxT lo2,
                                          IdxT hi2, uint32_t x, IdxT &p1, IdxT &p2) {
  IdxT l1 = lo1, h1 = hi1, l2 = lo2, h2 = hi2;
  p1 = hi1;
  p2 = hi2;
  while (l1 < h1 || l2 < h2) {
    const IdxT m1 = l1 < h1 ? l1 + ((h1 - l1) >> 1) : hi1 - 1;
    const IdxT m2 = l2 < h2 ? l2 + ((h2 - l2) >> 1) : hi2 - 1;
    const uint32_t v1 = a[m1], v2 = a[m2];
    if (l1 < h1) {
      if (v1 == x) {
        p1 = m1;
        h1 = l1;
      } else if (v1 < x) {
        l1 = m1 + 1;
      } else {
        h1 = m1;
      }
    }
    if (l2 < h2) {
      if (v2 == x) {
        p2 = m2;
        h2 = l2;
      } else if (v2 < x) {
        l2 = m2 + 1;
      } else {
        h2 = m2;
      }
    }
  }
}

// Last index i in [0, n) with a[i] <= x for a non-decreasing u64 array whose
// first element is <= x (segment search over exclusive offsets).
__device__ __forceinline__ uint32_t segment_of(const uint64_t *a, uint32_t n, uint64_t x) {
  uint32_t lo = 0, hi = n;   // invariant: a[lo] <= x, answer in [lo, hi)
  while (hi - lo > 1) {
    uint32_t mid = lo + ((hi - lo) >> 1);
    if (a[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// Wave-wide inclusive prefix sum of a 32-bit value (wave64).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(v, d, 64);
    if (lane >= (uint32_t)d) v += t;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ uint32_t wave_min32(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    uint32_t o = __shfl_xor(v, d, 64);
    v = o < v ? o : v;
  }
  return v;
}

// Wave-aggregated append: every lane with `want` gets a unique slot in a
// global list whose length is *counter. Returns the slot (undefined for
// lanes without `want`).
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool want) {
  uint64_t mask = ballot64(want);
  uint32_t total = __popcll(mask);
  if (total == 0) return 0;
  uint32_t lane = lane_id();
  uint32_t leader = __ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, total);
  base = __shfl(base, leader, 64);
  uint64_t below = mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane)));
  return base + __popcll(below);
}

// 20 s at the 100 MHz real-time counter: far beyond any legitimate wait.
constexpr uint64_t kBarrierTimeoutTicks = 2000000000ull;

// Grid-wide barrier state of a persistent launch, in 64-bit words: the
// release generation, the count of groups done, the residency gate's
// arrivals, then one arrival counter per group of workgroups, each word on
// a 128-byte line of its own. All words start at zero for every launch.
constexpr uint32_t kBarGroups = 8;     // workgroup b is in group b % 8
constexpr uint32_t kBarLine = 16;      // 64-bit words per 128-byte line
constexpr uint32_t kBarRelease = 0;
constexpr uint32_t kBarDone = kBarLine;
constexpr uint32_t kBarGate = 2 * kBarLine;
constexpr uint32_t kBarGroup0 = 3 * kBarLine;
constexpr uint32_t kBarWords = kBarGroup0 + kBarGroups * kBarLine;

// Grid-wide barrier for a persistent launch whose workgroups are all
// resident (checked by residency_gate at the kernel's start). Arrivals are counted per group (monotone
// counters: a workgroup's generation is its arrival index over the group's
// size); the last arrival of a group counts the group done, and the last
// group publishes the generation, which every workgroup waits for. Fences:
// release before the arrival, acquire after the wait (one each per
// workgroup: an agent-scope fence writes back or invalidates the caches, so
// none is taken inside the wait loop); the last arrivals, which carry the
// other workgroups' arrivals on, take both. A watchdog bound turns a stuck
// wait into an error flag instead of a hang: once `status` is non-zero
// every waiter leaves.
__device__ __forceinline__ bool grid_barrier(uint64_t *bar, uint32_t nblocks, uint32_t *status) {
  __syncthreads();
  __shared__ uint32_t s_ok;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t ng = nblocks < kBarGroups ? nblocks : kBarGroups;
    const uint32_t grp = blockIdx.x % ng;
    const uint32_t gsize = nblocks / ng + (grp < nblocks % ng ? 1u : 0u);
    const uint64_t arrived =
        atomicAdd((unsigned long long *)(bar + kBarGroup0 + kBarLine * grp), 1ull);
    const uint64_t gen = arrived / gsize + 1;
    if (arrived % gsize == gsize - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      const uint64_t done = atomicAdd((unsigned long long *)(bar + kBarDone), 1ull);
      if (done % ng == ng - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        __hip_atomic_store(bar + kBarRelease, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    uint32_t ok = 1;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();   // 100 MHz clock
    while (ld_acq64(bar + kBarRelease) < gen) {
      if (ld_acq32(status) != 0) { ok = 0; break; }
      if (__builtin_amdgcn_s_memrealtime() - t0 > kBarrierTimeoutTicks) {
        atomicOr(status, ND_DERR_WATCHDOG);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// First step of every persistent (grid-barrier) kernel, before it touches
// any state: all workgroups must arrive within 200 ms, else the grid is not
// fully resident (the device cannot run all of its workgroups at once, or
// other work holds part of it) and every workgroup leaves with
// ND_DERR_RESIDENCY, so that the host relaunches a smaller grid instead of
// the barriers waiting out their watchdog. A workgroup can see the last
// arrival just as another one gives up waiting; a grid barrier after the
// gate therefore lets the kernel go on only when every workgroup passed it
// (one that gave up never arrives there, and its status bit releases the
// others), so a grid that will be relaunched has written nothing.
constexpr uint64_t kResidencyTicks = 20000000ull;

__device__ __forceinline__ bool residency_gate(uint64_t *bar, uint32_t nblocks,
                                               uint32_t *status) {
  __syncthreads();
  __shared__ uint32_t s_in;
  if (threadIdx.x == 0) {
    atomicAdd((unsigned long long *)(bar + kBarGate), 1ull);
    uint32_t ok = 1;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    while (ld_acq64(bar + kBarGate) < (uint64_t)nblocks) {
      if (ld_acq32(status) != 0) { ok = 0; break; }
      if (__builtin_amdgcn_s_memrealtime() - t0 > kResidencyTicks) {
        atomicOr(status, ND_DERR_RESIDENCY);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_in = ok;
  }
  __syncthreads();
  if (s_in == 0) return false;
  return grid_barrier(bar, nblocks, status);
}

// ---------------------------------------------------------------------------
// Host context
// ---------------------------------------------------------------------------

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

struct BatchState;

struct nd_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int validate = 1;
  uint64_t mem_limit = 0;
  uint32_t peel_blocks = 0;
  uint32_t work_chunk = 0;
  std::vector<nd_schedule> sched;   // nd_set_schedule: peel grid by (kind, r, s, n_r)
  bool in_batch = false;            // the pipeline runs a batch group's union
  uint64_t watchdog = 0;
  uint32_t flags = 0;          // ND_FLAG_*
  // persistent grids take 1/grid_div of the device, so that as many
  // pipelines' persistent kernels fit on it at once (the server's workers)
  uint32_t grid_div = 1;
  uint32_t *progress = nullptr;   // pinned host words the peel kernel updates
  const char *report_phase = nullptr;   // name of the running persistent launch
  // largest grid of each persistent kernel found resident on this device
  std::vector<std::pair<const void *, uint32_t>> resident_cap;
  int cu_count = 0;
  std::string last_error;

  // graph
  bool have_graph = false;
  uint32_t n = 0;
  uint64_t nnz = 0, m = 0;
  uint32_t r = 0, s = 0;
  double approx_delta = 0;   // > 0: approximate decomposition (Algorithm 2)
  bool decomposed = false;
  bool info_valid = false;   // info holds the last decomposition or batch

  // results of the last nd_batch_decompose (nd_batch.hip)
  BatchState *batch = nullptr;

  // device memory: hipMalloc / hipFree, the caller's callbacks, or a fixed
  // arena (sub-allocated in order, released all at once by nd_arena_reset)
  nd_alloc_fn alloc_fn = nullptr;
  nd_free_fn free_fn = nullptr;
  void *alloc_user = nullptr;
  char *arena = nullptr;
  uint64_t arena_cap = 0, arena_used = 0;

  // named device buffers (grow-only)
  std::vector<DevBuf> bufs;
  uint64_t bytes_held = 0;
  uint64_t bytes_peak = 0;   // largest bytes_held since the run started

  // device views of the prepared tables (valid after a decomposition)
  GraphView gv{};

  // results
  nd_info info{};
  uint64_t n_r = 0;
  uint64_t n_int = 0;
  uint64_t gen_n_s = 0;   // s = 5..7: s-cliques listed by nd_prep_general
  // last hierarchy cut (nd_cut): valid until the next decomposition
  bool cut_valid = false;
  uint64_t cut_nuclei = 0, cut_verts = 0;

  // events for phase timing: 0 start, 1 prep, 2 count, 3 peel, 4 tree;
  // 5/6 around the peel kernel, 7/8 around the count kernel
  hipEvent_t ev[10] = {};
  bool events_ok = false;
};

// buffer slots held by the context
enum BufId : int {
  B_RP = 0, B_COL, B_EID, B_EU, B_EV, B_UPLO, B_DEG,
  B_OKEY, B_DGP, B_DGC, B_DGE,
  B_SUP, B_UPC, B_WP, B_TRIB, B_WC, B_WT, B_TE,
  B_CNT, B_CNT0, B_ROUND, B_UF, B_L,
  B_F0, B_F1, B_WSCAN, B_AL0, B_AL1, B_BTOT, B_LINKQ,
  B_SCAL, B_TMP64, B_TMP32A, B_TMP32B, B_TMP32C, B_TMP32D,
  B_SORTK0, B_SORTK1, B_SORTV0, B_SORTV1, B_HIST,
  B_PARENT, B_LEVEL, B_RCL, B_GCACHE, B_ACNT, B_NODEML, B_SORTOFF,
  B_BATCHDESC, B_WG, B_W24L, B_LHIST, B_LOFF, B_SG, B_TSEL, B_TG, B_PSTATE,
  // hierarchy cut (nd_cut.hip)
  B_CUT_TOP, B_CUT_POS, B_CUT_LEAF, B_CUT_NUC, B_CUT_RCL, B_CUT_K0, B_CUT_K1, B_CUT_V0,
  B_CUT_V1, B_CUT_FLAG, B_CUT_POS2, B_CUT_VERTS, B_CUT_VNUC, B_CUT_CNT,
  B_THR,   // approximate decomposition: bucket ends
  B_C2G,   // 4-clique counting: global C2 slices for rows above the LDS cap
  B_CSLOT, // peel: chunk -> frontier slot map of a large round
  B_FREC,  // peel, (2,3) and (3,4): per frontier slot, the list ranges its visits search
  // s = 5..7 (nd_gen.hip): clique levels, sorted tuples, r-clique table,
  // s-clique members and the incidence CSR
  B_GEN_L0, B_GEN_L1, B_GEN_CNT, B_GEN_OFF, B_GEN_RTUP, B_GEN_STUP, B_GEN_RCL, B_GEN_SM,
  B_GEN_IO, B_GEN_IL,
  B_COUNT
};

// hierarchy construction: Algorithm 5 during the peel ("EL"), or the
// two-pass descending-core construction after it ("TE"); by default TE when
// s - r >= 2 ((1,3), (1,4), (2,4): core numbers span thousands of levels),
// EL otherwise
inline bool nd_use_te(const nd_ctx *c);

// the (r,s) pairs whose peel is built: every 1 <= r < s <= 7 (s <= 4 with
// edge -> triangle lists, s = 5..7 with the s-cliques kept); index of a
// pair's batch slots
constexpr uint32_t kMaxS = 7;
inline bool nd_rs_supported(uint32_t r, uint32_t s) { return r >= 1 && r < s && s <= kMaxS; }
inline bool nd_rs_general(uint32_t s) { return s >= 5; }
inline int nd_rs_index(uint32_t r, uint32_t s) {
  if (r == 2 && s == 4) return 3;
  if (r == 1 && s == 3) return 4;
  if (r == 1 && s == 4) return 5;
  if (s <= 4) return (int)r - 1;
  // s = 5..7: after the six pairs above, in (s, r) order
  return 6 + (int)((s - 5) * (s + 2) / 2) + (int)r - 1;   // s = 5: 6..9, 6: 10..14, 7: 15..20
}

// batch arena: per (r,s) group, kBatchFields grow-only slots after B_COUNT
constexpr int kBatchFields = 10;
constexpr int kBatchGroups = 21;   // every pair r < s <= 7
inline int nd_batch_slot(int group, int field) { return B_COUNT + group * kBatchFields + field; }

// device scalars block (one per context)
struct DevScalars {
  uint64_t n_s;            // s-cliques counted
  uint64_t visits, decrements, links, unites;
  uint64_t bucket_scans;
  uint64_t link_calls;     // link calls issued after the redundancy filter
  uint64_t hier_visits;    // s-cliques found by the descending-core hierarchy pass
  uint64_t cas_retries;    // compare-and-swaps of unite / L that lost a race
  uint32_t status;         // ND_DERR_* bits
  uint32_t k;              // final level reached
  uint32_t rounds;         // peel rounds executed
  uint32_t fsize[2];       // frontier sizes (by round parity)
  uint32_t kmin[2];        // bucket scan minimum (by scan parity)
  uint32_t n_alive[2];     // alive list sizes (by scan parity)
  uint32_t linkq_head, linkq_tail;
  uint32_t max_outdeg;
  uint32_t orient_round;
  uint32_t n_kept;         // tree: kept nodes
  uint32_t max_sup;        // (2,4): largest number of triangles on one edge
  uint32_t pad[4];
  alignas(128) uint64_t bar[kBarWords];   // grid barrier state (zeroed before each launch)
};

// helpers implemented in nd_api.hip
nd_status nd_fail(nd_ctx *c, nd_status st, const std::string &msg);
void *nd_buf(nd_ctx *c, int id, size_t bytes, nd_status *st);
// sets the message nd_last_error(NULL) returns on this thread
void nd_thread_error(const char *msg);
// forgets every buffer of an arena context (its memory is reused from the
// start by the next nd_buf calls); the caller ensures no queued work uses it
void nd_arena_reset(nd_ctx *c);
nd_status nd_hip(nd_ctx *c, hipError_t e, const char *what);

// Launch of a persistent (grid-barrier) kernel that opens with
// residency_gate: *nb workgroups (the kernel reads the count from *nb_arg),
// the barrier counter reset first; if the grid turns out not to be resident
// it is relaunched with 3/4 of the workgroups (waits for the launch).
// `before` / `after` (may be null) are recorded around the last attempt.
nd_status nd_persistent_launch(nd_ctx *c, const void *kern, uint32_t *nb, uint32_t *nb_arg,
                         dim3 block, void **args, hipEvent_t before, hipEvent_t after,
                         const char *what);

// releases the host state of the last batch (nd_batch.hip)
void nd_batch_release(nd_ctx *c);

// a batch split in its host half (checks, grouping, union packing; no
// device) and its device half (nd_batch.hip); execute takes ownership
nd_status nd_batch_plan(uint32_t G, const nd_graph_desc *graphs, nd_mem where,
                        nd_graph_result *results, BatchState **out, std::string *err);
nd_status nd_batch_execute(nd_ctx *c, BatchState *bs, const nd_graph_desc *graphs,
                           nd_graph_result *results);
void nd_batch_state_free(BatchState *bs);

// progress reports (ND_FLAG_PROGRESS): a finished phase, and the peel's
// round / level while its kernel runs (nd_api.hip)
void nd_report(nd_ctx *c, const char *fmt, ...);
void nd_report_while_running(nd_ctx *c, const char *phase, const uint32_t *progress);

// the whole decomposition of the graph held in the context (nd_api.hip)
nd_status nd_run_pipeline(nd_ctx *c);
nd_status nd_validate_loaded(nd_ctx *c);

// pipeline stages (each returns ND_OK or an error already recorded in ctx)
nd_status nd_stage_prep(nd_ctx *c, GraphView *gv);
nd_status nd_prep_general(nd_ctx *c, GraphView *gv);
nd_status nd_stage_count(nd_ctx *c, const GraphView &gv);
nd_status nd_stage_peel(nd_ctx *c, const GraphView &gv);
nd_status nd_stage_tree(nd_ctx *c, const GraphView &gv);
nd_status nd_write_rcliques(nd_ctx *c, const GraphView &gv, uint32_t *out_dev);
nd_status nd_sort_pairs_u64(nd_ctx *c, uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1,
                            uint64_t n, uint32_t bits, uint64_t **out_k, uint32_t **out_v);

// small device utilities (nd_prep.hip)
nd_status nd_exclusive_scan_u64(nd_ctx *c, const uint64_t *in_dev, uint64_t *out_dev, uint64_t n,
                                uint64_t *total_host);
nd_status nd_exclusive_scan_u32_to_u64(nd_ctx *c, const uint32_t *in_dev, uint64_t *out_dev,
                                       uint64_t n, uint64_t *total_host);

inline uint32_t nd_grid(uint64_t work, uint32_t block, uint32_t cap = 1u << 20) {
  uint64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

inline bool nd_use_te(const nd_ctx *c) {
  if (c->flags & ND_FLAG_HIER_TE) return true;
  if (c->flags & ND_FLAG_HIER_EL) return false;
  return c->s - c->r >= 2;
}
