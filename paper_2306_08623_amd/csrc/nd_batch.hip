// nd_batch.hip -- many independent graphs per call.
//
// Graphs that share (r,s) are decomposed together as one disjoint union.
// That is exact: no s-clique spans two graphs, so every count, core number
// and hierarchy component of the union is one of a single graph (Section 3
// definitions are per connected structure). Lexicographic r-clique order of
// the union lists graph 0's r-cliques first, then graph 1's, and so on (the
// union numbers vertices graph after graph), so every graph owns one
// contiguous range of union r-clique ids. A canonical tree node belongs to
// the graph of its smallest leaf; ordering the union's nodes by (graph,
// union index) keeps each graph's nodes in (level, smallest leaf) order, i.e.
// in its own canonical order.
//
// A group therefore runs the single-graph pipeline once (one persistent peel
// launch for all of its graphs), after which small kernels derive per-graph
// offsets and the numbering of tree nodes, and the results are kept in an
// arena that nd_batch_get slices.
#include "nd_internal.h"

#include <algorithm>
#include <cstring>

namespace {

struct Member {
  uint32_t n;
  uint64_t nnz;
  const uint64_t *rp;
  const uint32_t *col;
  uint64_t voff, eoff;
};

__global__ void k_gather_union(const Member *__restrict__ mem, uint32_t G, uint32_t n_total,
                               uint64_t nnz_total, uint64_t *__restrict__ rp_u,
                               uint32_t *__restrict__ col_u) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint32_t g = blockIdx.y; g < G; g += gridDim.y) {
    const Member M = mem[g];
    // a member whose row_ptr does not run from 0 to nnz, or whose columns
    // leave 0..n-1, gets entries the union's validation rejects
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < M.n; i += stride) {
      uint64_t v = M.eoff + M.rp[i];
      if (i == 0 && (M.rp[0] != 0 || M.rp[M.n] != M.nnz)) v = ND_NONE64;
      rp_u[M.voff + i] = v;
    }
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < M.nnz; j += stride) {
      const uint32_t x = M.col[j];
      col_u[M.eoff + j] = x < M.n ? x + (uint32_t)M.voff : ND_NONE;
    }
  }
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) rp_u[n_total] = nnz_total;
}

// first triangle whose smallest vertex is >= voff[g]: triangle ids are
// lexicographic, so their smallest vertices never decrease
__global__ void k_tri_offsets(uint64_t n_tri, const uint32_t *__restrict__ te,
                              const uint32_t *__restrict__ eu, const uint64_t *__restrict__ voff,
                              uint32_t G, uint64_t *__restrict__ roff) {
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g <= G; g += gridDim.x * blockDim.x) {
    const uint64_t v = voff[g];
    uint64_t lo = 0, hi = n_tri;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (eu[te[3 * mid]] < v) lo = mid + 1;
      else hi = mid;
    }
    roff[g] = lo;
  }
}

// the same from a lexicographic r-clique table (s = 5..7, r >= 2): a
// graph's r-cliques start at the first tuple whose first vertex is its own
__global__ void k_rcl_offsets(uint64_t n_r, uint32_t r, const uint32_t *__restrict__ rcl,
                              const uint64_t *__restrict__ voff, uint32_t G,
                              uint64_t *__restrict__ roff) {
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g <= G; g += gridDim.x * blockDim.x) {
    const uint64_t v = voff[g];
    uint64_t lo = 0, hi = n_r;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (rcl[mid * r] < v) lo = mid + 1;
      else hi = mid;
    }
    roff[g] = lo;
  }
}

// graph of every union node (by its smallest leaf) as a sort key
__global__ void k_node_keys(uint64_t n_int, const uint32_t *__restrict__ node_ml,
                            const uint64_t *__restrict__ roff, uint32_t G,
                            uint64_t *__restrict__ key, uint32_t *__restrict__ val) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_int;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t leaf = node_ml[i];
    uint32_t lo = 0, hi = G;   // roff[lo] <= leaf < roff[hi]
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (roff[mid] <= leaf) lo = mid;
      else hi = mid;
    }
    key[i] = ((uint64_t)lo << 32) | i;
    val[i] = (uint32_t)i;
  }
}

// first sorted position of each graph's nodes, and the local index of every
// union node
__global__ void k_node_offsets(uint64_t n_int, const uint64_t *__restrict__ skey, uint32_t G,
                               uint64_t *__restrict__ noff) {
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g <= G; g += gridDim.x * blockDim.x) {
    uint64_t lo = 0, hi = n_int;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if ((skey[mid] >> 32) < g) lo = mid + 1;
      else hi = mid;
    }
    noff[g] = lo;
  }
}

__global__ void k_node_local(uint64_t n_int, const uint64_t *__restrict__ skey,
                             const uint32_t *__restrict__ sval,
                             const uint64_t *__restrict__ noff, uint32_t *__restrict__ local) {
  for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < n_int;
       p += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t g = (uint32_t)(skey[p] >> 32);
    local[sval[p]] = (uint32_t)(p - noff[g]);
  }
}

// per graph: number of s-cliques (sum of counts / C(s,r)) and max core
__global__ void k_member_stats(uint32_t G, const uint64_t *__restrict__ roff,
                               const uint32_t *__restrict__ cnt0, const uint32_t *__restrict__ core,
                               uint64_t *__restrict__ sum_out, uint32_t *__restrict__ max_out) {
  __shared__ uint64_t s_sum[4];
  __shared__ uint32_t s_max[4];
  for (uint32_t g = blockIdx.x; g < G; g += gridDim.x) {
    uint64_t sum = 0;
    uint32_t mx = 0;
    for (uint64_t x = roff[g] + threadIdx.x; x < roff[g + 1]; x += blockDim.x) {
      sum += cnt0[x];
      mx = core[x] > mx ? core[x] : mx;
    }
    sum = wave_sum64(sum);
    for (int d = 32; d >= 1; d >>= 1) {
      uint32_t o = __shfl_xor(mx, d, 64);
      mx = o > mx ? o : mx;
    }
    if (lane_id() == 0) {
      s_sum[threadIdx.x / 64] = sum;
      s_max[threadIdx.x / 64] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t S = 0;
      uint32_t Mx = 0;
      for (uint32_t w = 0; w < blockDim.x / 64; w++) {
        S += s_sum[w];
        Mx = s_max[w] > Mx ? s_max[w] : Mx;
      }
      sum_out[g] = S;
      max_out[g] = Mx;
    }
    __syncthreads();
  }
}

// graph j's slice of the union outputs, renumbered
__global__ void k_slice_rcliques(uint64_t n_r_g, uint32_t r, const uint32_t *__restrict__ rcl,
                                 uint64_t roff, uint32_t voff, uint32_t *__restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_r_g * r;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = rcl[roff * r + i] - voff;
}

__global__ void k_slice_tree(uint64_t n_r_u, uint64_t n_r_g, uint64_t n_int_g, uint64_t roff,
                             uint64_t noff, const uint64_t *__restrict__ parent_u,
                             const uint32_t *__restrict__ level_u,
                             const uint32_t *__restrict__ sval,
                             const uint32_t *__restrict__ local, uint64_t *__restrict__ parent,
                             uint32_t *__restrict__ level) {
  const uint64_t tot = n_r_g + n_int_g;
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < tot;
       x += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t p;
    if (x < n_r_g) {
      p = parent_u[roff + x];
    } else {
      const uint32_t i = sval[noff + (x - n_r_g)];
      p = parent_u[n_r_u + i];
      if (level) level[x - n_r_g] = level_u[i];
    }
    if (parent) parent[x] = p == ND_NONE64 ? ND_NONE64 : n_r_g + local[p - n_r_u];
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

enum BatchField {
  BF_VOFF = 0, BF_ROFF, BF_NOFF, BF_RCL, BF_CNT0, BF_CORE, BF_PARENT, BF_LEVEL, BF_SVAL, BF_LOCAL
};
static_assert(BF_LOCAL < kBatchFields, "batch slots");

struct BatchGroup {
  uint32_t r = 0, s = 0;
  int slot = 0;                           // result slots of this (r,s) pair
  std::vector<uint32_t> members;          // batch indices
  uint64_t n_r = 0, n_int = 0;
  std::vector<uint64_t> voff, roff, noff; // host copies, members + 1 entries
  std::vector<uint64_t> eoff;             // CSR-slot offsets, members + 1 entries
  // union CSR packed on the host by the plan (host inputs only)
  std::vector<uint64_t> hrp;
  std::vector<uint32_t> hcol;
  // device results of the group (context slots, valid until the next batch)
  uint32_t *rcl = nullptr, *cnt0 = nullptr, *core = nullptr, *level = nullptr;
  uint64_t *parent = nullptr;
  uint32_t *sval = nullptr, *local = nullptr;
};

struct BatchState {
  std::vector<BatchGroup> groups;
  std::vector<std::pair<uint32_t, uint32_t>> loc;   // batch index -> (group, position)
  const nd_graph_desc *graphs = nullptr;            // the caller's, during execution
  nd_mem where = ND_MEM_HOST;
};

void nd_batch_release(nd_ctx *c) {
  delete c->batch;
  c->batch = nullptr;
}

void nd_batch_state_free(BatchState *bs) { delete bs; }

static nd_status run_group(nd_ctx *c, int gi, BatchGroup &B, const nd_graph_desc *graphs,
                           nd_mem where, nd_graph_result *results) {
  nd_status st = ND_OK;
  const uint32_t G = (uint32_t)B.members.size();
  const std::vector<uint64_t> &eoff = B.eoff;
  const uint64_t n_tot = B.voff[G], nnz_tot = eoff[G];
  uint64_t *rp = (uint64_t *)nd_buf(c, B_RP, (n_tot + 1) * 8, &st);
  if (!rp) return st;
  uint32_t *col = (uint32_t *)nd_buf(c, B_COL, std::max<uint64_t>(nnz_tot, 1) * 4, &st);
  if (!col) return st;
  if (where == ND_MEM_DEVICE) {
    std::vector<Member> hm(G);
    for (uint32_t j = 0; j < G; j++) {
      const nd_graph_desc &d = graphs[B.members[j]];
      hm[j] = Member{d.n, d.nnz, d.row_ptr, d.col, B.voff[j], eoff[j]};
    }
    Member *dm = (Member *)nd_buf(c, B_BATCHDESC, G * sizeof(Member), &st);
    if (!dm) return st;
    if ((st = nd_hip(c, hipMemcpyAsync(dm, hm.data(), G * sizeof(Member), hipMemcpyHostToDevice,
                                       c->stream),
                     "batch descriptors")) != ND_OK)
      return st;
    hipLaunchKernelGGL(k_gather_union, dim3(16, std::min<uint32_t>(G, 8192)), dim3(256), 0,
                       c->stream, dm, G, (uint32_t)n_tot, nnz_tot, rp, col);
    if ((st = nd_hip(c, hipGetLastError(), "union gather")) != ND_OK) return st;
    // the descriptor upload reads pageable host memory
    if ((st = nd_hip(c, hipStreamSynchronize(c->stream), "union gather")) != ND_OK) return st;
  } else {
    if ((st = nd_hip(c, hipMemcpyAsync(rp, B.hrp.data(), (n_tot + 1) * 8, hipMemcpyHostToDevice,
                                       c->stream),
                     "union row_ptr")) != ND_OK)
      return st;
    if (nnz_tot && (st = nd_hip(c, hipMemcpyAsync(col, B.hcol.data(), nnz_tot * 4,
                                                  hipMemcpyHostToDevice, c->stream),
                                "union col")) != ND_OK)
      return st;
    if ((st = nd_hip(c, hipStreamSynchronize(c->stream), "union upload")) != ND_OK) return st;
    std::vector<uint64_t>().swap(B.hrp);
    std::vector<uint32_t>().swap(B.hcol);
  }
  c->n = (uint32_t)n_tot;
  c->nnz = nnz_tot;
  c->m = nnz_tot / 2;
  c->r = B.r;
  c->s = B.s;
  c->have_graph = true;
  if (c->validate && (st = nd_validate_loaded(c)) != ND_OK) return st;
  c->in_batch = true;
  st = nd_run_pipeline(c);
  c->in_batch = false;
  if (st != ND_OK) return st;

  // ---- per-graph offsets of r-cliques
  const uint64_t n_r = c->n_r, n_int = c->n_int;
  B.n_r = n_r;
  B.n_int = n_int;
  auto slot = [&](int field, size_t bytes) { return nd_buf(c, nd_batch_slot(gi, field), bytes, &st); };
  uint64_t *d_voff = (uint64_t *)slot(BF_VOFF, (G + 1) * 8);
  if (!d_voff) return st;
  uint64_t *d_roff = (uint64_t *)slot(BF_ROFF, (G + 1) * 8);
  if (!d_roff) return st;
  uint64_t *d_noff = (uint64_t *)slot(BF_NOFF, (G + 1) * 8);
  if (!d_noff) return st;
  B.rcl = (uint32_t *)slot(BF_RCL, n_r * B.r * 4);
  if (!B.rcl) return st;
  B.cnt0 = (uint32_t *)slot(BF_CNT0, n_r * 4);
  if (!B.cnt0) return st;
  B.core = (uint32_t *)slot(BF_CORE, n_r * 4);
  if (!B.core) return st;
  B.parent = (uint64_t *)slot(BF_PARENT, (n_r + n_int) * 8);
  if (!B.parent) return st;
  B.level = (uint32_t *)slot(BF_LEVEL, n_int * 4);
  if (!B.level) return st;
  B.sval = (uint32_t *)slot(BF_SVAL, n_int * 4);
  if (!B.sval) return st;
  B.local = (uint32_t *)slot(BF_LOCAL, n_int * 4);
  if (!B.local) return st;
  if ((st = nd_hip(c, hipMemcpyAsync(d_voff, B.voff.data(), (G + 1) * 8, hipMemcpyHostToDevice,
                                     c->stream),
                   "voff")) != ND_OK)
    return st;
  B.roff.assign(G + 1, 0);
  if (B.r == 1) {
    B.roff = B.voff;
  } else if (B.r == 2) {
    for (uint32_t j = 0; j <= G; j++) B.roff[j] = eoff[j] / 2;
  }
  if (B.r >= 3) {
    if (c->gv.rcl)
      hipLaunchKernelGGL(k_rcl_offsets, dim3(nd_grid(G + 1, 256, 1024)), dim3(256), 0, c->stream,
                         n_r, B.r, c->gv.rcl, d_voff, G, d_roff);
    else
      hipLaunchKernelGGL(k_tri_offsets, dim3(nd_grid(G + 1, 256, 1024)), dim3(256), 0, c->stream,
                         n_r, c->gv.te, c->gv.eu, d_voff, G, d_roff);
    if ((st = nd_hip(c, hipMemcpyAsync(B.roff.data(), d_roff, (G + 1) * 8, hipMemcpyDeviceToHost,
                                       c->stream),
                     "roff")) != ND_OK)
      return st;
  } else if ((st = nd_hip(c, hipMemcpyAsync(d_roff, B.roff.data(), (G + 1) * 8,
                                            hipMemcpyHostToDevice, c->stream),
                          "roff")) != ND_OK) {
    return st;
  }
  // ---- group copies of the union results
  if ((st = nd_write_rcliques(c, c->gv, B.rcl)) != ND_OK) return st;
  if (n_r) {
    if ((st = nd_hip(c, hipMemcpyAsync(B.cnt0, c->bufs[B_CNT0].p, n_r * 4,
                                       hipMemcpyDeviceToDevice, c->stream), "cnt0")) != ND_OK ||
        (st = nd_hip(c, hipMemcpyAsync(B.core, c->bufs[B_CNT].p, n_r * 4,
                                       hipMemcpyDeviceToDevice, c->stream), "core")) != ND_OK ||
        (st = nd_hip(c, hipMemcpyAsync(B.parent, c->bufs[B_PARENT].p, (n_r + n_int) * 8,
                                       hipMemcpyDeviceToDevice, c->stream), "parent")) != ND_OK)
      return st;
  }
  // ---- nodes grouped by graph (stable), local numbering
  B.noff.assign(G + 1, 0);
  if (n_int) {
    if ((st = nd_hip(c, hipMemcpyAsync(B.level, c->bufs[B_LEVEL].p, n_int * 4,
                                       hipMemcpyDeviceToDevice, c->stream), "level")) != ND_OK)
      return st;
    uint64_t *k0 = (uint64_t *)nd_buf(c, B_SORTK0, n_int * 8, &st);
    if (!k0) return st;
    uint64_t *k1 = (uint64_t *)nd_buf(c, B_SORTK1, n_int * 8, &st);
    if (!k1) return st;
    uint32_t *v0 = (uint32_t *)nd_buf(c, B_SORTV0, n_int * 4, &st);
    if (!v0) return st;
    uint32_t *v1 = (uint32_t *)nd_buf(c, B_SORTV1, n_int * 4, &st);
    if (!v1) return st;
    const uint32_t *node_ml = (const uint32_t *)c->bufs[B_NODEML].p;
    hipLaunchKernelGGL(k_node_keys, dim3(nd_grid(n_int, 256, 16384)), dim3(256), 0, c->stream,
                       n_int, node_ml, d_roff, G, k0, v0);
    uint32_t gbits = 1;
    while (gbits < 32 && (1ull << gbits) <= G) gbits++;
    uint64_t *ks = nullptr;
    uint32_t *vs = nullptr;
    if ((st = nd_sort_pairs_u64(c, k0, v0, k1, v1, n_int, 32 + gbits, &ks, &vs)) != ND_OK)
      return st;
    hipLaunchKernelGGL(k_node_offsets, dim3(nd_grid(G + 1, 256, 1024)), dim3(256), 0, c->stream,
                       n_int, ks, G, d_noff);
    hipLaunchKernelGGL(k_node_local, dim3(nd_grid(n_int, 256, 16384)), dim3(256), 0, c->stream,
                       n_int, ks, vs, d_noff, B.local);
    if ((st = nd_hip(c, hipMemcpyAsync(B.sval, vs, n_int * 4, hipMemcpyDeviceToDevice,
                                       c->stream), "sval")) != ND_OK ||
        (st = nd_hip(c, hipMemcpyAsync(B.noff.data(), d_noff, (G + 1) * 8,
                                       hipMemcpyDeviceToHost, c->stream), "noff")) != ND_OK)
      return st;
  }
  // ---- per-graph counts and levels
  uint64_t *d_sum = (uint64_t *)nd_buf(c, B_TMP64, G * 8 + 8, &st);
  if (!d_sum) return st;
  uint32_t *d_max = (uint32_t *)nd_buf(c, B_TMP32D, G * 4 + 4, &st);
  if (!d_max) return st;
  hipLaunchKernelGGL(k_member_stats, dim3(std::min<uint32_t>(G, 4096)), dim3(256), 0, c->stream,
                     G, d_roff, B.cnt0, B.core, d_sum, d_max);
  std::vector<uint64_t> hsum(G);
  std::vector<uint32_t> hmax(G);
  if ((st = nd_hip(c, hipGetLastError(), "batch group kernels")) != ND_OK ||
      (st = nd_hip(c, hipMemcpyAsync(hsum.data(), d_sum, G * 8, hipMemcpyDeviceToHost, c->stream),
                   "member sums")) != ND_OK ||
      (st = nd_hip(c, hipMemcpyAsync(hmax.data(), d_max, G * 4, hipMemcpyDeviceToHost, c->stream),
                   "member max")) != ND_OK)
    return st;
  if ((st = nd_hip(c, hipStreamSynchronize(c->stream), "batch group")) != ND_OK) return st;
  uint64_t csr = 1;   // C(s, r)
  for (uint32_t i = 0; i < B.r; i++) csr = csr * (B.s - i) / (i + 1);
  for (uint32_t j = 0; j < G; j++) {
    nd_graph_result &R = results[B.members[j]];
    R.status = ND_OK;
    R.n_r = B.roff[j + 1] - B.roff[j];
    R.n_int = B.noff[j + 1] - B.noff[j];
    R.n_s = hsum[j] / csr;
    R.k = hmax[j];
  }
  return ND_OK;
}

static void add_info(nd_info &T, const nd_info &I) {
  T.n += I.n;
  T.m += I.m;
  T.n_r += I.n_r;
  T.n_s += I.n_s;
  T.k = std::max(T.k, I.k);
  T.rounds += I.rounds;
  T.n_int += I.n_int;
  T.visits += I.visits;
  T.decrements += I.decrements;
  T.links += I.links;
  T.link_calls += I.link_calls;
  T.unites += I.unites;
  T.bucket_scans += I.bucket_scans;
  T.max_outdeg = std::max(T.max_outdeg, I.max_outdeg);
  T.orient_rounds += I.orient_rounds;
  T.ms_prep += I.ms_prep;
  T.ms_count += I.ms_count;
  T.ms_peel += I.ms_peel;
  T.ms_tree += I.ms_tree;
  T.ms_count_kernel += I.ms_count_kernel;
  T.ms_peel_kernel += I.ms_peel_kernel;
  T.hier_te |= I.hier_te;
  T.ms_hier += I.ms_hier;
  T.hier_visits += I.hier_visits;
  T.grid_retries += I.grid_retries;
  T.cascades += I.cascades;
  T.cas_retries += I.cas_retries;
  T.device_peak = std::max(T.device_peak, I.device_peak);
}

// Host half of a batch: checks, grouping by (r,s) and, for host inputs, the
// union CSRs packed on the host. Needs no device.
nd_status nd_batch_plan(uint32_t G, const nd_graph_desc *graphs, nd_mem where,
                        nd_graph_result *results, BatchState **out, std::string *err) {
  *out = nullptr;
  if (G && (!graphs || !results)) {
    *err = "NULL graph descriptors or results";
    return ND_E_INVALID_ARG;
  }
  if (where != ND_MEM_HOST && where != ND_MEM_DEVICE) {
    *err = "bad memory kind";
    return ND_E_INVALID_ARG;
  }
  for (uint32_t i = 0; i < G; i++) results[i] = nd_graph_result{};
  BatchState *bs = new BatchState();
  bs->loc.resize(G);
  bs->where = where;
  auto fail_graph = [&](uint32_t i, nd_status code, const char *what) {
    delete bs;
    results[i].status = code;
    *err = "graph " + std::to_string(i) + ": " + what;
    return code;
  };
  bool present[kBatchGroups] = {};
  for (uint32_t i = 0; i < G; i++) {
    const nd_graph_desc &d = graphs[i];
    if (d.r < 1 || d.s <= d.r) return fail_graph(i, ND_E_INVALID_ARG, "need 1 <= r < s");
    if (!nd_rs_supported(d.r, d.s))
      return fail_graph(i, ND_E_UNSUPPORTED, "this (r,s) pair is not built");
    if (!d.row_ptr || (d.nnz && !d.col))
      return fail_graph(i, ND_E_INVALID_ARG, "NULL row_ptr or col");
    if (d.nnz & 1) return fail_graph(i, ND_E_BAD_GRAPH, "nnz is odd");
    if (d.n == 0 && d.nnz) return fail_graph(i, ND_E_BAD_GRAPH, "edges without vertices");
    if (where == ND_MEM_HOST && (d.row_ptr[0] != 0 || d.row_ptr[d.n] != d.nnz))
      return fail_graph(i, ND_E_BAD_GRAPH, "row_ptr[0] must be 0 and row_ptr[n] must be nnz");
    // groups in the fixed order of nd_rs_index: each pair keeps its own
    // result slots from one batch to the next
    const int pi = nd_rs_index(d.r, d.s);
    present[pi] = true;
    bs->loc[i] = {(uint32_t)pi, 0};
  }
  uint32_t gidx[kBatchGroups];
  for (uint32_t p = 0; p < (uint32_t)kBatchGroups; p++) {
    gidx[p] = (uint32_t)bs->groups.size();
    if (present[p]) {
      bs->groups.emplace_back();
      for (uint32_t s = 2; s <= kMaxS; s++)
        for (uint32_t r = 1; r < s; r++)
          if (nd_rs_index(r, s) == (int)p) {
            bs->groups.back().r = r;
            bs->groups.back().s = s;
          }
      bs->groups.back().slot = (int)p;
    }
  }
  for (uint32_t i = 0; i < G; i++) {
    const uint32_t g = gidx[bs->loc[i].first];
    bs->loc[i] = {g, (uint32_t)bs->groups[g].members.size()};
    bs->groups[g].members.push_back(i);
  }
  for (BatchGroup &B : bs->groups) {
    const uint32_t M = (uint32_t)B.members.size();
    B.voff.assign(M + 1, 0);
    B.eoff.assign(M + 1, 0);
    for (uint32_t j = 0; j < M; j++) {
      const nd_graph_desc &d = graphs[B.members[j]];
      B.voff[j + 1] = B.voff[j] + d.n;
      B.eoff[j + 1] = B.eoff[j] + d.nnz;
    }
    const uint64_t n_tot = B.voff[M], nnz_tot = B.eoff[M];
    if (n_tot >= 0xFFFFFFFFull || nnz_tot / 2 >= 0xFFFFFFFFull) {
      for (uint32_t i : B.members) results[i].status = ND_E_UNSUPPORTED;
      delete bs;
      *err = "a batch group exceeds 32-bit vertex or edge ids";
      return ND_E_UNSUPPORTED;
    }
    if (where == ND_MEM_HOST) {
      // members whose columns leave 0..n-1 get entries the validation rejects
      B.hrp.resize(n_tot + 1);
      B.hcol.resize(std::max<uint64_t>(nnz_tot, 1));
      for (uint32_t j = 0; j < M; j++) {
        const nd_graph_desc &d = graphs[B.members[j]];
        for (uint32_t u = 0; u < d.n; u++) B.hrp[B.voff[j] + u] = B.eoff[j] + d.row_ptr[u];
        const uint32_t vo = (uint32_t)B.voff[j];
        uint32_t *dst = B.hcol.data() + B.eoff[j];
        for (uint64_t x = 0; x < d.nnz; x++) dst[x] = d.col[x] < d.n ? d.col[x] + vo : ND_NONE;
      }
      B.hrp[n_tot] = nnz_tot;
    }
  }
  *out = bs;
  return ND_OK;
}

// Device half: takes ownership of the plan (kept as the context's batch on
// success). `graphs` must be the descriptors the plan was made from.
nd_status nd_batch_execute(nd_ctx *c, BatchState *bs, const nd_graph_desc *graphs,
                           nd_graph_result *results) {
  nd_status st = nd_hip(c, hipSetDevice(c->device), "hipSetDevice");
  nd_batch_release(c);
  c->have_graph = false;
  c->decomposed = false;
  c->info_valid = false;
  if (st != ND_OK) {
    delete bs;
    return st;
  }
  c->batch = bs;
  nd_info total{};
  for (size_t g = 0; g < bs->groups.size(); g++) {
    BatchGroup &B = bs->groups[g];
    st = run_group(c, B.slot, B, graphs, bs->where, results);
    if (st != ND_OK) {
      for (uint32_t i : B.members) results[i].status = st;
      nd_batch_release(c);
      c->have_graph = false;
      c->decomposed = false;
      return st;
    }
    add_info(total, c->info);
  }
  // the context's own graph buffers now hold the last group's union: the
  // single-graph getters are invalid until the next nd_load_csr
  c->have_graph = false;
  c->decomposed = false;
  total.r = bs->groups.size() == 1 ? bs->groups[0].r : 0;
  total.s = bs->groups.size() == 1 ? bs->groups[0].s : 0;
  total.device_bytes = c->bytes_held;
  c->info = total;
  c->info_valid = true;
  return ND_OK;
}

extern "C" {

nd_status nd_batch_decompose(nd_ctx *c, uint32_t G, const nd_graph_desc *graphs, nd_mem where,
                             nd_graph_result *results) {
  if (!c) return ND_E_INVALID_ARG;
  c->last_error.clear();
  if (c->approx_delta > 0)
    return nd_fail(c, ND_E_UNSUPPORTED,
                   "batches peel exactly: the approximate rounds of a union are not those of "
                   "its graphs (nd_set_approx(ctx, 0) first)");
  nd_batch_release(c);
  c->have_graph = false;
  c->decomposed = false;
  c->info_valid = false;
  BatchState *bs = nullptr;
  std::string err;
  nd_status st = nd_batch_plan(G, graphs, where, results, &bs, &err);
  if (st != ND_OK) return nd_fail(c, st, err);
  return nd_batch_execute(c, bs, graphs, results);
}

nd_status nd_batch_get(nd_ctx *c, uint32_t i, uint32_t *rcliques, uint32_t *counts,
                       uint32_t *coreness, uint64_t *parent, uint32_t *level, nd_mem where) {
  if (!c) return ND_E_INVALID_ARG;
  if (!c->batch || i >= c->batch->loc.size())
    return nd_fail(c, ND_E_STATE, "no such graph in the last batch");
  if (where != ND_MEM_HOST && where != ND_MEM_DEVICE)
    return nd_fail(c, ND_E_INVALID_ARG, "bad memory kind");
  nd_status st = nd_hip(c, hipSetDevice(c->device), "hipSetDevice");
  if (st != ND_OK) return st;
  const BatchGroup &B = c->batch->groups[c->batch->loc[i].first];
  const uint32_t j = c->batch->loc[i].second;
  const uint64_t roff = B.roff[j], n_r = B.roff[j + 1] - roff;
  const uint64_t noff = B.noff[j], n_int = B.noff[j + 1] - noff;
  const hipMemcpyKind kind = where == ND_MEM_HOST ? hipMemcpyDeviceToHost
                                                  : hipMemcpyDeviceToDevice;
  if (rcliques && n_r) {
    uint32_t *dst = rcliques;
    if (where == ND_MEM_HOST && !(dst = (uint32_t *)nd_buf(c, B_RCL, n_r * B.r * 4, &st)))
      return st;
    hipLaunchKernelGGL(k_slice_rcliques, dim3(nd_grid(n_r * B.r, 256, 16384)), dim3(256), 0,
                       c->stream, n_r, B.r, B.rcl, roff, (uint32_t)B.voff[j], dst);
    if (where == ND_MEM_HOST &&
        (st = nd_hip(c, hipMemcpyAsync(rcliques, dst, n_r * B.r * 4, kind, c->stream),
                     "rcliques out")) != ND_OK)
      return st;
  }
  if (counts && n_r &&
      (st = nd_hip(c, hipMemcpyAsync(counts, B.cnt0 + roff, n_r * 4, kind, c->stream),
                   "counts out")) != ND_OK)
    return st;
  if (coreness && n_r &&
      (st = nd_hip(c, hipMemcpyAsync(coreness, B.core + roff, n_r * 4, kind, c->stream),
                   "coreness out")) != ND_OK)
    return st;
  if (parent && n_r) {
    uint64_t *dp = parent;
    uint32_t *dl = (level && n_int) ? level : nullptr;
    if (where == ND_MEM_HOST) {
      if (!(dp = (uint64_t *)nd_buf(c, B_SORTK1, (n_r + n_int) * 8, &st))) return st;
      if (dl && !(dl = (uint32_t *)nd_buf(c, B_SORTV1, n_int * 4, &st))) return st;
    }
    hipLaunchKernelGGL(k_slice_tree, dim3(nd_grid(n_r + n_int, 256, 16384)), dim3(256), 0,
                       c->stream, B.n_r, n_r, n_int, roff, noff, B.parent, B.level, B.sval,
                       B.local, dp, dl);
    if (where == ND_MEM_HOST) {
      if ((st = nd_hip(c, hipMemcpyAsync(parent, dp, (n_r + n_int) * 8, kind, c->stream),
                       "parent out")) != ND_OK)
        return st;
      if (dl && (st = nd_hip(c, hipMemcpyAsync(level, dl, n_int * 4, kind, c->stream),
                             "level out")) != ND_OK)
        return st;
    }
  } else if (level && n_int) {
    uint32_t *dl = level;
    if (where == ND_MEM_HOST && !(dl = (uint32_t *)nd_buf(c, B_SORTV1, n_int * 4, &st)))
      return st;
    hipLaunchKernelGGL(k_slice_tree, dim3(nd_grid(n_r + n_int, 256, 16384)), dim3(256), 0,
                       c->stream, B.n_r, n_r, n_int, roff, noff, B.parent, B.level, B.sval,
                       B.local, (uint64_t *)nullptr, dl);
    if (where == ND_MEM_HOST &&
        (st = nd_hip(c, hipMemcpyAsync(level, dl, n_int * 4, kind, c->stream), "level out")) !=
            ND_OK)
      return st;
  }
  if ((st = nd_hip(c, hipGetLastError(), "batch slice")) != ND_OK) return st;
  return nd_hip(c, hipStreamSynchronize(c->stream), "batch get");
}

}  // extern "C"
