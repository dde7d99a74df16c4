// nd_cut.hip -- hierarchy cut: the c-(r,s) nuclei of the last decomposition,
// read off the canonical tree (Section 8, on the usefulness of the
// hierarchy). Dropping every tree node of level below c leaves maximal
// subtrees whose roots are the nodes of level >= c with no parent of level
// >= c; each such subtree is one c-(r,s) nucleus and holds all of its
// leaves (an r-clique of core >= 1 has as parent the node of its own core
// number, so every r-clique of core >= c lands in exactly one nucleus).
//
//   1. top[x]: for every internal node of level >= c, its parent while that
//      parent's level is >= c, then pointer jumping until every entry names
//      a cut root; cut roots are numbered in node order.
//   2. every r-clique takes the nucleus of its parent node; its vertices
//      become (nucleus << 32 | vertex) keys, radix-sorted and deduplicated
//      into the nuclei's vertex sets.
//   3. one wave per (nucleus, vertex) entry counts the neighbours w > v of
//      the vertex that lie in the same vertex set (binary search): the edges
//      of the graph induced on the nucleus's vertices.
#include "nd_internal.h"

#include <algorithm>

namespace {

constexpr uint32_t kCB = 256;

__global__ void k_cut_top(uint64_t n_r, uint64_t n_int, uint32_t c,
                          const uint64_t *__restrict__ parent, const uint32_t *__restrict__ level,
                          uint32_t *__restrict__ top) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n_int;
       x += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t t = ND_NONE;
    if (level[x] >= c) {
      const uint64_t p = parent[n_r + x];
      // a parent's level is below its child's: p < n_r + x in node order
      t = (p == ND_NONE64 || level[p - n_r] < c) ? (uint32_t)x : (uint32_t)(p - n_r);
    }
    top[x] = t;
  }
}

// one round of pointer jumping toward the cut roots; *changed counts moves
__global__ void k_cut_jump(uint64_t n_int, uint32_t *top, uint32_t *changed) {
  uint32_t moved = 0;
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n_int;
       x += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t t = top[x];
    if (t == ND_NONE) continue;
    const uint32_t tt = top[t];
    if (tt != t) {
      top[x] = tt;
      moved = 1;
    }
  }
  if (__popcll(ballot64(moved != 0)) && lane_id() == 0) atomicAdd(changed, 1u);
}

__global__ void k_cut_rootflag(uint64_t n_int, const uint32_t *__restrict__ top,
                               uint32_t *__restrict__ flag) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n_int;
       x += (uint64_t)gridDim.x * blockDim.x)
    flag[x] = top[x] == (uint32_t)x;
}

__global__ void k_cut_nuclei(uint64_t n_r, uint64_t n_int, const uint32_t *__restrict__ top,
                             const uint64_t *__restrict__ pos, const uint32_t *__restrict__ level,
                             const uint32_t *__restrict__ node_ml, nd_nucleus *__restrict__ nuc) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n_int;
       x += (uint64_t)gridDim.x * blockDim.x) {
    if (top[x] != (uint32_t)x) continue;
    nd_nucleus q;
    q.node = n_r + x;
    q.min_leaf = node_ml[x];
    q.n_rcliques = 0;
    q.n_vertices = 0;
    q.n_edges = 0;
    q.vert_off = 0;
    q.level = level[x];
    q.reserved = 0;
    nuc[pos[x]] = q;
  }
}

// Groups the active lanes of a wave by key; the lowest lane of a group gets
// the group's size (the others 0), so one atomic per group and wave
// suffices when a few nuclei hold most r-cliques.
__device__ __forceinline__ uint32_t group_count(uint32_t key, bool active) {
  const uint32_t lane = lane_id();
  uint64_t pending = ballot64(active);
  uint32_t count = 0;
  while (pending) {
    const uint32_t leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t k = __shfl(key, leader, 64);
    const uint64_t same = ballot64(active && key == k);
    if (lane == leader) count = __popcll(same);
    pending &= ~same;
  }
  return count;
}

__global__ void k_cut_leaves(uint64_t n_r, uint32_t r, const uint64_t *__restrict__ parent,
                             const uint32_t *__restrict__ top, const uint64_t *__restrict__ pos,
                             const uint32_t *__restrict__ rcl, uint32_t *__restrict__ leaf_nuc,
                             nd_nucleus *__restrict__ nuc, uint64_t *__restrict__ keys,
                             uint32_t *__restrict__ nkeys) {
  for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x; base < n_r;
       base += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t R = base + threadIdx.x;
    uint32_t id = ND_NONE;
    if (R < n_r) {
      const uint64_t p = parent[R];
      if (p != ND_NONE64) {
        const uint32_t t = top[p - n_r];
        if (t != ND_NONE) id = (uint32_t)pos[t];
      }
      leaf_nuc[R] = id;
    }
    const bool in = id != ND_NONE;
    const uint32_t cnt = group_count(id, in);
    if (cnt) atomicAdd((unsigned long long *)&nuc[id].n_rcliques, (unsigned long long)cnt);
    for (uint32_t j = 0; j < r; j++) {
      const uint32_t slot = wave_append(nkeys, in);
      if (in) keys[slot] = ((uint64_t)id << 32) | rcl[R * r + j];
    }
  }
}

__global__ void k_cut_uniqflag(uint64_t n, const uint64_t *__restrict__ k,
                               uint32_t *__restrict__ flag) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    flag[i] = (i == 0 || k[i] != k[i - 1]) ? 1u : 0u;
}

__global__ void k_cut_compact(uint64_t n, const uint64_t *__restrict__ k,
                              const uint32_t *__restrict__ flag, const uint64_t *__restrict__ pos,
                              uint32_t *__restrict__ verts, uint32_t *__restrict__ vnuc) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    if (!flag[i]) continue;
    verts[pos[i]] = (uint32_t)k[i];
    vnuc[pos[i]] = (uint32_t)(k[i] >> 32);
  }
}

// vertex sets are contiguous and ordered by nucleus: their starts, then
// (after all starts are written) their sizes
__global__ void k_cut_starts(uint64_t n, const uint32_t *__restrict__ vnuc,
                             nd_nucleus *__restrict__ nuc) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    if (i == 0 || vnuc[i] != vnuc[i - 1]) nuc[vnuc[i]].vert_off = i;
}

__global__ void k_cut_sizes(uint64_t n, const uint32_t *__restrict__ vnuc,
                            nd_nucleus *__restrict__ nuc) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    if (i + 1 == n || vnuc[i + 1] != vnuc[i]) nuc[vnuc[i]].n_vertices = i + 1 - nuc[vnuc[i]].vert_off;
}

// one wave per (nucleus, vertex v) entry: neighbours w > v of v found in
// the nucleus's sorted vertex set
__global__ void k_cut_edges(uint64_t n, const uint32_t *__restrict__ verts,
                            const uint32_t *__restrict__ vnuc, nd_nucleus *__restrict__ nuc,
                            const uint64_t *__restrict__ rp, const uint32_t *__restrict__ col) {
  const uint32_t lane = lane_id();
  const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
  for (uint64_t i = blockIdx.x * (uint64_t)(blockDim.x / 64) + threadIdx.x / 64; i < n;
       i += waves) {
    const uint32_t v = verts[i], id = vnuc[i];
    const uint64_t lo = nuc[id].vert_off, hi = lo + nuc[id].n_vertices;
    const uint64_t b = rp[v], e = rp[v + 1];
    uint64_t cnt = 0;
    for (uint64_t j = b + lane; j < e; j += 64) {
      const uint32_t w = col[j];
      if (w <= v) continue;
      if (find_u32<uint64_t>(verts, lo, hi, w) != hi) cnt++;
    }
    cnt = wave_sum64(cnt);
    if (lane == 0 && cnt) atomicAdd((unsigned long long *)&nuc[id].n_edges, (unsigned long long)cnt);
  }
}

uint32_t cut_bits(uint64_t v) {
  uint32_t b = 0;
  while (b < 64 && (v >> b) != 0) b++;
  return b;
}

}  // namespace

extern "C" {

nd_status nd_cut(nd_ctx *c, uint32_t level_c, uint64_t *n_nuclei, uint64_t *n_vertices) {
  if (!c) return ND_E_INVALID_ARG;
  nd_status st = nd_hip(c, hipSetDevice(c->device), "hipSetDevice");
  if (st != ND_OK) return st;
  c->cut_valid = false;
  if (!c->decomposed) return nd_fail(c, ND_E_STATE, "no decomposition result");
  if (level_c < 1) return nd_fail(c, ND_E_INVALID_ARG, "the cut level c must be at least 1");
  const uint64_t nr = c->n_r, ni = c->n_int;
  uint64_t N = 0, U = 0;
  if (ni) {
    const uint64_t *parent = (const uint64_t *)c->bufs[B_PARENT].p;
    const uint32_t *level = (const uint32_t *)c->bufs[B_LEVEL].p;
    const uint32_t *node_ml = (const uint32_t *)c->bufs[B_NODEML].p;
    uint32_t *top = (uint32_t *)nd_buf(c, B_CUT_TOP, ni * 4, &st);
    if (!top) return st;
    uint32_t *cnt = (uint32_t *)nd_buf(c, B_CUT_CNT, 8, &st);
    if (!cnt) return st;
    const uint32_t gi = nd_grid(ni, kCB, 16384);
    hipLaunchKernelGGL(k_cut_top, dim3(gi), dim3(kCB), 0, c->stream, nr, ni, level_c, parent,
                       level, top);
    // pointer jumping: each round halves the remaining chain lengths
    for (int round = 0;; round++) {
      if (round > 64) return nd_fail(c, ND_E_WATCHDOG, "cut: pointer jumping did not settle");
      uint32_t moved = 0;
      if ((st = nd_hip(c, hipMemsetAsync(cnt, 0, 4, c->stream), "cut jump")) != ND_OK) return st;
      hipLaunchKernelGGL(k_cut_jump, dim3(gi), dim3(kCB), 0, c->stream, ni, top, cnt);
      if ((st = nd_hip(c, hipMemcpyAsync(&moved, cnt, 4, hipMemcpyDeviceToHost, c->stream),
                       "cut jump")) != ND_OK ||
          (st = nd_hip(c, hipStreamSynchronize(c->stream), "cut jump")) != ND_OK)
        return st;
      if (!moved) break;
    }
    uint32_t *flag = (uint32_t *)nd_buf(c, B_CUT_FLAG, ni * 4, &st);
    if (!flag) return st;
    uint64_t *pos = (uint64_t *)nd_buf(c, B_CUT_POS, (ni + 1) * 8, &st);
    if (!pos) return st;
    hipLaunchKernelGGL(k_cut_rootflag, dim3(gi), dim3(kCB), 0, c->stream, ni, top, flag);
    if ((st = nd_exclusive_scan_u32_to_u64(c, flag, pos, ni, &N)) != ND_OK) return st;
  }
  if (N) {
    const uint32_t *level = (const uint32_t *)c->bufs[B_LEVEL].p;
    const uint32_t *node_ml = (const uint32_t *)c->bufs[B_NODEML].p;
    const uint64_t *parent = (const uint64_t *)c->bufs[B_PARENT].p;
    const uint32_t *top = (const uint32_t *)c->bufs[B_CUT_TOP].p;
    const uint64_t *pos = (const uint64_t *)c->bufs[B_CUT_POS].p;
    uint32_t *cnt = (uint32_t *)c->bufs[B_CUT_CNT].p;
    nd_nucleus *nuc = (nd_nucleus *)nd_buf(c, B_CUT_NUC, N * sizeof(nd_nucleus), &st);
    if (!nuc) return st;
    uint32_t *leaf = (uint32_t *)nd_buf(c, B_CUT_LEAF, nr * 4, &st);
    if (!leaf) return st;
    uint32_t *rcl = (uint32_t *)nd_buf(c, B_CUT_RCL, nr * c->r * 4ull, &st);
    if (!rcl) return st;
    const uint64_t maxk = nr * c->r;
    uint64_t *k0 = (uint64_t *)nd_buf(c, B_CUT_K0, maxk * 8, &st);
    if (!k0) return st;
    hipLaunchKernelGGL(k_cut_nuclei, dim3(nd_grid(ni, kCB, 16384)), dim3(kCB), 0, c->stream, nr,
                       ni, top, pos, level, node_ml, nuc);
    if ((st = nd_write_rcliques(c, c->gv, rcl)) != ND_OK) return st;
    if ((st = nd_hip(c, hipMemsetAsync(cnt, 0, 4, c->stream), "cut keys")) != ND_OK) return st;
    hipLaunchKernelGGL(k_cut_leaves, dim3(nd_grid(nr, kCB, 16384)), dim3(kCB), 0, c->stream, nr,
                       c->r, parent, top, pos, rcl, leaf, nuc, k0, cnt);
    uint32_t nk = 0;
    if ((st = nd_hip(c, hipMemcpyAsync(&nk, cnt, 4, hipMemcpyDeviceToHost, c->stream),
                     "cut keys")) != ND_OK ||
        (st = nd_hip(c, hipStreamSynchronize(c->stream), "cut keys")) != ND_OK)
      return st;
    const uint64_t np = nk;
    uint64_t *k1 = (uint64_t *)nd_buf(c, B_CUT_K1, std::max<uint64_t>(np, 1) * 8, &st);
    if (!k1) return st;
    uint32_t *v0 = (uint32_t *)nd_buf(c, B_CUT_V0, std::max<uint64_t>(np, 1) * 4, &st);
    if (!v0) return st;
    uint32_t *v1 = (uint32_t *)nd_buf(c, B_CUT_V1, std::max<uint64_t>(np, 1) * 4, &st);
    if (!v1) return st;
    if ((st = nd_hip(c, hipMemsetAsync(v0, 0, std::max<uint64_t>(np, 1) * 4, c->stream),
                     "cut values")) != ND_OK)
      return st;
    uint64_t *ks = nullptr;
    uint32_t *vs = nullptr;
    // keys: nucleus in bits 32 and up, vertex id below
    const uint32_t nbits = std::max<uint32_t>(1, cut_bits(N - 1));
    if ((st = nd_sort_pairs_u64(c, k0, v0, k1, v1, np, 32 + nbits, &ks, &vs)) != ND_OK) return st;
    uint32_t *flag = (uint32_t *)nd_buf(c, B_CUT_FLAG, std::max<uint64_t>(np, 1) * 4, &st);
    if (!flag) return st;
    uint64_t *pos2 = (uint64_t *)nd_buf(c, B_CUT_POS2, (np + 1) * 8, &st);
    if (!pos2) return st;
    const uint32_t gp = nd_grid(np, kCB, 16384);
    hipLaunchKernelGGL(k_cut_uniqflag, dim3(gp), dim3(kCB), 0, c->stream, np, ks, flag);
    if ((st = nd_exclusive_scan_u32_to_u64(c, flag, pos2, np, &U)) != ND_OK) return st;
    uint32_t *verts = (uint32_t *)nd_buf(c, B_CUT_VERTS, std::max<uint64_t>(U, 1) * 4, &st);
    if (!verts) return st;
    uint32_t *vnuc = (uint32_t *)nd_buf(c, B_CUT_VNUC, std::max<uint64_t>(U, 1) * 4, &st);
    if (!vnuc) return st;
    hipLaunchKernelGGL(k_cut_compact, dim3(gp), dim3(kCB), 0, c->stream, np, ks, flag, pos2,
                       verts, vnuc);
    const uint32_t gu = nd_grid(U, kCB, 16384);
    hipLaunchKernelGGL(k_cut_starts, dim3(gu), dim3(kCB), 0, c->stream, U, vnuc, nuc);
    hipLaunchKernelGGL(k_cut_sizes, dim3(gu), dim3(kCB), 0, c->stream, U, vnuc, nuc);
    hipLaunchKernelGGL(k_cut_edges, dim3(nd_grid(U * 64, kCB, 16384)), dim3(kCB), 0, c->stream,
                       U, verts, vnuc, nuc, (const uint64_t *)c->bufs[B_RP].p,
                       (const uint32_t *)c->bufs[B_COL].p);
    if ((st = nd_hip(c, hipGetLastError(), "cut kernels")) != ND_OK) return st;
  } else if (nr) {
    uint32_t *leaf = (uint32_t *)nd_buf(c, B_CUT_LEAF, nr * 4, &st);
    if (!leaf) return st;
    if ((st = nd_hip(c, hipMemsetAsync(leaf, 0xFF, nr * 4, c->stream), "cut leaves")) != ND_OK)
      return st;
  }
  if ((st = nd_hip(c, hipStreamSynchronize(c->stream), "cut sync")) != ND_OK) return st;
  c->cut_nuclei = N;
  c->cut_verts = U;
  c->cut_valid = true;
  if (n_nuclei) *n_nuclei = N;
  if (n_vertices) *n_vertices = U;
  return ND_OK;
}

nd_status nd_get_cut(nd_ctx *c, nd_nucleus *nuclei, uint32_t *verts, uint32_t *leaf_nucleus,
                     nd_mem where) {
  if (!c) return ND_E_INVALID_ARG;
  nd_status st = nd_hip(c, hipSetDevice(c->device), "hipSetDevice");
  if (st != ND_OK) return st;
  if (!c->cut_valid || !c->decomposed) return nd_fail(c, ND_E_STATE, "no hierarchy cut");
  if (where != ND_MEM_HOST && where != ND_MEM_DEVICE)
    return nd_fail(c, ND_E_INVALID_ARG, "bad memory kind");
  const hipMemcpyKind kind = where == ND_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  struct Part {
    void *dst;
    int buf;
    uint64_t bytes;
  } parts[3] = {{nuclei, B_CUT_NUC, c->cut_nuclei * sizeof(nd_nucleus)},
                {verts, B_CUT_VERTS, c->cut_verts * 4},
                {leaf_nucleus, B_CUT_LEAF, c->n_r * 4}};
  for (const Part &p : parts) {
    if (!p.dst || !p.bytes) continue;
    if ((st = nd_hip(c, hipMemcpyAsync(p.dst, c->bufs[p.buf].p, p.bytes, kind, c->stream),
                     "cut copy")) != ND_OK)
      return st;
  }
  return nd_hip(c, hipStreamSynchronize(c->stream), "cut copy sync");
}

}  // extern "C"
