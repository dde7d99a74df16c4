// nd_tree.hip -- hierarchy tree from uf and L (CONSTRUCT-TREE-EFFICIENT,
// Algorithm 5, Section 7.3) and its canonical numbering.
//
//   1. root[x] = find(x) for every r-clique; every uf component is a
//      candidate node at level ND[root].
//   2. The parent of the node of component C is the node of find(L[C]) when
//      L[C] is set, else none.
//   3. A node with a single child is dropped (Section 7.3 remark): that is a
//      component of one r-clique that no other component points to; its leaf
//      is attached to the node's parent instead. No two such nodes can chain,
//      because every component keeps at least one leaf.
//   4. Every remaining node gets the smallest leaf index of its subtree: each
//      leaf walks up with atomicMin and stops at the first ancestor that
//      already holds a smaller leaf (that leaf's own walk covers the rest).
//   5. Nodes are numbered by ascending (level, smallest leaf) with a stable
//      LSD radix sort, which yields the canonical tree.
#include "nd_internal.h"

#include <algorithm>

namespace {

constexpr uint32_t kTB = 256;

__device__ __forceinline__ uint32_t tfind(const uint32_t *uf, uint32_t x) {
  // the peel has finished: no concurrent writers, plain loads suffice
  for (;;) {
    uint32_t p = uf[x];
    if (p == x) return x;
    x = p;
  }
}

// Groups the active lanes of a wave by key: returns the group's size in its
// lowest lane (`first` set there), 0 elsewhere. A few large components or
// nodes take most updates; one atomic per group and wave instead of one per
// lane takes the contention off them.
__device__ __forceinline__ uint32_t wave_group(uint32_t key, bool active, bool &first) {
  const uint32_t lane = lane_id();
  uint64_t pending = ballot64(active);
  uint32_t count = 0;
  first = false;
  while (pending) {
    const uint32_t leader = __ffsll((unsigned long long)pending) - 1;
    const uint32_t k = __shfl(key, leader, 64);
    const uint64_t same = ballot64(active && key == k);
    if (lane == leader) {
      first = true;
      count = __popcll(same);
    }
    pending &= ~same;
  }
  return count;
}

__global__ void k_roots(uint64_t n, const uint32_t *__restrict__ uf, uint32_t *__restrict__ root,
                        uint32_t *__restrict__ sz) {
  for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x; base < n;
       base += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = base + threadIdx.x;
    const bool active = x < n;
    const uint32_t rt = active ? tfind(uf, (uint32_t)x) : 0;
    if (active) root[x] = rt;
    bool first;
    const uint32_t cnt = wave_group(rt, active, first);
    if (first) atomicAdd(&sz[rt], cnt);
  }
}

__global__ void k_node_parent(uint64_t n, const uint32_t *__restrict__ root,
                              const uint32_t *__restrict__ L, uint32_t *__restrict__ npar,
                              uint32_t *__restrict__ nkid) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n;
       x += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t p = ND_NONE;
    if (root[x] == x && L[x] != ND_NONE) {
      p = root[L[x]];
      atomicAdd(&nkid[p], 1u);
    }
    npar[x] = p;
  }
}

__device__ __forceinline__ bool kept(const uint32_t *root, const uint32_t *sz,
                                     const uint32_t *nkid, uint32_t c) {
  return root[c] == c && sz[c] + nkid[c] >= 2;
}

// parent node (as a component root id) of leaf x, or NONE
__device__ __forceinline__ uint32_t leaf_parent(const uint32_t *root, const uint32_t *sz,
                                                const uint32_t *nkid, const uint32_t *npar,
                                                uint32_t x) {
  uint32_t c = root[x];
  return kept(root, sz, nkid, c) ? c : npar[c];
}

__global__ void k_minleaf(uint64_t n, const uint32_t *__restrict__ root,
                          const uint32_t *__restrict__ sz, const uint32_t *__restrict__ nkid,
                          const uint32_t *__restrict__ npar, uint32_t *__restrict__ ml,
                          uint32_t *status) {
  for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x; base < n;
       base += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = base + threadIdx.x;
    uint32_t node = x < n ? leaf_parent(root, sz, nkid, npar, (uint32_t)x) : ND_NONE;
    // of the lanes that start at one node only the lowest (the smallest leaf
    // id, lanes take consecutive leaves) can lower a minimum on its path
    bool first;
    (void)wave_group(node, node != ND_NONE, first);
    if (!first) continue;
    // levels strictly decrease along npar, so the walk is finite; the cap
    // only guards against a corrupted table
    for (uint32_t hop = 0; node != ND_NONE; hop++) {
      if (hop > (1u << 24)) {
        atomicOr(status, ND_DERR_WATCHDOG);
        break;
      }
      uint32_t old = atomicMin(&ml[node], (uint32_t)x);
      if (old <= (uint32_t)x) break;
      node = npar[node];
    }
  }
}

__global__ void k_kept_flag(uint64_t n, const uint32_t *__restrict__ root,
                            const uint32_t *__restrict__ sz, const uint32_t *__restrict__ nkid,
                            uint32_t *__restrict__ flag) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n;
       x += (uint64_t)gridDim.x * blockDim.x)
    flag[x] = kept(root, sz, nkid, (uint32_t)x) ? 1u : 0u;
}

__global__ void k_kept_keys(uint64_t n, const uint32_t *__restrict__ flag,
                            const uint64_t *__restrict__ pos, const uint32_t *__restrict__ nd,
                            const uint32_t *__restrict__ ml, uint32_t lbits,
                            uint64_t *__restrict__ key, uint32_t *__restrict__ val) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n;
       x += (uint64_t)gridDim.x * blockDim.x) {
    if (!flag[x]) continue;
    uint64_t i = pos[x];
    key[i] = ((uint64_t)nd[x] << lbits) | ml[x];
    val[i] = (uint32_t)x;
  }
}

// ---- stable LSD radix sort of (u64 key, u32 value), 8 bits per pass ------

constexpr uint32_t kSortTile = 4096;

__global__ void __launch_bounds__(kTB) k_radix_hist(const uint64_t *__restrict__ key, uint64_t n,
                                                    uint32_t shift, uint32_t ntiles,
                                                    uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t b = (uint64_t)blockIdx.x * kSortTile;
  const uint64_t e = b + kSortTile < n ? b + kSortTile : n;
  for (uint64_t i = b + threadIdx.x; i < e; i += kTB) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
  __syncthreads();
  hist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(kTB) k_radix_scatter(const uint64_t *__restrict__ kin,
                                                       const uint32_t *__restrict__ vin,
                                                       uint64_t n, uint32_t shift,
                                                       uint32_t ntiles,
                                                       const uint64_t *__restrict__ off,
                                                       uint64_t *__restrict__ kout,
                                                       uint32_t *__restrict__ vout) {
  __shared__ uint32_t run[256];          // elements of each digit placed so far
  __shared__ uint32_t wcnt[kTB / 64][256];
  const uint32_t lane = lane_id(), wv = threadIdx.x / 64;
  run[threadIdx.x] = 0;
  const uint64_t b = (uint64_t)blockIdx.x * kSortTile;
  const uint64_t e = b + kSortTile < n ? b + kSortTile : n;
  __syncthreads();
  for (uint64_t base = b; base < e; base += kTB) {
    for (uint32_t d = threadIdx.x; d < (kTB / 64) * 256; d += kTB) (&wcnt[0][0])[d] = 0;
    __syncthreads();
    const uint64_t i = base + threadIdx.x;
    const bool valid = i < e;
    uint64_t k = 0;
    uint32_t v = 0, dig = 0;
    if (valid) {
      k = kin[i];
      v = vin[i];
      dig = (uint32_t)(k >> shift) & 255u;
    }
    // lanes of this wave holding the same digit
    uint64_t same = ballot64(valid);
    for (uint32_t bit = 0; bit < 8; bit++) {
      uint64_t m = ballot64(valid && ((dig >> bit) & 1u));
      same &= ((dig >> bit) & 1u) ? m : ~m;
    }
    const uint64_t below = same & ((lane == 0) ? 0ull : (~0ull >> (64 - lane)));
    const uint32_t rank = __popcll(below);
    if (valid && rank == 0) wcnt[wv][dig] = __popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t pre = run[dig];
      for (uint32_t w = 0; w < wv; w++) pre += wcnt[w][dig];
      const uint64_t dst = off[(uint64_t)dig * ntiles + blockIdx.x] + pre + rank;
      kout[dst] = k;
      vout[dst] = v;
    }
    __syncthreads();
    {
      uint32_t add = 0;
      for (uint32_t w = 0; w < kTB / 64; w++) add += wcnt[w][threadIdx.x];
      run[threadIdx.x] += add;
    }
    __syncthreads();
  }
}

__global__ void k_write_tree(uint64_t n_r, uint64_t n_int, const uint32_t *__restrict__ root,
                             const uint32_t *__restrict__ sz, const uint32_t *__restrict__ nkid,
                             const uint32_t *__restrict__ npar, const uint32_t *__restrict__ canon,
                             const uint32_t *__restrict__ sorted_val, const uint32_t *__restrict__ nd,
                             uint64_t *__restrict__ parent, uint32_t *__restrict__ level) {
  const uint64_t tot = n_r + n_int;
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < tot;
       x += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t p;
    if (x < n_r) {
      p = leaf_parent(root, sz, nkid, npar, (uint32_t)x);
    } else {
      const uint32_t c = sorted_val[x - n_r];
      p = npar[c];
      level[x - n_r] = nd[c];
    }
    parent[x] = p == ND_NONE ? ND_NONE64 : n_r + canon[p];
  }
}

__global__ void k_canon(uint64_t n_int, const uint32_t *__restrict__ sorted_val,
                        const uint32_t *__restrict__ ml, uint32_t *__restrict__ canon,
                        uint32_t *__restrict__ node_ml) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_int;
       i += (uint64_t)gridDim.x * blockDim.x) {
    canon[sorted_val[i]] = (uint32_t)i;
    node_ml[i] = ml[sorted_val[i]];
  }
}

__global__ void k_rcliques(uint32_t r, uint64_t n_r, const uint32_t *__restrict__ eu,
                           const uint32_t *__restrict__ ev, const uint32_t *__restrict__ te,
                           uint32_t *__restrict__ out) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n_r;
       x += (uint64_t)gridDim.x * blockDim.x) {
    if (r == 1) {
      out[x] = (uint32_t)x;
    } else if (r == 2) {
      out[2 * x] = eu[x];
      out[2 * x + 1] = ev[x];
    } else {
      const uint32_t e_ab = te[3 * x], e_ac = te[3 * x + 1];
      out[3 * x] = eu[e_ab];
      out[3 * x + 1] = ev[e_ab];
      out[3 * x + 2] = ev[e_ac];
    }
  }
}

uint32_t bits_for(uint64_t v) {
  uint32_t b = 0;
  while (b < 64 && (v >> b) != 0) b++;
  return b;
}

}  // namespace

// Stable LSD radix sort of n (u64 key, u32 value) pairs on the context's
// stream, `bits` low key bits significant; k1/v1 are scratch of the same
// size. *out_k / *out_v point at whichever buffers hold the result.
nd_status nd_sort_pairs_u64(nd_ctx *c, uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1,
                            uint64_t n, uint32_t bits, uint64_t **out_k, uint32_t **out_v) {
  nd_status st = ND_OK;
  if (n) {
    const uint32_t ntiles = (uint32_t)((n + kSortTile - 1) / kSortTile);
    uint32_t *hist = (uint32_t *)nd_buf(c, B_HIST, 256ull * ntiles * 4, &st);
    if (!hist) return st;
    uint64_t *hoff = (uint64_t *)nd_buf(c, B_SORTOFF, (256ull * ntiles + 1) * 8, &st);
    if (!hoff) return st;
    for (uint32_t shift = 0; shift < bits; shift += 8) {
      hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(kTB), 0, c->stream, k0, n, shift,
                         ntiles, hist);
      st = nd_exclusive_scan_u32_to_u64(c, hist, hoff, 256ull * ntiles, nullptr);
      if (st != ND_OK) return st;
      hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kTB), 0, c->stream, k0, v0, n,
                         shift, ntiles, hoff, k1, v1);
      std::swap(k0, k1);
      std::swap(v0, v1);
    }
  }
  *out_k = k0;
  *out_v = v0;
  return nd_hip(c, hipGetLastError(), "radix sort");
}

nd_status nd_stage_tree(nd_ctx *c, const GraphView &g) {
  (void)g;
  nd_status st;
  const uint64_t nr = c->n_r;
  c->n_int = 0;
  if (nr == 0) return ND_OK;
  const uint32_t *uf = (const uint32_t *)c->bufs[B_UF].p;
  const uint32_t *L = (const uint32_t *)c->bufs[B_L].p;
  const uint32_t *nd = (const uint32_t *)c->bufs[B_CNT].p;
  // reuse the peel's frontier / alive buffers as scratch
  uint32_t *root = (uint32_t *)c->bufs[B_F0].p;
  uint32_t *sz = (uint32_t *)c->bufs[B_F1].p;
  uint32_t *npar = (uint32_t *)c->bufs[B_AL0].p;
  uint32_t *nkid = (uint32_t *)c->bufs[B_AL1].p;
  uint32_t *ml = (uint32_t *)nd_buf(c, B_TMP32A, nr * 4, &st);   // min leaf per node
  if (!ml) return st;
  uint64_t *pos = (uint64_t *)c->bufs[B_WSCAN].p;   // n_r + 1 needed
  uint32_t *flag = (uint32_t *)nd_buf(c, B_TMP32D, nr * 4, &st);
  if (!flag) return st;
  if (c->bufs[B_WSCAN].bytes < (nr + 1) * 8) {
    pos = (uint64_t *)nd_buf(c, B_WSCAN, (nr + 1) * 8, &st);
    if (!pos) return st;
  }
  const uint32_t grid = nd_grid(nr, kTB, 16384);
  if ((st = nd_hip(c, hipMemsetAsync(sz, 0, nr * 4, c->stream), "sz")) != ND_OK) return st;
  if ((st = nd_hip(c, hipMemsetAsync(nkid, 0, nr * 4, c->stream), "nkid")) != ND_OK) return st;
  if ((st = nd_hip(c, hipMemsetAsync(ml, 0xFF, nr * 4, c->stream), "ml")) != ND_OK) return st;
  hipLaunchKernelGGL(k_roots, dim3(grid), dim3(kTB), 0, c->stream, nr, uf, root, sz);
  hipLaunchKernelGGL(k_node_parent, dim3(grid), dim3(kTB), 0, c->stream, nr, root, L, npar, nkid);
  DevScalars *sc = (DevScalars *)c->bufs[B_SCAL].p;
  hipLaunchKernelGGL(k_minleaf, dim3(grid), dim3(kTB), 0, c->stream, nr, root, sz, nkid, npar, ml,
                     &sc->status);
  hipLaunchKernelGGL(k_kept_flag, dim3(grid), dim3(kTB), 0, c->stream, nr, root, sz, nkid, flag);
  uint64_t nint = 0;
  st = nd_exclusive_scan_u32_to_u64(c, flag, pos, nr, &nint);
  if (st != ND_OK) return st;
  c->n_int = nint;
  uint64_t *parent = (uint64_t *)nd_buf(c, B_PARENT, (nr + nint) * 8, &st);
  if (!parent) return st;
  uint32_t *level = (uint32_t *)nd_buf(c, B_LEVEL, std::max<uint64_t>(nint, 1) * 4, &st);
  if (!level) return st;
  uint32_t *canon = (uint32_t *)nd_buf(c, B_TMP32C, nr * 4, &st);
  if (!canon) return st;
  const uint32_t *sorted_val = nullptr;
  if (nint) {
    uint64_t *k0 = (uint64_t *)nd_buf(c, B_SORTK0, nint * 8, &st);
    if (!k0) return st;
    uint64_t *k1 = (uint64_t *)nd_buf(c, B_SORTK1, nint * 8, &st);
    if (!k1) return st;
    uint32_t *v0 = (uint32_t *)nd_buf(c, B_SORTV0, nint * 4, &st);
    if (!v0) return st;
    uint32_t *v1 = (uint32_t *)nd_buf(c, B_SORTV1, nint * 4, &st);
    if (!v1) return st;
    const uint32_t lbits = std::max<uint32_t>(1, bits_for(nr - 1));
    hipLaunchKernelGGL(k_kept_keys, dim3(grid), dim3(kTB), 0, c->stream, nr, flag, pos, nd, ml,
                       lbits, k0, v0);
    // key bits: level < 2^32, min leaf < 2^lbits
    uint64_t *ks = nullptr;
    uint32_t *vs = nullptr;
    st = nd_sort_pairs_u64(c, k0, v0, k1, v1, nint, lbits + 32, &ks, &vs);
    if (st != ND_OK) return st;
    sorted_val = vs;
    uint32_t *node_ml = (uint32_t *)nd_buf(c, B_NODEML, nint * 4, &st);
    if (!node_ml) return st;
    hipLaunchKernelGGL(k_canon, dim3(nd_grid(nint, kTB, 16384)), dim3(kTB), 0, c->stream, nint,
                       sorted_val, ml, canon, node_ml);
  }
  hipLaunchKernelGGL(k_write_tree, dim3(nd_grid(nr + nint, kTB, 16384)), dim3(kTB), 0, c->stream,
                     nr, nint, root, sz, nkid, npar, canon, sorted_val, nd, parent, level);
  return nd_hip(c, hipGetLastError(), "tree kernels");
}

nd_status nd_write_rcliques(nd_ctx *c, const GraphView &g, uint32_t *out_dev) {
  if (c->n_r == 0) return ND_OK;
  if (g.rcl)   // s = 5..7, r >= 2: the lexicographic table built in prep
    return nd_hip(c, hipMemcpyAsync(out_dev, g.rcl, c->n_r * c->r * 4ull, hipMemcpyDeviceToDevice,
                                    c->stream), "rclique copy");
  hipLaunchKernelGGL(k_rcliques, dim3(nd_grid(c->n_r, kTB, 16384)), dim3(kTB), 0, c->stream, c->r,
                     c->n_r, g.eu, g.ev, g.te, out_dev);
  return nd_hip(c, hipGetLastError(), "rclique kernel");
}
