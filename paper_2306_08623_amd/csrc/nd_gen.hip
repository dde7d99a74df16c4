// nd_gen.hip -- tables for the (r,s) pairs with s = 5..7.
//
// The paper's framework takes any r < s (Section 3 defines the decomposition
// for every pair; its evaluation runs r < s <= 7). For s <= 4 the library
// keeps no s-clique: the peel finds them again from edge -> triangle lists.
// For larger s it lists them once here and keeps them in HBM, as two
// arrays:
//
//   sm[q * C + j]  the C = C(s,r) r-clique ids of s-clique q (its r-subsets
//                  in lexicographic order of positions)
//   io / il        the s-cliques of every r-clique, as a CSR: il[io[R] ..
//                  io[R + 1]) are the ids q of the s-cliques containing R
//
// so a peeled r-clique's visit (Algorithm 3's loop over the s-cliques
// containing it) reads its list and the C - 1 other members of each entry.
// This costs 8 C n_s bytes; the decomposition fails with ND_E_OOM when the
// device cannot hold them.
//
// Cliques are listed level by level in the oriented graph: a k-clique is
// a tuple of vertices in ascending orientation order; it extends by every
// out-neighbour x of its last vertex that is an out-neighbour of all its
// other vertices, so every (k+1)-clique is listed exactly once (from its
// first k vertices in that order). r-clique ids are lexicographic: the
// level-r tuples, each sorted by vertex id, are sorted by an LSD radix sort
// of two vertex ids per pass.
#include "nd_internal.h"

#include <algorithm>

namespace {

constexpr uint32_t kGB = 256;

__device__ __forceinline__ bool out_adj(const GraphView &g, uint32_t v, uint32_t x) {
  const uint64_t b = g.dgp[v], f = g.dgp[v + 1];
  return find_u32<uint64_t>(g.dgc, b, f, x) != f;
}

// level 2: the oriented edges (u, x), u -> x, in out-slot order
__global__ void k_gen_level2(GraphView g, uint32_t *__restrict__ out) {
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < g.m;
       j += (uint64_t)gridDim.x * blockDim.x) {
    out[2 * j] = segment_of(g.dgp, g.n, j);
    out[2 * j + 1] = g.dgc[j];
  }
}

// number of extensions of every k-clique (k >= 2); at most the out-degree
// of its last vertex
__global__ void k_gen_count(GraphView g, uint64_t nt, uint32_t k, const uint32_t *__restrict__ tup,
                            uint32_t *__restrict__ cnt) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < nt;
       t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t *T = tup + t * k;
    const uint32_t last = T[k - 1];
    uint32_t c = 0;
    for (uint64_t p = g.dgp[last]; p < g.dgp[last + 1]; p++) {
      const uint32_t x = g.dgc[p];
      bool ok = true;
      for (uint32_t i = 0; i + 1 < k && ok; i++) ok = out_adj(g, T[i], x);
      c += ok ? 1u : 0u;
    }
    cnt[t] = c;
  }
}

// the (k+1)-cliques: tuple t's extensions at off[t] .. in out-slot order
__global__ void k_gen_fill(GraphView g, uint64_t nt, uint32_t k, const uint32_t *__restrict__ tup,
                           const uint64_t *__restrict__ off, uint32_t *__restrict__ out) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < nt;
       t += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t *T = tup + t * k;
    const uint32_t last = T[k - 1];
    uint64_t o = off[t];
    for (uint64_t p = g.dgp[last]; p < g.dgp[last + 1]; p++) {
      const uint32_t x = g.dgc[p];
      bool ok = true;
      for (uint32_t i = 0; i + 1 < k && ok; i++) ok = out_adj(g, T[i], x);
      if (!ok) continue;
      uint32_t *O = out + o * (k + 1);
      for (uint32_t i = 0; i < k; i++) O[i] = T[i];
      O[k] = x;
      o++;
    }
  }
}

// every tuple sorted by vertex id (insertion sort, k <= 7)
__global__ void k_gen_sort_tuples(uint64_t nt, uint32_t k, const uint32_t *__restrict__ in,
                                  uint32_t *__restrict__ out) {
  for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < nt;
       t += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t v[kMaxS];
    for (uint32_t i = 0; i < k; i++) {
      const uint32_t x = in[t * k + i];
      uint32_t j = i;
      while (j > 0 && v[j - 1] > x) {
        v[j] = v[j - 1];
        j--;
      }
      v[j] = x;
    }
    for (uint32_t i = 0; i < k; i++) out[t * k + i] = v[i];
  }
}

__global__ void k_gen_iota(uint32_t *__restrict__ a, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    a[i] = (uint32_t)i;
}

// radix key of sorted tuple perm[i]: components a (high) and b (low, or
// none when b == a), each `bits` wide
__global__ void k_gen_keys(uint64_t nt, uint32_t k, const uint32_t *__restrict__ tup,
                           const uint32_t *__restrict__ perm, uint32_t a, uint32_t b,
                           uint32_t bits, uint64_t *__restrict__ key) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nt;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t *T = tup + (uint64_t)perm[i] * k;
    key[i] = a == b ? (uint64_t)T[a] : ((uint64_t)T[a] << bits) | T[b];
  }
}

__global__ void k_gen_gather(uint64_t nt, uint32_t k, const uint32_t *__restrict__ tup,
                             const uint32_t *__restrict__ perm, uint32_t *__restrict__ out) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nt;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t *T = tup + (uint64_t)perm[i] * k;
    for (uint32_t j = 0; j < k; j++) out[i * k + j] = T[j];
  }
}

// id of the sorted r-tuple `key` in the lexicographic table, ND_NONE if
// absent
__device__ uint32_t rcl_find(const uint32_t *__restrict__ rcl, uint64_t n_r, uint32_t r,
                             const uint32_t *key) {
  uint64_t lo = 0, hi = n_r;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    const uint32_t *T = rcl + mid * r;
    int cmp = 0;
    for (uint32_t j = 0; j < r && cmp == 0; j++) cmp = T[j] < key[j] ? -1 : (T[j] > key[j] ? 1 : 0);
    if (cmp < 0) lo = mid + 1;
    else hi = mid;
  }
  if (lo == n_r) return ND_NONE;
  const uint32_t *T = rcl + lo * r;
  for (uint32_t j = 0; j < r; j++)
    if (T[j] != key[j]) return ND_NONE;
  return (uint32_t)lo;
}

// the C(s,r) r-clique ids of every s-clique (r-subsets of its sorted tuple
// in lexicographic order of positions), and the s-clique count of every
// r-clique
__global__ void k_gen_members(uint64_t ns, uint32_t r, uint32_t s, uint32_t C,
                              const uint32_t *__restrict__ stup, const uint32_t *__restrict__ rcl,
                              uint64_t n_r, uint32_t *__restrict__ sm, uint32_t *__restrict__ cnt,
                              uint32_t *status) {
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < ns;
       q += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t *S = stup + q * s;
    uint32_t pos[kMaxS], key[kMaxS];
    for (uint32_t i = 0; i < r; i++) pos[i] = i;
    for (uint32_t j = 0; j < C; j++) {
      for (uint32_t i = 0; i < r; i++) key[i] = S[pos[i]];
      const uint32_t id = r == 1 ? key[0] : rcl_find(rcl, n_r, r, key);
      sm[q * C + j] = id;
      if (id == ND_NONE) atomicOr(status, ND_DERR_BADGRAPH);   // tables disagree
      else if (atomicAdd(&cnt[id], 1u) == 0xFFFFFFFFu) atomicOr(status, ND_DERR_OVERFLOW);
      // next combination: the rightmost position that can still advance
      int i = (int)r - 1;
      while (i >= 0 && pos[i] == s - r + (uint32_t)i) i--;
      if (i < 0) break;
      pos[i]++;
      for (uint32_t t = (uint32_t)i + 1; t < r; t++) pos[t] = pos[t - 1] + 1;
    }
  }
}

// il: the s-cliques of every r-clique, one thread per (s-clique, member);
// the order inside a row is whatever the atomics give (the peel's results do
// not depend on it)
__global__ void k_gen_inc_fill(uint64_t ns, uint32_t C, const uint32_t *__restrict__ sm,
                               const uint64_t *__restrict__ io, uint32_t *__restrict__ cur,
                               uint32_t *__restrict__ il) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < ns * C;
       x += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t id = sm[x];
    if (id == ND_NONE) continue;
    il[io[id] + atomicAdd(&cur[id], 1u)] = (uint32_t)(x / C);
  }
}

uint32_t bits_of(uint64_t v) {
  uint32_t b = 0;
  while (b < 64 && (v >> b) != 0) b++;
  return b;
}

}  // namespace

nd_status nd_prep_general(nd_ctx *c, GraphView *gv) {
  nd_status st;
  DevScalars *sc = (DevScalars *)c->bufs[B_SCAL].p;
  const uint32_t r = c->r, s = c->s, n = c->n;
  const uint64_t m = c->m;
  uint64_t C = 1;
  for (uint32_t i = 0; i < r; i++) C = C * (s - i) / (i + 1);
  gv->nsm = (uint32_t)C;
  gv->rcl = nullptr;
  gv->sm = nullptr;
  gv->io = nullptr;
  gv->il = nullptr;
  // levels 2 .. s; level r's sorted tuples become the r-clique table
  uint64_t nt = m;   // tuples of the current level
  uint32_t *cur = nullptr;
  uint32_t *stup = nullptr;   // level s, sorted tuples
  uint64_t n_s = 0;
  c->n_r = r == 1 ? n : 0;
  if (m) {
    cur = (uint32_t *)nd_buf(c, B_GEN_L0, m * 2 * 4, &st);
    if (!cur) return st;
    hipLaunchKernelGGL(k_gen_level2, dim3(nd_grid(m, kGB, 16384)), dim3(kGB), 0, c->stream, *gv,
                       cur);
  }
  int which = 0;
  for (uint32_t k = 2; k <= s && nt; k++) {
    if (k == r || k == s) {
      // this level's tuples sorted by vertex id
      const int bid = k == r ? B_GEN_RTUP : B_GEN_STUP;
      uint32_t *srt = (uint32_t *)nd_buf(c, bid, nt * k * 4, &st);
      if (!srt) return st;
      hipLaunchKernelGGL(k_gen_sort_tuples, dim3(nd_grid(nt, kGB, 16384)), dim3(kGB), 0, c->stream,
                         nt, k, cur, srt);
      if (k == r) {
        if (nt >= 0xFFFFFFFFull)
          return nd_fail(c, ND_E_OVERFLOW, "r-clique ids exceed 32 bits");
        c->n_r = nt;
        // lexicographic order: LSD passes over pairs of tuple positions
        uint32_t *perm = (uint32_t *)nd_buf(c, B_SORTV0, nt * 4, &st);
        if (!perm) return st;
        uint32_t *v1 = (uint32_t *)nd_buf(c, B_SORTV1, nt * 4, &st);
        if (!v1) return st;
        uint64_t *k0 = (uint64_t *)nd_buf(c, B_SORTK0, nt * 8, &st);
        if (!k0) return st;
        uint64_t *k1 = (uint64_t *)nd_buf(c, B_SORTK1, nt * 8, &st);
        if (!k1) return st;
        hipLaunchKernelGGL(k_gen_iota, dim3(nd_grid(nt, kGB, 16384)), dim3(kGB), 0, c->stream,
                           perm, nt);
        const uint32_t vb = std::max<uint32_t>(1, bits_of(n));
        for (int hi = (int)k - 1; hi >= 0; hi -= 2) {
          const uint32_t b = (uint32_t)hi, a = hi >= 1 ? (uint32_t)hi - 1 : (uint32_t)hi;
          hipLaunchKernelGGL(k_gen_keys, dim3(nd_grid(nt, kGB, 16384)), dim3(kGB), 0, c->stream,
                             nt, k, srt, perm, a, b, vb, k0);
          uint64_t *ok;
          uint32_t *ov;
          st = nd_sort_pairs_u64(c, k0, perm, k1, v1, nt, a == b ? vb : 2 * vb, &ok, &ov);
          if (st != ND_OK) return st;
          if (ov != perm) std::swap(perm, v1);
          if (ok != k0) std::swap(k0, k1);
        }
        uint32_t *rcl = (uint32_t *)nd_buf(c, B_GEN_RCL, nt * k * 4, &st);
        if (!rcl) return st;
        hipLaunchKernelGGL(k_gen_gather, dim3(nd_grid(nt, kGB, 16384)), dim3(kGB), 0, c->stream,
                           nt, k, srt, perm, rcl);
        gv->rcl = rcl;
      } else {
        stup = srt;
        n_s = nt;
      }
    }
    if (k == s) break;
    // extend to level k + 1
    uint32_t *cnt = (uint32_t *)nd_buf(c, B_GEN_CNT, nt * 4, &st);
    if (!cnt) return st;
    uint64_t *off = (uint64_t *)nd_buf(c, B_GEN_OFF, (nt + 1) * 8, &st);
    if (!off) return st;
    hipLaunchKernelGGL(k_gen_count, dim3(nd_grid(nt, kGB, 65536)), dim3(kGB), 0, c->stream, *gv,
                       nt, k, cur, cnt);
    uint64_t nxt = 0;
    if ((st = nd_exclusive_scan_u32_to_u64(c, cnt, off, nt, &nxt)) != ND_OK) return st;
    which ^= 1;
    uint32_t *dst = nullptr;
    if (nxt) {
      dst = (uint32_t *)nd_buf(c, which ? B_GEN_L1 : B_GEN_L0, nxt * (k + 1) * 4, &st);
      if (!dst) return st;
      hipLaunchKernelGGL(k_gen_fill, dim3(nd_grid(nt, kGB, 65536)), dim3(kGB), 0, c->stream, *gv,
                         nt, k, cur, off, dst);
    }
    cur = dst;
    nt = nxt;
  }
  if ((st = nd_hip(c, hipGetLastError(), "clique levels")) != ND_OK) return st;
  const uint64_t n_r = c->n_r;
  if (n_s >= 0xFFFFFFFFull)
    return nd_fail(c, ND_E_OVERFLOW, "more than 2^32-2 s-cliques: s-clique ids exceed 32 bits");
  c->gen_n_s = n_s;
  // incidence: member ids and counts, then the CSR of each r-clique's s-cliques
  uint32_t *cnt = (uint32_t *)nd_buf(c, B_GEN_CNT, std::max<uint64_t>(n_r, 1) * 4, &st);
  if (!cnt) return st;
  uint64_t *io = (uint64_t *)nd_buf(c, B_GEN_IO, (n_r + 1) * 8, &st);
  if (!io) return st;
  if (n_r && (st = nd_hip(c, hipMemsetAsync(cnt, 0, n_r * 4, c->stream), "gen counts")) != ND_OK)
    return st;
  uint32_t *sm = (uint32_t *)nd_buf(c, B_GEN_SM, std::max<uint64_t>(n_s * C, 1) * 4, &st);
  if (!sm) return st;
  if (n_s)
    hipLaunchKernelGGL(k_gen_members, dim3(nd_grid(n_s, kGB, 65536)), dim3(kGB), 0, c->stream,
                       n_s, r, s, (uint32_t)C, stup, gv->rcl, n_r, sm, cnt, &sc->status);
  uint64_t total = 0;
  if (n_r) {
    if ((st = nd_exclusive_scan_u32_to_u64(c, cnt, io, n_r, &total)) != ND_OK) return st;
  } else if ((st = nd_hip(c, hipMemsetAsync(io, 0, 8, c->stream), "gen io")) != ND_OK) {
    return st;
  }
  uint32_t *il = (uint32_t *)nd_buf(c, B_GEN_IL, std::max<uint64_t>(total, 1) * 4, &st);
  if (!il) return st;
  if (total) {
    if ((st = nd_hip(c, hipMemsetAsync(cnt, 0, n_r * 4, c->stream), "gen cursor")) != ND_OK)
      return st;
    hipLaunchKernelGGL(k_gen_inc_fill, dim3(nd_grid(n_s * C, kGB, 65536)), dim3(kGB), 0,
                       c->stream, n_s, (uint32_t)C, sm, io, cnt, il);
  }
  gv->sm = sm;
  gv->io = io;
  gv->il = il;
  return nd_hip(c, hipGetLastError(), "incidence kernels");
}
