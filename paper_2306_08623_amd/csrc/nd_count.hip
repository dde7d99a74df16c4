// nd_count.hip -- s-clique counting per r-clique (Algorithm 3: the s-clique
// counts stored per r-clique before peeling starts).
//
// Every s-clique is listed exactly once in the oriented graph DG, from its
// two lowest vertices u -> v (Section 3 low out-degree orientation; the
// recursive listing of Algorithm 3's counting step): the remaining s-2
// vertices are common out-neighbours of u and v. For each listed s-clique
// the kernel resolves the ids of its C(s,r) r-cliques and adds one to each
// count with an atomic.
//
//   s = 2: the count of a vertex is its degree.
//   s = 3: one lane per DG edge u -> v; every common out-neighbour w is a
//          triangle {u, v, w}; edge ids come from the DG slots.
//   s = 4: one wave per DG edge; the common out-neighbourhood C2 is built in
//          LDS (ballot compaction keeps it ascending) -- for rows of
//          out-degree above 1024, in a global slice of the wave; lanes then test the
//          pairs {w, x} of C2 for adjacency; every adjacent pair closes a
//          4-clique {u, v, w, x}. Triangle ids (r = 3) are read from W(e) of
//          the triangle's lexicographically first edge by binary search.
#include "nd_internal.h"

#include <algorithm>

namespace {

constexpr uint32_t kCountBlock = 256;
constexpr uint32_t kC2Cap = 1024;   // largest C2 (oriented out-degree) kept on chip

__global__ void k_count_degree(uint32_t n, const uint64_t *__restrict__ rp,
                               uint32_t *__restrict__ cnt) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
    cnt[v] = (uint32_t)(rp[v + 1] - rp[v]);
}

// triangle id of {a, b, c} given the ids of its three edges, via W of the
// edge joining the two smallest vertices
__device__ __forceinline__ uint32_t tri_lookup(const GraphView &g, uint32_t a, uint32_t b,
                                               uint32_t c, uint32_t e_ab, uint32_t e_ac,
                                               uint32_t e_bc) {
  // sort (a,b,c) ascending, carrying the edge opposite each vertex
  // opposite(a) = e_bc, opposite(b) = e_ac, opposite(c) = e_ab
  uint32_t x0 = a, x1 = b, x2 = c;
  uint32_t o0 = e_bc, o1 = e_ac, o2 = e_ab;
  if (x0 > x1) { uint32_t t = x0; x0 = x1; x1 = t; t = o0; o0 = o1; o1 = t; }
  if (x1 > x2) { uint32_t t = x1; x1 = x2; x2 = t; t = o1; o1 = o2; o2 = t; }
  if (x0 > x1) { uint32_t t = x0; x0 = x1; x1 = t; t = o0; o0 = o1; o1 = t; }
  // first edge {x0, x1} is opposite x2
  const uint64_t b0 = g.wp[o2], b1 = g.wp[o2 + 1];
  uint64_t p = lower_bound_u32<uint64_t>(g.wc, b0, b1, x2);
  if (p == b1 || g.wc[p] != x2) return ND_NONE;   // impossible for a real triangle
  return g.wt[p];
}

template <int R>
__global__ void __launch_bounds__(kCountBlock) k_count_s3(GraphView g, uint32_t *__restrict__ cnt,
                                                          DevScalars *sc) {
  uint64_t local = 0;
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < g.m;
       j += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t v = g.dgc[j];
    const uint32_t e_uv = g.dge[j];
    const uint32_t u = g.eu[e_uv] ^ g.ev[e_uv] ^ v;   // the endpoint other than v
    uint64_t bu = g.dgp[u], eu = g.dgp[u + 1], bv = g.dgp[v], ev = g.dgp[v + 1];
    uint64_t lo = bv;
    for (uint64_t i = bu; i < eu && lo < ev; i++) {
      const uint32_t w = g.dgc[i];
      lo = lower_bound_u32<uint64_t>(g.dgc, lo, ev, w);
      if (lo < ev && g.dgc[lo] == w) {
        local++;
        if (R == 1) {
          atomicAdd(&cnt[u], 1u);
          atomicAdd(&cnt[v], 1u);
          atomicAdd(&cnt[w], 1u);
        } else {
          atomicAdd(&cnt[e_uv], 1u);
          atomicAdd(&cnt[g.dge[i]], 1u);
          atomicAdd(&cnt[g.dge[lo]], 1u);
        }
      }
    }
  }
  local = wave_sum64(local);
  if (lane_id() == 0 && local) atomicAdd((unsigned long long *)&sc->n_s, (unsigned long long)local);
}

// LDS arrays of `cap` entries per wave: C2 vertices, their edge ids to u and
// to v, and for r = 3 the 4-cliques found so far through the triangle
// {u, v, w} of each entry (its id is looked up when that count is flushed,
// only for entries that have 4-cliques)
__global__ void k_count_inc(uint64_t nr, const uint64_t *__restrict__ io, uint32_t *__restrict__ cnt) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < nr;
       x += (uint64_t)gridDim.x * blockDim.x)
    cnt[x] = (uint32_t)(io[x + 1] - io[x]);
}

// one 4-clique's increments of its six edges' counts; with kWrap, a count
// that wraps past 2^32 - 1 sets ND_DERR_OVERFLOW (returning atomics, which
// wait for their result: only used when the bound allows a wrap)
template <bool kWrap>
__device__ __forceinline__ void count_edges6(uint32_t *cnt, const uint32_t (&e6)[6],
                                             DevScalars *sc) {
  if (kWrap) {
    bool wrap = false;
#pragma unroll
    for (int z = 0; z < 6; z++) wrap |= atomicAdd(&cnt[e6[z]], 1u) == 0xFFFFFFFFu;
    if (wrap) atomicOr(&sc->status, ND_DERR_OVERFLOW);
  } else {
#pragma unroll
    for (int z = 0; z < 6; z++) atomicAdd(&cnt[e6[z]], 1u);
  }
}

template <int R>
constexpr uint32_t count_s4_arrays() { return R == 3 ? 4 : 3; }

// kGlobal = false: the C2 arrays are in LDS (cap entries per wave) and the
// kernel takes the edges u -> v whose u has out-degree in (small, cap];
// kGlobal = true: they are in global memory (gbuf, one slice of cap entries
// per wave of the grid) and the kernel takes the edges whose u has
// out-degree above `light` (those the LDS kernel left; all of them when
// light = 0).
template <int R, bool kGlobal, bool kWrap>
__global__ void __launch_bounds__(kCountBlock) k_count_s4(GraphView g, uint32_t *__restrict__ cnt,
                                                          DevScalars *sc, uint32_t cap,
                                                          uint32_t *__restrict__ gbuf,
                                                          uint32_t light, uint32_t small) {
  extern __shared__ uint32_t s_c2[];
  const uint32_t wv = threadIdx.x / 64;
  const uint32_t lane = lane_id();
  uint32_t *cv = kGlobal
      ? gbuf + (uint64_t)count_s4_arrays<R>() * cap *
                   ((uint64_t)blockIdx.x * (kCountBlock / 64) + wv)
      : s_c2 + (uint64_t)count_s4_arrays<R>() * cap * wv;
  uint32_t *ceu = cv + cap;
  uint32_t *cev = ceu + cap;
  uint32_t *cn = cev + cap;   // r = 3 only
  uint64_t local = 0;
  const uint64_t nwaves = (uint64_t)gridDim.x * (kCountBlock / 64);
  for (uint64_t j = blockIdx.x * (uint64_t)(kCountBlock / 64) + wv; j < g.m; j += nwaves) {
    // the slot's source vertex: the endpoint of its edge other than v
    const uint32_t v = g.dgc[j];
    const uint32_t e_uv = g.dge[j];
    const uint32_t u = g.eu[e_uv] ^ g.ev[e_uv] ^ v;
    const uint64_t bu = g.dgp[u], eu = g.dgp[u + 1];
    // the other kernels' edges: rows up to `small` out-neighbours go to
    // k_count_s4_small, rows above `light` to the global-memory variant
    if (kGlobal ? eu - bu <= light : (eu - bu > cap || eu - bu <= small)) continue;
    const uint64_t bv = g.dgp[v], ev = g.dgp[v + 1];
    // C2 = N+(u) intersect N+(v), ascending, with the edge ids to u and v
    uint32_t c = 0;
    for (uint64_t base = bu; base < eu; base += 64) {
      const uint64_t i = base + lane;
      bool hit = false;
      uint32_t w = 0, e_uw = 0, e_vw = 0;
      if (i < eu) {
        w = g.dgc[i];
        uint64_t p = find_u32<uint64_t>(g.dgc, bv, ev, w);
        if (p < ev) {
          hit = true;
          e_uw = g.dge[i];
          e_vw = g.dge[p];
        }
      }
      uint64_t mask = ballot64(hit);
      if (hit) {
        uint64_t below = mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane)));
        uint32_t slot = c + __popcll(below);
        if (slot < cap) {
          cv[slot] = w;
          ceu[slot] = e_uw;
          cev[slot] = e_vw;
          if (R == 3) cn[slot] = 0;
        }
      }
      c += __popcll(mask);
    }
    if (c > cap) {   // C2 is within u's out-row, at most cap entries: cannot happen
      if (lane == 0) atomicOr(&sc->status, ND_DERR_OVERFLOW);
      continue;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    // pairs {cv[a], cv[b]}, a < b, all c(c-1)/2 of them spread over the
    // lanes: lane l takes pair numbers l, l + 64, ... in row-major order
    const uint64_t npairs = (uint64_t)c * (c - 1) / 2;
    uint32_t a = 0, b = 1 + lane;
    for (uint64_t q = lane; q < npairs; q += 64, b += 64) {
      while (b >= c) {   // next row: row a + 1 starts at b = a + 2
        const uint32_t over = b - c;
        a++;
        b = a + 1 + over;
      }
      const uint32_t w = cv[a], x = cv[b];
      if (R == 3) {
        // x is a neighbour of u and of v; it lies in W(uw), the common
        // neighbours of u and w, exactly when w and x are adjacent, and its
        // slot there names triangle {u, w, x}; its slot in W(vw) names
        // {v, w, x}. Both lists hold v or u, so neither is empty; the two
        // searches advance in lockstep.
        const uint32_t euw = ceu[a], evw = cev[a];
        const uint64_t b1 = g.wp[euw], f1 = g.wp[euw + 1], b2 = g.wp[evw], f2 = g.wp[evw + 1];
        uint64_t p1, p2;
        find2_u32<uint64_t>(g.wc, b1, f1, b2, f2, x, p1, p2);
        if (p1 == f1) continue;   // w and x are not adjacent
        local++;
        // triangles {u,v,w} and {u,v,x} are counted per C2 entry (LDS),
        // {u,w,x} and {v,w,x} per 4-clique
        atomicAdd(&cn[a], 1u);
        atomicAdd(&cn[b], 1u);
        atomicAdd(&cnt[g.wt[p1]], 1u);
        if (p2 == f2) atomicOr(&sc->status, ND_DERR_BADGRAPH);   // tables disagree
        else atomicAdd(&cnt[g.wt[p2]], 1u);
        continue;
      }
      // adjacency of w and x through the out-row of the lower-key vertex
      uint32_t lowv = w, highv = x;
      if (g.okey[x] < g.okey[w]) { lowv = x; highv = w; }
      const uint64_t bl = g.dgp[lowv], el = g.dgp[lowv + 1];
      const uint64_t p = find_u32<uint64_t>(g.dgc, bl, el, highv);
      if (p == el) continue;
      local++;
      if (R == 1) {
        // (1,4) counts are guarded before counting (probe ranges below 2^32)
        atomicAdd(&cnt[u], 1u);
        atomicAdd(&cnt[v], 1u);
        atomicAdd(&cnt[w], 1u);
        atomicAdd(&cnt[x], 1u);
      } else if (R == 2) {
        // (2,4): an edge's count is at most C(|common neighbours|, 2); when
        // that can pass 2^32 (kWrap) a wrap is caught where it happens, else
        // the increments need no result
        const uint32_t e6[6] = {e_uv, ceu[a], cev[a], ceu[b], cev[b], g.dge[p]};
        count_edges6<kWrap>(cnt, e6, sc);
      }
    }
    if (R == 3) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (uint32_t e = lane; e < c; e += 64) {
        if (cn[e] == 0) continue;
        const uint32_t t = tri_lookup(g, u, v, cv[e], e_uv, ceu[e], cev[e]);
        if (t == ND_NONE) atomicOr(&sc->status, ND_DERR_BADGRAPH);
        else atomicAdd(&cnt[t], cn[e]);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  local = wave_sum64(local);
  if (lane == 0 && local) atomicAdd((unsigned long long *)&sc->n_s, (unsigned long long)local);
}

// Rows of small out-degree: a wave per edge would leave most lanes idle
// (graphs of average degree 8 have out-degrees of a few), so groups of
// kSmallG lanes take one edge u -> v each, for the edges whose u has
// out-degree <= kSmallG: C2 in one ballot pass, its pairs over the group's
// lanes, then the per-entry triangle counts. The wave's loop over its
// groups' edges, and its barriers, stay wave-uniform; a group without an
// edge in a pass has c = 0.
constexpr uint32_t kSmallG = 16;

template <int R, bool kWrap>
__global__ void __launch_bounds__(kCountBlock) k_count_s4_small(GraphView g,
                                                                uint32_t *__restrict__ cnt,
                                                                DevScalars *sc) {
  constexpr uint32_t kGroups = 64 / kSmallG;
  constexpr uint32_t A = count_s4_arrays<R>();
  __shared__ uint32_t s_c2[(kCountBlock / 64) * kGroups * A * kSmallG];
  const uint32_t wv = threadIdx.x / 64;
  const uint32_t lane = lane_id();
  const uint32_t gi = lane / kSmallG, gl = lane % kSmallG;
  uint32_t *cv = s_c2 + ((uint64_t)wv * kGroups + gi) * A * kSmallG;
  uint32_t *ceu = cv + kSmallG;
  uint32_t *cev = ceu + kSmallG;
  uint32_t *cn = cev + kSmallG;   // r = 3 only
  uint64_t local = 0;
  const uint64_t stride = (uint64_t)gridDim.x * (kCountBlock / 64) * kGroups;
  for (uint64_t jb = ((uint64_t)blockIdx.x * (kCountBlock / 64) + wv) * kGroups; jb < g.m;
       jb += stride) {
    const uint64_t j = jb + gi;
    uint32_t u = 0, v = 0, e_uv = 0;
    uint64_t bu = 0, deg = 0;
    if (j < g.m) {
      v = g.dgc[j];
      e_uv = g.dge[j];
      u = g.eu[e_uv] ^ g.ev[e_uv] ^ v;
      bu = g.dgp[u];
      deg = g.dgp[u + 1] - bu;
      if (deg > kSmallG) deg = 0;   // left to the wave-per-edge kernel
    }
    // C2 = N+(u) intersect N+(v) in one pass of the group
    bool hit = false;
    uint32_t w = 0, e_uw = 0, e_vw = 0;
    if (gl < deg) {
      const uint64_t bv = g.dgp[v], ev = g.dgp[v + 1];
      w = g.dgc[bu + gl];
      const uint64_t p = find_u32<uint64_t>(g.dgc, bv, ev, w);
      if (p < ev) {
        hit = true;
        e_uw = g.dge[bu + gl];
        e_vw = g.dge[p];
      }
    }
    const uint32_t gmask = (uint32_t)(ballot64(hit) >> (gi * kSmallG)) & ((1u << kSmallG) - 1);
    const uint32_t c = __popc(gmask);
    if (hit) {
      const uint32_t slot = __popc(gmask & ((1u << gl) - 1));
      cv[slot] = w;
      ceu[slot] = e_uw;
      cev[slot] = e_vw;
      if (R == 3) cn[slot] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // pairs {cv[a], cv[b]}, a < b, over the group's lanes in row-major order
    const uint32_t npairs = c * (c - 1) / 2;
    uint32_t a = 0, b = 1 + gl;
    for (uint32_t q = gl; q < npairs; q += kSmallG, b += kSmallG) {
      while (b >= c) {   // next row: row a + 1 starts at b = a + 2
        const uint32_t over = b - c;
        a++;
        b = a + 1 + over;
      }
      const uint32_t x = cv[b];
      const uint32_t wa = cv[a];
      if (R == 3) {
        // as in k_count_s4: x in W(u wa) iff wa and x are adjacent; the two
        // slots name triangles {u, wa, x} and {v, wa, x}
        const uint32_t euw = ceu[a], evw = cev[a];
        const uint64_t b1 = g.wp[euw], f1 = g.wp[euw + 1], b2 = g.wp[evw], f2 = g.wp[evw + 1];
        uint64_t p1, p2;
        find2_u32<uint64_t>(g.wc, b1, f1, b2, f2, x, p1, p2);
        if (p1 == f1) continue;
        local++;
        atomicAdd(&cn[a], 1u);
        atomicAdd(&cn[b], 1u);
        atomicAdd(&cnt[g.wt[p1]], 1u);
        if (p2 == f2) atomicOr(&sc->status, ND_DERR_BADGRAPH);
        else atomicAdd(&cnt[g.wt[p2]], 1u);
        continue;
      }
      uint32_t lowv = wa, highv = x;
      if (g.okey[x] < g.okey[wa]) { lowv = x; highv = wa; }
      const uint64_t bl = g.dgp[lowv], el = g.dgp[lowv + 1];
      const uint64_t p = find_u32<uint64_t>(g.dgc, bl, el, highv);
      if (p == el) continue;
      local++;
      if (R == 1) {
        atomicAdd(&cnt[u], 1u);
        atomicAdd(&cnt[v], 1u);
        atomicAdd(&cnt[wa], 1u);
        atomicAdd(&cnt[x], 1u);
      } else if (R == 2) {
        const uint32_t e6[6] = {e_uv, ceu[a], cev[a], ceu[b], cev[b], g.dge[p]};
        count_edges6<kWrap>(cnt, e6, sc);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (R == 3 && gl < c && cn[gl] != 0) {
      const uint32_t t = tri_lookup(g, u, v, cv[gl], e_uv, ceu[gl], cev[gl]);
      if (t == ND_NONE) atomicOr(&sc->status, ND_DERR_BADGRAPH);
      else atomicAdd(&cnt[t], cn[gl]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  local = wave_sum64(local);
  if (lane == 0 && local) atomicAdd((unsigned long long *)&sc->n_s, (unsigned long long)local);
}

// The three 4-clique kernels of one r: rows of at most kSmallG
// out-neighbours in 16-lane groups, rows up to kC2Cap with C2 on chip, heavier
// rows (a graph of degeneracy above kC2Cap, or every row with
// ND_FLAG_COUNT_GLOBAL) with C2 in a global slice per wave.
template <int R, bool kWrap>
nd_status launch_count_s4(nd_ctx *c, const GraphView &g, uint32_t *cnt, DevScalars *sc,
                          uint32_t maxd, bool force_global) {
  nd_status st;
  const uint32_t light = force_global ? 0u : std::min<uint32_t>(maxd, kC2Cap);
  const uint32_t small = force_global ? 0u : kSmallG;
  constexpr uint32_t arrays = count_s4_arrays<R>();
  if (small) {
    const uint32_t grid = nd_grid(g.m, (kCountBlock / 64) * (64 / kSmallG), 65536);
    hipLaunchKernelGGL((k_count_s4_small<R, kWrap>), dim3(grid), dim3(kCountBlock), 0, c->stream,
                       g, cnt, sc);
  }
  if (light > small) {
    const uint32_t cap = std::max<uint32_t>(64, (light + 63) / 64 * 64);
    const uint32_t grid = nd_grid(g.m, kCountBlock / 64, 65536);
    const size_t lds = (size_t)(kCountBlock / 64) * arrays * cap * 4;
    if ((st = nd_hip(c, hipFuncSetAttribute((const void *)k_count_s4<R, false, kWrap>,
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                     "count LDS size")) != ND_OK)
      return st;
    hipLaunchKernelGGL((k_count_s4<R, false, kWrap>), dim3(grid), dim3(kCountBlock), lds,
                       c->stream, g, cnt, sc, cap, nullptr, 0u, small);
  }
  if (force_global || maxd > kC2Cap) {
    const uint32_t cap = std::max<uint32_t>(64, (maxd + 63) / 64 * 64);
    // waves of the global kernel: as many as 1 GiB of C2 slices holds,
    // between 64 and 65,536
    const uint64_t per_wave = (uint64_t)arrays * cap * 4;
    const uint64_t waves = std::max<uint64_t>(64, std::min<uint64_t>(65536, (1ull << 30) / per_wave));
    uint32_t *gbuf = (uint32_t *)nd_buf(c, B_C2G, waves * per_wave, &st);
    if (!gbuf) return st;
    const uint32_t grid = (uint32_t)(waves / (kCountBlock / 64));
    hipLaunchKernelGGL((k_count_s4<R, true, kWrap>), dim3(grid), dim3(kCountBlock), 0, c->stream,
                       g, cnt, sc, cap, gbuf, light, 0u);
  }
  return ND_OK;
}

}  // namespace

nd_status nd_stage_count(nd_ctx *c, const GraphView &g) {
  nd_status st;
  DevScalars *sc = (DevScalars *)c->bufs[B_SCAL].p;
  const uint64_t nr = c->n_r;
  uint32_t *cnt = (uint32_t *)nd_buf(c, B_CNT, std::max<uint64_t>(nr, 1) * 4, &st);
  if (!cnt) return st;
  uint32_t *cnt0 = (uint32_t *)nd_buf(c, B_CNT0, std::max<uint64_t>(nr, 1) * 4, &st);
  if (!cnt0) return st;
  st = nd_hip(c, hipMemsetAsync(&sc->n_s, 0, 8, c->stream), "memset n_s");
  if (st != ND_OK) return st;
  if (nr) {
    st = nd_hip(c, hipMemsetAsync(cnt, 0, nr * 4, c->stream), "memset cnt");
    if (st != ND_OK) return st;
  }
  const uint32_t r = c->r, s = c->s;
  if (c->events_ok) (void)hipEventRecord(c->ev[7], c->stream);
  if (nd_rs_general(s)) {
    // s = 5..7: the s-cliques were listed once in prep; a count is the
    // length of the r-clique's incidence list
    if (nr)
      hipLaunchKernelGGL(k_count_inc, dim3(nd_grid(nr, 256, 16384)), dim3(256), 0, c->stream, nr,
                         g.io, cnt);
    const uint64_t ns = c->gen_n_s;
    st = nd_hip(c, hipMemcpyAsync(&sc->n_s, &ns, 8, hipMemcpyHostToDevice, c->stream), "n_s");
    if (st != ND_OK) return st;
    st = nd_hip(c, hipStreamSynchronize(c->stream), "n_s");
    if (st != ND_OK) return st;
  } else if (s == 2) {
    if (g.n)
      hipLaunchKernelGGL(k_count_degree, dim3(nd_grid(g.n, 256, 8192)), dim3(256), 0, c->stream,
                         g.n, g.rp, cnt);
    uint64_t ns = g.m;
    st = nd_hip(c, hipMemcpyAsync(&sc->n_s, &ns, 8, hipMemcpyHostToDevice, c->stream), "n_s");
    if (st != ND_OK) return st;
  } else if (s == 3 && g.m) {
    const uint32_t grid = nd_grid(g.m, kCountBlock, 16384);
    if (r == 1)
      hipLaunchKernelGGL(k_count_s3<1>, dim3(grid), dim3(kCountBlock), 0, c->stream, g, cnt, sc);
    else
      hipLaunchKernelGGL(k_count_s3<2>, dim3(grid), dim3(kCountBlock), 0, c->stream, g, cnt, sc);
  } else if (s == 4 && g.m) {
    // C2 (common out-neighbours of an edge) has at most max-out-degree
    // entries: the LDS arrays are sized to it, so that more workgroups fit;
    // (2,4) also reads the largest triangle count of an edge, which bounds
    // its counts by C(t, 2)
    uint32_t maxd = 0, maxsup = 0;
    if ((st = nd_hip(c, hipMemcpyAsync(&maxd, &sc->max_outdeg, 4, hipMemcpyDeviceToHost,
                                       c->stream), "max out-degree")) != ND_OK ||
        (st = nd_hip(c, hipMemcpyAsync(&maxsup, &sc->max_sup, 4, hipMemcpyDeviceToHost,
                                       c->stream), "max support")) != ND_OK ||
        (st = nd_hip(c, hipStreamSynchronize(c->stream), "max out-degree")) != ND_OK)
      return st;
    c->info.max_outdeg = maxd;
    const bool force_global = (c->flags & ND_FLAG_COUNT_GLOBAL) != 0;
    if (r == 1) {
      st = launch_count_s4<1, false>(c, g, cnt, sc, maxd, force_global);
    } else if (r == 2) {
      const bool wrap = (uint64_t)maxsup * (maxsup - (maxsup ? 1 : 0)) / 2 > 0xFFFFFFFFull;
      st = wrap ? launch_count_s4<2, true>(c, g, cnt, sc, maxd, force_global)
                : launch_count_s4<2, false>(c, g, cnt, sc, maxd, force_global);
    } else {
      st = launch_count_s4<3, false>(c, g, cnt, sc, maxd, force_global);
    }
    if (st != ND_OK) return st;
  }
  st = nd_hip(c, hipGetLastError(), "count kernels");
  if (c->events_ok) (void)hipEventRecord(c->ev[8], c->stream);
  if (st != ND_OK) return st;
  if (nr)
    st = nd_hip(c, hipMemcpyAsync(cnt0, cnt, nr * 4, hipMemcpyDeviceToDevice, c->stream),
                "copy counts");
  return st;
}
