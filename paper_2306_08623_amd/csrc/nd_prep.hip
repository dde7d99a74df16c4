// nd_prep.hip -- graph preparation on the device:
//   * CSR validation (simple undirected graph, Section 3);
//   * dense edge ids: the id of undirected edge {u<v} is its rank in
//     lexicographic order, and every CSR slot knows the id of its edge;
//   * low out-degree orientation (Section 3: an O(alpha)-orientation, as used
//     by Algorithm 3's Arb-Orient): rounds that remove every remaining vertex
//     whose remaining degree is at most (1+eps) times the remaining average;
//     vertices are ordered by (removal round, degree, id) and each edge points
//     from the earlier to the later vertex;
//   * the oriented out-CSR (DG);
//   * for r = 3, the edge -> triangle tables: for every edge e = {u<v} the
//     ascending list W(e) of common neighbours of u and v with the id of each
//     triangle; triangle ids are lexicographic in (a<b<c).
#include "nd_internal.h"

#include <algorithm>

namespace {

constexpr uint32_t kScanBlock = 256;
constexpr uint32_t kScanItems = 8;
constexpr uint64_t kScanTile = (uint64_t)kScanBlock * kScanItems;

// ---------------------------------------------------------------------------
// exclusive scan (u32 or u64 input -> u64 output with the total at out[n])
// ---------------------------------------------------------------------------

template <typename InT>
__global__ void __launch_bounds__(kScanBlock) k_scan_tile(const InT *__restrict__ in,
                                                          uint64_t *__restrict__ out, uint64_t n,
                                                          uint64_t *__restrict__ tile_sums) {
  __shared__ uint64_t s_in[kScanTile];
  __shared__ uint64_t s_part[kScanBlock];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  // coalesced load into LDS
  for (uint32_t i = threadIdx.x; i < kScanTile; i += kScanBlock) {
    uint64_t idx = base + i;
    s_in[i] = idx < n ? (uint64_t)in[idx] : 0;
  }
  __syncthreads();
  uint64_t sum = 0;
#pragma unroll
  for (uint32_t i = 0; i < kScanItems; i++) sum += s_in[threadIdx.x * kScanItems + i];
  s_part[threadIdx.x] = sum;
  __syncthreads();
  for (uint32_t d = 1; d < kScanBlock; d <<= 1) {
    uint64_t t = threadIdx.x >= d ? s_part[threadIdx.x - d] : 0;
    __syncthreads();
    s_part[threadIdx.x] += t;
    __syncthreads();
  }
  uint64_t run = s_part[threadIdx.x] - sum;
#pragma unroll
  for (uint32_t i = 0; i < kScanItems; i++) {
    uint64_t v = s_in[threadIdx.x * kScanItems + i];
    s_in[threadIdx.x * kScanItems + i] = run;
    run += v;
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < kScanTile; i += kScanBlock) {
    uint64_t idx = base + i;
    if (idx < n) out[idx] = s_in[i];
  }
  if (threadIdx.x == kScanBlock - 1) tile_sums[blockIdx.x] = s_part[kScanBlock - 1];
}

__global__ void k_scan_add(uint64_t *__restrict__ out, uint64_t n,
                           const uint64_t *__restrict__ tile_off) {
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  const uint64_t add = tile_off[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < kScanTile; i += blockDim.x) {
    uint64_t idx = base + i;
    if (idx < n) out[idx] += add;
  }
}

__global__ void k_scan_total(uint64_t *out, uint64_t n, const uint64_t *tile_sums,
                             const uint64_t *tile_off, uint32_t ntiles) {
  // total = offset of the last tile + its sum
  out[n] = tile_off[ntiles - 1] + tile_sums[ntiles - 1];
}

__global__ void k_scan_single_total(uint64_t *out, uint64_t n, const uint64_t *tile_sums) {
  out[n] = tile_sums[0];
}

template <typename InT>
nd_status scan_impl(nd_ctx *c, const InT *in, uint64_t *out, uint64_t n, uint64_t *scratch) {
  // out must have n+1 entries; scratch holds the tile sums of all levels
  if (n == 0) {
    uint64_t z = 0;
    return nd_hip(c, hipMemcpyAsync(out, &z, sizeof(z), hipMemcpyHostToDevice, c->stream),
                  "scan zero");
  }
  const uint32_t ntiles = (uint32_t)((n + kScanTile - 1) / kScanTile);
  uint64_t *tile_sums = scratch;
  uint64_t *tile_off = scratch + ntiles;
  hipLaunchKernelGGL(k_scan_tile<InT>, dim3(ntiles), dim3(kScanBlock), 0, c->stream, in, out, n,
                     tile_sums);
  if (ntiles == 1) {
    hipLaunchKernelGGL(k_scan_single_total, dim3(1), dim3(1), 0, c->stream, out, n, tile_sums);
    return nd_hip(c, hipGetLastError(), "scan");
  }
  nd_status st = scan_impl<uint64_t>(c, tile_sums, tile_off, ntiles, scratch + 2 * ntiles + 1);
  if (st != ND_OK) return st;
  hipLaunchKernelGGL(k_scan_add, dim3(ntiles), dim3(kScanBlock), 0, c->stream, out, n, tile_off);
  hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, c->stream, out, n, tile_sums, tile_off,
                     ntiles);
  return nd_hip(c, hipGetLastError(), "scan");
}

size_t scan_scratch_elems(uint64_t n) {
  size_t tot = 0;
  while (n > 1) {
    uint64_t nt = (n + kScanTile - 1) / kScanTile;
    tot += 2 * nt + 1;
    n = nt;
  }
  return tot + 4;
}

// ---------------------------------------------------------------------------
// validation and edge ids
// ---------------------------------------------------------------------------

__global__ void k_check_rowptr(uint32_t n, uint64_t nnz, const uint64_t *__restrict__ rp,
                               uint32_t *status) {
  for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u <= n;
       u += (uint64_t)gridDim.x * blockDim.x) {
    bool bad = false;
    if (u == 0 && rp[0] != 0) bad = true;
    if (u == n && rp[n] != nnz) bad = true;
    if (u < n && rp[u] > rp[u + 1]) bad = true;
    if (rp[u] > nnz) bad = true;
    if (bad) atomicOr(status, ND_DERR_BADGRAPH);
  }
}

// Row u: ids < n, strictly ascending, no self-loop, twin slot present.
__global__ void k_check_slots(uint32_t n, uint64_t nnz, const uint64_t *__restrict__ rp,
                              const uint32_t *__restrict__ col, uint32_t *status) {
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < nnz;
       j += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t u = segment_of(rp, n, j);
    uint32_t v = col[j];
    bool bad = v >= n || v == u || (j > rp[u] && col[j - 1] >= v);
    if (!bad) bad = find_u32<uint64_t>(col, rp[v], rp[v + 1], u) == rp[v + 1];
    if (bad) atomicOr(status, ND_DERR_BADGRAPH);
  }
}

// uplo[u] = number of neighbours of u smaller than u; upcnt[u] = the rest.
__global__ void k_uplo(uint32_t n, const uint64_t *__restrict__ rp, const uint32_t *__restrict__ col,
                       uint32_t *__restrict__ uplo, uint32_t *__restrict__ upcnt,
                       uint32_t *__restrict__ deg) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    uint64_t b = rp[u], e = rp[u + 1];
    uint64_t p = lower_bound_u32<uint64_t>(col, b, e, u);
    uplo[u] = (uint32_t)(p - b);
    upcnt[u] = (uint32_t)(e - p);
    deg[u] = (uint32_t)(e - b);
  }
}

__global__ void k_edge_ids(uint32_t n, uint64_t nnz, const uint64_t *__restrict__ rp,
                           const uint32_t *__restrict__ col, const uint32_t *__restrict__ uplo,
                           const uint64_t *__restrict__ eoff, uint32_t *__restrict__ eid,
                           uint32_t *__restrict__ eu, uint32_t *__restrict__ ev) {
  for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < nnz;
       j += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t u = segment_of(rp, n, j);
    uint32_t v = col[j];
    uint32_t id;
    if (v > u) {
      id = (uint32_t)(eoff[u] + (j - rp[u] - uplo[u]));
      eu[id] = u;
      ev[id] = v;
    } else {
      uint64_t jj = find_u32<uint64_t>(col, rp[v], rp[v + 1], u);
      id = (uint32_t)(eoff[v] + (jj - rp[v] - uplo[v]));
    }
    eid[j] = id;
  }
}

// ---------------------------------------------------------------------------
// orientation: persistent rounds with grid barriers
// ---------------------------------------------------------------------------

struct OrientArgs {
  uint32_t n;
  const uint64_t *rp;
  const uint32_t *col;
  uint32_t *rdeg;     // remaining degree
  uint32_t *orank;    // removal round (ND_NONE while present)
  DevScalars *sc;
  uint64_t *sums;     // [2 * 2]: (left, degsum) by round parity
  uint32_t nblocks;
};

constexpr uint32_t kOrientBlock = 256;
constexpr uint32_t kOrientMaxRounds = 255;

__global__ void __launch_bounds__(kOrientBlock) k_orient(OrientArgs a) {
  __shared__ uint64_t s_left[kOrientBlock / 64], s_sum[kOrientBlock / 64];
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nth = gridDim.x * blockDim.x;
  if (!residency_gate(a.sc->bar, a.nblocks, &a.sc->status)) return;
  for (uint32_t round = 0;; round++) {
    uint64_t *cur = a.sums + 2 * (round & 1);
    uint64_t *nxt = a.sums + 2 * ((round + 1) & 1);
    // phase 1: remaining count and degree sum
    uint64_t left = 0, sum = 0;
    for (uint32_t v = tid; v < a.n; v += nth) {
      if (a.orank[v] == ND_NONE) {
        left++;
        sum += a.rdeg[v];
      }
    }
    left = wave_sum64(left);
    sum = wave_sum64(sum);
    if (lane_id() == 0) {
      s_left[threadIdx.x / 64] = left;
      s_sum[threadIdx.x / 64] = sum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t L = 0, S = 0;
      for (uint32_t w = 0; w < kOrientBlock / 64; w++) {
        L += s_left[w];
        S += s_sum[w];
      }
      if (L) atomicAdd((unsigned long long *)&cur[0], (unsigned long long)L);
      if (S) atomicAdd((unsigned long long *)&cur[1], (unsigned long long)S);
      if (blockIdx.x == 0) {   // clear next round's slots (nobody reads them now)
        nxt[0] = 0;
        nxt[1] = 0;
      }
    }
    if (!grid_barrier(a.sc->bar, a.nblocks, &a.sc->status)) return;
    const uint64_t L = ld_acq64(&cur[0]);
    const uint64_t S = ld_acq64(&cur[1]);
    if (L == 0) {
      if (tid == 0) a.sc->orient_round = round;
      return;
    }
    // phase 2: remove vertices with remaining degree <= 1.5 * average
    const bool last = round >= kOrientMaxRounds;
    for (uint32_t v = tid; v < a.n; v += nth) {
      if (a.orank[v] == ND_NONE && (last || 2ull * a.rdeg[v] * L <= 3ull * S)) a.orank[v] = round;
    }
    if (!grid_barrier(a.sc->bar, a.nblocks, &a.sc->status)) return;
    // phase 3: removed vertices lower their remaining neighbours' degrees
    for (uint32_t v = tid; v < a.n; v += nth) {
      if (a.orank[v] != round) continue;
      for (uint64_t j = a.rp[v]; j < a.rp[v + 1]; j++) {
        uint32_t w = a.col[j];
        if (a.orank[w] == ND_NONE) atomicSub(&a.rdeg[w], 1u);
      }
    }
    if (!grid_barrier(a.sc->bar, a.nblocks, &a.sc->status)) return;
  }
}

__global__ void k_okey(uint32_t n, const uint32_t *__restrict__ orank,
                       const uint32_t *__restrict__ deg, uint64_t *__restrict__ okey) {
  for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    uint64_t d = deg[v] > 0xFFFFFFu ? 0xFFFFFFu : deg[v];
    okey[v] = ((uint64_t)orank[v] << 56) | (d << 32) | v;
  }
}

__global__ void k_dg_count(uint32_t n, const uint64_t *__restrict__ rp,
                           const uint32_t *__restrict__ col, const uint64_t *__restrict__ okey,
                           uint32_t *__restrict__ dgcnt, DevScalars *sc) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    uint64_t ku = okey[u];
    uint32_t c = 0;
    for (uint64_t j = rp[u]; j < rp[u + 1]; j++) c += okey[col[j]] > ku;
    dgcnt[u] = c;
    if (c) atomicMax(&sc->max_outdeg, c);
  }
}

__global__ void k_dg_fill(uint32_t n, const uint64_t *__restrict__ rp,
                          const uint32_t *__restrict__ col, const uint32_t *__restrict__ eid,
                          const uint64_t *__restrict__ okey, const uint64_t *__restrict__ dgp,
                          uint32_t *__restrict__ dgc, uint32_t *__restrict__ dge) {
  for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
    uint64_t ku = okey[u];
    uint64_t o = dgp[u];
    for (uint64_t j = rp[u]; j < rp[u + 1]; j++) {
      uint32_t v = col[j];
      if (okey[v] > ku) {
        dgc[o] = v;
        dge[o] = eid[j];
        o++;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// edge -> triangle tables (r = 3)
// ---------------------------------------------------------------------------

// Triangle lists W(e) of every edge e = {u, v}, one wave per edge: the lanes
// take the entries of the shorter of N(u), N(v), 64 at a time in ascending
// order, and binary-search them in the longer list, so that an edge between
// two hubs is spread over the wave instead of one thread. Common neighbours
// come out in ascending order (ballot compaction in lane order).
constexpr uint32_t kEtlBlock = 256;

struct CommonScan {
  uint64_t as, ae, bs, be;   // probed (shorter) list, searched list
  bool u_short;              // the probed list is N(u)
};

__device__ __forceinline__ CommonScan common_scan(const uint64_t *rp, uint32_t u, uint32_t v) {
  CommonScan c;
  const uint64_t bu = rp[u], eu_ = rp[u + 1], bv = rp[v], ev_ = rp[v + 1];
  c.u_short = eu_ - bu <= ev_ - bv;
  c.as = c.u_short ? bu : bv;
  c.ae = c.u_short ? eu_ : ev_;
  c.bs = c.u_short ? bv : bu;
  c.be = c.u_short ? ev_ : eu_;
  return c;
}

// Edge -> triangle lists, in groups of G lanes per edge: G = 64 for edges
// whose shorter adjacency list has more than kEtlSmall entries, G = 16 for
// the others (four edges per wave; sparse graphs have mostly short lists).
// A group probes the shorter list G entries at a time and binary-searches
// each entry in the longer one; hits are compacted in lane order, so W(e)
// comes out ascending.
constexpr uint32_t kEtlSmall = 32;
constexpr uint32_t kEtlSmallG = 16;

template <uint32_t G>
__device__ __forceinline__ uint64_t group_bits(uint64_t mask, uint32_t gi) {
  return G == 64 ? mask : (mask >> (gi * G)) & ((1ull << G) - 1);
}

template <uint32_t G>
__device__ __forceinline__ bool etl_mine(const CommonScan &c) {
  return G == 64 ? c.ae - c.as > kEtlSmall : c.ae - c.as <= kEtlSmall;
}

template <uint32_t G>
__global__ void __launch_bounds__(kEtlBlock) k_etl_count(uint64_t m, const uint64_t *__restrict__ rp,
                                                         const uint32_t *__restrict__ col,
                                                         const uint32_t *__restrict__ eu,
                                                         const uint32_t *__restrict__ ev,
                                                         uint32_t *__restrict__ sup,
                                                         uint32_t *__restrict__ upc) {
  constexpr uint32_t kGroups = 64 / G;
  const uint32_t lane = lane_id(), gi = lane / G, gl = lane % G;
  const uint64_t ngroups = (uint64_t)gridDim.x * (kEtlBlock / 64) * kGroups;
  for (uint64_t e = ((uint64_t)blockIdx.x * (kEtlBlock / 64) + threadIdx.x / 64) * kGroups + gi;
       e < m; e += ngroups) {
    const uint32_t u = eu[e], v = ev[e];
    const CommonScan c = common_scan(rp, u, v);
    if (!etl_mine<G>(c)) continue;
    uint32_t s = 0, up = 0;
    for (uint64_t base = c.as; base < c.ae; base += G) {
      const uint64_t i = base + gl;
      bool hit = false, above = false;
      if (i < c.ae) {
        const uint32_t w = col[i];
        hit = find_u32<uint64_t>(col, c.bs, c.be, w) < c.be;
        above = hit && w > v;
      }
      s += __popcll(group_bits<G>(ballot64(hit), gi));
      up += __popcll(group_bits<G>(ballot64(above), gi));
    }
    if (gl == 0) {
      sup[e] = s;
      upc[e] = up;
    }
  }
}

template <uint32_t G>
__global__ void __launch_bounds__(kEtlBlock) k_etl_fill(uint64_t m, const uint64_t *__restrict__ rp,
                                                        const uint32_t *__restrict__ col,
                                                        const uint32_t *__restrict__ eid,
                                                        const uint32_t *__restrict__ eu,
                                                        const uint32_t *__restrict__ ev,
                                                        const uint32_t *__restrict__ sup,
                                                        const uint32_t *__restrict__ upc,
                                                        const uint64_t *__restrict__ wp,
                                                        const uint64_t *__restrict__ trib,
                                                        uint32_t *__restrict__ wc,
                                                        uint32_t *__restrict__ wt,
                                                        uint32_t *__restrict__ te) {
  constexpr uint32_t kGroups = 64 / G;
  const uint32_t lane = lane_id(), gi = lane / G, gl = lane % G;
  const uint64_t ngroups = (uint64_t)gridDim.x * (kEtlBlock / 64) * kGroups;
  for (uint64_t e = ((uint64_t)blockIdx.x * (kEtlBlock / 64) + threadIdx.x / 64) * kGroups + gi;
       e < m; e += ngroups) {
    const uint32_t u = eu[e], v = ev[e];
    const CommonScan c = common_scan(rp, u, v);
    if (!etl_mine<G>(c)) continue;
    uint64_t o = wp[e];
    const uint64_t first_up = wp[e] + (sup[e] - upc[e]);
    const uint64_t tb = trib[e];
    for (uint64_t base = c.as; base < c.ae; base += G) {
      const uint64_t i = base + gl;
      bool hit = false;
      uint32_t w = 0;
      uint64_t p = 0;
      if (i < c.ae) {
        w = col[i];
        p = find_u32<uint64_t>(col, c.bs, c.be, w);
        hit = p < c.be;
      }
      const uint64_t mask = group_bits<G>(ballot64(hit), gi);
      if (hit) {
        const uint64_t below = mask & ((1ull << gl) - 1);
        const uint64_t slot = o + __popcll(below);
        const uint64_t su = c.u_short ? i : p, sv = c.u_short ? p : i;   // w's slots in N(u), N(v)
        wc[slot] = w;
        if (w > v) {
          // triangle (u, v, w) owned by this edge
          const uint64_t t = tb + (slot - first_up);
          wt[slot] = (uint32_t)t;
          te[3 * t + 0] = (uint32_t)e;
          te[3 * t + 1] = eid[su];
          te[3 * t + 2] = eid[sv];
        } else {
          // owner is edge {u, w}: resolved once every list is filled
          wt[slot] = eid[su];
        }
      }
      o += __popcll(mask);
    }
  }
}

__global__ void k_etl_resolve(uint64_t m, uint64_t nw, const uint32_t *__restrict__ ev,
                              const uint64_t *__restrict__ wp, const uint32_t *__restrict__ wc,
                              uint32_t *__restrict__ wt, uint32_t *status) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nw;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t e = segment_of(wp, (uint32_t)m, i);
    uint32_t v = ev[e];
    if (wc[i] < v) {
      uint32_t owner = wt[i];
      const uint64_t end = wp[owner + 1];
      uint64_t p = find_u32<uint64_t>(wc, wp[owner], end, v);
      if (p == end) {   // impossible for a valid graph; never read past the list
        atomicOr(status, ND_DERR_BADGRAPH);
        continue;
      }
      wt[i] = wt[p];
    }
  }
}

__global__ void k_max_u32(const uint32_t *__restrict__ a, uint64_t n, uint32_t *out) {
  uint32_t mx = 0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    mx = a[i] > mx ? a[i] : mx;
  for (int d = 32; d >= 1; d >>= 1) {
    uint32_t o = __shfl_xor(mx, d, 64);
    mx = o > mx ? o : mx;
  }
  if (lane_id() == 0 && mx) atomicMax(out, mx);
}

}  // namespace

nd_status nd_exclusive_scan_u64(nd_ctx *c, const uint64_t *in, uint64_t *out, uint64_t n,
                                uint64_t *total_host) {
  nd_status st;
  uint64_t *scratch = (uint64_t *)nd_buf(c, B_TMP64, scan_scratch_elems(n) * 8, &st);
  if (!scratch) return st;
  st = scan_impl<uint64_t>(c, in, out, n, scratch);
  if (st != ND_OK || !total_host) return st;
  st = nd_hip(c, hipMemcpyAsync(total_host, out + n, 8, hipMemcpyDeviceToHost, c->stream),
              "scan total");
  if (st != ND_OK) return st;
  return nd_hip(c, hipStreamSynchronize(c->stream), "scan sync");
}

nd_status nd_exclusive_scan_u32_to_u64(nd_ctx *c, const uint32_t *in, uint64_t *out, uint64_t n,
                                       uint64_t *total_host) {
  nd_status st;
  uint64_t *scratch = (uint64_t *)nd_buf(c, B_TMP64, scan_scratch_elems(n) * 8, &st);
  if (!scratch) return st;
  st = scan_impl<uint32_t>(c, in, out, n, scratch);
  if (st != ND_OK || !total_host) return st;
  st = nd_hip(c, hipMemcpyAsync(total_host, out + n, 8, hipMemcpyDeviceToHost, c->stream),
              "scan total");
  if (st != ND_OK) return st;
  return nd_hip(c, hipStreamSynchronize(c->stream), "scan sync");
}

// Validation of a CSR already resident in the context's buffers.
nd_status nd_validate_loaded(nd_ctx *c) {
  nd_status st;
  DevScalars *sc = (DevScalars *)nd_buf(c, B_SCAL, sizeof(DevScalars), &st);
  if (!sc) return st;
  const uint64_t *rp = (const uint64_t *)c->bufs[B_RP].p;
  const uint32_t *col = (const uint32_t *)c->bufs[B_COL].p;
  st = nd_hip(c, hipMemsetAsync(sc, 0, sizeof(DevScalars), c->stream), "memset scalars");
  if (st != ND_OK) return st;
  hipLaunchKernelGGL(k_check_rowptr, dim3(nd_grid(c->n + 1ull, 256, 4096)), dim3(256), 0,
                     c->stream, c->n, c->nnz, rp, &sc->status);
  uint32_t status = 0;
  st = nd_hip(c, hipMemcpyAsync(&status, &sc->status, 4, hipMemcpyDeviceToHost, c->stream),
              "validate readback");
  if (st != ND_OK) return st;
  st = nd_hip(c, hipStreamSynchronize(c->stream), "validate sync");
  if (st != ND_OK) return st;
  if (status) return nd_fail(c, ND_E_BAD_GRAPH, "row_ptr is not a valid offset array");
  if (c->nnz) {
    hipLaunchKernelGGL(k_check_slots, dim3(nd_grid(c->nnz, 256, 16384)), dim3(256), 0, c->stream,
                       c->n, c->nnz, rp, col, &sc->status);
    st = nd_hip(c, hipMemcpyAsync(&status, &sc->status, 4, hipMemcpyDeviceToHost, c->stream),
                "validate readback");
    if (st != ND_OK) return st;
    st = nd_hip(c, hipStreamSynchronize(c->stream), "validate sync");
    if (st != ND_OK) return st;
    if (status)
      return nd_fail(c, ND_E_BAD_GRAPH,
                     "CSR is not a simple undirected graph (unsorted row, duplicate, self-loop, "
                     "id >= n or missing reverse edge)");
  }
  return ND_OK;
}

// (2,4): for each W entry (edge e = {u,v}, third vertex w, triangle t), the
// candidates x > w of t's 4-cliques lie in the parts above w of W(e),
// W(x1), W(x2) (x1, x2 = t's other edges, in te order); the shortest of the
// three parts is probed. sel[p] = (list index << 30) | start offset of the
// part inside its list; len[p] = its length. One thread per edge.
__global__ void k_w24_len(uint64_t m, const uint64_t *__restrict__ wp,
                          const uint32_t *__restrict__ wc, const uint32_t *__restrict__ wt,
                          const uint32_t *__restrict__ te, uint32_t *__restrict__ len,
                          uint32_t *__restrict__ sel) {
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t b = wp[e], f = wp[e + 1];
    for (uint64_t p = b; p < f; p++) {
      const uint32_t w = wc[p];
      const uint64_t t = wt[p];
      uint32_t xs[2], nx = 0;
      for (int q = 0; q < 3; q++) {
        const uint32_t z = te[3 * t + q];
        if (z != (uint32_t)e && nx < 2) xs[nx++] = z;
      }
      uint64_t best = f - p - 1;   // W(e) above w: the entries after p
      uint32_t bsel = 0, boff = (uint32_t)(p + 1 - b);
      for (int q = 0; q < 2; q++) {
        const uint64_t lb = wp[xs[q]], lf = wp[xs[q] + 1];
        const uint64_t first = upper_bound_u32(wc, lb, lf, w);
        if (lf - first < best) {
          best = lf - first;
          bsel = (uint32_t)q + 1;
          boff = (uint32_t)(first - lb);
        }
      }
      len[p] = (uint32_t)best;
      sel[p] = (bsel << 30) | boff;
    }
  }
}

// (1,3): for CSR slot q = (v -> w), the entries of W(vw) above w
__global__ void k_slot_tris(uint64_t nnz, const uint32_t *__restrict__ col,
                            const uint32_t *__restrict__ eid, const uint64_t *__restrict__ wp,
                            const uint32_t *__restrict__ wc, uint32_t *__restrict__ scnt) {
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < nnz;
       q += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t e = eid[q], w = col[q];
    const uint64_t b = wp[e], f = wp[e + 1];
    scnt[q] = (uint32_t)(f - upper_bound_u32(wc, b, f, w));
  }
}

// (1,4): one thread per CSR slot v -> w; for each triangle probe (entry x
// above w of W(vw)) the shortest of the parts above x of W(vw), W(vx), W(wx)
__global__ void k_t14_len(uint64_t nnz, const uint64_t *__restrict__ rp,
                          const uint32_t *__restrict__ col, const uint32_t *__restrict__ eid,
                          const uint32_t *__restrict__ eu, const uint32_t *__restrict__ ev,
                          const uint64_t *__restrict__ wp,
                          const uint32_t *__restrict__ wc, const uint32_t *__restrict__ wt,
                          const uint32_t *__restrict__ te, const uint64_t *__restrict__ sg,
                          uint32_t *__restrict__ tlen, uint32_t *__restrict__ tsel, uint32_t n) {
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < nnz;
       q += (uint64_t)gridDim.x * blockDim.x) {
    // the row v of slot q
    uint64_t lo = 0, hi = n;   // last v with rp[v] <= q
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (rp[mid] <= q) lo = mid;
      else hi = mid;
    }
    const uint32_t v = (uint32_t)lo, w = col[q], e = eid[q];
    const uint64_t b = wp[e], f = wp[e + 1];
    const uint64_t first = upper_bound_u32(wc, b, f, w);
    uint64_t gi = sg[q];
    for (uint64_t p = first; p < f; p++, gi++) {
      const uint32_t x = wc[p];
      const uint64_t t = wt[p];
      // the triangle's edges other than {v,w}: {v,x} (contains v) and {w,x}
      uint32_t evx = ND_NONE, ewx = ND_NONE;
      for (int k = 0; k < 3; k++) {
        const uint32_t z = te[3 * t + k];
        if (z == e) continue;
        if (eu[z] == v || ev[z] == v) evx = z;
        else ewx = z;
      }
      uint64_t best = f - p - 1;   // W(vw) above x: the entries after p
      uint32_t bsel = 0, boff = (uint32_t)(p + 1 - b);
      const uint32_t lists[2] = {evx, ewx};
      for (int k = 0; k < 2; k++) {
        const uint64_t lb = wp[lists[k]], lf = wp[lists[k] + 1];
        const uint64_t fst = upper_bound_u32(wc, lb, lf, x);
        if (lf - fst < best) {
          best = lf - fst;
          bsel = (uint32_t)k + 1;
          boff = (uint32_t)(fst - lb);
        }
      }
      tlen[gi] = (uint32_t)best;
      tsel[gi] = (bsel << 30) | boff;
    }
  }
}

// a vertex's triangles ((1,3): its s-clique count and probe range) must
// stay below 2^32
__global__ void k_t13_check(uint32_t n, const uint64_t *__restrict__ rp,
                            const uint64_t *__restrict__ sg, uint32_t *status) {
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n;
       v += (uint64_t)gridDim.x * blockDim.x)
    if (sg[rp[v + 1]] - sg[rp[v]] >= 0xFFFFFFFFull) atomicOr(status, ND_DERR_OVERFLOW);
}

// a vertex's (1,4) probe range must stay below 2^32 entries
__global__ void k_t14_check(uint32_t n, const uint64_t *__restrict__ rp,
                            const uint64_t *__restrict__ sg, const uint64_t *__restrict__ tg,
                            uint32_t *status) {
  for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n;
       v += (uint64_t)gridDim.x * blockDim.x)
    if (tg[sg[rp[v + 1]]] - tg[sg[rp[v]]] >= 0xFFFFFFFFull) atomicOr(status, ND_DERR_OVERFLOW);
}

// an edge's probe range must stay below 2^32 entries (32-bit work items)
__global__ void k_w24_check(uint64_t m, const uint64_t *__restrict__ wp,
                            const uint64_t *__restrict__ wg, uint32_t *status) {
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
       e += (uint64_t)gridDim.x * blockDim.x)
    if (wg[wp[e + 1]] - wg[wp[e]] >= 0xFFFFFFFFull) atomicOr(status, ND_DERR_OVERFLOW);
}

static uint32_t coop_blocks(nd_ctx *c, const void *kernel, uint32_t block, uint32_t want) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  uint64_t cap = std::max<uint64_t>(1, (uint64_t)per_cu * (uint64_t)c->cu_count / c->grid_div);
  for (const auto &e : c->resident_cap)
    if (e.first == kernel) cap = std::min<uint64_t>(cap, e.second);
  uint64_t g = want ? std::min<uint64_t>(want, cap) : cap;
  return (uint32_t)std::max<uint64_t>(1, g);
}

nd_status nd_stage_prep(nd_ctx *c, GraphView *gv) {
  nd_status st;
  const uint32_t n = c->n;
  const uint64_t nnz = c->nnz, m = c->m;
  DevScalars *sc = (DevScalars *)c->bufs[B_SCAL].p;
  uint32_t *uplo = (uint32_t *)nd_buf(c, B_UPLO, (n + 1ull) * 4, &st);
  if (!uplo) return st;
  uint32_t *deg = (uint32_t *)nd_buf(c, B_DEG, (n + 1ull) * 4, &st);
  if (!deg) return st;
  uint32_t *upcnt = (uint32_t *)nd_buf(c, B_TMP32A, (n + 1ull) * 4, &st);
  if (!upcnt) return st;
  uint64_t *eoff = (uint64_t *)nd_buf(c, B_DGP, (n + 1ull) * 8, &st);   // reused for dgp below
  if (!eoff) return st;
  uint32_t *eid = (uint32_t *)nd_buf(c, B_EID, std::max<uint64_t>(nnz, 1) * 4, &st);
  if (!eid) return st;
  uint32_t *eu = (uint32_t *)nd_buf(c, B_EU, std::max<uint64_t>(m, 1) * 4, &st);
  if (!eu) return st;
  uint32_t *ev = (uint32_t *)nd_buf(c, B_EV, std::max<uint64_t>(m, 1) * 4, &st);
  if (!ev) return st;
  const uint64_t *rp = (const uint64_t *)c->bufs[B_RP].p;
  const uint32_t *col = (const uint32_t *)c->bufs[B_COL].p;

  gv->n = n;
  gv->nnz = nnz;
  gv->m = m;
  gv->rp = rp;
  gv->col = col;
  gv->eid = eid;
  gv->eu = eu;
  gv->ev = ev;

  if (n) {
    hipLaunchKernelGGL(k_uplo, dim3(nd_grid(n, 256, 8192)), dim3(256), 0, c->stream, n, rp, col,
                       uplo, upcnt, deg);
    st = nd_exclusive_scan_u32_to_u64(c, upcnt, eoff, n, nullptr);
    if (st != ND_OK) return st;
  }
  if (nnz) {
    hipLaunchKernelGGL(k_edge_ids, dim3(nd_grid(nnz, 256, 16384)), dim3(256), 0, c->stream, n, nnz,
                       rp, col, uplo, eoff, eid, eu, ev);
  }

  // orientation
  uint32_t *orank = (uint32_t *)nd_buf(c, B_TMP32B, (n + 1ull) * 4, &st);
  if (!orank) return st;
  uint32_t *rdeg = (uint32_t *)nd_buf(c, B_TMP32C, (n + 1ull) * 4, &st);
  if (!rdeg) return st;
  uint64_t *sums = (uint64_t *)nd_buf(c, B_SORTK0, 64, &st);
  if (!sums) return st;
  if (n) {
    st = nd_hip(c, hipMemsetAsync(orank, 0xFF, n * 4ull, c->stream), "memset orank");
    if (st != ND_OK) return st;
    st = nd_hip(c, hipMemcpyAsync(rdeg, deg, n * 4ull, hipMemcpyDeviceToDevice, c->stream),
                "copy deg");
    if (st != ND_OK) return st;
    st = nd_hip(c, hipMemsetAsync(sums, 0, 64, c->stream), "memset sums");
    if (st != ND_OK) return st;
    OrientArgs oa{};
    oa.n = n;
    oa.rp = rp;
    oa.col = col;
    oa.rdeg = rdeg;
    oa.orank = orank;
    oa.sc = sc;
    oa.sums = sums;
    uint32_t nb = coop_blocks(c, (const void *)k_orient, kOrientBlock,
                              (uint32_t)std::min<uint64_t>(2048, (n + kOrientBlock - 1) / kOrientBlock));
    void *args[] = {&oa};
    st = nd_persistent_launch(c, (const void *)k_orient, &nb, &oa.nblocks, dim3(kOrientBlock), args,
                        nullptr, nullptr, "orientation launch");
    if (st != ND_OK) return st;
  }
  uint32_t *dgcnt = upcnt;   // reuse
  uint64_t *dgp = eoff;
  uint32_t *dgc = (uint32_t *)nd_buf(c, B_DGC, std::max<uint64_t>(m, 1) * 4, &st);
  if (!dgc) return st;
  uint32_t *dge = (uint32_t *)nd_buf(c, B_DGE, std::max<uint64_t>(m, 1) * 4, &st);
  if (!dge) return st;
  uint64_t *okey = (uint64_t *)nd_buf(c, B_OKEY, (n + 1ull) * 8, &st);
  if (!okey) return st;
  if (n) {
    hipLaunchKernelGGL(k_okey, dim3(nd_grid(n, 256, 8192)), dim3(256), 0, c->stream, n, orank, deg,
                       okey);
    hipLaunchKernelGGL(k_dg_count, dim3(nd_grid(n, 256, 8192)), dim3(256), 0, c->stream, n, rp,
                       col, okey, dgcnt, sc);
    st = nd_exclusive_scan_u32_to_u64(c, dgcnt, dgp, n, nullptr);
    if (st != ND_OK) return st;
    hipLaunchKernelGGL(k_dg_fill, dim3(nd_grid(n, 256, 8192)), dim3(256), 0, c->stream, n, rp, col,
                       eid, okey, dgp, dgc, dge);
  } else {
    st = nd_hip(c, hipMemsetAsync(dgp, 0, 8, c->stream), "dgp");
    if (st != ND_OK) return st;
  }
  gv->okey = okey;
  gv->dgp = dgp;
  gv->dgc = dgc;
  gv->dge = dge;
  gv->wp = nullptr;
  gv->wc = nullptr;
  gv->wt = nullptr;
  gv->te = nullptr;

  gv->wg = nullptr;
  gv->wsel = nullptr;
  gv->sg = nullptr;
  gv->tsel = nullptr;
  gv->tg = nullptr;
  if (nd_rs_general(c->s)) {
    if ((st = nd_hip(c, hipGetLastError(), "prep kernels")) != ND_OK) return st;
    return nd_prep_general(c, gv);
  }
  const bool tri_tables = c->r == 3 || (c->r == 2 && c->s == 4) || (c->r == 1 && c->s >= 3);
  if (tri_tables && m) {
    uint32_t *sup = (uint32_t *)nd_buf(c, B_SUP, m * 4, &st);
    if (!sup) return st;
    uint32_t *upc = (uint32_t *)nd_buf(c, B_UPC, m * 4, &st);
    if (!upc) return st;
    uint64_t *wp = (uint64_t *)nd_buf(c, B_WP, (m + 1) * 8, &st);
    if (!wp) return st;
    uint64_t *trib = (uint64_t *)nd_buf(c, B_TRIB, (m + 1) * 8, &st);
    if (!trib) return st;
    hipLaunchKernelGGL(k_etl_count<kEtlSmallG>,
                       dim3(nd_grid(m, (kEtlBlock / 64) * (64 / kEtlSmallG), 65536)),
                       dim3(kEtlBlock), 0, c->stream, m, rp, col, eu, ev, sup, upc);
    hipLaunchKernelGGL(k_etl_count<64>, dim3(nd_grid(m, kEtlBlock / 64, 65536)), dim3(kEtlBlock), 0,
                       c->stream, m, rp, col, eu, ev, sup, upc);
    if (c->r == 2 && c->s == 4)   // bounds the (2,4) counts: C(triangles on the edge, 2)
      hipLaunchKernelGGL(k_max_u32, dim3(nd_grid(m, 256, 4096)), dim3(256), 0, c->stream, sup, m,
                         &sc->max_sup);
    uint64_t nw = 0, ntri = 0;
    st = nd_exclusive_scan_u32_to_u64(c, sup, wp, m, &nw);
    if (st != ND_OK) return st;
    st = nd_exclusive_scan_u32_to_u64(c, upc, trib, m, &ntri);
    if (st != ND_OK) return st;
    if (ntri >= 0xFFFFFFFFull)
      return nd_fail(c, ND_E_OVERFLOW, "more than 2^32-2 triangles: 32-bit triangle ids overflow");
    c->n_r = c->r == 3 ? ntri : (c->r == 2 ? m : n);
    uint32_t *wc = (uint32_t *)nd_buf(c, B_WC, std::max<uint64_t>(nw, 1) * 4, &st);
    if (!wc) return st;
    uint32_t *wt = (uint32_t *)nd_buf(c, B_WT, std::max<uint64_t>(nw, 1) * 4, &st);
    if (!wt) return st;
    uint32_t *te = (uint32_t *)nd_buf(c, B_TE, std::max<uint64_t>(3 * ntri, 1) * 4, &st);
    if (!te) return st;
    if (nw) {
      hipLaunchKernelGGL(k_etl_fill<kEtlSmallG>,
                         dim3(nd_grid(m, (kEtlBlock / 64) * (64 / kEtlSmallG), 65536)),
                         dim3(kEtlBlock), 0, c->stream, m, rp, col, eid, eu, ev, sup, upc, wp,
                         trib, wc, wt, te);
      hipLaunchKernelGGL(k_etl_fill<64>, dim3(nd_grid(m, kEtlBlock / 64, 65536)), dim3(kEtlBlock),
                         0, c->stream, m, rp, col, eid, eu, ev, sup, upc, wp, trib, wc, wt, te);
      hipLaunchKernelGGL(k_etl_resolve, dim3(nd_grid(nw, 256, 65536)), dim3(256), 0, c->stream, m,
                         nw, ev, wp, wc, wt, &sc->status);
    }
    gv->wp = wp;
    gv->wc = wc;
    gv->wt = wt;
    gv->te = te;
    if (c->r == 1) {
      // (1,3): per CSR slot v -> w, the triangles at v with smaller other
      // vertex w (entries of W(vw) above w), summed over all slots
      uint32_t *scnt = (uint32_t *)nd_buf(c, B_TMP32D, std::max<uint64_t>(nnz, 1) * 4, &st);
      if (!scnt) return st;
      uint64_t *sgl = (uint64_t *)nd_buf(c, B_SG, (nnz + 1) * 8, &st);
      if (!sgl) return st;
      hipLaunchKernelGGL(k_slot_tris, dim3(nd_grid(nnz, 256, 65536)), dim3(256), 0, c->stream, nnz,
                         col, eid, wp, wc, scnt);
      uint64_t total = 0;
      st = nd_exclusive_scan_u32_to_u64(c, scnt, sgl, nnz, &total);
      if (st != ND_OK) return st;
      if (n)
        hipLaunchKernelGGL(k_t13_check, dim3(nd_grid(n, 256, 16384)), dim3(256), 0, c->stream, n,
                           rp, sgl, &sc->status);
      gv->sg = sgl;
      if (c->s == 4) {
        // (1,4): for every triangle probe (v, w, x) of (1,3), the probed part
        // above x of W(vw), W(vx), W(wx), and the running sum of its length
        const uint64_t ntp = total;   // triangle probes = 3 n_tri
        uint32_t *tlen = (uint32_t *)nd_buf(c, B_W24L, std::max<uint64_t>(ntp, 1) * 4, &st);
        if (!tlen) return st;
        uint32_t *tsel = (uint32_t *)nd_buf(c, B_TSEL, std::max<uint64_t>(ntp, 1) * 4, &st);
        if (!tsel) return st;
        uint64_t *tg = (uint64_t *)nd_buf(c, B_TG, (ntp + 1) * 8, &st);
        if (!tg) return st;
        hipLaunchKernelGGL(k_t14_len, dim3(nd_grid(nnz, 256, 65536)), dim3(256), 0, c->stream,
                           nnz, rp, col, eid, eu, ev, wp, wc, wt, te, sgl, tlen, tsel, n);
        uint64_t t2 = 0;
        st = nd_exclusive_scan_u32_to_u64(c, tlen, tg, ntp, &t2);
        if (st != ND_OK) return st;
        hipLaunchKernelGGL(k_t14_check, dim3(nd_grid(n, 256, 16384)), dim3(256), 0, c->stream, n,
                           rp, sgl, tg, &sc->status);
        gv->tsel = tsel;
        gv->tg = tg;
      }
    }
    if (c->r == 2) {
      // (2,4): probe length of every W entry's triangle, summed over all
      // entries, so a peeled edge can hand out the candidate 4th vertices of
      // all its triangles as one flat range
      uint32_t *len3 = (uint32_t *)nd_buf(c, B_TMP32D, std::max<uint64_t>(nw, 1) * 4, &st);
      if (!len3) return st;
      uint32_t *wsel = (uint32_t *)nd_buf(c, B_W24L, std::max<uint64_t>(nw, 1) * 4, &st);
      if (!wsel) return st;
      uint64_t *wg = (uint64_t *)nd_buf(c, B_WG, (nw + 1) * 8, &st);
      if (!wg) return st;
      if (nw)
        hipLaunchKernelGGL(k_w24_len, dim3(nd_grid(m, 256, 16384)), dim3(256), 0, c->stream, m,
                           wp, wc, wt, te, len3, wsel);
      uint64_t total = 0;
      st = nd_exclusive_scan_u32_to_u64(c, len3, wg, nw, &total);
      if (st != ND_OK) return st;
      hipLaunchKernelGGL(k_w24_check, dim3(nd_grid(m, 256, 16384)), dim3(256), 0, c->stream, m,
                         wp, wg, &sc->status);
      gv->wg = wg;
      gv->wsel = wsel;
    }
  } else if (c->r == 3) {
    c->n_r = 0;
  } else if (c->r == 2) {
    c->n_r = m;
  } else {
    c->n_r = n;
    if (c->s >= 3) {
      // no edges: every vertex's triangle range is empty (sg = tg = {0})
      uint64_t *sgl = (uint64_t *)nd_buf(c, B_SG, 8, &st);
      if (!sgl) return st;
      if ((st = nd_hip(c, hipMemsetAsync(sgl, 0, 8, c->stream), "sg")) != ND_OK) return st;
      gv->sg = sgl;
      if (c->s == 4) {
        uint64_t *tg = (uint64_t *)nd_buf(c, B_TG, 8, &st);
        if (!tg) return st;
        if ((st = nd_hip(c, hipMemsetAsync(tg, 0, 8, c->stream), "tg")) != ND_OK) return st;
        gv->tg = tg;
      }
    }
  }
  return nd_hip(c, hipGetLastError(), "prep kernels");
}
