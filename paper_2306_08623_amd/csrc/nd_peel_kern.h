// nd_peel_kern.h -- the peel and hierarchy kernels and their launch
// helpers, shared by the files that instantiate them for the (r,s) pairs
// (nd_peel.hip: s <= 4; nd_peel_gen_a.hip / nd_peel_gen_b.hip: s = 5..7).
//
// Peeling rounds interleaved with hierarchy linking
// (Algorithm 3, Section 7.1, with LINK-EFFICIENT of Algorithm 5,
// Section 7.3), as one persistent launch.
//
// Round t at level k:
//   bucket  When the frontier is empty, the remaining r-cliques are scanned
//           for their minimum count k' (> k), and the frontier becomes every
//           remaining r-clique with count k'. The scan also compacts the list
//           of remaining r-cliques, so each scan only touches survivors.
//   mark    Every frontier r-clique R gets core number k and peel round t.
//   visit   For every frontier R and every s-clique S containing R (found by
//           intersecting the adjacency lists of R's members), each other
//           r-clique R' of S is classified by its peel round:
//             - R' peeled earlier or in this round: link(R', R) -- R and R'
//               are s-clique-adjacent and both core numbers are final;
//             - R' still present: if no member of S was peeled before round t
//               (S still exists) and R is the smallest-id member of S peeled
//               in round t (so S is removed exactly once), decrement R''s
//               count; the decrement that lowers it from k+1 to k puts R'
//               into the next frontier (same level k).
//   A grid barrier separates the phases. The next round starts with the
//   collected frontier or, if it is empty, with a bucket scan.
//
// Work balance: every frontier r-clique contributes "probe elements" (the
// entries of its shortest adjacency list); a per-block prefix sum over the
// frontier lets every lane take one probe element of the global sequence.
//
// The link routine keeps uf (components of equal core number) and L (for a
// component root, an r-clique of the nearest lower core it is connected to)
// consistent with compare-and-swap; its recursive calls become a small
// per-lane stack that spills into a global queue drained between rounds.
#pragma once

#include "nd_internal.h"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <type_traits>

// Arguments of the persistent peel kernel (one definition for every file
// that includes this header).
struct PeelArgs {
  GraphView g;
  uint64_t n_r;
  uint32_t *cnt;      // s-clique count; the core number once peeled
  uint32_t *round;    // peel round, ND_ALIVE while present
  uint8_t *pst;       // peel state: kAlive, kPeeledNow (this round), kPeeledBefore
  uint32_t *uf;       // union-find parent
  uint32_t *L;        // nearest lower core link of a uf root
  uint64_t *frec;     // (2,3), (3,4): per frontier slot, 32 B of list ranges (Shape::len_rec)
  uint32_t *F0, *F1;  // frontiers by round parity
  uint64_t *wscan;    // per frontier slot: inclusive work prefix in its segment
  uint32_t *al0, *al1;  // remaining r-cliques by scan parity, one segment per block
  uint32_t *acnt;       // [2 * nblocks] length of each block's segment list
  uint64_t *btot;     // per block: work total of its frontier segment
  uint32_t *linkq;    // spilled link pairs
  uint32_t linkq_cap;
  uint64_t *gcache;   // device-wide table of linked root pairs
  uint64_t gcache_mask;
  DevScalars *sc;
  uint32_t nblocks;
  uint32_t max_rounds;
  uint32_t *progress;   // host-visible [round, level, frontier], or null
  // approximate decomposition (Algorithm 2): the upper ends of the
  // geometric buckets (n_thr of them; 0 = exact peeling) and the most rounds
  // a bucket is processed before the next bucket takes over
  const uint32_t *thr;
  uint32_t n_thr;
  uint32_t round_cap;
  // chunk map of a large round: the frontier slot holding probe unit 64 c,
  // for every chunk c (cslot_cap entries at most)
  uint32_t *cslot;
  uint64_t cslot_cap;
};

namespace {

constexpr uint32_t kPeelBlock = 256;
constexpr uint32_t kMaxPeelBlocks = 2048;
constexpr uint32_t kScanU = 4;   // bucket scan: entries per thread and pass
// Peel state of an r-clique as the visits of a round read it: all they need
// of the round number, in a byte (a quarter of the lines of the round array)
constexpr uint8_t kAlive = 0, kPeeledNow = 1, kPeeledBefore = 2;
constexpr uint32_t kLocalStack = 8;
constexpr uint32_t kLinkStepCap = 1u << 24;


// ---------------------------------------------------------------------------
// union-find (lock-free: CAS link of roots by index, path halving)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t uf_find(uint32_t *uf, uint32_t x) {
  for (;;) {
    uint32_t p = ld_acq32(&uf[x]);
    if (p == x) return x;
    uint32_t gp = ld_acq32(&uf[p]);
    if (gp == p) return p;
    cas32(&uf[x], p, gp);
    x = gp;
  }
}

// The roots of x and y, the two walks in lockstep (their dependent loads
// overlap), each with the path halving of uf_find.
__device__ __forceinline__ void uf_find2(uint32_t *uf, uint32_t &x, uint32_t &y) {
  bool dx = false, dy = false;
  for (;;) {
    uint32_t px = x, py = y;
    if (!dx) px = ld_acq32(&uf[x]);
    if (!dy) py = ld_acq32(&uf[y]);
    dx |= px == x;
    dy |= py == y;
    if (dx && dy) return;
    uint32_t gx = px, gy = py;
    if (!dx) gx = ld_acq32(&uf[px]);
    if (!dy) gy = ld_acq32(&uf[py]);
    if (!dx) {
      if (gx == px) {
        x = px;
        dx = true;
      } else {
        cas32(&uf[x], px, gx);
        x = gx;
      }
    }
    if (!dy) {
      if (gy == py) {
        y = py;
        dy = true;
      } else {
        cas32(&uf[y], py, gy);
        y = gy;
      }
    }
    if (dx && dy) return;
  }
}

// Joins the sets of a and b; the smaller root id survives. Returns the root
// whose parent pointer this call changed (the loser), or ND_NONE when a and b
// were already in one set. Lost races are counted in *retries, a counter
// of the workgroup in LDS (summed into the device scalars once per launch,
// so counting costs neither registers nor global atomics).
__device__ __forceinline__ uint32_t uf_unite(uint32_t *uf, uint32_t a, uint32_t b,
                                             uint32_t *retries) {
  for (;;) {
    uf_find2(uf, a, b);
    if (a == b) return ND_NONE;
    if (a > b) { uint32_t t = a; a = b; b = t; }
    if (cas32(&uf[b], b, a)) return b;
    atomicAdd(retries, 1u);
  }
}

struct LinkCtx {
  uint32_t *uf;
  uint32_t *L;
  const uint32_t *nd;
  uint32_t *linkq;
  uint32_t linkq_cap;
  DevScalars *sc;
  uint64_t links, unites;
  uint32_t *retries;  // LDS: compare-and-swaps of unite / L that lost a race
};

// The spill queue is a ring of linkq_cap (a power of two) pairs addressed by
// monotone head/tail counters; head only moves between grid barriers.
__device__ __forceinline__ void spill(LinkCtx &c, uint32_t R, uint32_t Q) {
  const uint32_t i = atomicAdd(&c.sc->linkq_tail, 1u);
  const uint32_t h = ld_acq32(&c.sc->linkq_head);
  if (i - h < c.linkq_cap) {
    const uint64_t slot = i & (c.linkq_cap - 1);
    c.linkq[2 * slot] = R;
    c.linkq[2 * slot + 1] = Q;
  } else {
    atomicOr(&c.sc->status, ND_DERR_LINKQ);
  }
}

__device__ __forceinline__ uint64_t min64(uint64_t a, uint64_t b) { return a < b ? a : b; }

// One step of LINK-EFFICIENT (Algorithm 5) on the pair (R, Q): the same
// transitions as link_efficient below, but the recursive calls it makes
// (at most two) are returned in out[] instead of being run, so that a whole
// wave can work through a queue of pending steps together.
__device__ __forceinline__ uint32_t link_step(LinkCtx &c, uint32_t R, uint32_t Q, uint64_t *out) {
  uint32_t no = 0;
  auto push = [&](uint32_t a, uint32_t b) {
    if (a != ND_NONE && b != ND_NONE) out[no++] = ((uint64_t)a << 32) | b;
  };
  if (R == ND_NONE || Q == ND_NONE) return 0;
  c.links++;
  // roots first, then the order by core number: a union-find set only ever
  // joins r-cliques of one core number, so a root's is its members'
  uf_find2(c.uf, R, Q);
  uint32_t ndR = c.nd[R], ndQ = c.nd[Q];
  if (ndQ < ndR) {
    const uint32_t t = R, tn = ndR;
    R = Q;
    Q = t;
    ndR = ndQ;
    ndQ = tn;
  }
  if (ndR == ndQ) {
    if (R == Q) return 0;
    const uint32_t loser = uf_unite(c.uf, R, Q, c.retries);   // hand-over as in link_efficient
    if (loser != ND_NONE) {
      c.unites++;
      const uint32_t w = uf_find(c.uf, loser);
      push(ld_acq32(&c.L[loser]), w);
    }
    return no;
  }
  for (uint32_t spins = 0;; spins++) {
    if (spins > kLinkStepCap) {
      atomicOr(&c.sc->status, ND_DERR_WATCHDOG);
      return no;
    }
    Q = uf_find(c.uf, Q);
    const uint32_t LQ = ld_acq32(&c.L[Q]);
    if (LQ == ND_NONE) {
      if (cas32(&c.L[Q], ND_NONE, R)) {
        const uint32_t pQ = uf_find(c.uf, Q);
        if (pQ != Q) push(R, pQ);
        return no;
      }
      atomicAdd(c.retries, 1u);
      continue;
    }
    if (c.nd[LQ] < ndR) {
      if (cas32(&c.L[Q], LQ, R)) {
        const uint32_t pQ = uf_find(c.uf, Q);
        if (pQ != Q) push(R, pQ);
        push(R, LQ);
        return no;
      }
      atomicAdd(c.retries, 1u);
    } else {
      push(R, LQ);
      return no;
    }
  }
}

// Per-wave LDS queue of pending link steps (pairs R << 32 | Q); `qn` is the
// same in every lane. Each pass gives one pending step to each lane.
constexpr uint32_t kWaveQ = 128;

// appends one optional pair per lane; the caller leaves room for 64
__device__ __forceinline__ void wave_q_push(uint64_t *q, uint32_t &qn, bool has, uint64_t v) {
  const uint64_t m = ballot64(has);
  if (has) {
    const uint32_t lane = lane_id();
    const uint64_t below = m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane)));
    q[qn + __popcll(below)] = v;
  }
  qn += __popcll(m);
  __builtin_amdgcn_wave_barrier();
}

// runs queued steps while at least `need` are pending (need = 1: until empty)
__device__ void wave_q_drain(LinkCtx &c, uint64_t *q, uint32_t &qn, uint32_t need) {
  const uint32_t lane = lane_id();
  uint32_t passes = 0;
  while (qn >= need && qn > 0) {
    if (++passes > kLinkStepCap) {   // a runaway cascade: give up with an error
      if (lane == 0) atomicOr(&c.sc->status, ND_DERR_WATCHDOG);
      qn = 0;
      break;
    }
    const uint32_t take = qn < 64 ? qn : 64;
    uint64_t mine = ~0ull;
    if (lane < take) mine = q[qn - take + lane];
    __builtin_amdgcn_wave_barrier();
    qn -= take;
    uint64_t out[2];
    uint32_t no = 0;
    if (mine != ~0ull) no = link_step(c, (uint32_t)(mine >> 32), (uint32_t)mine, out);
#pragma unroll
    for (int o = 0; o < 2; o++) {
      const bool has = (uint32_t)o < no;
      const uint32_t cnt = __popcll(ballot64(has));
      if (qn + cnt <= kWaveQ) {
        wave_q_push(q, qn, has, has ? out[o] : 0);
      } else if (has) {
        spill(c, (uint32_t)(out[o] >> 32), (uint32_t)out[o]);
      }
    }
  }
}

// LINK-EFFICIENT (Algorithm 5) for the pair (R0, Q0), whose core numbers are
// both final. Recursive calls are pushed on a small stack; pairs that do not
// fit go to the global queue.
__device__ void link_efficient(LinkCtx &c, uint32_t R0, uint32_t Q0) {
  uint32_t stR[kLocalStack], stQ[kLocalStack];
  uint32_t sp = 0;
  stR[sp] = R0;
  stQ[sp] = Q0;
  sp++;
  uint32_t steps = 0;
  while (sp > 0) {
    sp--;
    uint32_t R = stR[sp], Q = stQ[sp];
    if (R == ND_NONE || Q == ND_NONE) continue;
    if (++steps > kLinkStepCap) {
      atomicOr(&c.sc->status, ND_DERR_WATCHDOG);
      return;
    }
    c.links++;
    auto push = [&](uint32_t a, uint32_t b) {
      if (a == ND_NONE || b == ND_NONE) return;
      if (sp < kLocalStack) {
        stR[sp] = a;
        stQ[sp] = b;
        sp++;
      } else {
        spill(c, a, b);
      }
    };
    if (c.nd[Q] < c.nd[R]) { uint32_t t = R; R = Q; Q = t; }
    R = uf_find(c.uf, R);
    Q = uf_find(c.uf, Q);
    const uint32_t ndR = c.nd[R];
    if (ndR == c.nd[Q]) {
      if (R == Q) continue;
      // The root that lost its role hands its nearest-lower-core link to the
      // merged set. The loser is the root whose parent this unite changed:
      // R or Q may have been merged elsewhere after they were read, in which
      // case unite joins their current roots, and it is one of those whose L
      // must move (a CAS on L[loser] that lands after this read is handed
      // over by its own writer, which then sees loser is no longer a root).
      const uint32_t loser = uf_unite(c.uf, R, Q, c.retries);
      if (loser != ND_NONE) {
        c.unites++;
        const uint32_t w = uf_find(c.uf, loser);
        push(ld_acq32(&c.L[loser]), w);
      }
    } else {
      // ND[R] < ND[Q]: R may become Q's nearest lower core, and R must be
      // connected with Q's current nearest lower core
      // (L[Q] is read at Q's current root; a CAS is only tried when its
      // expected value was just observed, since L never returns to empty)
      uint32_t spins = 0;
      for (;;) {
        if (++spins > kLinkStepCap) {
          atomicOr(&c.sc->status, ND_DERR_WATCHDOG);
          return;
        }
        Q = uf_find(c.uf, Q);
        const uint32_t LQ = ld_acq32(&c.L[Q]);
        if (LQ == ND_NONE) {
          if (cas32(&c.L[Q], ND_NONE, R)) {
            uint32_t pQ = uf_find(c.uf, Q);
            if (pQ != Q) push(R, pQ);   // Q was merged meanwhile
            break;
          }
          atomicAdd(c.retries, 1u);
          continue;                      // L[Q] was set concurrently: read again
        }
        if (c.nd[LQ] < ndR) {
          if (cas32(&c.L[Q], LQ, R)) {
            uint32_t pQ = uf_find(c.uf, Q);
            if (pQ != Q) push(R, pQ);
            push(R, LQ);
            break;
          }
          atomicAdd(c.retries, 1u);
        } else {
          push(R, LQ);
          break;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// per-(r,s) s-clique discovery around a frontier r-clique
// ---------------------------------------------------------------------------

// First index x in [lo, hi) with a[x] > v for a non-decreasing array, when
// the answer is known to be >= lo: doubling steps from lo, then a binary
// search inside the last step.
__device__ __forceinline__ uint64_t gallop_u64(const uint64_t *a, uint64_t lo, uint64_t hi,
                                               uint64_t v) {
  if (lo >= hi || a[lo] > v) return lo;
  uint64_t base = lo, step = 1;   // a[base] <= v
  while (base + step < hi && a[base + step] <= v) {
    base += step;
    step <<= 1;
  }
  uint64_t l = base + 1, h = base + step + 1 < hi ? base + step + 1 : hi;
  while (l < h) {
    const uint64_t mid = (l + h) >> 1;
    if (a[mid] <= v) l = mid + 1;
    else h = mid;
  }
  return l;
}

// Every shape lists, for a frontier r-clique R, its "probe" list: the
// shortest adjacency-like list whose entries extend R to s-clique
// candidates. len() is its length; visit() tests probe entry i and, when it
// closes an s-clique, writes the ids of the other r-cliques of that s-clique.
template <int R_, int S_>
struct Shape;

// Shapes with kRec = true have the mark pass store, per frontier slot, what
// their visits need of the r-clique (len_rec), and visit from that record
// (visit_rec) instead of re-reading the r-clique's tables on every probe.
template <class S, class = void>
struct RecOf : std::false_type {};
template <class S>
struct RecOf<S, std::void_t<decltype(S::kRec)>> : std::integral_constant<bool, S::kRec> {};

// (1,2): R = vertex v; every neighbour x closes an s-clique {v, x}.
template <>
struct Shape<1, 2> {
  static constexpr int kOthers = 1;
  __device__ static uint32_t len(const GraphView &g, uint32_t R) {
    return (uint32_t)(g.rp[R + 1] - g.rp[R]);
  }
  __device__ static bool visit(const GraphView &g, uint32_t R, uint32_t i, uint32_t *o) {
    o[0] = g.col[g.rp[R] + i];
    return true;
  }
};

// (2,3): R = edge {u, v}; probe the shorter row, search the longer; the two
// slots give the ids of edges {u, x} and {v, x}.
template <>
struct Shape<2, 3> {
  static constexpr int kOthers = 2;
  static constexpr bool kRec = true;
  // record: the CSR start of the endpoint with the shorter list (probed),
  // the start and length of the other one's list
  __device__ static uint32_t len_rec(const GraphView &g, uint32_t R, uint64_t *rec) {
    const uint32_t u = g.eu[R], v = g.ev[R];
    uint64_t bp = g.rp[u], ep = g.rp[u + 1], bq = g.rp[v], eq = g.rp[v + 1];
    // the same choice of the probed endpoint as visit() below
    if (eq - bq < ep - bp) {
      uint64_t t = bp; bp = bq; bq = t;
      t = ep; ep = eq; eq = t;
    }
    rec[0] = bp;
    rec[1] = bq;
    rec[2] = eq - bq;
    return (uint32_t)(ep - bp);
  }
  __device__ static bool visit_rec(const GraphView &g, const uint64_t *rec, uint32_t i,
                                   uint32_t *o) {
    const uint64_t sp = rec[0] + i, bq = rec[1], eq = rec[1] + rec[2];
    const uint32_t x = g.col[sp];
    const uint64_t sq = find_u32<uint64_t>(g.col, bq, eq, x);
    if (sq == eq) return false;
    o[0] = g.eid[sp];
    o[1] = g.eid[sq];
    return true;
  }
  __device__ static uint32_t len(const GraphView &g, uint32_t R) {
    const uint32_t u = g.eu[R], v = g.ev[R];
    const uint64_t du = g.rp[u + 1] - g.rp[u], dv = g.rp[v + 1] - g.rp[v];
    return (uint32_t)(du < dv ? du : dv);
  }
  __device__ static bool visit(const GraphView &g, uint32_t R, uint32_t i, uint32_t *o) {
    uint32_t p = g.eu[R], q = g.ev[R];
    if (g.rp[q + 1] - g.rp[q] < g.rp[p + 1] - g.rp[p]) { uint32_t t = p; p = q; q = t; }
    const uint64_t sp = g.rp[p] + i;
    const uint32_t x = g.col[sp];
    const uint64_t bq = g.rp[q], eq = g.rp[q + 1];
    const uint64_t sq = find_u32<uint64_t>(g.col, bq, eq, x);
    if (sq == eq) return false;
    o[0] = g.eid[sp];
    o[1] = g.eid[sq];
    return true;
  }
};

// (1,3): R = vertex v. A triangle {v, w, x} at v is taken from the CSR slot
// v -> w of its smaller other vertex w, as the entry x > w of W(vw); the
// probe entries of v are these, slot after slot (sg holds the running sums),
// so every probe is a triangle. The other r-cliques are the vertices w, x.
template <>
struct Shape<1, 3> {
  static constexpr int kOthers = 2;
  __device__ static uint32_t len(const GraphView &g, uint32_t R) {
    return (uint32_t)(g.sg[g.rp[R + 1]] - g.sg[g.rp[R]]);
  }
  __device__ static bool visit(const GraphView &g, uint32_t R, uint32_t i, uint32_t *o) {
    const uint64_t b = g.rp[R], f = g.rp[R + 1];
    const uint64_t target = g.sg[b] + i;
    uint64_t lo = b, hi = f;   // last slot q with sg[q] <= target
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (g.sg[mid] <= target) lo = mid;
      else hi = mid;
    }
    const uint32_t w = g.col[lo], e = g.eid[lo];
    const uint64_t wb = g.wp[e], wf = g.wp[e + 1];
    const uint64_t first = upper_bound_u32(g.wc, wb, wf, w);
    o[0] = w;
    o[1] = g.wc[first + (target - g.sg[lo])];
    return true;
  }
};

// (1,4): R = vertex v. A 4-clique {v, w, x, y} with w < x < y is taken
// from the triangle probe (v, w, x) of (1,3) with a 4th vertex y > x from
// the shortest of the parts above x of W(vw), W(vx), W(wx) (chosen in prep:
// tsel); tg holds the running sums over all triangle probes, so a vertex's
// probe entries are one flat range. The other r-cliques are w, x, y.
template <>
struct Shape<1, 4> {
  static constexpr int kOthers = 3;
  __device__ static uint32_t len(const GraphView &g, uint32_t R) {
    return (uint32_t)(g.tg[g.sg[g.rp[R + 1]]] - g.tg[g.sg[g.rp[R]]]);
  }
  __device__ static bool visit(const GraphView &g, uint32_t R, uint32_t i, uint32_t *o) {
    const uint64_t gb = g.sg[g.rp[R]], gf = g.sg[g.rp[R + 1]];
    const uint64_t target = g.tg[gb] + i;
    uint64_t lo = gb, hi = gf;   // the triangle probe: last gi with tg[gi] <= target
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (g.tg[mid] <= target) lo = mid;
      else hi = mid;
    }
    const uint64_t gi = lo, jj = target - g.tg[gi];
    uint64_t qlo = g.rp[R], qhi = g.rp[R + 1];   // its slot: last q with sg[q] <= gi
    while (qhi - qlo > 1) {
      const uint64_t mid = (qlo + qhi) >> 1;
      if (g.sg[mid] <= gi) qlo = mid;
      else qhi = mid;
    }
    const uint32_t w = g.col[qlo], e = g.eid[qlo];
    const uint64_t b = g.wp[e], f = g.wp[e + 1];
    const uint64_t p = upper_bound_u32(g.wc, b, f, w) + (gi - g.sg[qlo]);
    const uint32_t x = g.wc[p], t = g.wt[p];
    uint32_t evx = ND_NONE, ewx = ND_NONE;   // the triangle's edges {v,x}, {w,x}
    for (int k = 0; k < 3; k++) {
      const uint32_t z = g.te[3ull * t + k];
      if (z == e) continue;
      if (g.eu[z] == R || g.ev[z] == R) evx = z;
      else ewx = z;
    }
    if (evx == ND_NONE || ewx == ND_NONE) return false;   // unreachable for consistent tables
    const uint32_t sl = g.tsel[gi];
    const uint32_t which = sl >> 30, off = sl & 0x3FFFFFFFu;
    const uint32_t el[3] = {e, evx, ewx};
    const uint32_t ep = el[which];
    const uint32_t y = g.wc[g.wp[ep] + off + jj];
#pragma unroll
    for (int k = 0; k < 3; k++) {
      if ((uint32_t)k == which) continue;
      const uint64_t lb = g.wp[el[k]], lf = g.wp[el[k] + 1];
      if (find_u32<uint64_t>(g.wc, lb, lf, y) == lf) return false;
    }
    o[0] = w;
    o[1] = x;
    o[2] = y;
    return true;
  }
};

// (3,4): R = triangle with edges e0, e1, e2; the common neighbours of its
// vertices are the entries common to W(e0), W(e1), W(e2); the positions give
// the ids of the three other triangles.
template <>
struct Shape<3, 4> {
  static constexpr int kOthers = 3;
  static constexpr bool kRec = true;
  // record: the start of the shortest of the three W lists, the starts of
  // the other two, and their two lengths (32 B); a probe then needs one
  // record read before its list entry instead of the triangle's edge ids
  // and six W offsets
  __device__ static uint32_t len_rec(const GraphView &g, uint32_t R, uint64_t *rec) {
    const uint32_t e0 = g.te[3ull * R], e1 = g.te[3ull * R + 1], e2 = g.te[3ull * R + 2];
    uint64_t b0 = g.wp[e0], f0 = g.wp[e0 + 1], b1 = g.wp[e1], f1 = g.wp[e1 + 1],
             b2 = g.wp[e2], f2 = g.wp[e2 + 1];
    const uint64_t s0 = f0 - b0, s1 = f1 - b1, s2 = f2 - b2;
    // the same choice of the probed list as visit() below
    if (s1 < s0 && s1 <= s2) {
      uint64_t t = b0; b0 = b1; b1 = t;
      t = f0; f0 = f1; f1 = t;
    } else if (s2 < s0 && s2 < s1) {
      uint64_t t = b0; b0 = b2; b2 = t;
      t = f0; f0 = f2; f2 = t;
    }
    rec[0] = b0;
    rec[1] = b1;
    rec[2] = b2;
    rec[3] = (f1 - b1) | ((f2 - b2) << 32);
    return (uint32_t)(f0 - b0);
  }
  __device__ static bool visit_rec(const GraphView &g, const uint64_t *rec, uint32_t i,
                                   uint32_t *o) {
    const uint64_t b0 = rec[0], b1 = rec[1], b2 = rec[2], ln = rec[3];
    const uint64_t f1 = b1 + (uint32_t)ln, f2 = b2 + (ln >> 32);
    const uint64_t p0 = b0 + i;
    const uint32_t x = g.wc[p0];
    if (b1 == f1 || b2 == f2) return false;   // never: each holds R's third vertex
    uint64_t p1, p2;
    find2_u32<uint64_t>(g.wc, b1, f1, b2, f2, x, p1, p2);
    if (p1 == f1 || p2 == f2) return false;
    o[0] = g.wt[p0];
    o[1] = g.wt[p1];
    o[2] = g.wt[p2];
    return true;
  }
  __device__ static uint32_t len(const GraphView &g, uint32_t R) {
    const uint32_t e0 = g.te[3ull * R], e1 = g.te[3ull * R + 1], e2 = g.te[3ull * R + 2];
    uint64_t s0 = g.wp[e0 + 1] - g.wp[e0], s1 = g.wp[e1 + 1] - g.wp[e1],
             s2 = g.wp[e2 + 1] - g.wp[e2];
    uint64_t mn = s0 < s1 ? s0 : s1;
    mn = mn < s2 ? mn : s2;
    return (uint32_t)mn;
  }
  __device__ static bool visit(const GraphView &g, uint32_t R, uint32_t i, uint32_t *o) {
    uint32_t e0 = g.te[3ull * R], e1 = g.te[3ull * R + 1], e2 = g.te[3ull * R + 2];
    uint64_t s0 = g.wp[e0 + 1] - g.wp[e0], s1 = g.wp[e1 + 1] - g.wp[e1],
             s2 = g.wp[e2 + 1] - g.wp[e2];
    // probe the shortest list: rotate it into e0
    if (s1 < s0 && s1 <= s2) {
      uint32_t t = e0; e0 = e1; e1 = t;
    } else if (s2 < s0 && s2 < s1) {
      uint32_t t = e0; e0 = e2; e2 = t;
    }
    const uint64_t p0 = g.wp[e0] + i;
    const uint32_t x = g.wc[p0];
    const uint64_t b1 = g.wp[e1], f1 = g.wp[e1 + 1];
    const uint64_t b2 = g.wp[e2], f2 = g.wp[e2 + 1];
    if (b1 == f1 || b2 == f2) return false;   // never: each holds R's third vertex
    uint64_t p1, p2;
    find2_u32<uint64_t>(g.wc, b1, f1, b2, f2, x, p1, p2);
    if (p1 == f1 || p2 == f2) return false;
    o[0] = g.wt[p0];
    o[1] = g.wt[p1];
    o[2] = g.wt[p2];
    return true;
  }
};

// (2,4): R = edge e = {u, v}. A 4-clique {u, v, w, x} containing e is a
// triangle t = {u, v, w} on e (an entry of W(e)) extended by a common
// neighbour x of t, taken from the triangle with the smaller extra vertex
// (w < x) so that it is met once. Probe entries are, for every triangle t of
// e in W(e) order, the entries above w of t's shortest W list part (chosen
// in prep: wsel), as one flat range (wg holds the running sums). The other
// five edges are {u,w}, {v,w} (from t), {u,x}, {v,x} (from triangle {u,v,x},
// x's entry in W(e)) and {w,x} (from triangle {u,w,x}, x's entry in W(x1)).
template <>
struct Shape<2, 4> {
  static constexpr int kOthers = 5;
  __device__ static uint32_t len(const GraphView &g, uint32_t R) {
    return (uint32_t)(g.wg[g.wp[R + 1]] - g.wg[g.wp[R]]);
  }
  __device__ static bool visit(const GraphView &g, uint32_t R, uint32_t i, uint32_t *o) {
    const uint64_t b = g.wp[R], f = g.wp[R + 1];
    const uint64_t target = g.wg[b] + i;
    // the W entry whose probe range holds `target`: last p with wg[p] <= target
    uint64_t lo = b, hi = f;
    while (hi - lo > 1) {
      const uint64_t mid = (lo + hi) >> 1;
      if (g.wg[mid] <= target) lo = mid;
      else hi = mid;
    }
    const uint64_t pt = lo;
    const uint64_t j = target - g.wg[pt];
    const uint32_t t = g.wt[pt];
    const uint32_t sl = g.wsel[pt];
    // t's edges other than R, in te order
    uint32_t xs[2], nx = 0;
    for (int q = 0; q < 3; q++) {
      const uint32_t z = g.te[3ull * t + q];
      if (z != R && nx < 2) xs[nx++] = z;
    }
    const uint32_t x1 = xs[0], x2 = xs[1];
    const uint32_t which = sl >> 30, off = sl & 0x3FFFFFFFu;
    uint64_t pR, p1;
    // the two list searches of either case advance in lockstep (all lists
    // searched hold t's third vertex, so none is empty)
    if (which == 0) {
      pR = b + off + j;
      const uint32_t x = g.wc[pR];
      const uint64_t b1 = g.wp[x1], f1 = g.wp[x1 + 1], b2 = g.wp[x2], f2 = g.wp[x2 + 1];
      if (b1 == f1 || b2 == f2) return false;
      uint64_t p2;
      find2_u32<uint64_t>(g.wc, b1, f1, b2, f2, x, p1, p2);
      if (p1 == f1 || p2 == f2) return false;
    } else {
      const uint32_t ep = which == 1 ? x1 : x2, eo = which == 1 ? x2 : x1;
      const uint64_t pp = g.wp[ep] + off + j;
      const uint32_t x = g.wc[pp];
      const uint64_t bo = g.wp[eo], fo = g.wp[eo + 1];
      if (bo == fo || b == f) return false;
      uint64_t po;
      find2_u32<uint64_t>(g.wc, bo, fo, b, f, x, po, pR);
      if (po == fo || pR == f) return false;
      p1 = which == 1 ? pp : po;
    }
    // triangle {u,v,x}: its edges other than R are {u,x}, {v,x}
    const uint32_t tx = g.wt[pR];
    uint32_t ys[2], ny = 0;
    for (int q = 0; q < 3; q++) {
      const uint32_t z = g.te[3ull * tx + q];
      if (z != R && ny < 2) ys[ny++] = z;
    }
    // triangle on x1 with x: its edges are x1, one of ys, and {w,x}
    const uint32_t tw = g.wt[p1];
    uint32_t wx = ND_NONE;
    for (int q = 0; q < 3; q++) {
      const uint32_t z = g.te[3ull * tw + q];
      if (z != x1 && z != ys[0] && z != ys[1]) wx = z;
    }
    if (wx == ND_NONE) return false;   // unreachable for consistent tables
    o[0] = x1;
    o[1] = x2;
    o[2] = ys[0];
    o[3] = ys[1];
    o[4] = wx;
    return true;
  }
};

// s = 5..7 (tables from nd_gen.hip): R's probe list is its list of
// s-cliques; every probe closes one, whose other NO = C(s,r) - 1 members are
// its r-clique ids without R (in their stored order). Shapes of this kind
// are instantiated by NO alone, as Shape<0, NO>.
template <int NO>
struct Shape<0, NO> {
  static constexpr int kOthers = NO;
  __device__ static uint32_t len(const GraphView &g, uint32_t R) {
    return (uint32_t)(g.io[R + 1] - g.io[R]);
  }
  __device__ static bool visit(const GraphView &g, uint32_t R, uint32_t i, uint32_t *o) {
    const uint32_t *mem = g.sm + (uint64_t)g.il[g.io[R] + i] * (NO + 1);
    // members before R in place, the ones after it shifted down by one
    bool seen = false;
#pragma unroll
    for (int j = 0; j < NO; j++) {
      const uint32_t x = mem[j];
      seen = seen || x == R;
      o[j] = seen ? mem[j + 1] : x;
    }
    return true;
  }
};

// ---------------------------------------------------------------------------
// redundant-link filter
// ---------------------------------------------------------------------------

// A block keeps a small LDS table of root pairs (x, q) it has already linked:
// link(R', R) was completed with find(R') = x and find(R) = q. Union-find
// roots never become roots again after losing a union and sets only grow, so
// a later call whose partner and frontier r-clique still have roots x and q
// adds no information (its partner lies in x's set, which is connected to
// q's set at x's level) and is skipped. Entries are single 64-bit LDS words,
// so a lookup never sees half of an entry.
constexpr uint32_t kLinkCache = 1024;

__device__ __forceinline__ uint32_t lcache_slot(uint32_t x, uint32_t q) {
  return ((x * 0x9E3779B1u) ^ (q * 0x85EBCA77u) ^ (q >> 15)) & (kLinkCache - 1);
}

__device__ __forceinline__ bool lcache_hit(const uint64_t *cache, uint32_t x, uint32_t q) {
  const uint64_t key = ((uint64_t)x << 32) | q;
  const uint32_t h = lcache_slot(x, q);
  return cache[h] == key || cache[h ^ 1] == key;
}

__device__ __forceinline__ void lcache_put(uint64_t *cache, uint32_t x, uint32_t q) {
  const uint64_t key = ((uint64_t)x << 32) | q;
  const uint32_t h = lcache_slot(x, q);
  // keep the other way of the pair if it already holds this key
  if (cache[h ^ 1] == key) return;
  atomicExch((unsigned long long *)&cache[h], (unsigned long long)key);
}

// Second level: a lossy device-wide table of the same pairs (2^k entries,
// cleared per decomposition). Every key ever stored names a completed link,
// so a lookup may use plain (possibly stale) loads: an old word is either
// empty (a miss, costing one redundant link) or another valid pair.
__device__ __forceinline__ uint64_t gcache_slot(uint32_t x, uint32_t q, uint64_t mask) {
  uint64_t h = ((uint64_t)x * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)q * 0xC2B2AE3D27D4EB4Full);
  return (h >> 17) & mask;
}

// Root of x from plain loads, without compression. Parent pointers only
// ever point to smaller ids, so the walk ends even on stale values, and any
// node it returns was, at some time, a root whose set contained x (so x is
// connected to it at their common core number). Used only to form cache
// keys, where such an ancestor is as good as the current root.
__device__ __forceinline__ uint32_t key_root(const uint32_t *uf, uint32_t x) {
  for (;;) {
    const uint32_t p = uf[x];
    if (p == x) return x;
    x = p;
  }
}

// key_root of x and of y, the two walks in lockstep
__device__ __forceinline__ void key_root2(const uint32_t *uf, uint32_t &x, uint32_t &y) {
  bool dx = false, dy = false;
  for (;;) {
    uint32_t px = x, py = y;
    if (!dx) px = uf[x];
    if (!dy) py = uf[y];
    dx |= px == x;
    dy |= py == y;
    x = px;
    y = py;
    if (dx && dy) return;
  }
}

// ---------------------------------------------------------------------------
// the persistent kernel
// ---------------------------------------------------------------------------

// Occupancy: 5 workgroups per CU (at most 96 VGPRs) without linking; 4 (128
// VGPRs) with it, which keeps the link path's state in registers instead
// of spilling it to scratch (measured faster than 5 with spills).
template <int R_, int S_, bool kLink>
__global__ void __launch_bounds__(kPeelBlock, kLink ? 4 : 5) k_peel(PeelArgs a) {
  using Sh = Shape<R_, S_>;
  constexpr int NO = Sh::kOthers;
  __shared__ uint64_t s_boff[kMaxPeelBlocks + 1];
  __shared__ uint32_t s_red[kPeelBlock / 64];
  __shared__ uint32_t s_cnt[kPeelBlock / 64];
  __shared__ uint32_t s_bmin;   // this workgroup's minimum at the last bucket scan
  __shared__ uint64_t s_red64[kPeelBlock / 64];
  __shared__ uint64_t s_lcache[kLinkCache];
  __shared__ uint64_t s_lq[kLink ? kPeelBlock / 64 : 1][kLink ? kWaveQ : 1];

  DevScalars *sc = a.sc;
  const GraphView &g = a.g;
  const uint32_t nb = a.nblocks;
  const uint32_t lane = lane_id();
  const uint32_t wv = threadIdx.x / 64;
  const uint64_t gtid = blockIdx.x * (uint64_t)kPeelBlock + threadIdx.x;
  const uint64_t nthreads = (uint64_t)nb * kPeelBlock;

  LinkCtx lc;
  lc.uf = a.uf;
  lc.L = a.L;
  lc.nd = a.cnt;
  lc.linkq = a.linkq;
  lc.linkq_cap = a.linkq_cap;
  lc.sc = sc;
  lc.links = 0;
  lc.unites = 0;
  __shared__ uint32_t s_retries;
  if (threadIdx.x == 0) s_retries = 0;
  lc.retries = &s_retries;
  uint64_t visits = 0, decs = 0, scans = 0, calls = 0;
  for (uint32_t i = threadIdx.x; i < kLinkCache; i += kPeelBlock) s_lcache[i] = ~0ull;
  if (!residency_gate(sc->bar, nb, &sc->status)) return;

  uint32_t k = 0;
  uint32_t t = 0;
  uint32_t nscan = 0;   // bucket scans done
  uint32_t fprev = 0;   // frontier size of the previous round
  uint32_t bi = 0;      // approximate mode: current bucket
  uint32_t rib = 0;     // approximate mode: rounds in the current bucket
  const bool approx = a.n_thr != 0;
  bool done = false;

  while (!done) {
    if (t >= a.max_rounds) {
      if (gtid == 0) atomicOr(&sc->status, ND_DERR_WATCHDOG);
      break;
    }
    uint32_t *F = (t & 1) ? a.F1 : a.F0;
    uint32_t *Fn = (t & 1) ? a.F0 : a.F1;
    uint32_t f = ld_acq32(&sc->fsize[t & 1]);
    // approximate mode: a bucket that has had its rounds passes its
    // remaining r-cliques to the next bucket; the scan rebuilds the frontier
    // from the remaining list, so the collected one is dropped (every
    // workgroup takes this branch: rib is the same everywhere)
    const bool forced = approx && rib >= a.round_cap;
    if (forced && gtid == 0) sc->fsize[t & 1] = 0;

    if (f == 0 || forced) {
      // ---- bucket scan: new level = minimum count of the remaining r-cliques.
      // Every workgroup owns one segment of the id range and keeps the list
      // of its still-present r-cliques compacted in place (order preserved),
      // so a scan needs one global atomic per workgroup, not per wave.
      const uint32_t qp = nscan & 1;
      const uint64_t bseg = (a.n_r + nb - 1) / nb;
      const uint64_t rbeg = min64((uint64_t)blockIdx.x * bseg, a.n_r);
      const uint32_t *in = (qp ? a.al1 : a.al0) + rbeg;
      uint32_t *out = (qp ? a.al0 : a.al1) + rbeg;
      const uint32_t nin = (nscan == 0) ? (uint32_t)(min64(rbeg + bseg, a.n_r) - rbeg)
                                        : a.acnt[qp * nb + blockIdx.x];
      // each thread takes kScanU consecutive entries per pass (more loads in
      // flight); a block-wide exclusive scan of the kept counts preserves order
      uint32_t mn = ND_NONE;
      uint32_t nkeep = 0;
      for (uint32_t base = 0; base < nin; base += kPeelBlock * kScanU) {
        const uint32_t i0 = base + threadIdx.x * kScanU;
        uint32_t id[kScanU], rv[kScanU];
#pragma unroll
        for (uint32_t u = 0; u < kScanU; u++)
          id[u] = (i0 + u < nin) ? ((nscan == 0) ? (uint32_t)(rbeg + i0 + u) : in[i0 + u]) : 0;
#pragma unroll
        for (uint32_t u = 0; u < kScanU; u++) rv[u] = (i0 + u < nin) ? a.pst[id[u]] : kPeeledBefore;
        uint32_t nk = 0;
#pragma unroll
        for (uint32_t u = 0; u < kScanU; u++) {
          if (i0 + u < nin && rv[u] == kAlive) {
            const uint32_t cv = a.cnt[id[u]];
            mn = cv < mn ? cv : mn;
            nk++;
          }
        }
        const uint32_t incl = wave_incl_scan(nk);
        if (lane == 63) s_cnt[wv] = incl;
        __syncthreads();
        uint32_t woff = 0, tot = 0;
        for (uint32_t w = 0; w < kPeelBlock / 64; w++) {
          woff += w < wv ? s_cnt[w] : 0;
          tot += s_cnt[w];
        }
        uint32_t o = nkeep + woff + incl - nk;
#pragma unroll
        for (uint32_t u = 0; u < kScanU; u++)
          if (i0 + u < nin && rv[u] == kAlive) out[o++] = id[u];
        nkeep += tot;
        __syncthreads();
      }
      mn = wave_min32(mn);
      if (lane == 0) s_red[wv] = mn;
      __syncthreads();
      if (threadIdx.x == 0) {
        uint32_t bm = ND_NONE;
        for (uint32_t w = 0; w < kPeelBlock / 64; w++) bm = s_red[w] < bm ? s_red[w] : bm;
        if (bm != ND_NONE) atomicMin(&sc->kmin[qp], bm);
        a.acnt[(qp ^ 1) * nb + blockIdx.x] = nkeep;
        if (nkeep) atomicAdd(&sc->n_alive[qp ^ 1], nkeep);
        s_bmin = bm;
      }
      if (!grid_barrier(sc->bar, nb, &sc->status)) break;
      const uint32_t nout = ld_acq32(&sc->n_alive[qp ^ 1]);
      if (nout == 0) {
        done = true;
        break;
      }
      const uint32_t kq = ld_acq32(&sc->kmin[qp]);
      if (gtid == 0) {
        sc->n_alive[qp] = 0;         // becomes the total of the next scan
        sc->kmin[qp ^ 1] = ND_NONE;  // minimum of the next scan
      }
      // the new level: exact, the minimum; approximate, the end of the first
      // bucket (from the current one, or the next when forced) that reaches
      // the minimum, 0 for r-cliques in no s-clique
      uint32_t lvl = kq;
      if (approx && kq != 0) {
        uint32_t b = bi + (forced ? 1u : 0u);
        while (b < a.n_thr && a.thr[b] < kq) b++;
        if (b >= a.n_thr) {   // a bucket end beyond 32 bits
          if (gtid == 0) atomicOr(&sc->status, ND_DERR_OVERFLOW);
          break;
        }
        bi = b;
        lvl = a.thr[b];
      }
      rib = 0;
      // the new frontier: remaining entries at or below the new level (none
      // in a segment whose minimum is above it)
      if (s_bmin <= lvl) {
        for (uint32_t base = 0; base < nkeep; base += kPeelBlock * kScanU) {
          const uint32_t i0 = base + threadIdx.x * kScanU;
          uint32_t id[kScanU];
#pragma unroll
          for (uint32_t u = 0; u < kScanU; u++) id[u] = (i0 + u < nkeep) ? out[i0 + u] : 0;
          bool take[kScanU];
          uint32_t nt = 0;
#pragma unroll
          for (uint32_t u = 0; u < kScanU; u++) {
            take[u] = i0 + u < nkeep && a.cnt[id[u]] <= lvl;
            nt += take[u];
          }
          const uint32_t incl = wave_incl_scan(nt);
          uint32_t wbase = 0;
          if (lane == 63 && incl) wbase = atomicAdd(&sc->fsize[t & 1], incl);
          wbase = __shfl(wbase, 63, 64);
          uint32_t o = wbase + incl - nt;
#pragma unroll
          for (uint32_t u = 0; u < kScanU; u++)
            if (take[u]) F[o++] = id[u];
        }
      }
      scans++;
      nscan++;
      k = lvl;
      if (!grid_barrier(sc->bar, nb, &sc->status)) break;
      f = ld_acq32(&sc->fsize[t & 1]);
    }

    if (a.progress && gtid == 0) {
      // progress for a host that reports long runs (system-scope stores into
      // pinned host memory; read by the host while the kernel runs)
      __hip_atomic_store(&a.progress[0], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&a.progress[1], k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&a.progress[2], f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }

    // ---- mark: core number and peel round; per-segment work prefix sums
    const uint64_t seg = (f + nb - 1) / nb;
    const uint64_t sbeg = min64((uint64_t)blockIdx.x * seg, f);
    const uint64_t send = min64(sbeg + seg, f);
    // the previous round's frontier (in Fn, which takes pushes only after the
    // barrier below) becomes peeled-before
    for (uint64_t i = gtid; i < fprev; i += nthreads) a.pst[Fn[i]] = kPeeledBefore;
    fprev = f;
    uint64_t run = 0;
    for (uint64_t base = sbeg; base < send; base += kPeelBlock) {
      const uint64_t i = base + threadIdx.x;
      uint32_t w = 0;
      if (i < send) {
        const uint32_t R = F[i];
        a.round[R] = t;
        a.pst[R] = kPeeledNow;
        a.cnt[R] = k;
        if constexpr (RecOf<Sh>::value) w = Sh::len_rec(g, R, &a.frec[4 * i]);
        else w = Sh::len(g, R);
      }
      // block-wide inclusive scan of w
      uint32_t incl = wave_incl_scan(w);
      if (lane == 63) s_red64[wv] = incl;
      __syncthreads();
      uint64_t wpre = 0, btot = 0;
      for (uint32_t x = 0; x < kPeelBlock / 64; x++) {
        if (x < wv) wpre += s_red64[x];
        btot += s_red64[x];
      }
      if (i < send) a.wscan[i] = run + wpre + incl;
      run += btot;
      __syncthreads();
    }
    if (threadIdx.x == 0) a.btot[blockIdx.x] = run;
    if (gtid == 0) sc->fsize[(t + 1) & 1] = 0;
    if (!grid_barrier(sc->bar, nb, &sc->status)) break;

    // ---- visit: one probe element per lane over the whole frontier
    {
      // exclusive scan of the block totals into LDS (each thread owns a run)
      const uint32_t per = (nb + kPeelBlock - 1) / kPeelBlock;
      const uint32_t j0 = threadIdx.x * per;
      uint64_t mine = 0;
      for (uint32_t j = j0; j < j0 + per && j < nb; j++) mine += a.btot[j];
      uint64_t incl = mine;
      for (int d = 1; d < 64; d <<= 1) {
        uint64_t y = __shfl_up(incl, d, 64);
        if (lane >= (uint32_t)d) incl += y;
      }
      if (lane == 63) s_red64[wv] = incl;
      __syncthreads();
      uint64_t acc = incl - mine;
      for (uint32_t x = 0; x < wv; x++) acc += s_red64[x];
      for (uint32_t j = j0; j < j0 + per && j < nb; j++) {
        s_boff[j] = acc;
        acc += a.btot[j];
      }
      if (threadIdx.x == kPeelBlock - 1) s_boff[nb] = acc;
      __syncthreads();
    }
    const uint64_t P = s_boff[nb];
    // A large round first maps every chunk of 64 probe units to the frontier
    // slot of its first unit (each slot writes the chunks that start inside
    // it; one more grid barrier), so a lane finds its slot from the map in a
    // short search instead of a block search and a slot search. Small rounds
    // skip the map: the barrier would cost more than it saves.
    const uint64_t nchunks = (P + 63) >> 6;
    const bool use_map = P >= 16ull * nthreads && nchunks <= a.cslot_cap;
    if (use_map) {
      const uint64_t ub = s_boff[blockIdx.x];
      for (uint64_t i = sbeg + threadIdx.x; i < send; i += kPeelBlock) {
        const uint64_t u0 = ub + (i > sbeg ? a.wscan[i - 1] : 0);
        const uint64_t u1 = ub + a.wscan[i];
        for (uint64_t ch = (u0 + 63) >> 6; (ch << 6) < u1; ch++) a.cslot[ch] = (uint32_t)i;
      }
      if (!grid_barrier(sc->bar, nb, &sc->status)) break;
    }
    uint64_t *wq = s_lq[kLink ? wv : 0];
    uint32_t qn = 0;   // pending link steps of this wave (uniform)
    uint32_t seg_hint = 0;   // this lane's segment in its previous pass (units only grow)
    for (uint64_t base = blockIdx.x * (uint64_t)kPeelBlock + wv * 64ull; base < P;
         base += nthreads) {
      const uint64_t p = base + lane;
      uint32_t others[NO];
      bool push[NO];
      uint64_t lpair[NO];   // link calls of this lane's probe, queued below
#pragma unroll
      for (int j = 0; j < NO; j++) {
        push[j] = false;
        lpair[j] = ~0ull;
      }
      uint32_t R = 0, idx = 0;
      uint64_t slot = 0;   // R's frontier slot
      bool have = false;
      if (p < P && use_map) {
        // the slot holding p lies between the slots of p's chunk and of the
        // next chunk: the last slot there whose first unit is <= p
        const uint64_t ch = p >> 6;
        uint64_t lo = a.cslot[ch];
        uint64_t hi = ch + 1 < nchunks ? (uint64_t)a.cslot[ch + 1] + 1 : f;
        auto start = [&](uint64_t i) -> uint64_t {
          const uint64_t blk = i / seg;
          return s_boff[blk] + (i > blk * seg ? a.wscan[i - 1] : 0);
        };
        while (hi - lo > 1) {
          const uint64_t mid = (lo + hi) >> 1;
          if (start(mid) <= p) lo = mid;
          else hi = mid;
        }
        R = F[lo];
        slot = lo;
        idx = (uint32_t)(p - start(lo));
      } else if (p < P) {
        // block segment holding unit p (s_boff[lo] <= p < s_boff[hi]): a
        // binary search in the first pass, a gallop from the previous
        // segment after it; then the frontier slot inside the segment
        uint32_t lo = seg_hint, hi = nb;
        if (lo != 0) {
          uint32_t step = 1;
          while (lo + step < nb && s_boff[lo + step] <= p) {
            lo += step;
            step <<= 1;
          }
          hi = lo + step < nb ? lo + step : nb;
        }
        while (hi - lo > 1) {
          uint32_t mid = (lo + hi) >> 1;
          if (s_boff[mid] <= p) lo = mid;
          else hi = mid;
        }
        seg_hint = lo;
        const uint64_t qoff = p - s_boff[lo];
        const uint64_t b0 = min64((uint64_t)lo * seg, f);
        const uint64_t b1 = min64(b0 + seg, f);
        // first slot with wscan > qoff: every lane searches for itself (the
        // lanes take consecutive units, so their loads mostly share lines)
        uint64_t x0 = b0;
        {
          uint64_t x1 = b1;
          while (x0 < x1) {
            uint64_t mid = (x0 + x1) >> 1;
            if (a.wscan[mid] <= qoff) x0 = mid + 1;
            else x1 = mid;
          }
        }
        R = F[x0];
        slot = x0;
        const uint64_t before = (x0 > b0) ? a.wscan[x0 - 1] : 0;
        idx = (uint32_t)(qoff - before);
      }
      have = p < P;
      bool hit = false;
      if constexpr (RecOf<Sh>::value) hit = have && Sh::visit_rec(g, &a.frec[4 * slot], idx, others);
      else hit = have && Sh::visit(g, R, idx, others);
      if (hit) {
        visits++;
        uint32_t rr[NO];   // peel states
        bool dead = false, lead = true;
#pragma unroll
        for (int j = 0; j < NO; j++) {
          rr[j] = a.pst[others[j]];
          dead |= rr[j] == kPeeledBefore;
          lead &= !(rr[j] == kPeeledNow && others[j] < R);
        }
        // decrements first; their old values are only compared after the
        // link checks below, so the atomics stay in flight meanwhile
        uint32_t oldc[NO];
        bool dec[NO];
#pragma unroll
        for (int j = 0; j < NO; j++) {
          dec[j] = !dead && lead && rr[j] == kAlive;
          oldc[j] = 0;
          if (dec[j]) {
            oldc[j] = atomicSub(&a.cnt[others[j]], 1u);
            decs++;
          }
        }
        uint32_t qroot = ND_NONE;   // cache key of R's set, formed on first use
#pragma unroll
        for (int j = 0; j < NO; j++) {
          if (kLink && (rr[j] == kPeeledBefore || (rr[j] == kPeeledNow && R < others[j]))) {
            uint32_t x = others[j];
            if (qroot == ND_NONE) {
              qroot = R;
              key_root2(a.uf, qroot, x);
            } else {
              x = key_root(a.uf, x);
            }
            if (x == qroot || lcache_hit(s_lcache, x, qroot)) continue;
            const uint64_t key = ((uint64_t)x << 32) | qroot;
            uint64_t *gslot = &a.gcache[gcache_slot(x, qroot, a.gcache_mask)];
            if (*gslot == key) {
              lcache_put(s_lcache, x, qroot);
              continue;
            }
            calls++;
            lpair[j] = ((uint64_t)others[j] << 32) | R;
            lcache_put(s_lcache, x, qroot);
            atomicExch((unsigned long long *)gslot, (unsigned long long)key);
          }
        }
#pragma unroll
        for (int j = 0; j < NO; j++) push[j] = dec[j] && oldc[j] == k + 1;
      }
#pragma unroll
      for (int j = 0; j < NO; j++) {
        uint32_t slot = wave_append(&sc->fsize[(t + 1) & 1], push[j]);
        if (push[j]) Fn[slot] = others[j];
      }
      if (kLink) {
        // queue this pass's link calls; run them whenever a full pass of
        // 64 steps is pending
#pragma unroll
        for (int j = 0; j < NO; j++) {
          if (qn > kWaveQ - 64) wave_q_drain(lc, wq, qn, 64);
          wave_q_push(wq, qn, lpair[j] != ~0ull, lpair[j]);
        }
        wave_q_drain(lc, wq, qn, 64);
      }
    }
    if (kLink) wave_q_drain(lc, wq, qn, 1);
    if (!grid_barrier(sc->bar, nb, &sc->status)) break;

    // ---- drain spilled link pairs (rare): repeat until the queue is empty
    bool ok = true;
    for (; kLink;) {
      const uint32_t h = ld_acq32(&sc->linkq_head);
      const uint32_t tl = ld_acq32(&sc->linkq_tail);
      if (h == tl) break;
      if (tl - h > a.linkq_cap) {   // overflowed: the status bit is already set
        ok = false;
        break;
      }
      for (uint64_t d = gtid; d < (uint32_t)(tl - h); d += nthreads) {
        const uint64_t slot = (h + (uint32_t)d) & (a.linkq_cap - 1);
        link_efficient(lc, a.linkq[2 * slot], a.linkq[2 * slot + 1]);
      }
      if (!grid_barrier(sc->bar, nb, &sc->status)) { ok = false; break; }
      if (gtid == 0) sc->linkq_head = tl;
      if (!grid_barrier(sc->bar, nb, &sc->status)) { ok = false; break; }
    }
    if (!ok) break;
    t++;
    rib++;
  }

  // statistics
  uint64_t v = wave_sum64(visits), d = wave_sum64(decs), l = wave_sum64(lc.links),
           u = wave_sum64(lc.unites), cl = wave_sum64(calls);
  __syncthreads();
  if (threadIdx.x == 0 && s_retries)
    atomicAdd((unsigned long long *)&sc->cas_retries, (unsigned long long)s_retries);
  if (lane == 0) {
    if (cl) atomicAdd((unsigned long long *)&sc->link_calls, (unsigned long long)cl);
    if (v) atomicAdd((unsigned long long *)&sc->visits, (unsigned long long)v);
    if (d) atomicAdd((unsigned long long *)&sc->decrements, (unsigned long long)d);
    if (l) atomicAdd((unsigned long long *)&sc->links, (unsigned long long)l);
    if (u) atomicAdd((unsigned long long *)&sc->unites, (unsigned long long)u);
  }
  if (gtid == 0) {
    sc->rounds = t;
    sc->k = k;
    sc->bucket_scans = scans;
  }
}

// ---------------------------------------------------------------------------
// Hierarchy by descending core number (the two-pass construction, "TE"):
// after a peel without linking, the same union-find uf (same-core
// components) and nearest-lower-core table L that Algorithm 5 builds are
// built level by level, c = k down to 1. When level c starts, every part of
// the hierarchy above c is final and forms trees; a second union-find (tuf)
// groups r-cliques by tree and remembers each tree's lowest component
// (bottom). An r-clique R of core c that shares an s-clique with R' (core
// >= c) either joins R''s component (same core), or hangs R''s tree below
// R's component: L[bottom] = R, set once by CAS; a later r-clique of core c
// that reaches the same tree finds L taken and joins the component that took
// it. Each pair costs a few union-find operations, independent of the depth
// of the hierarchy; Algorithm 5 instead walks L chains level by level, which
// is slow when core numbers span thousands of levels.
// ---------------------------------------------------------------------------

struct HierArgs {
  GraphView g;
  uint64_t n_r;
  const uint32_t *nd;      // core numbers
  const uint32_t *ord;     // r-cliques by core number, descending
  const uint64_t *loff;    // [k + 2]: core c occupies ord[loff[k - c], loff[k - c + 1])
  uint32_t *uf, *L, *tuf, *bottom;
  uint64_t *wscan;
  uint64_t *btot;
  DevScalars *sc;
  uint32_t nblocks;
  uint32_t k;
  uint32_t *progress;
};

// rootR: a root R had during this visit. Sets only grow, so finding the
// partner side at rootR proves both are joined already; a rootR that has
// since lost its root status only sends the pair down the full path.
__device__ __forceinline__ void hier_pair(const HierArgs &a, uint32_t R, uint32_t rootR,
                                          uint32_t R2, uint32_t c, uint64_t &unites,
                                          uint32_t *retries) {
  // Every uf union is paired with a tuf union of the same two sets (or of
  // sets containing them), so a uf set always lies inside one tuf set once
  // the level's unions are done: when the uf union finds both sides already
  // joined, the tuf union would join nothing either and is skipped.
  const uint32_t n2 = a.nd[R2];
  if (n2 == c) {   // same core: one component, one tree
    if (uf_find(a.uf, R2) == rootR) return;
    if (uf_unite(a.uf, R, R2, retries) != ND_NONE) {
      unites++;
      uf_unite(a.tuf, R, R2, retries);
    }
    return;
  }
  const uint32_t T = uf_find(a.tuf, R2);
  const uint32_t B = ld_acq32(&a.bottom[T]);
  if (a.nd[B] == c) {   // R2's tree already hangs below a core-c component
    if (uf_find(a.uf, B) == rootR) return;
    if (uf_unite(a.uf, B, R, retries) != ND_NONE) {
      unites++;
      uf_unite(a.tuf, T, R, retries);
    }
    return;
  }
  // R2's tree still ends at a component of a higher core: hang it below R
  const uint32_t Bs = uf_find(a.uf, B);   // final: that core is finished
  const uint32_t old = atomicCAS(&a.L[Bs], ND_NONE, R);
  if (old == ND_NONE) {
    uf_unite(a.tuf, T, R, retries);
    const uint32_t w = uf_find(a.tuf, R);
    __hip_atomic_store(&a.bottom[w], R, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {   // taken at this level by the component of `old`
    unites += uf_unite(a.uf, old, R, retries) != ND_NONE;
    uf_unite(a.tuf, T, R, retries);
  }
}

template <int R_, int S_>
__global__ void __launch_bounds__(kPeelBlock) k_hier(HierArgs a) {
  using Sh = Shape<R_, S_>;
  constexpr int NO = Sh::kOthers;
  __shared__ uint64_t s_boff[kMaxPeelBlocks + 1];
  __shared__ uint64_t s_red64[kPeelBlock / 64];

  DevScalars *sc = a.sc;
  const GraphView &g = a.g;
  const uint32_t nb = a.nblocks;
  const uint32_t lane = lane_id();
  const uint32_t wv = threadIdx.x / 64;
  const uint64_t gtid = blockIdx.x * (uint64_t)kPeelBlock + threadIdx.x;
  const uint64_t nthreads = (uint64_t)nb * kPeelBlock;
  uint64_t visits = 0, pairs = 0, unites = 0;
  __shared__ uint32_t s_retries;
  if (threadIdx.x == 0) s_retries = 0;
  uint32_t *retries = &s_retries;
  if (!residency_gate(sc->bar, nb, &sc->status)) return;

  for (uint32_t c = a.k; c >= 1; c--) {
    const uint64_t fb = a.loff[a.k - c], fe = a.loff[a.k - c + 1];
    const uint64_t f = fe - fb;
    if (f == 0) continue;   // the same decision in every workgroup
    const uint32_t *F = a.ord + fb;
    if (a.progress && gtid == 0) {
      __hip_atomic_store(&a.progress[0], a.k - c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&a.progress[1], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&a.progress[2], (uint32_t)f, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    }
    // per-segment inclusive prefix of the probe work of this level's r-cliques
    const uint64_t seg = (f + nb - 1) / nb;
    const uint64_t sbeg = min64((uint64_t)blockIdx.x * seg, f);
    const uint64_t send = min64(sbeg + seg, f);
    uint64_t run = 0;
    for (uint64_t base = sbeg; base < send; base += kPeelBlock) {
      const uint64_t i = base + threadIdx.x;
      const uint32_t w = i < send ? Sh::len(g, F[i]) : 0;
      const uint32_t incl = wave_incl_scan(w);
      if (lane == 63) s_red64[wv] = incl;
      __syncthreads();
      uint64_t wpre = 0, btot = 0;
      for (uint32_t x = 0; x < kPeelBlock / 64; x++) {
        if (x < wv) wpre += s_red64[x];
        btot += s_red64[x];
      }
      if (i < send) a.wscan[i] = run + wpre + incl;
      run += btot;
      __syncthreads();
    }
    if (threadIdx.x == 0) a.btot[blockIdx.x] = run;
    if (!grid_barrier(sc->bar, nb, &sc->status)) break;
    {
      const uint32_t per = (nb + kPeelBlock - 1) / kPeelBlock;
      const uint32_t j0 = threadIdx.x * per;
      uint64_t mine = 0;
      for (uint32_t j = j0; j < j0 + per && j < nb; j++) mine += a.btot[j];
      uint64_t incl = mine;
      for (int d = 1; d < 64; d <<= 1) {
        uint64_t y = __shfl_up(incl, d, 64);
        if (lane >= (uint32_t)d) incl += y;
      }
      if (lane == 63) s_red64[wv] = incl;
      __syncthreads();
      uint64_t acc = incl - mine;
      for (uint32_t x = 0; x < wv; x++) acc += s_red64[x];
      for (uint32_t j = j0; j < j0 + per && j < nb; j++) {
        s_boff[j] = acc;
        acc += a.btot[j];
      }
      if (threadIdx.x == kPeelBlock - 1) s_boff[nb] = acc;
      __syncthreads();
    }
    const uint64_t P = s_boff[nb];
    for (uint64_t base = blockIdx.x * (uint64_t)kPeelBlock + wv * 64ull; base < P;
         base += nthreads) {
      const uint64_t p = base + lane;
      if (p < P) {
        uint32_t lo = 0, hi = nb;   // s_boff[lo] <= p < s_boff[hi]
        while (hi - lo > 1) {
          uint32_t mid = (lo + hi) >> 1;
          if (s_boff[mid] <= p) lo = mid;
          else hi = mid;
        }
        const uint64_t qoff = p - s_boff[lo];
        const uint64_t b0 = min64((uint64_t)lo * seg, f);
        const uint64_t b1 = min64(b0 + seg, f);
        const uint64_t x0 = gallop_u64(a.wscan, b0, b1, qoff);
        const uint32_t R = F[x0];
        const uint64_t before = (x0 > b0) ? a.wscan[x0 - 1] : 0;
        uint32_t others[NO];
        if (Sh::visit(g, R, (uint32_t)(qoff - before), others)) {
          visits++;
          const uint32_t rootR = uf_find(a.uf, R);
#pragma unroll
          for (int j = 0; j < NO; j++) {
            if (a.nd[others[j]] >= c) {
              pairs++;
              hier_pair(a, R, rootR, others[j], c, unites, retries);
            }
          }
        }
      }
    }
    if (!grid_barrier(sc->bar, nb, &sc->status)) break;
  }
  const uint64_t v = wave_sum64(visits), l = wave_sum64(pairs), u = wave_sum64(unites);
  __syncthreads();
  if (threadIdx.x == 0 && s_retries)
    atomicAdd((unsigned long long *)&sc->cas_retries, (unsigned long long)s_retries);
  if (lane == 0) {
    if (v) atomicAdd((unsigned long long *)&sc->hier_visits, (unsigned long long)v);
    if (l) atomicAdd((unsigned long long *)&sc->links, (unsigned long long)l);
    if (u) atomicAdd((unsigned long long *)&sc->unites, (unsigned long long)u);
  }
}

// r-cliques by core number, descending (counting sort; order inside a level
// is free)
__global__ void k_level_hist(uint64_t n, const uint32_t *__restrict__ nd, uint32_t k,
                             uint32_t *__restrict__ hist) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n;
       x += (uint64_t)gridDim.x * blockDim.x)
    atomicAdd(&hist[k - nd[x]], 1u);
}

__global__ void k_level_scatter(uint64_t n, const uint32_t *__restrict__ nd, uint32_t k,
                                const uint64_t *__restrict__ loff, uint32_t *__restrict__ fill,
                                uint32_t *__restrict__ ord) {
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < n;
       x += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t b = k - nd[x];
    ord[loff[b] + atomicAdd(&fill[b], 1u)] = (uint32_t)x;
  }
}

__global__ void k_iota(uint32_t *a, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    a[i] = (uint32_t)i;
}

// persistent grid: as many workgroups as fit on the device at once. The
// occupancy query is bounded by the kernel's registers at a 16-register
// allocation granule (the query's own figure was not resident for a
// 68-register kernel), and by the largest grid this context has seen
// resident; the kernels' residency gate catches anything still too large.
template <typename K>
uint32_t coop_grid(nd_ctx *c, K kern, uint32_t *nb) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kern, kPeelBlock, 0) !=
          hipSuccess ||
      per_cu < 1)
    return 0;
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, (const void *)kern) == hipSuccess && fa.numRegs > 0) {
    const int regs = (fa.numRegs + 15) / 16 * 16;
    const int waves_per_simd = std::min(8, 512 / regs);
    const int waves_per_block = kPeelBlock / 64;
    per_cu = std::max(1, std::min(per_cu, waves_per_simd * 4 / waves_per_block));
  } else {
    (void)hipGetLastError();
  }
  uint64_t cap = std::max<uint64_t>(1, (uint64_t)per_cu * (uint64_t)c->cu_count / c->grid_div);
  for (const auto &e : c->resident_cap)
    if (e.first == (const void *)kern) cap = std::min<uint64_t>(cap, e.second);
  cap = std::min<uint64_t>(cap, kMaxPeelBlocks);
  uint64_t want = c->peel_blocks;
  if (!want)
    for (const nd_schedule &e : c->sched)
      if (e.kind == (c->in_batch ? ND_SCHED_BATCH : ND_SCHED_SINGLE) && e.r == c->r &&
          e.s == c->s && c->n_r <= e.n_r_max) {
        want = e.peel_blocks;
        break;
      }
  if (!want) want = cap;
  *nb = (uint32_t)std::max<uint64_t>(1, std::min(want, cap));
  return *nb;
}

template <int R_, int S_, bool kLink>
nd_status launch_peel(nd_ctx *c, PeelArgs &pa) {
  const void *kern = (const void *)k_peel<R_, S_, kLink>;
  uint32_t nb = 0;
  if (!coop_grid(c, k_peel<R_, S_, kLink>, &nb))
    return nd_fail(c, ND_E_DEVICE, "occupancy query failed for the peel kernel");
  void *args[] = {&pa};
  if (pa.progress) c->report_phase = "peel";
  nd_status st = nd_persistent_launch(c, kern, &nb, &pa.nblocks, dim3(kPeelBlock), args,
                                c->events_ok ? c->ev[5] : nullptr,
                                c->events_ok ? c->ev[6] : nullptr, "peel launch");
  c->report_phase = nullptr;
  return st;
}

// Two passes: the peel without linking, then k_hier over the core numbers.
template <int R_, int S_>
nd_status run_te(nd_ctx *c, PeelArgs &pa) {
  nd_status st = launch_peel<R_, S_, false>(c, pa);
  if (st != ND_OK) return st;
  DevScalars *sc = pa.sc;
  uint32_t hk[2] = {0, 0};
  if ((st = nd_hip(c, hipMemcpyAsync(hk, &sc->status, 8, hipMemcpyDeviceToHost, c->stream),
                   "peel result")) != ND_OK ||
      (st = nd_hip(c, hipStreamSynchronize(c->stream), "peel result")) != ND_OK)
    return st;
  if (hk[0]) return ND_OK;   // device error: reported by the status check that follows
  const uint32_t k = hk[1];
  nd_report(c, "peel (no links) done: k=%u; hierarchy by descending core", k);
  const uint64_t nr = pa.n_r;
  HierArgs h{};
  h.g = pa.g;
  h.n_r = nr;
  h.nd = pa.cnt;
  h.uf = pa.uf;
  h.L = pa.L;
  h.ord = pa.F0;
  h.tuf = pa.al0;
  h.bottom = pa.al1;
  h.wscan = pa.wscan;
  h.btot = pa.btot;
  h.sc = sc;
  h.k = k;
  h.progress = pa.progress;
  uint32_t *hist = (uint32_t *)nd_buf(c, B_LHIST, (k + 2ull) * 4, &st);
  if (!hist) return st;
  uint64_t *loff = (uint64_t *)nd_buf(c, B_LOFF, (k + 2ull) * 8, &st);
  if (!loff) return st;
  h.loff = loff;
  if ((st = nd_hip(c, hipMemsetAsync(hist, 0, (k + 2ull) * 4, c->stream), "level hist")) != ND_OK)
    return st;
  hipLaunchKernelGGL(k_level_hist, dim3(nd_grid(nr, 256, 16384)), dim3(256), 0, c->stream, nr,
                     pa.cnt, k, hist);
  uint64_t total = 0;
  if ((st = nd_exclusive_scan_u32_to_u64(c, hist, loff, k + 1ull, &total)) != ND_OK) return st;
  if ((st = nd_hip(c, hipMemsetAsync(hist, 0, (k + 2ull) * 4, c->stream), "level fill")) != ND_OK)
    return st;
  hipLaunchKernelGGL(k_level_scatter, dim3(nd_grid(nr, 256, 16384)), dim3(256), 0, c->stream, nr,
                     pa.cnt, k, loff, hist, pa.F0);
  hipLaunchKernelGGL(k_iota, dim3(nd_grid(nr, 256, 16384)), dim3(256), 0, c->stream, pa.al0, nr);
  hipLaunchKernelGGL(k_iota, dim3(nd_grid(nr, 256, 16384)), dim3(256), 0, c->stream, pa.al1, nr);
  if ((st = nd_hip(c, hipGetLastError(), "level sort")) != ND_OK) return st;
  if (pa.progress) memset(pa.progress, 0, 4 * sizeof(uint32_t));
  uint32_t nb = 0;
  if (!coop_grid(c, k_hier<R_, S_>, &nb))
    return nd_fail(c, ND_E_DEVICE, "occupancy query failed for the hierarchy kernel");
  void *args[] = {&h};
  if (h.progress) c->report_phase = "hierarchy";
  st = nd_persistent_launch(c, (const void *)k_hier<R_, S_>, &nb, &h.nblocks, dim3(kPeelBlock), args,
                      nullptr, c->events_ok ? c->ev[9] : nullptr, "hierarchy launch");
  c->report_phase = nullptr;
  return st;
}

}  // namespace

// s = 5..7: the peel (or, with te, the peel and the two-pass hierarchy) of
// the pairs with `others` = C(s,r) - 1 other r-cliques per s-clique
nd_status nd_peel_general_a(nd_ctx *c, PeelArgs &pa, bool te, uint32_t others);
nd_status nd_peel_general_b(nd_ctx *c, PeelArgs &pa, bool te, uint32_t others);
