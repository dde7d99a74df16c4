// nd_peel.hip -- the peel stage: buffers, scalars and the dispatch to the
// persistent peel (and hierarchy) kernels of nd_peel_kern.h.
#include "nd_peel_kern.h"

nd_status nd_stage_peel(nd_ctx *c, const GraphView &g) {
  nd_status st;
  const uint64_t nr = c->n_r;
  DevScalars *sc = (DevScalars *)c->bufs[B_SCAL].p;
  if (nr == 0) return ND_OK;
  if (nr >= 0xFFFFFFFFull) return nd_fail(c, ND_E_OVERFLOW, "r-clique ids exceed 32 bits");
  PeelArgs pa{};
  pa.g = g;
  pa.n_r = nr;
  pa.cnt = (uint32_t *)c->bufs[B_CNT].p;
  if (!(pa.round = (uint32_t *)nd_buf(c, B_ROUND, nr * 4, &st))) return st;
  if (!(pa.pst = (uint8_t *)nd_buf(c, B_PSTATE, nr, &st))) return st;
  if (!(pa.uf = (uint32_t *)nd_buf(c, B_UF, nr * 4, &st))) return st;
  if (!(pa.L = (uint32_t *)nd_buf(c, B_L, nr * 4, &st))) return st;
  if (((c->r == 3 && c->s == 4) || (c->r == 2 && c->s == 3)) &&
      !(pa.frec = (uint64_t *)nd_buf(c, B_FREC, nr * 32, &st)))
    return st;
  if (!(pa.F0 = (uint32_t *)nd_buf(c, B_F0, nr * 4, &st))) return st;
  if (!(pa.F1 = (uint32_t *)nd_buf(c, B_F1, nr * 4, &st))) return st;
  if (!(pa.wscan = (uint64_t *)nd_buf(c, B_WSCAN, nr * 8, &st))) return st;
  if (!(pa.al0 = (uint32_t *)nd_buf(c, B_AL0, nr * 4, &st))) return st;
  if (!(pa.al1 = (uint32_t *)nd_buf(c, B_AL1, nr * 4, &st))) return st;
  if (!(pa.btot = (uint64_t *)nd_buf(c, B_BTOT, (kMaxPeelBlocks + 1) * 8, &st))) return st;
  if (!(pa.acnt = (uint32_t *)nd_buf(c, B_ACNT, 2 * kMaxPeelBlocks * 4, &st))) return st;
  pa.linkq_cap = 1u << 16;
  while (pa.linkq_cap < nr && pa.linkq_cap < (1u << 26)) pa.linkq_cap <<= 1;
  if (!(pa.linkq = (uint32_t *)nd_buf(c, B_LINKQ, pa.linkq_cap * 8ull, &st))) return st;
  {
    // 2^k entries, about one per 16 r-cliques, between 2^16 and 2^22
    uint64_t ge = 1u << 16;
    while (ge < (1u << 22) && ge * 16 < nr) ge <<= 1;
    if (!(pa.gcache = (uint64_t *)nd_buf(c, B_GCACHE, ge * 8, &st))) return st;
    pa.gcache_mask = ge - 1;
    if ((st = nd_hip(c, hipMemsetAsync(pa.gcache, 0xFF, ge * 8, c->stream), "gcache")) != ND_OK)
      return st;
  }
  // chunk map of large rounds (one entry per 64 probe units of a round);
  // rounds with more chunks fall back to the two searches
  pa.cslot_cap = nr / 2 + (1u << 16);
  if (!(pa.cslot = (uint32_t *)nd_buf(c, B_CSLOT, pa.cslot_cap * 4, &st))) return st;
  if (c->approx_delta > 0) {
    // Algorithm 2's geometric buckets: ends floor((C + delta)(1 + delta)^(i+1)),
    // the product by repeated multiplication in double precision, while they
    // fit 32 bits; a bucket is processed at most
    // floor(ln n_r / ln(1 + delta / C)) + 1 rounds (Lemma 2: each round leaves
    // at most a C / (C + delta) share of the r-cliques of the bucket's core
    // range outside it)
    uint64_t C = 1;   // C(s, r)
    for (uint32_t i = 0; i < c->r; i++) C = C * (c->s - i) / (i + 1);
    const double d = c->approx_delta;
    uint32_t host_thr[4096];
    uint32_t nt = 0;
    double t = (double)C + d;
    while (nt < 4096) {
      t *= 1.0 + d;
      if (t >= 4294967296.0) break;
      host_thr[nt++] = (uint32_t)t;
    }
    if (nt == 0) return nd_fail(c, ND_E_OVERFLOW, "approximate buckets exceed 32 bits");
    uint32_t *dthr = (uint32_t *)nd_buf(c, B_THR, nt * 4ull, &st);
    if (!dthr) return st;
    if ((st = nd_hip(c, hipMemcpyAsync(dthr, host_thr, nt * 4ull, hipMemcpyHostToDevice,
                                       c->stream), "bucket ends")) != ND_OK)
      return st;
    pa.thr = dthr;
    pa.n_thr = nt;
    uint64_t cap = 1;
    if (nr > 1) cap = (uint64_t)(std::log((double)nr) / std::log(1.0 + d / (double)C)) + 1;
    pa.round_cap = (uint32_t)std::min<uint64_t>(cap, 0xFFFFFFFFull);
    c->info.round_cap = pa.round_cap;
  }
  pa.sc = sc;
  pa.progress = c->progress;
  if (pa.progress) memset(pa.progress, 0, 4 * sizeof(uint32_t));
  uint64_t wd = c->watchdog ? c->watchdog : nr + 2;
  pa.max_rounds = (uint32_t)std::min<uint64_t>(wd, 0xFFFFFFF0ull);

  if ((st = nd_hip(c, hipMemsetAsync(pa.round, 0xFF, nr * 4, c->stream), "round")) != ND_OK)
    return st;
  if ((st = nd_hip(c, hipMemsetAsync(pa.pst, kAlive, nr, c->stream), "peel state")) != ND_OK)
    return st;
  if ((st = nd_hip(c, hipMemsetAsync(pa.L, 0xFF, nr * 4, c->stream), "L")) != ND_OK) return st;
  hipLaunchKernelGGL(k_iota, dim3(nd_grid(nr, 256, 16384)), dim3(256), 0, c->stream, pa.uf, nr);
  // scalars: counters zero, kmin = NONE (the barrier words are cleared per launch)
  DevScalars init;
  memset(&init, 0, sizeof(init));
  init.kmin[0] = init.kmin[1] = ND_NONE;
  // keep n_s and max_outdeg: copy only the fields the peel owns
  const size_t off_lo = offsetof(DevScalars, visits);
  const size_t off_hi = offsetof(DevScalars, max_outdeg);
  if ((st = nd_hip(c,
                   hipMemcpyAsync((char *)sc + off_lo, (char *)&init + off_lo, off_hi - off_lo,
                                  hipMemcpyHostToDevice, c->stream),
                   "peel scalars")) != ND_OK)
    return st;
  if ((st = nd_hip(c, hipStreamSynchronize(c->stream), "peel scalars sync")) != ND_OK) return st;

  const uint32_t r = c->r, s = c->s;
  const bool te = nd_use_te(c);
  c->info.hier_te = te ? 1 : 0;
  if (r == 1 && s == 2) return te ? run_te<1, 2>(c, pa) : launch_peel<1, 2, true>(c, pa);
  if (r == 2 && s == 3) return te ? run_te<2, 3>(c, pa) : launch_peel<2, 3, true>(c, pa);
  if (r == 3 && s == 4) return te ? run_te<3, 4>(c, pa) : launch_peel<3, 4, true>(c, pa);
  if (r == 2 && s == 4) return te ? run_te<2, 4>(c, pa) : launch_peel<2, 4, true>(c, pa);
  if (r == 1 && s == 3) return te ? run_te<1, 3>(c, pa) : launch_peel<1, 3, true>(c, pa);
  if (r == 1 && s == 4) return te ? run_te<1, 4>(c, pa) : launch_peel<1, 4, true>(c, pa);
  if (nd_rs_general(s)) {
    const uint32_t others = g.nsm - 1;   // C(s,r) - 1
    return others <= 9 ? nd_peel_general_a(c, pa, te, others)
                       : nd_peel_general_b(c, pa, te, others);
  }
  return nd_fail(c, ND_E_UNSUPPORTED, "peeling for this (r,s) is not built");
}
