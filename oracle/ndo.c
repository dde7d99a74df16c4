/*
 * ndo.c -- plain sequential CPU oracle for exact (r,s) nucleus decomposition
 * and its hierarchy. TEST INFRASTRUCTURE ONLY (see ndo.h): the product
 * library never includes, links or calls this file.
 *
 * Deliberately simple: every step follows a definition from the paper with
 * plain loops, sorted-array binary searches and no parallelism, blocking or
 * fusion. Speed is not a goal.
 *
 * Steps (arXiv 2306.08623):
 *   O1  list r-cliques as ascending tuples in lexicographic order
 *       (the canonical r-clique id is the index in this order);
 *   O2  list every s-clique once and add one to the count of each of its
 *       C(s,r) r-cliques (Section 3: s-clique degree);
 *   O3  sequential minimum-degree peel (Section 6, proof of Lemma 1):
 *       core number = running maximum of the minimum current degree;
 *   O4  hierarchy from the definition (Section 5, Algorithm 1 semantics;
 *       Section 7.4 practical form): descending levels, one union-find;
 *   O5  canonical numbering of the internal nodes by (level, min leaf).
 */
#define _POSIX_C_SOURCE 199309L
#include "ndo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define MAXS 7
#define NONE UINT64_MAX

typedef struct {
  uint32_t n;
  const uint64_t *rp;
  const uint32_t *col;
  uint64_t maxdeg;
} graph;

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* ---- growable arrays ---------------------------------------------------- */

typedef struct { uint32_t *a; uint64_t n, cap; int oom; } vec32;
typedef struct { uint64_t *a; uint64_t n, cap; int oom; } vec64;

static void v32_push(vec32 *v, uint32_t x) {
  if (v->oom) return;
  if (v->n == v->cap) {
    uint64_t nc = v->cap ? v->cap * 2 : 1024;
    uint32_t *p = (uint32_t *)realloc(v->a, nc * sizeof(uint32_t));
    if (!p) { v->oom = 1; return; }
    v->a = p; v->cap = nc;
  }
  v->a[v->n++] = x;
}

static void v64_push(vec64 *v, uint64_t x) {
  if (v->oom) return;
  if (v->n == v->cap) {
    uint64_t nc = v->cap ? v->cap * 2 : 1024;
    uint64_t *p = (uint64_t *)realloc(v->a, nc * sizeof(uint64_t));
    if (!p) { v->oom = 1; return; }
    v->a = p; v->cap = nc;
  }
  v->a[v->n++] = x;
}

/* ---- graph helpers ------------------------------------------------------ */

static int adjacent(const graph *g, uint32_t u, uint32_t v) {
  uint64_t lo = g->rp[u], hi = g->rp[u + 1];
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    uint32_t x = g->col[mid];
    if (x == v) return 1;
    if (x < v) lo = mid + 1; else hi = mid;
  }
  return 0;
}

int ndo_validate_csr(uint32_t n, const uint64_t *row_ptr, const uint32_t *col) {
  if (!row_ptr) return NDO_E_INVALID_ARG;
  if (row_ptr[0] != 0) return NDO_E_BAD_GRAPH;
  for (uint32_t u = 0; u < n; u++)
    if (row_ptr[u + 1] < row_ptr[u]) return NDO_E_BAD_GRAPH;
  if (row_ptr[n] && !col) return NDO_E_INVALID_ARG;
  graph g = {n, row_ptr, col, 0};
  for (uint32_t u = 0; u < n; u++) {
    for (uint64_t j = row_ptr[u]; j < row_ptr[u + 1]; j++) {
      uint32_t v = col[j];
      if (v >= n || v == u) return NDO_E_BAD_GRAPH;
      if (j > row_ptr[u] && col[j - 1] >= v) return NDO_E_BAD_GRAPH;
      if (!adjacent(&g, v, u)) return NDO_E_BAD_GRAPH;
    }
  }
  return NDO_OK;
}

/* ---- clique listing by depth-first search over forward neighbours ------- */

/* out = the elements of the sorted list a[0..na) that are neighbours of v,
 * ascending. Three equivalent ways, whichever touches the fewest entries: a
 * linear merge of a with the sorted row of v, a binary search of the row for
 * each element of a, or a binary search of a for each entry of the row. */
static uint64_t lower_bound32(const uint32_t *a, uint64_t lo, uint64_t hi, uint32_t x) {
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

static uint64_t log2ceil(uint64_t x) {
  uint64_t lg = 1;
  while ((1ull << lg) < x) lg++;
  return lg;
}

static uint64_t intersect_row(const graph *g, const uint32_t *a, uint64_t na, uint32_t v,
                              uint32_t *out) {
  uint64_t b = g->rp[v], be = g->rp[v + 1], k = 0;
  uint64_t deg = be - b;
  uint64_t c_merge = na + deg;
  uint64_t c_probe_a = na * log2ceil(deg);
  uint64_t c_probe_row = deg * log2ceil(na);
  if (c_probe_a <= c_merge && c_probe_a <= c_probe_row) {
    for (uint64_t i = 0; i < na; i++)
      if (adjacent(g, v, a[i])) out[k++] = a[i];
    return k;
  }
  if (c_probe_row < c_merge) {
    for (uint64_t j = b; j < be; j++) {
      uint32_t y = g->col[j];
      uint64_t p = lower_bound32(a, 0, na, y);
      if (p < na && a[p] == y) out[k++] = y;
    }
    return k;
  }
  uint64_t i = 0;
  while (i < na && b < be) {
    uint32_t x = a[i], y = g->col[b];
    if (x == y) { out[k++] = x; i++; b++; }
    else if (x < y) i++;
    else b++;
  }
  return k;
}

/* Lists every q-clique once as an ascending tuple, in lexicographic order:
 * tuple[0] runs over all vertices; tuple[d+1] runs over the common
 * neighbours of tuple[0..d] that are larger than tuple[d]. */
typedef void (*emit_fn)(const uint32_t *tuple, void *ctx);

typedef struct {
  const graph *g;
  uint32_t q;
  uint32_t tuple[MAXS];
  uint32_t *cand[MAXS];
  uint64_t ncand[MAXS];
  emit_fn emit;
  void *ctx;
} lister;

static void lister_rec(lister *L, uint32_t d) {
  if (d == L->q) { L->emit(L->tuple, L->ctx); return; }
  const graph *g = L->g;
  for (uint64_t i = 0; i < L->ncand[d]; i++) {
    uint32_t v = L->cand[d][i];
    L->tuple[d] = v;
    if (d + 1 < L->q)
      L->ncand[d + 1] = intersect_row(g, L->cand[d] + i + 1, L->ncand[d] - i - 1, v,
                                      L->cand[d + 1]);
    lister_rec(L, d + 1);
  }
}

static int list_cliques(const graph *g, uint32_t q, emit_fn emit, void *ctx) {
  lister L;
  memset(&L, 0, sizeof(L));
  L.g = g; L.q = q; L.emit = emit; L.ctx = ctx;
  uint64_t cap = g->maxdeg ? g->maxdeg : 1;
  for (uint32_t d = 0; d < q; d++) {
    L.cand[d] = (uint32_t *)malloc(cap * sizeof(uint32_t));
    if (!L.cand[d]) { for (uint32_t e = 0; e < d; e++) free(L.cand[e]); return NDO_E_OOM; }
  }
  for (uint32_t v0 = 0; v0 < g->n; v0++) {
    L.tuple[0] = v0;
    if (q == 1) { emit(L.tuple, ctx); continue; }
    uint64_t k = 0;
    for (uint64_t j = g->rp[v0]; j < g->rp[v0 + 1]; j++)
      if (g->col[j] > v0) L.cand[1][k++] = g->col[j];
    L.ncand[1] = k;
    lister_rec(&L, 1);
  }
  for (uint32_t d = 0; d < q; d++) free(L.cand[d]);
  return NDO_OK;
}

/* ---- r-clique table (O1) and lookup ------------------------------------ */

typedef struct {
  uint32_t r;
  uint64_t n_r;
  uint32_t *t;       /* n_r * r, lexicographic */
  uint64_t *first;   /* n+1: tuples starting with vertex a are [first[a], first[a+1]) */
} rtable;

typedef struct { vec32 v; uint32_t r; } rcollect;

static void emit_rcollect(const uint32_t *tuple, void *ctx) {
  rcollect *c = (rcollect *)ctx;
  for (uint32_t i = 0; i < c->r; i++) v32_push(&c->v, tuple[i]);
}

static int tuple_cmp(const uint32_t *a, const uint32_t *b, uint32_t r) {
  for (uint32_t i = 0; i < r; i++) {
    if (a[i] < b[i]) return -1;
    if (a[i] > b[i]) return 1;
  }
  return 0;
}

/* id of an ascending r-tuple, or NONE if it is not an r-clique: binary
 * search among the tuples that start with tuple[0] */
static uint64_t rlookup(const rtable *T, const uint32_t *tuple) {
  if (T->r == 1) return tuple[0];
  uint64_t lo = T->first[tuple[0]], hi = T->first[tuple[0] + 1];
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    int c = tuple_cmp(T->t + mid * T->r, tuple, T->r);
    if (c == 0) return mid;
    if (c < 0) lo = mid + 1; else hi = mid;
  }
  return NONE;
}

/* ---- s-cliques containing a given r-clique ------------------------------ */

/* For r-clique R (ascending tuple), calls fn(S, ctx) for every s-clique S
 * containing R, with S as an ascending s-tuple. C(R) is the set of vertices
 * adjacent to every vertex of R; the s-cliques containing R are R plus an
 * (s-r)-clique inside C(R). */
typedef void (*sfn)(const uint32_t *S, void *ctx);

typedef struct {
  const graph *g;
  uint32_t r, s;
  uint32_t *cand[MAXS + 1];
  uint64_t ncand[MAXS + 1];
  uint32_t ext[MAXS];
  const uint32_t *R;
  sfn fn;
  void *ctx;
} sscan;

static void sscan_emit(sscan *X) {
  uint32_t S[MAXS];
  uint32_t i = 0, j = 0, k = 0, q = X->s - X->r;
  while (i < X->r || j < q) {
    if (j >= q || (i < X->r && X->R[i] < X->ext[j])) S[k++] = X->R[i++];
    else S[k++] = X->ext[j++];
  }
  X->fn(S, X->ctx);
}

static void sscan_rec(sscan *X, uint32_t d) {
  uint32_t q = X->s - X->r;
  if (d == q) { sscan_emit(X); return; }
  const graph *g = X->g;
  for (uint64_t i = 0; i < X->ncand[d]; i++) {
    uint32_t v = X->cand[d][i];
    X->ext[d] = v;
    if (d + 1 < q)
      X->ncand[d + 1] = intersect_row(g, X->cand[d] + i + 1, X->ncand[d] - i - 1, v,
                                      X->cand[d + 1]);
    sscan_rec(X, d + 1);
  }
}

static void for_each_sclique(sscan *X, const uint32_t *R) {
  const graph *g = X->g;
  X->R = R;
  /* C(R): scan the row of the member of R with the fewest neighbours and
   * keep the vertices adjacent to every other member */
  uint32_t base = 0;
  for (uint32_t t = 1; t < X->r; t++)
    if (g->rp[R[t] + 1] - g->rp[R[t]] < g->rp[R[base] + 1] - g->rp[R[base]]) base = t;
  uint64_t k = 0;
  for (uint64_t j = g->rp[R[base]]; j < g->rp[R[base] + 1]; j++) {
    uint32_t w = g->col[j];
    int ok = 1;
    for (uint32_t t = 0; t < X->r && ok; t++)
      if (t != base) ok = adjacent(g, R[t], w);
    if (ok) X->cand[0][k++] = w;
  }
  X->ncand[0] = k;
  sscan_rec(X, 0);
}

static int sscan_init(sscan *X, const graph *g, uint32_t r, uint32_t s, sfn fn, void *ctx) {
  memset(X, 0, sizeof(*X));
  X->g = g; X->r = r; X->s = s; X->fn = fn; X->ctx = ctx;
  uint64_t cap = g->maxdeg ? g->maxdeg : 1;
  for (uint32_t d = 0; d <= s - r; d++) {
    X->cand[d] = (uint32_t *)malloc(cap * sizeof(uint32_t));
    if (!X->cand[d]) return NDO_E_OOM;
  }
  return NDO_OK;
}

static void sscan_free(sscan *X) {
  for (uint32_t d = 0; d <= MAXS; d++) free(X->cand[d]);
}

/* r-subsets of an s-set, as bit masks */
typedef struct { uint32_t nm; uint32_t mask[128]; } subsets;

static void make_subsets(subsets *sb, uint32_t r, uint32_t s) {
  sb->nm = 0;
  for (uint32_t m = 0; m < (1u << s); m++)
    if ((uint32_t)__builtin_popcount(m) == r) sb->mask[sb->nm++] = m;
}

static void subset_tuple(const uint32_t *S, uint32_t s, uint32_t mask, uint32_t *out) {
  uint32_t k = 0;
  for (uint32_t i = 0; i < s; i++)
    if (mask & (1u << i)) out[k++] = S[i];
}

/* ---- O2: counting -------------------------------------------------------- */

typedef struct {
  const rtable *T;
  uint32_t s;
  subsets sb;
  uint64_t *count;
  uint64_t n_s;
} counter;

static void emit_count(const uint32_t *S, void *ctx) {
  counter *c = (counter *)ctx;
  uint32_t sub[MAXS];
  c->n_s++;
  for (uint32_t i = 0; i < c->sb.nm; i++) {
    subset_tuple(S, c->s, c->sb.mask[i], sub);
    uint64_t id = rlookup(c->T, sub);
    c->count[id]++;   /* every subset of a clique is a clique, so id != NONE */
  }
}

/* ---- union-find (sequential) -------------------------------------------- */

static uint64_t uf_find(uint64_t *p, uint64_t x) {
  uint64_t root = x;
  while (p[root] != root) root = p[root];
  while (p[x] != root) { uint64_t nx = p[x]; p[x] = root; x = nx; }
  return root;
}

static void uf_union(uint64_t *p, uint64_t a, uint64_t b) {
  a = uf_find(p, a);
  b = uf_find(p, b);
  if (a == b) return;
  if (a < b) p[b] = a; else p[a] = b;
}

/* ---- O3: sequential peel ------------------------------------------------- */

typedef struct {
  const rtable *T;
  uint32_t s;
  uint64_t self;
  subsets sb;
  uint64_t *deg;     /* current degree */
  uint8_t *gone;     /* 1 once peeled */
  uint64_t *vert, *pos, *bin;
  uint64_t nbin;
  uint64_t floor_deg;  /* degree of the r-clique being peeled */
  /* scratch for the current s-clique */
  uint64_t others[128];
} peeler;

/* Batagelj-Zaversnik bucket move of x from bin d to bin d-1. Degrees are
 * never lowered below the degree of the r-clique being peeled, which leaves
 * every core number unchanged: a core number is the running maximum of the
 * minimum degree, and that maximum is already at least the current one. */
static void bz_decrement(peeler *P, uint64_t x, uint64_t floor_deg) {
  uint64_t dx = P->deg[x];
  if (dx <= floor_deg) return;
  uint64_t px = P->pos[x];
  uint64_t pw = P->bin[dx];
  uint64_t w = P->vert[pw];
  if (w != x) {
    P->pos[x] = pw; P->vert[pw] = x;
    P->pos[w] = px; P->vert[px] = w;
  }
  P->bin[dx]++;
  P->deg[x] = dx - 1;
}

static void emit_peel(const uint32_t *S, void *ctx) {
  peeler *P = (peeler *)ctx;
  uint32_t sub[MAXS];
  uint32_t no = 0;
  for (uint32_t i = 0; i < P->sb.nm; i++) {
    subset_tuple(S, P->s, P->sb.mask[i], sub);
    uint64_t id = rlookup(P->T, sub);
    if (id == P->self) continue;
    if (P->gone[id]) return;           /* S was destroyed earlier */
    P->others[no++] = id;
  }
  for (uint32_t i = 0; i < no; i++) bz_decrement(P, P->others[i], P->floor_deg);
}

/* ---- O4: hierarchy --------------------------------------------------------- */

typedef struct {
  const rtable *T;
  uint32_t s;
  uint64_t self;
  subsets sb;
  const uint8_t *active;
  uint64_t *uf;
  uint64_t *stamp;
  uint64_t level;
  vec64 *pieces;
  int do_union;
} linker;

static void emit_link(const uint32_t *S, void *ctx) {
  linker *K = (linker *)ctx;
  uint32_t sub[MAXS];
  for (uint32_t i = 0; i < K->sb.nm; i++) {
    subset_tuple(S, K->s, K->sb.mask[i], sub);
    uint64_t id = rlookup(K->T, sub);
    if (id == K->self || !K->active[id]) continue;
    if (K->do_union) {
      uf_union(K->uf, K->self, id);
    } else {
      uint64_t p = uf_find(K->uf, id);
      if (K->stamp[p] != K->level) { K->stamp[p] = K->level; v64_push(K->pieces, p); }
    }
  }
}

typedef struct { uint64_t key; uint64_t val; } kv;

static int kv_cmp(const void *a, const void *b) {
  const kv *x = (const kv *)a, *y = (const kv *)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->val != y->val) return x->val < y->val ? -1 : 1;
  return 0;
}

typedef struct { uint64_t level, minleaf, node; } nodekey;

static int nodekey_cmp(const void *a, const void *b) {
  const nodekey *x = (const nodekey *)a, *y = (const nodekey *)b;
  if (x->level != y->level) return x->level < y->level ? -1 : 1;
  if (x->minleaf != y->minleaf) return x->minleaf < y->minleaf ? -1 : 1;
  return 0;
}

/* ---- driver ---------------------------------------------------------------- */

void ndo_free(ndo_result *res) {
  if (!res) return;
  free(res->rcliques);
  free(res->count);
  free(res->coreness);
  free(res->peel_order);
  free(res->parent);
  free(res->level);
  memset(res, 0, sizeof(*res));
}

static int build_graph(graph *g, uint32_t n, const uint64_t *row_ptr, const uint32_t *col) {
  int st = ndo_validate_csr(n, row_ptr, col);
  if (st != NDO_OK) return st;
  g->n = n; g->rp = row_ptr; g->col = col; g->maxdeg = 0;
  for (uint32_t u = 0; u < n; u++) {
    uint64_t d = row_ptr[u + 1] - row_ptr[u];
    if (d > g->maxdeg) g->maxdeg = d;
  }
  return NDO_OK;
}

static int do_count(const graph *g, uint32_t r, uint32_t s, ndo_result *out, rtable *T) {
  rcollect rc;
  memset(&rc, 0, sizeof(rc));
  rc.r = r;
  int st = list_cliques(g, r, emit_rcollect, &rc);
  if (st != NDO_OK || rc.v.oom) { free(rc.v.a); return NDO_E_OOM; }
  T->r = r;
  T->n_r = rc.v.n / r;
  T->t = rc.v.a;
  out->n_r = T->n_r;
  out->rcliques = T->t;
  if (!out->rcliques) out->rcliques = (uint32_t *)malloc(sizeof(uint32_t));
  T->t = out->rcliques;
  T->first = (uint64_t *)calloc((uint64_t)g->n + 1, sizeof(uint64_t));
  out->count = (uint64_t *)calloc(T->n_r ? T->n_r : 1, sizeof(uint64_t));
  if (!out->count || !T->first) return NDO_E_OOM;
  /* first[a] = number of tuples whose first vertex is below a */
  for (uint64_t i = 0; i < T->n_r; i++) T->first[T->t[i * r] + 1]++;
  for (uint32_t a = 0; a < g->n; a++) T->first[a + 1] += T->first[a];
  counter c;
  memset(&c, 0, sizeof(c));
  c.T = T; c.s = s; c.count = out->count;
  make_subsets(&c.sb, r, s);
  st = list_cliques(g, s, emit_count, &c);
  if (st != NDO_OK) return st;
  out->n_s = c.n_s;
  return NDO_OK;
}

/* O4 + O5 for the core numbers in out->coreness, peeled in the order
 * out->peel_order (core numbers non-decreasing along it): the hierarchy of
 * Section 5 / 7.4 by one union-find over descending levels, then canonical
 * numbering. Takes ownership of `gone` (n_r bytes, reused as the active
 * flags). X is a scan of the graph whose fn is emit_link. */
static int build_tree(const rtable *T, uint32_t r, uint32_t s, ndo_result *out, sscan *X,
                      uint8_t *gone) {
  const uint64_t nr = T->n_r;
  const uint64_t nr1 = nr ? nr : 1;
  uint32_t tup[MAXS];
  /* O4: hierarchy, levels from k down to 1 (reverse peel order is sorted by
   * non-increasing core number). */
  uint64_t *uf = (uint64_t *)malloc(nr1 * sizeof(uint64_t));
  uint64_t *stamp = (uint64_t *)malloc(nr1 * sizeof(uint64_t));
  uint64_t *top = (uint64_t *)malloc(nr1 * sizeof(uint64_t));
  uint64_t *par = (uint64_t *)malloc(2 * nr1 * sizeof(uint64_t));
  uint64_t *minleaf = (uint64_t *)malloc(2 * nr1 * sizeof(uint64_t));
  uint64_t *nlevel = (uint64_t *)malloc(nr1 * sizeof(uint64_t));
  uint8_t *active = gone;     /* reused: cleared below */
  vec64 pieces;
  memset(&pieces, 0, sizeof(pieces));
  if (!uf || !stamp || !top || !par || !minleaf || !nlevel) {
    free(uf); free(stamp); free(top); free(par); free(minleaf); free(nlevel); free(active);
    return NDO_E_OOM;
  }
  memset(active, 0, nr1);
  for (uint64_t i = 0; i < nr; i++) { uf[i] = i; stamp[i] = NONE; top[i] = i; }
  for (uint64_t i = 0; i < 2 * nr1; i++) { par[i] = NONE; minleaf[i] = i; }
  uint64_t nint = 0;
  linker K;
  memset(&K, 0, sizeof(K));
  K.T = T; K.s = s; K.active = active; K.uf = uf; K.stamp = stamp; K.pieces = &pieces;
  make_subsets(&K.sb, r, s);
  X->ctx = &K;
  uint64_t hi = nr;   /* process peel_order[lo..hi) in reverse */
  int oom = 0;
  while (hi > 0) {
    uint64_t c = out->coreness[out->peel_order[hi - 1]];
    uint64_t lo = hi;
    while (lo > 0 && out->coreness[out->peel_order[lo - 1]] == c) lo--;
    if (c == 0) break;   /* core-0 r-cliques lie in no s-clique: root leaves */
    for (uint64_t i = lo; i < hi; i++) active[out->peel_order[i]] = 1;
    /* pieces: the level-c r-cliques themselves and the current components
     * (of levels > c) they touch */
    pieces.n = 0;
    K.level = c;
    K.do_union = 0;
    for (uint64_t i = lo; i < hi; i++) {
      uint64_t R = out->peel_order[i];
      if (stamp[R] != c) { stamp[R] = c; v64_push(&pieces, R); }
      K.self = R;
      memcpy(tup, T->t + R * r, r * sizeof(uint32_t));
      for_each_sclique(X, tup);
    }
    K.do_union = 1;
    for (uint64_t i = lo; i < hi; i++) {
      uint64_t R = out->peel_order[i];
      K.self = R;
      memcpy(tup, T->t + R * r, r * sizeof(uint32_t));
      for_each_sclique(X, tup);
    }
    if (pieces.oom) { oom = 1; break; }
    /* group the pieces by their new root; groups of >= 2 pieces are the new
     * components of size >= 2, i.e. the level-c tree nodes */
    kv *grp = (kv *)malloc((pieces.n ? pieces.n : 1) * sizeof(kv));
    if (!grp) { oom = 1; break; }
    for (uint64_t i = 0; i < pieces.n; i++) {
      grp[i].key = uf_find(uf, pieces.a[i]);
      grp[i].val = pieces.a[i];
    }
    qsort(grp, pieces.n, sizeof(kv), kv_cmp);
    for (uint64_t i = 0; i < pieces.n;) {
      uint64_t j = i;
      while (j < pieces.n && grp[j].key == grp[i].key) j++;
      if (j - i >= 2) {
        uint64_t node = nr + nint;
        nlevel[nint] = c;
        nint++;
        uint64_t ml = NONE;
        for (uint64_t t = i; t < j; t++) {
          uint64_t child = top[grp[t].val];
          par[child] = node;
          if (minleaf[child] < ml) ml = minleaf[child];
        }
        minleaf[node] = ml;
        top[grp[i].key] = node;
      }
      i = j;
    }
    free(grp);
    hi = lo;
  }
  free(pieces.a); free(uf); free(stamp); free(top); free(active);
  if (oom) { free(par); free(minleaf); free(nlevel); return NDO_E_OOM; }

  /* O5: canonical numbering by (level, min leaf) */
  nodekey *keys = (nodekey *)malloc((nint ? nint : 1) * sizeof(nodekey));
  uint64_t *canon = (uint64_t *)malloc((nint ? nint : 1) * sizeof(uint64_t));
  out->parent = (uint64_t *)malloc((nr + nint ? nr + nint : 1) * sizeof(uint64_t));
  out->level = (uint64_t *)malloc((nint ? nint : 1) * sizeof(uint64_t));
  if (!keys || !canon || !out->parent || !out->level) {
    free(keys); free(canon); free(par); free(minleaf); free(nlevel);
    return NDO_E_OOM;
  }
  for (uint64_t i = 0; i < nint; i++) {
    keys[i].level = nlevel[i];
    keys[i].minleaf = minleaf[nr + i];
    keys[i].node = i;
  }
  qsort(keys, nint, sizeof(nodekey), nodekey_cmp);
  for (uint64_t i = 0; i < nint; i++) canon[keys[i].node] = nr + i;
  for (uint64_t x = 0; x < nr; x++)
    out->parent[x] = par[x] == NONE ? NONE : canon[par[x] - nr];
  for (uint64_t i = 0; i < nint; i++) {
    uint64_t p = par[nr + i];
    out->parent[canon[i]] = p == NONE ? NONE : canon[p - nr];
    out->level[canon[i] - nr] = nlevel[i];
  }
  out->n_int = nint;
  free(keys); free(canon); free(par); free(minleaf); free(nlevel);
  return NDO_OK;
}

int ndo_count(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
              uint32_t r, uint32_t s, ndo_result *out) {
  if (!out) return NDO_E_INVALID_ARG;
  memset(out, 0, sizeof(*out));
  if (r < 1 || s <= r || s > MAXS) return NDO_E_INVALID_ARG;
  graph g;
  int st = build_graph(&g, n, row_ptr, col);
  if (st != NDO_OK) return st;
  out->n = n; out->r = r; out->s = s;
  rtable T;
  memset(&T, 0, sizeof(T));
  st = do_count(&g, r, s, out, &T);
  free(T.first);
  if (st != NDO_OK) ndo_free(out);
  return st;
}

int ndo_decompose(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                  uint32_t r, uint32_t s, ndo_result *out) {
  if (!out) return NDO_E_INVALID_ARG;
  memset(out, 0, sizeof(*out));
  if (r < 1 || s <= r || s > MAXS) return NDO_E_INVALID_ARG;
  graph g;
  int st = build_graph(&g, n, row_ptr, col);
  if (st != NDO_OK) return st;
  out->n = n; out->r = r; out->s = s;

  /* O1 + O2 */
  double t0 = now_s();
  rtable T;
  memset(&T, 0, sizeof(T));
  st = do_count(&g, r, s, out, &T);
  if (st != NDO_OK) { free(T.first); ndo_free(out); return st; }
  const uint64_t nr = T.n_r;
  const uint64_t nr1 = nr ? nr : 1;
  double t1 = now_s();
  out->t_count = t1 - t0;

  /* O3: sequential peel with Batagelj-Zaversnik bins */
  out->coreness = (uint64_t *)calloc(nr1, sizeof(uint64_t));
  out->peel_order = (uint64_t *)calloc(nr1, sizeof(uint64_t));
  peeler P;
  memset(&P, 0, sizeof(P));
  P.T = &T; P.s = s;
  make_subsets(&P.sb, r, s);
  P.deg = (uint64_t *)malloc(nr1 * sizeof(uint64_t));
  P.gone = (uint8_t *)calloc(nr1, 1);
  P.vert = (uint64_t *)malloc(nr1 * sizeof(uint64_t));
  P.pos = (uint64_t *)malloc(nr1 * sizeof(uint64_t));
  uint64_t maxd = 0;
  for (uint64_t i = 0; i < nr; i++) if (out->count[i] > maxd) maxd = out->count[i];
  P.nbin = maxd + 2;
  P.bin = (uint64_t *)calloc(P.nbin, sizeof(uint64_t));
  sscan X;
  int sst = sscan_init(&X, &g, r, s, emit_peel, &P);
  if (!out->coreness || !out->peel_order || !P.deg || !P.gone || !P.vert || !P.pos ||
      !P.bin || sst != NDO_OK) {
    free(P.deg); free(P.gone); free(P.vert); free(P.pos); free(P.bin); sscan_free(&X);
    free(T.first); ndo_free(out);
    return NDO_E_OOM;
  }
  for (uint64_t i = 0; i < nr; i++) { P.deg[i] = out->count[i]; P.bin[P.deg[i]]++; }
  {
    uint64_t start = 0;
    for (uint64_t d = 0; d < P.nbin; d++) { uint64_t c = P.bin[d]; P.bin[d] = start; start += c; }
    for (uint64_t i = 0; i < nr; i++) { P.pos[i] = P.bin[P.deg[i]]++; P.vert[P.pos[i]] = i; }
    for (uint64_t d = P.nbin - 1; d > 0; d--) P.bin[d] = P.bin[d - 1];
    P.bin[0] = 0;
  }
  uint64_t k = 0;
  uint32_t tup[MAXS];
  for (uint64_t i = 0; i < nr; i++) {
    uint64_t R = P.vert[i];
    uint64_t d = P.deg[R];
    if (d > k) k = d;
    out->coreness[R] = k;
    out->peel_order[i] = R;
    P.gone[R] = 1;
    P.self = R;
    P.floor_deg = d;
    memcpy(tup, T.t + R * r, r * sizeof(uint32_t));
    for_each_sclique(&X, tup);
  }
  out->k = k;
  free(P.deg); free(P.vert); free(P.pos); free(P.bin);
  double t2 = now_s();
  out->t_peel = t2 - t1;

  /* O4 + O5: the hierarchy of these core numbers */
  X.fn = emit_link;
  st = build_tree(&T, r, s, out, &X, P.gone);
  sscan_free(&X);
  if (st != NDO_OK) { free(T.first); ndo_free(out); return st; }
  out->t_tree = now_s() - t2;
  free(T.first);
  return NDO_OK;
}

/* ---- approximate decomposition (Section 6, Algorithm 2) ------------------ */

/* Upper ends of the geometric buckets: thr[i] = floor((C + delta) *
 * (1 + delta)^(i+1)), the product formed by repeated multiplication in
 * double precision; the list ends with the first value of 2^32 or more
 * (stored as 2^32). Returns the number of entries (at most cap). */
static uint32_t approx_thresholds(uint64_t C, double delta, uint64_t *thr, uint32_t cap) {
  double t = (double)C + delta;
  uint32_t nb = 0;
  while (nb < cap) {
    t *= 1.0 + delta;
    if (t >= 4294967296.0) { thr[nb++] = 4294967296ull; break; }
    thr[nb++] = (uint64_t)t;   /* floor of a positive value */
  }
  return nb;
}

/* Rounds a bucket is processed at most: the smallest T with
 * n_r * (C / (C + delta))^T < 1 (Lemma 2: each round leaves at most a
 * C / (C + delta) share of the r-cliques of core <= l outside the bucket). */
static uint64_t approx_round_cap(uint64_t C, double delta, uint64_t nr) {
  if (nr <= 1) return 1;
  return (uint64_t)(log((double)nr) / log(1.0 + delta / (double)C)) + 1;
}

typedef struct {
  const rtable *T;
  uint32_t s;
  uint64_t self;
  uint64_t t;           /* current round */
  subsets sb;
  const uint64_t *round;  /* peel round, NONE while unpeeled */
  uint64_t *deg;
} approx_peeler;

/* s-clique S of a peeled r-clique R in round t: if no member of S was
 * peeled in an earlier round (S still exists) and R is the smallest member
 * of S peeled in round t, S is removed once: every member not peeled yet
 * loses one s-clique */
static void emit_approx(const uint32_t *S, void *ctx) {
  approx_peeler *P = (approx_peeler *)ctx;
  uint32_t sub[MAXS];
  uint64_t ids[128];
  uint32_t no = 0;
  for (uint32_t i = 0; i < P->sb.nm; i++) {
    subset_tuple(S, P->s, P->sb.mask[i], sub);
    uint64_t id = rlookup(P->T, sub);
    if (id == P->self) continue;
    uint64_t rd = P->round[id];
    if (rd != NONE && rd < P->t) return;            /* S was destroyed earlier */
    if (rd == P->t && id < P->self) return;        /* a smaller member removes S */
    ids[no++] = id;
  }
  for (uint32_t i = 0; i < no; i++)
    if (P->round[ids[i]] == NONE) P->deg[ids[i]]--;
}

int ndo_approx_decompose(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t r,
                         uint32_t s, double delta, ndo_result *out) {
  if (!out) return NDO_E_INVALID_ARG;
  memset(out, 0, sizeof(*out));
  if (r < 1 || s <= r || s > MAXS || !(delta > 0.0)) return NDO_E_INVALID_ARG;
  graph g;
  int st = build_graph(&g, n, row_ptr, col);
  if (st != NDO_OK) return st;
  out->n = n; out->r = r; out->s = s;
  double t0 = now_s();
  rtable T;
  memset(&T, 0, sizeof(T));
  st = do_count(&g, r, s, out, &T);
  if (st != NDO_OK) { free(T.first); ndo_free(out); return st; }
  const uint64_t nr = T.n_r, nr1 = nr ? nr : 1;
  double t1 = now_s();
  out->t_count = t1 - t0;

  subsets sb;
  make_subsets(&sb, r, s);
  const uint64_t C = sb.nm;   /* C(s, r) */
  uint64_t thr[4096];
  const uint32_t nb = approx_thresholds(C, delta, thr, 4096);
  const uint64_t cap = approx_round_cap(C, delta, nr);
  out->coreness = (uint64_t *)calloc(nr1, sizeof(uint64_t));
  out->peel_order = (uint64_t *)calloc(nr1, sizeof(uint64_t));
  uint64_t *deg = (uint64_t *)malloc(nr1 * sizeof(uint64_t));
  uint64_t *round = (uint64_t *)malloc(nr1 * sizeof(uint64_t));
  uint64_t *A = (uint64_t *)malloc(nr1 * sizeof(uint64_t));
  uint8_t *gone = (uint8_t *)calloc(nr1, 1);
  approx_peeler P;
  memset(&P, 0, sizeof(P));
  P.T = &T; P.s = s; P.sb = sb; P.round = round; P.deg = deg;
  sscan X;
  int sst = sscan_init(&X, &g, r, s, emit_approx, &P);
  if (!out->coreness || !out->peel_order || !deg || !round || !A || !gone || sst != NDO_OK) {
    free(deg); free(round); free(A); free(gone); sscan_free(&X); free(T.first); ndo_free(out);
    return NDO_E_OOM;
  }
  for (uint64_t i = 0; i < nr; i++) { deg[i] = out->count[i]; round[i] = NONE; }
  /* r-cliques in no s-clique: core 0, peeled first */
  uint64_t done = 0, t = 0;
  for (uint64_t R = 0; R < nr; R++)
    if (deg[R] == 0) { round[R] = 0; out->coreness[R] = 0; out->peel_order[done++] = R; }
  if (done) t = 1;
  /* buckets in order; a bucket is left when it is empty or after `cap`
   * rounds, its remaining r-cliques carried into the next */
  uint32_t b = 0;
  uint64_t rounds_here = 0, kmax = 0;
  int overflow = 0;
  while (done < nr) {
    if (b >= nb || thr[b] >= 4294967296ull) { overflow = 1; break; }
    const uint64_t lvl = thr[b];
    uint64_t na = 0;
    for (uint64_t R = 0; R < nr; R++)
      if (round[R] == NONE && deg[R] <= lvl) A[na++] = R;
    if (na == 0) { b++; rounds_here = 0; continue; }
    for (uint64_t i = 0; i < na; i++) {
      round[A[i]] = t;
      out->coreness[A[i]] = lvl;
      out->peel_order[done++] = A[i];
    }
    kmax = lvl;
    uint32_t tup[MAXS];
    P.t = t;
    for (uint64_t i = 0; i < na; i++) {
      P.self = A[i];
      memcpy(tup, T.t + A[i] * r, r * sizeof(uint32_t));
      for_each_sclique(&X, tup);
    }
    t++;
    if (++rounds_here >= cap) { b++; rounds_here = 0; }
  }
  free(deg); free(round); free(A);
  if (overflow) {
    free(gone); sscan_free(&X); free(T.first); ndo_free(out);
    return NDO_E_INVALID_ARG;
  }
  out->k = kmax;
  double t2 = now_s();
  out->t_peel = t2 - t1;
  X.fn = emit_link;
  st = build_tree(&T, r, s, out, &X, gone);
  sscan_free(&X);
  if (st != NDO_OK) { free(T.first); ndo_free(out); return st; }
  out->t_tree = now_s() - t2;
  free(T.first);
  return NDO_OK;
}

/* ---- the c-(r,s) nuclei from the definition ------------------------------- */

typedef struct {
  const rtable *T;
  uint32_t s;
  uint64_t self;
  subsets sb;
  const uint64_t *coreness;
  uint64_t c;
  uint64_t *uf;
} cutter;

/* R and every other r-clique R' of the s-clique S with core >= c are
 * s-clique-adjacent members of the graph G_c: join them */
static void emit_cut(const uint32_t *S, void *ctx) {
  cutter *K = (cutter *)ctx;
  uint32_t sub[MAXS];
  for (uint32_t i = 0; i < K->sb.nm; i++) {
    subset_tuple(S, K->s, K->sb.mask[i], sub);
    uint64_t id = rlookup(K->T, sub);
    if (id != K->self && K->coreness[id] >= K->c) uf_union(K->uf, K->self, id);
  }
}

static int u64_cmp(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

void ndo_cut_free(ndo_cut *cut) {
  if (!cut) return;
  free(cut->leaf_nucleus);
  free(cut->min_leaf);
  free(cut->level);
  free(cut->n_rcliques);
  free(cut->n_vertices);
  free(cut->n_edges);
  free(cut->vert_off);
  free(cut->verts);
  memset(cut, 0, sizeof(*cut));
}

int ndo_nuclei(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t r, uint32_t s,
               const uint64_t *coreness, uint64_t c, ndo_cut *out) {
  if (!out) return NDO_E_INVALID_ARG;
  memset(out, 0, sizeof(*out));
  if (r < 1 || s <= r || s > MAXS || c < 1 || !coreness) return NDO_E_INVALID_ARG;
  graph g;
  int st = build_graph(&g, n, row_ptr, col);
  if (st != NDO_OK) return st;
  /* O1: the r-cliques and their lexicographic ids */
  rcollect rc;
  memset(&rc, 0, sizeof(rc));
  rc.r = r;
  st = list_cliques(&g, r, emit_rcollect, &rc);
  if (st != NDO_OK || rc.v.oom) { free(rc.v.a); return NDO_E_OOM; }
  rtable T;
  T.r = r;
  T.n_r = rc.v.n / r;
  T.t = rc.v.a;
  T.first = (uint64_t *)calloc((uint64_t)n + 1, sizeof(uint64_t));
  const uint64_t nr = T.n_r, nr1 = nr ? nr : 1;
  uint64_t *uf = (uint64_t *)malloc(nr1 * sizeof(uint64_t));
  out->leaf_nucleus = (uint64_t *)malloc(nr1 * sizeof(uint64_t));
  sscan X;
  int sst = sscan_init(&X, &g, r, s, emit_cut, NULL);
  if (!T.first || !uf || !out->leaf_nucleus || sst != NDO_OK) {
    free(T.t); free(T.first); free(uf); sscan_free(&X); ndo_cut_free(out);
    return NDO_E_OOM;
  }
  for (uint64_t i = 0; i < nr; i++) T.first[T.t[i * r] + 1]++;
  for (uint32_t a = 0; a < n; a++) T.first[a + 1] += T.first[a];
  out->n_r = nr;
  double t0 = now_s();

  /* components of G_c: every s-clique of an r-clique of core >= c joins its
   * members of core >= c */
  cutter K;
  memset(&K, 0, sizeof(K));
  K.T = &T; K.s = s; K.coreness = coreness; K.c = c; K.uf = uf;
  make_subsets(&K.sb, r, s);
  X.ctx = &K;
  for (uint64_t i = 0; i < nr; i++) uf[i] = i;
  uint32_t tup[MAXS];
  for (uint64_t R = 0; R < nr; R++) {
    if (coreness[R] < c) continue;
    K.self = R;
    memcpy(tup, T.t + R * r, r * sizeof(uint32_t));
    for_each_sclique(&X, tup);
  }
  sscan_free(&X);

  /* nuclei numbered by their smallest r-clique: the first member met in
   * ascending id order names the component */
  uint64_t nn = 0;
  uint64_t *comp_of_root = (uint64_t *)malloc(nr1 * sizeof(uint64_t));
  if (!comp_of_root) { free(T.t); free(T.first); free(uf); ndo_cut_free(out); return NDO_E_OOM; }
  for (uint64_t i = 0; i < nr; i++) comp_of_root[i] = NONE;
  for (uint64_t R = 0; R < nr; R++) {
    out->leaf_nucleus[R] = NONE;
    if (coreness[R] < c) continue;
    uint64_t root = uf_find(uf, R);
    if (comp_of_root[root] == NONE) comp_of_root[root] = nn++;
    out->leaf_nucleus[R] = comp_of_root[root];
  }
  free(comp_of_root);
  free(uf);
  out->n_nuclei = nn;
  uint64_t nn1 = nn ? nn : 1;
  out->min_leaf = (uint64_t *)malloc(nn1 * sizeof(uint64_t));
  out->level = (uint64_t *)malloc(nn1 * sizeof(uint64_t));
  out->n_rcliques = (uint64_t *)calloc(nn1, sizeof(uint64_t));
  out->n_vertices = (uint64_t *)calloc(nn1, sizeof(uint64_t));
  out->n_edges = (uint64_t *)calloc(nn1, sizeof(uint64_t));
  out->vert_off = (uint64_t *)calloc(nn1 + 1, sizeof(uint64_t));
  /* (nucleus, vertex) pairs of every member r-clique, sorted, duplicates
   * dropped: the vertex sets */
  uint64_t np = 0;
  for (uint64_t R = 0; R < nr; R++) np += out->leaf_nucleus[R] != NONE ? r : 0;
  uint64_t *pairs = (uint64_t *)malloc((np ? np : 1) * sizeof(uint64_t));
  if (!out->min_leaf || !out->level || !out->n_rcliques || !out->n_vertices || !out->n_edges ||
      !out->vert_off || !pairs) {
    free(pairs); free(T.t); free(T.first); ndo_cut_free(out);
    return NDO_E_OOM;
  }
  for (uint64_t i = 0; i < nn; i++) { out->min_leaf[i] = NONE; out->level[i] = NONE; }
  np = 0;
  for (uint64_t R = 0; R < nr; R++) {
    uint64_t q = out->leaf_nucleus[R];
    if (q == NONE) continue;
    if (R < out->min_leaf[q]) out->min_leaf[q] = R;
    if (coreness[R] < out->level[q]) out->level[q] = coreness[R];
    out->n_rcliques[q]++;
    for (uint32_t j = 0; j < r; j++) pairs[np++] = (q << 32) | T.t[R * r + j];
  }
  qsort(pairs, np, sizeof(uint64_t), u64_cmp);
  uint64_t nv = 0;
  for (uint64_t i = 0; i < np; i++)
    if (i == 0 || pairs[i] != pairs[i - 1]) pairs[nv++] = pairs[i];
  out->verts = (uint32_t *)malloc((nv ? nv : 1) * sizeof(uint32_t));
  if (!out->verts) { free(pairs); free(T.t); free(T.first); ndo_cut_free(out); return NDO_E_OOM; }
  for (uint64_t i = 0; i < nv; i++) {
    out->verts[i] = (uint32_t)(pairs[i] & 0xFFFFFFFFu);
    out->n_vertices[pairs[i] >> 32]++;
  }
  free(pairs);
  for (uint64_t q = 0; q < nn; q++) out->vert_off[q + 1] = out->vert_off[q] + out->n_vertices[q];
  /* edges of G with both ends in the nucleus's vertex set, each counted
   * once from its smaller end */
  for (uint64_t q = 0; q < nn; q++) {
    const uint32_t *V = out->verts + out->vert_off[q];
    const uint64_t nvq = out->n_vertices[q];
    for (uint64_t i = 0; i < nvq; i++) {
      uint32_t v = V[i];
      for (uint64_t j = row_ptr[v]; j < row_ptr[v + 1]; j++) {
        uint32_t w = col[j];
        if (w <= v) continue;
        uint64_t p = lower_bound32(V, 0, nvq, w);
        if (p < nvq && V[p] == w) out->n_edges[q]++;
      }
    }
  }
  out->t_cut = now_s() - t0;
  free(T.t);
  free(T.first);
  return NDO_OK;
}

/* ---- per-r-clique queries -------------------------------------------------- */

struct ndo_graph {
  graph g;
  rtable T;
  uint32_t r, s;
  subsets sb;
  sscan X;
  uint64_t self, nS, cap, nout;
  uint64_t *out;
};

static void emit_incident(const uint32_t *S, void *ctx) {
  struct ndo_graph *G = (struct ndo_graph *)ctx;
  uint32_t sub[MAXS];
  G->nS++;
  for (uint32_t i = 0; i < G->sb.nm; i++) {
    subset_tuple(S, G->s, G->sb.mask[i], sub);
    uint64_t id = rlookup(&G->T, sub);
    if (id == G->self) continue;
    if (G->nout < G->cap) G->out[G->nout] = id;
    G->nout++;
  }
}

int ndo_open(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t r, uint32_t s,
             ndo_graph **out) {
  if (!out) return NDO_E_INVALID_ARG;
  *out = NULL;
  if (r < 1 || s <= r || s > MAXS) return NDO_E_INVALID_ARG;
  struct ndo_graph *G = (struct ndo_graph *)calloc(1, sizeof(*G));
  if (!G) return NDO_E_OOM;
  int st = build_graph(&G->g, n, row_ptr, col);
  if (st != NDO_OK) { free(G); return st; }
  G->r = r;
  G->s = s;
  rcollect rc;
  memset(&rc, 0, sizeof(rc));
  rc.r = r;
  st = list_cliques(&G->g, r, emit_rcollect, &rc);
  if (st != NDO_OK || rc.v.oom) { free(rc.v.a); free(G); return NDO_E_OOM; }
  G->T.r = r;
  G->T.n_r = rc.v.n / r;
  G->T.t = rc.v.a ? rc.v.a : (uint32_t *)malloc(sizeof(uint32_t));
  G->T.first = (uint64_t *)calloc((uint64_t)n + 1, sizeof(uint64_t));
  if (!G->T.t || !G->T.first) { ndo_close(G); return NDO_E_OOM; }
  for (uint64_t i = 0; i < G->T.n_r; i++) G->T.first[G->T.t[i * r] + 1]++;
  for (uint32_t a = 0; a < n; a++) G->T.first[a + 1] += G->T.first[a];
  make_subsets(&G->sb, r, s);
  if (sscan_init(&G->X, &G->g, r, s, emit_incident, G) != NDO_OK) { ndo_close(G); return NDO_E_OOM; }
  *out = G;
  return NDO_OK;
}

uint64_t ndo_graph_n_r(const ndo_graph *G) { return G ? G->T.n_r : 0; }

void ndo_graph_rcliques(const ndo_graph *G, uint32_t *out) {
  if (G && out && G->T.n_r) memcpy(out, G->T.t, G->T.n_r * G->r * sizeof(uint32_t));
}

uint64_t ndo_incident(ndo_graph *G, uint64_t id, uint64_t *out, uint64_t cap) {
  if (!G || id >= G->T.n_r) return 0;
  uint32_t tup[MAXS];
  memcpy(tup, G->T.t + id * G->r, G->r * sizeof(uint32_t));
  G->self = id;
  G->nS = 0;
  G->nout = 0;
  G->out = out;
  G->cap = out ? cap : 0;
  for_each_sclique(&G->X, tup);
  return G->nS;
}

void ndo_close(ndo_graph *G) {
  if (!G) return;
  sscan_free(&G->X);
  free(G->T.t);
  free(G->T.first);
  free(G);
}
