/*
 * ndo.h -- plain sequential CPU oracle for exact (r,s) nucleus decomposition
 * and its hierarchy.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library may include,
 * link or call this code; only the tests, the smoke check and the CPU
 * baseline of the benchmark use it. It shares no source with the GPU path.
 *
 * What it computes (Shi, Dhulipala, Shun, "Parallel Algorithms for
 * Hierarchical Nucleus Decomposition", arXiv 2306.08623):
 *
 *  - r-cliques in lexicographic order of their ascending vertex tuples; the
 *    position in that order is the canonical r-clique id.
 *  - the s-clique degree of every r-clique (Section 3, the number of
 *    s-cliques containing it) and the number of s-cliques n_s.
 *  - the (r,s)-clique core number of every r-clique (Section 3 definition),
 *    computed by the sequential minimum-degree peeling that Section 6 (proof
 *    of Lemma 1) describes: repeatedly remove an unpeeled r-clique of minimum
 *    current s-clique degree; its core number is the largest minimum seen so
 *    far; removing it destroys every s-clique it belongs to, which lowers the
 *    degree of the other still-present r-cliques of those s-cliques.
 *  - the nucleus hierarchy (Section 5, Algorithm 1 semantics; Section 7.4
 *    practical form): for c = k down to 1, union-find over r-cliques with
 *    core number >= c, joining two r-cliques when one s-clique contains both
 *    (s-clique-adjacent, Section 3); every component of that graph that
 *    contains a core-c r-clique and has at least two r-cliques is a tree node
 *    of level c. Parents with a single child are not created (Section 7.3,
 *    the remark on unary parents).
 *  - the canonical tree: leaves 0..n_r-1 are the canonical r-clique ids;
 *    internal nodes are numbered n_r + rank of (level, smallest leaf id in
 *    the node) ascending; parent = UINT64_MAX for roots.
 *
 * Everything is integer arithmetic; counts and core numbers are uint64.
 * Supported: 1 <= r < s <= 7.
 */
#ifndef NDO_H
#define NDO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  NDO_OK = 0,
  NDO_E_INVALID_ARG = 1,
  NDO_E_BAD_GRAPH = 2,
  NDO_E_OOM = 3,
};

typedef struct ndo_result {
  uint32_t n, r, s;
  uint64_t n_r;          /* number of r-cliques */
  uint64_t n_s;          /* number of s-cliques */
  uint32_t *rcliques;    /* n_r * r vertex ids, tuples ascending, lexicographic */
  uint64_t *count;       /* n_r: s-clique degree before any peeling */
  uint64_t *coreness;    /* n_r: (r,s)-clique core number */
  uint64_t *peel_order;  /* n_r: r-clique ids in the order the peel removed them */
  uint64_t k;            /* max core number (0 if n_r == 0) */
  uint64_t n_int;        /* internal nodes of the canonical tree */
  uint64_t *parent;      /* n_r + n_int: parent node, UINT64_MAX for roots */
  uint64_t *level;       /* n_int: level of internal node n_r + i */
  double t_count;        /* seconds: r-clique listing + s-clique counting */
  double t_peel;         /* seconds: sequential peel */
  double t_tree;         /* seconds: hierarchy + canonical numbering */
} ndo_result;

/* Returns NDO_OK if (row_ptr, col) is a symmetric CSR over 0..n-1 with each
 * row strictly increasing (so no duplicates) and no self-loops. */
int ndo_validate_csr(uint32_t n, const uint64_t *row_ptr, const uint32_t *col);

/* Full decomposition. On success *out owns heap arrays; release with
 * ndo_free. On error *out is zeroed. */
int ndo_decompose(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                  uint32_t r, uint32_t s, ndo_result *out);

/* Only the r-clique listing and the s-clique counts (rcliques, count, n_r,
 * n_s); coreness / tree fields stay NULL. */
int ndo_count(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
              uint32_t r, uint32_t s, ndo_result *out);

void ndo_free(ndo_result *res);

/* Approximate decomposition and its hierarchy (Section 6, Algorithm 2;
 * hierarchy as for exact core numbers). Buckets of s-clique degree with
 * upper ends thr[i] = floor((C(s,r) + delta) * (1 + delta)^(i+1)) (double
 * precision, the power by repeated multiplication); rounds are synchronous:
 * a round at bucket i peels every unpeeled r-clique of current degree
 * <= thr[i], assigns it thr[i], and removes each s-clique that still exists
 * once (from its smallest member peeled in that round). A bucket is left
 * when it is empty or after T = floor(ln n_r / ln(1 + delta / C(s,r))) + 1
 * rounds. r-cliques in no s-clique get 0. The approximation satisfies
 * core <= approx <= (C(s,r) + delta)(1 + delta) core (Theorem 6.1).
 * peel_order lists r-cliques in round order; k is the largest value
 * assigned. NDO_E_INVALID_ARG also when a bucket end would pass 2^32 - 1. */
int ndo_approx_decompose(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t r,
                         uint32_t s, double delta, ndo_result *out);

/* The c-(r,s) nuclei from the definition (Section 8, on the usefulness of
 * the hierarchy: without a hierarchy, the nuclei of level c are the
 * connected components of the r-cliques of core number >= c under s-clique
 * adjacency, Section 3). No tree is used: the components are found by a
 * union-find over every s-clique of those r-cliques. `coreness` is indexed
 * by the canonical r-clique id (as ndo_decompose returns it); c >= 1.
 * Nuclei are numbered by their smallest r-clique id. */
typedef struct ndo_cut {
  uint64_t n_r;
  uint64_t n_nuclei;
  uint64_t *leaf_nucleus;  /* n_r: nucleus of each r-clique, UINT64_MAX if core < c */
  uint64_t *min_leaf;      /* n_nuclei: smallest r-clique id in the nucleus */
  uint64_t *level;         /* n_nuclei: smallest core number in it */
  uint64_t *n_rcliques;    /* n_nuclei: its r-cliques */
  uint64_t *n_vertices;    /* n_nuclei: vertices of its r-cliques */
  uint64_t *n_edges;       /* n_nuclei: edges of G with both ends among them */
  uint64_t *vert_off;      /* n_nuclei + 1: its vertices are verts[vert_off[i] ..) */
  uint32_t *verts;         /* ascending within each nucleus */
  double t_cut;            /* seconds: components, vertex sets and edges */
} ndo_cut;

int ndo_nuclei(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t r, uint32_t s,
               const uint64_t *coreness, uint64_t c, ndo_cut *out);
void ndo_cut_free(ndo_cut *cut);

/* Per-r-clique queries on a graph too large for a full decomposition.
 * ndo_open lists the r-cliques (O1) once; ndo_incident then enumerates the
 * s-cliques containing one r-clique. */
typedef struct ndo_graph ndo_graph;

int ndo_open(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, uint32_t r, uint32_t s,
             ndo_graph **out);
uint64_t ndo_graph_n_r(const ndo_graph *G);
/* copies the n_r * r lexicographic r-clique tuples */
void ndo_graph_rcliques(const ndo_graph *G, uint32_t *out);
/* For r-clique `id`: the number of s-cliques containing it. If cap is large
 * enough, out receives, for each such s-clique in listing order, the ids of
 * its other C(s,r)-1 r-cliques (cap counts uint64 slots). */
uint64_t ndo_incident(ndo_graph *G, uint64_t id, uint64_t *out, uint64_t cap);
void ndo_close(ndo_graph *G);

#ifdef __cplusplus
}
#endif

#endif /* NDO_H */
