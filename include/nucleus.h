/*
 * nucleus.h -- C ABI of the MI355X (gfx950) exact (r,s) nucleus decomposition
 * library: coreness of every r-clique plus the nucleus hierarchy tree.
 *
 * Method: Shi, Dhulipala, Shun, "Parallel Algorithms for Hierarchical Nucleus
 * Decomposition" (arXiv 2306.08623). The library runs the interleaved
 * framework of Section 7.1 (Algorithm 3) with the efficient link and tree
 * construction of Section 7.3 (Algorithm 5) on one GPU:
 *   orient the graph (Section 3, low out-degree orientation), count the
 *   s-cliques of every r-clique, peel r-cliques in rounds of minimum count
 *   while linking s-clique-adjacent r-cliques into a union-find plus the
 *   "nearest lower core" table L, then build the tree from uf and L.
 *
 * Definitions (Section 3):
 *   - an r-clique's s-clique degree is the number of s-cliques containing it;
 *   - its core number is the largest c such that it lies in a c-(r,s)
 *     nucleus;
 *   - two r-cliques are s-clique-adjacent when one s-clique contains both;
 *   - the hierarchy nests, for every c, the connected components of the
 *     graph on r-cliques of core >= c under s-clique adjacency.
 *
 * Output conventions (identical to the reference CPU oracle used by the
 * tests):
 *   - r-cliques are ascending vertex tuples; their canonical index is their
 *     position in lexicographic order;
 *   - the tree is canonical: leaves 0..n_r-1 are the r-cliques; internal
 *     nodes n_r..n_r+n_int-1 are the components of size >= 2, each labelled
 *     with its level (the smallest core number inside it), numbered by
 *     ascending (level, smallest leaf index); a node's parent is the
 *     smallest node strictly containing it; roots have parent UINT64_MAX.
 *     Parents with a single child do not appear (Section 7.3 remark).
 *
 * Threading: one context per host thread; all device work of a context is
 * ordered on the context's HIP stream. No exception crosses this ABI.
 * Errors: every call returns an nd_status; after an error the context stays
 * usable but the results of the failed decomposition are invalid.
 */
#ifndef NUCLEUS_H
#define NUCLEUS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum nd_status {
  ND_OK = 0,
  ND_E_INVALID_ARG = 1,   /* NULL pointer, r/s out of range, bad sizes       */
  ND_E_BAD_GRAPH = 2,     /* CSR not symmetric / sorted / simple             */
  ND_E_UNSUPPORTED = 3,   /* (r,s) pair or size the library does not handle  */
  ND_E_OOM = 4,           /* device allocation failed or memory limit hit    */
  ND_E_OVERFLOW = 5,      /* a 32-bit count or id would overflow             */
  ND_E_DEVICE = 6,        /* a HIP runtime call failed                       */
  ND_E_WATCHDOG = 7,      /* a device loop exceeded its iteration bound      */
  ND_E_STATE = 8,         /* call out of order (e.g. no graph loaded)        */
  ND_E_CANCELLED = 9      /* the host cancelled the request                  */
} nd_status;

typedef enum nd_mem {
  ND_MEM_HOST = 0,        /* pointer is ordinary host memory                 */
  ND_MEM_DEVICE = 1       /* pointer is device memory of the context's GPU   */
} nd_mem;

typedef struct nd_ctx nd_ctx;

/* Device memory callbacks. alloc returns `bytes` of device memory of the
 * context's GPU (at least 256-byte aligned) usable by work queued on
 * `hip_stream`, or NULL when it cannot (the call then fails with ND_E_OOM);
 * free gives back a block that alloc returned, with the same size and
 * stream. `user` is nd_options.alloc_user. The library never frees a block
 * that queued work may still read: it waits for its stream first. */
typedef void *(*nd_alloc_fn)(size_t bytes, void *hip_stream, void *user);
typedef void (*nd_free_fn)(void *ptr, size_t bytes, void *hip_stream, void *user);

typedef struct nd_options {
  int device;             /* HIP device ordinal                               */
  void *hip_stream;       /* hipStream_t to order work on; NULL = null stream */
  int validate;           /* nonzero: check the CSR on the device             */
  uint64_t mem_limit;     /* max bytes of device workspace; 0 = no limit      */
  uint32_t peel_blocks;   /* workgroups of the persistent peel launch; 0=auto */
  uint32_t work_chunk;    /* reserved, ignored: the peel hands out one probe
                             element per lane and pass                        */
  uint64_t watchdog;      /* max peel rounds before ND_E_WATCHDOG; 0 = auto   */
  uint32_t flags;         /* ND_FLAG_* bits                                   */
  /* Where the context's device workspace comes from: both NULL = hipMalloc /
   * hipFree; both set = these callbacks (e.g. a framework's caching
   * allocator, so that it accounts for and reuses the memory); one of the
   * two alone is ND_E_INVALID_ARG. */
  nd_alloc_fn alloc;
  nd_free_fn free;
  void *alloc_user;
} nd_options;

/* nd_options.flags: print a line to stderr when a pipeline phase ends, and
 * every 10 s of a running peel launch its round and level (read from pinned
 * host memory the kernel updates), for runs that take minutes. */
#define ND_FLAG_PROGRESS 1u
/* How the hierarchy is built (the result is the same canonical tree):
 *  EL: during the peel, by Algorithm 5's link-efficient (Section 7.3);
 *  TE: after a peel without linking, level by level from the largest core
 *      number down (the paper's two-pass alternative, Section 7.4), with a
 *      union-find of partial trees that keeps each step independent of the
 *      depth of the hierarchy.
 * Neither flag: TE when s - r >= 2 ((1,3), (1,4), (2,4)), whose core
 * numbers span thousands of levels (Algorithm 5's link chains grow with
 * them), EL for (1,2), (2,3), (3,4). */
#define ND_FLAG_HIER_EL 2u
#define ND_FLAG_HIER_TE 4u
/* s = 4 counting keeps a row's common out-neighbourhood (at most its
 * out-degree) in on-chip memory when that is at most 1024, else in a slice
 * of global memory per wave (about 1 GiB in all). This flag sends every
 * row to the global slices (the same counts; for testing that path). */
#define ND_FLAG_COUNT_GLOBAL 8u

/* Per-decomposition statistics. Counters are totals over the whole run. */
typedef struct nd_info {
  uint32_t n, r, s;
  uint64_t m;             /* undirected edges                                 */
  uint64_t n_r;           /* r-cliques                                        */
  uint64_t n_s;           /* s-cliques                                        */
  uint32_t k;             /* maximum core number                              */
  uint32_t rounds;        /* peeling rounds executed                          */
  uint64_t n_int;         /* internal nodes of the canonical tree             */
  uint64_t visits;        /* (r-clique, s-clique) pairs traversed while peeling */
  uint64_t decrements;    /* count decrements                                 */
  uint64_t links;         /* EL: link steps (Algorithm 5 calls, cascades
                             included); TE: pairs handled by the hierarchy    */
  uint64_t link_calls;    /* top-level link calls issued (after skipping pairs
                             of roots already linked)                         */
  uint64_t unites;        /* successful union-find unions                     */
  uint64_t bucket_scans;  /* scans of the remaining r-cliques for a new k     */
  uint32_t max_outdeg;    /* out-degree bound reached by the orientation      */
  uint32_t orient_rounds; /* rounds of the orientation                        */
  float ms_prep;          /* device time: validation, ids, orientation, tables */
  float ms_count;         /* device time: s-clique counting                   */
  float ms_peel;          /* device time: peel + link rounds                  */
  float ms_tree;          /* device time: tree construction + canonical form  */
  float ms_count_kernel;  /* device time of the s-clique counting kernel      */
  float ms_peel_kernel;   /* device time of the persistent peel+link kernel   */
  uint64_t device_bytes;  /* workspace bytes held by the context              */
  uint32_t hier_te;       /* 1 if the hierarchy was built by the TE pass      */
  float ms_hier;          /* TE: device time of level sort + hierarchy kernel */
  uint64_t hier_visits;   /* TE: s-cliques met by the hierarchy kernel        */
  uint32_t grid_retries;  /* persistent launches repeated with a smaller grid
                             because the first was not fully resident         */
  uint64_t cascades;      /* EL: link steps run as recursive calls of
                             Algorithm 5 (links - link_calls)                 */
  uint64_t cas_retries;   /* failed compare-and-swaps that were retried: the
                             union of two roots, and the L updates of
                             Algorithm 5 (EL) / of the hierarchy pass (TE)    */
  uint64_t device_peak;   /* largest workspace held during this run (bytes)   */
  double approx_delta;    /* delta of an approximate run (0: exact)           */
  uint32_t round_cap;     /* approximate run: rounds a bucket is processed at
                             most (Algorithm 2)                               */
} nd_info;

/* Create a context on opt->device (opt may be NULL: device 0, null stream,
 * validation on). The context owns every device buffer it allocates (through
 * opt->alloc when set) and releases all of them in nd_destroy. */
nd_status nd_create(nd_ctx **out, const nd_options *opt);
void nd_destroy(nd_ctx *ctx);

/* Copy a CSR graph into the context. row_ptr: uint64[n+1] with row_ptr[0]=0
 * and row_ptr[n]=nnz; col: uint32[nnz], rows sorted ascending, symmetric, no
 * self-loops or duplicates (a simple undirected graph, Section 3); nnz = 2m.
 * `where` tells whether both pointers are host or device memory. The caller
 * keeps ownership. Structural errors are reported here when validation is on
 * (this call then waits for the device). */
nd_status nd_load_csr(nd_ctx *ctx, uint32_t n, uint64_t nnz, const uint64_t *row_ptr,
                      const uint32_t *col, nd_mem where);

/* Choose (r,s): every 1 <= r < s <= 7 (Section 3 defines the decomposition
 * for any pair; the paper's evaluation runs r < s <= 7), e.g. (1,2)
 * (k-core), (2,3) (k-truss), (3,4). Pairs with s <= 4 find the s-cliques
 * containing an r-clique again from edge -> triangle lists whenever they are
 * needed; pairs with s = 5..7 list every s-clique once and keep the
 * r-clique / s-clique incidence in device memory (8 C(s,r) bytes per
 * s-clique, plus the clique levels up to s while they are listed), so their
 * size is bounded by the device's memory (ND_E_OOM) and by 32-bit r- and
 * s-clique ids (ND_E_OVERFLOW). s > 7 returns ND_E_UNSUPPORTED; r < 1 or
 * r >= s returns ND_E_INVALID_ARG. */
nd_status nd_set_rs(nd_ctx *ctx, uint32_t r, uint32_t s);

/* Approximate decomposition (Section 6, Algorithm 2): with delta > 0 the
 * next nd_decompose calls peel by geometric buckets instead of exact levels;
 * delta = 0 restores exact peeling (the default). Bucket i holds current
 * s-clique degrees up to thr[i] = floor((C(s,r) + delta) (1 + delta)^(i+1))
 * (double precision, the power by repeated multiplication). A round at
 * bucket i peels every remaining r-clique of degree <= thr[i] and gives it
 * thr[i] as its (approximate) core number; the s-cliques it removes lower
 * the degrees of the others as in exact peeling. A bucket is left when it
 * is empty or after T = floor(ln n_r / ln(1 + delta / C(s,r))) + 1 rounds,
 * its remaining r-cliques carried into the next. r-cliques in no s-clique
 * get 0. Theorem 6.1: core <= approx <= (C(s,r) + delta)(1 + delta) core.
 * The hierarchy and every getter work on these values exactly as on exact
 * core numbers. Batches (nd_batch_decompose) always peel exactly: the
 * rounds of a union are not those of its graphs; a context in approximate
 * mode refuses them (ND_E_UNSUPPORTED). delta must be finite and in
 * [0, 64], else ND_E_INVALID_ARG. Bucket ends that would pass 2^32 - 1
 * stop the run with ND_E_UNSUPPORTED. */
nd_status nd_set_approx(nd_ctx *ctx, double delta);

/* Schedules: the persistent peel's grid size (workgroups) by kind, (r,s)
 * and size. The grid changes no result (only which lanes do which work): a
 * small grid makes each of the peel's grid barriers cheaper (a run has
 * thousands of rounds, two or three barriers each), a large one gives big
 * rounds more lanes. An entry applies to decompositions of its kind (a
 * single graph, or the disjoint union of one (r,s) group of a batch) of
 * pair (r,s) with at most n_r_max r-cliques; the first matching entry in
 * table order wins. The entries are written by an autotuner that times
 * candidate grids on the device (paper_2306_08623_amd/autotune.py, table
 * paper_2306_08623_amd/schedules.json). */
#define ND_SCHED_SINGLE 0u
#define ND_SCHED_BATCH 1u
typedef struct nd_schedule {
  uint32_t r, s;
  uint64_t n_r_max;       /* largest n_r the entry applies to                 */
  uint32_t peel_blocks;   /* workgroups of the persistent peel; 0 = resident
                             capacity of the device                           */
  uint32_t kind;          /* ND_SCHED_SINGLE or ND_SCHED_BATCH                */
} nd_schedule;

/* Replace the context's schedule table (copied; n = 0 clears it). An
 * nd_options.peel_blocks other than 0 overrides every entry. Entries with
 * r < 1, s <= r, s > 7 or an unknown kind are ND_E_INVALID_ARG. */
nd_status nd_set_schedule(nd_ctx *ctx, const nd_schedule *table, uint32_t n);

/* Run the whole pipeline on the context's stream: orientation, r-clique
 * tables, s-clique counting, peel rounds with linking, tree construction and
 * canonical numbering. Two kernels of the pipeline (orientation, peel) are
 * persistent grids that synchronise all their workgroups: while they run,
 * no other kernel should occupy the GPU (they stop with ND_E_WATCHDOG after
 * 20 s without progress instead of hanging). Blocks on small readbacks of
 * the r-clique count (needed to size the per-r-clique arrays) and, for s = 4,
 * of the largest out-degree of the orientation (it sizes the counting
 * kernel's buffers: on chip up to 1024, global memory beyond), and at the
 * end; results stay on the device until read with nd_get_*. A 32-bit count
 * that would wrap ((1,3), (1,4), (2,4) on very dense graphs) stops the run
 * with ND_E_UNSUPPORTED. */
nd_status nd_decompose(nd_ctx *ctx);

/* Wait for the context's stream and report device-side errors. */
nd_status nd_sync(nd_ctx *ctx);

nd_status nd_get_info(nd_ctx *ctx, nd_info *out);

/* r-cliques: n_r * r uint32 vertex ids, each tuple ascending, tuples in
 * lexicographic order (this order defines the r-clique index). */
nd_status nd_get_rcliques(nd_ctx *ctx, uint32_t *out, nd_mem where);

/* s-clique degree of every r-clique before peeling: uint32[n_r]. */
nd_status nd_get_counts(nd_ctx *ctx, uint32_t *out, nd_mem where);

/* Core numbers: uint32[n_r], indexed by r-clique index. */
nd_status nd_get_coreness(nd_ctx *ctx, uint32_t *out, nd_mem where);

/* Peel round of every r-clique: uint32[n_r]. Rounds are numbered from 0;
 * all r-cliques peeled in one round share a core number, and core numbers
 * never decrease from one round to the next (Algorithm 3's loop). With the
 * counts this certifies the core numbers: for every r-clique R, at least
 * ND[R] s-cliques containing R have all members of core >= ND[R], and at
 * most ND[R] have all members peeled in R's round or later. */
nd_status nd_get_peel_rounds(nd_ctx *ctx, uint32_t *out, nd_mem where);

/* Canonical tree: parent uint64[n_r + n_int] (UINT64_MAX for roots) and
 * level uint32[n_int] (level of node n_r + i). Either pointer may be NULL. */
nd_status nd_get_tree(nd_ctx *ctx, uint64_t *parent, uint32_t *level, nd_mem where);

/* ---- Hierarchy cut: the c-(r,s) nuclei ---------------------------------
 *
 * With the hierarchy, the nuclei of any level c come from the tree alone
 * (Section 8, on the usefulness of the hierarchy): drop every node of level
 * below c; each remaining maximal subtree is one c-(r,s) nucleus and holds
 * all of its leaves. Without it one would rerun connected components over
 * the r-cliques of core >= c. For every nucleus the library also gives the
 * vertices of its r-cliques and the number of graph edges among them (its
 * edge density is n_edges / C(n_vertices, 2)). */

typedef struct nd_nucleus {
  uint64_t node;          /* its canonical tree node (n_r .. n_r + n_int - 1) */
  uint64_t min_leaf;      /* its smallest r-clique index                      */
  uint64_t n_rcliques;    /* r-cliques in it (the leaves of its subtree)      */
  uint64_t n_vertices;    /* distinct vertices of those r-cliques             */
  uint64_t n_edges;       /* edges of the graph with both ends among them     */
  uint64_t vert_off;      /* its vertices: verts[vert_off .. + n_vertices)    */
  uint32_t level;         /* the node's level (>= c): smallest core inside    */
  uint32_t reserved;
} nd_nucleus;

/* Cut the tree of the last nd_decompose at level c >= 1 (ND_E_INVALID_ARG
 * for c = 0; ND_E_STATE without a decomposition, e.g. after a batch).
 * Computes on the device and waits; *n_nuclei and *n_vertices (either may
 * be NULL) receive the number of nuclei and the total length of their
 * vertex lists. c above the maximum core number gives no nucleus. The
 * result stays on the device until the next decomposition or cut. */
nd_status nd_cut(nd_ctx *ctx, uint32_t c, uint64_t *n_nuclei, uint64_t *n_vertices);

/* Copy the last cut out (any pointer may be NULL): nuclei[n_nuclei] in
 * ascending node order; verts[n_vertices], each nucleus's vertex ids
 * ascending at its vert_off; leaf_nucleus[n_r], the index of the nucleus
 * holding each r-clique, UINT32_MAX for r-cliques of core below c. */
nd_status nd_get_cut(nd_ctx *ctx, nd_nucleus *nuclei, uint32_t *verts, uint32_t *leaf_nucleus,
                     nd_mem where);

/* ---- Batches of independent graphs ------------------------------------
 *
 * One call decomposes many graphs. Graphs sharing (r,s) run together as one
 * disjoint union: the decomposition of a union is the union of the
 * decompositions (no s-clique spans two graphs, so counts, core numbers and
 * hierarchy components are each those of one graph; Section 3 definitions),
 * so each (r,s) group costs one pipeline with one persistent peel launch.
 * Every graph's results are exactly those of decomposing it alone. */

typedef struct nd_graph_desc {
  uint32_t n;                /* vertices                                         */
  uint32_t r, s;             /* (r,s) of this graph                              */
  uint64_t nnz;              /* entries of col (2m)                              */
  const uint64_t *row_ptr;   /* uint64[n+1], same rules as nd_load_csr           */
  const uint32_t *col;       /* uint32[nnz]                                      */
} nd_graph_desc;

typedef struct nd_graph_result {
  nd_status status;          /* ND_OK, or the error of this graph's group        */
  uint32_t k;                /* max core number (0 if no r-clique)               */
  uint64_t n_r;              /* r-cliques                                        */
  uint64_t n_s;              /* s-cliques                                        */
  uint64_t n_int;            /* internal nodes of the canonical tree             */
} nd_graph_result;

/* Decompose graphs[0..G) (all host or all device pointers, per `where`; the
 * caller keeps ownership and may free them when the call returns). Fills
 * results[0..G). Validation (when on) checks every graph: a graph whose
 * row_ptr does not run from 0 to nnz, or whose columns leave 0..n-1, fails
 * its group with ND_E_BAD_GRAPH. Supported (r,s) as for nd_set_rs. The sum of
 * n over one (r,s) group must stay below 2^32-1, and so must its edges.
 * Results stay on the device until the next nd_batch_decompose; the call
 * replaces the context's loaded graph (load again before nd_decompose).
 * nd_get_info afterwards reports totals over the batch (r = s = 0 when the
 * batch mixes pairs). On error the batch results are released. */
nd_status nd_batch_decompose(nd_ctx *ctx, uint32_t G, const nd_graph_desc *graphs, nd_mem where,
                             nd_graph_result *results);

/* Results of graph i of the last batch, in that graph's own numbering (its
 * vertices 0..n-1, its r-cliques 0..n_r-1 in lexicographic order, its tree
 * nodes n_r..n_r+n_int-1 in canonical order): identical to nd_get_rcliques /
 * nd_get_counts / nd_get_coreness / nd_get_tree after decomposing graph i
 * alone. Sizes come from results[i]; any pointer may be NULL. */
nd_status nd_batch_get(nd_ctx *ctx, uint32_t i, uint32_t *rcliques, uint32_t *counts,
                       uint32_t *coreness, uint64_t *parent, uint32_t *level, nd_mem where);

/* Device-memory estimate of decomposing one graph, from its size and a
 * bound on its clique counts (the number of r-cliques, and of triangles
 * where the tables need them, bounded from the degree sequence: each edge
 * {u,v} lies in at most min(deg u, deg v) - 1 triangles; for s = 5..7 every
 * k-clique level up to s is bounded by sum_v C(deg v, k - 1) / k, which is
 * loose on graphs with hubs). workspace: bytes
 * the pipeline holds while the graph runs (alone or as part of a batch
 * union, plus 4 MiB per batch); result: bytes of its outputs. Reads the CSR
 * on the host (device inputs are copied back first). Either output may be
 * NULL. */
nd_status nd_estimate_footprint(const nd_graph_desc *g, nd_mem where, uint64_t *workspace,
                                uint64_t *result);

/* ---- Serving: a request loop with continuous batching ------------------
 *
 * A server owns `workers` device pipelines (contexts on streams of their own
 * on one GPU) and a FIFO of requests. A request is admitted when its
 * estimated workspace (nd_estimate_footprint) fits the free part of its
 * pipeline's workspace share and its result fits the free part of the result
 * share. Each pipeline repeatedly takes every admissible waiting request, up
 * to max_batch, and decomposes them together (nd_batch_decompose), so
 * requests that arrive while others run join the next batch of whichever
 * pipeline frees first. The pipelines' batches run on the device at the same
 * time: each pipeline's persistent grid-barrier kernels take 1/workers of the
 * device, so all of them are resident together, and the other kernels share
 * what is left (nd_server_stats reports the measured device overlap).
 * Results stay in device memory until released. Every result is exactly the
 * one nd_decompose gives for the graph alone. */

typedef struct nd_server nd_server;

typedef struct nd_server_options {
  int device;             /* HIP device ordinal                               */
  uint32_t workers;       /* device pipelines; 0 = 2                          */
  uint32_t max_batch;     /* most requests decomposed together; 0 = 512       */
  uint64_t mem_budget;    /* device bytes for workspaces + held results;
                             0 = half of the free memory at creation          */
  int validate;           /* nonzero: check every request's CSR               */
} nd_server_options;

typedef struct nd_request_info {
  nd_status status;       /* outcome once done (ND_E_CANCELLED if cancelled)  */
  int done;               /* 0 = waiting or running, 1 = finished             */
  uint32_t k;             /* max core number                                  */
  uint64_t n_r, n_s, n_int;
  uint64_t workspace;     /* admission estimate of its workspace (bytes)      */
  uint64_t result_bytes;  /* device bytes its results hold                    */
  double t_submit_ms;     /* host clock, ms since the server started          */
  double t_start_ms;      /* its batch started                                */
  double t_done_ms;       /* results ready                                    */
  uint32_t batch_size;    /* requests in its batch                            */
  uint32_t worker;        /* pipeline that ran it                             */
} nd_request_info;

/* opt may be NULL (device 0, defaults above, validation on). */
nd_status nd_server_create(nd_server **out, const nd_server_options *opt);

/* Stops accepting requests, finishes the running batches, frees everything
 * (results not yet released included). */
void nd_server_destroy(nd_server *srv);

/* Queue one decomposition. The CSR (host or device memory per `where`) is
 * copied before the call returns; the caller keeps ownership. Checks as in
 * nd_batch_decompose; a request that could never be admitted (estimate above
 * the pipeline or result share) returns ND_E_OOM. *ticket identifies it. */
nd_status nd_server_submit(nd_server *srv, const nd_graph_desc *req, nd_mem where,
                           uint64_t *ticket);

/* State of a request without waiting (info->done tells whether it ended). */
nd_status nd_server_poll(nd_server *srv, uint64_t ticket, nd_request_info *info);

/* Wait for a request to end; timeout_ms < 0 waits without limit. Returns
 * ND_E_STATE if the time ran out first. */
nd_status nd_server_wait(nd_server *srv, uint64_t ticket, double timeout_ms,
                         nd_request_info *info);

/* Copy a finished request's results out, in the layout of nd_batch_get
 * (sizes from its nd_request_info); any pointer may be NULL. */
nd_status nd_server_get(nd_server *srv, uint64_t ticket, uint32_t *rcliques, uint32_t *counts,
                        uint32_t *coreness, uint64_t *parent, uint32_t *level, nd_mem where);

/* Free a finished request's device results and forget the ticket. */
nd_status nd_server_release(nd_server *srv, uint64_t ticket);

/* Withdraw a waiting request (it ends with ND_E_CANCELLED). A running one
 * finishes, and its results are dropped. */
nd_status nd_server_cancel(nd_server *srv, uint64_t ticket);

typedef struct nd_server_stats {
  uint64_t submitted, completed, failed, cancelled;
  uint64_t batches;           /* batches run, all pipelines                     */
  uint64_t max_batch_seen;    /* largest batch                                  */
  uint64_t waiting, running;  /* requests now waiting / in a running batch      */
  uint64_t result_bytes;      /* device bytes of results not yet released       */
  uint64_t workspace_share;   /* workspace bytes each pipeline may hold         */
  uint64_t result_share;      /* result bytes the server may hold               */
  uint64_t overlapped;        /* requests admitted while another pipeline ran   */
  /* device time of the batches run so far (the last 65,536), from HIP events
   * recorded on each pipeline's stream around its device work: the sum of
   * the batches' intervals, the time covered by at least one, and the time
   * covered by at least two (batches of different pipelines overlapping on
   * the GPU) */
  double device_batch_ms;
  double device_busy_ms;
  double device_overlap_ms;
} nd_server_stats;

nd_status nd_server_get_stats(nd_server *srv, nd_server_stats *out);

/* Message of the server's last error (empty if none). */
const char *nd_server_last_error(const nd_server *srv);

/* ---- Decomposition without device allocation ---------------------------
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The same
 * pipeline and kernels as nd_load_csr + nd_set_rs + nd_decompose +
 * nd_get_coreness / nd_get_tree (results identical), but every intermediate
 * buffer lives in one fixed device array of ND_NOALLOC_SCRATCH_BYTES per GPU
 * (the library reserves it, on every GPU it runs on, until the process
 * ends); no device memory is allocated or freed, not even on first use.
 *
 *   device, hip_stream  GPU ordinal and the hipStream_t to run on (NULL =
 *                       null stream); the call returns after the stream
 *                       finished its work.
 *   n, nnz, row_ptr, col  the CSR, as for nd_load_csr, in DEVICE memory of
 *                       that GPU (validated on the device).
 *   r, s                as for nd_set_rs.
 *   cap                 capacity of the outputs, in r-cliques.
 *   coreness            device uint32[cap]: core numbers (nd_get_coreness).
 *   parent, level       device uint64[2 cap] / uint32[cap]: the canonical
 *                       tree (nd_get_tree; n_r + n_int <= 2 n_r - 1 nodes).
 *   info                host, may be NULL: the run's nd_info (n_r, n_int ...).
 *
 * Errors: ND_E_OOM when the graph does not fit the scratch (the CSR and its
 * edge ids alone must take at most ND_NOALLOC_SCRATCH_BYTES; larger tables
 * are found as the pipeline sizes them), ND_E_INVALID_ARG when n_r > cap
 * (info still tells n_r), and every error of the calls it stands for. The
 * message is nd_last_error(NULL) on the calling thread. Calls on one GPU
 * share its scratch, which keeps the last call's contents; the library runs
 * them one at a time (a second caller waits), so they never overlap there.
 * Graphs up to about 10^5 edges fit for s = 3, fewer triangles for s = 4. */
#define ND_NOALLOC_SCRATCH_BYTES (64ull << 20)
nd_status nd_decompose_noalloc(int device, void *hip_stream, uint32_t n, uint64_t nnz,
                               const uint64_t *row_ptr, const uint32_t *col, uint32_t r,
                               uint32_t s, uint64_t cap, uint32_t *coreness, uint64_t *parent,
                               uint32_t *level, nd_info *info);

const char *nd_status_str(nd_status st);

/* Message of the last error of this context (empty string if none). With
 * ctx == NULL: the message of the last failed nd_create or
 * nd_decompose_noalloc on this thread. */
const char *nd_last_error(const nd_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* NUCLEUS_H */
