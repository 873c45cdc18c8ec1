/*
 * gsmart.h — C ABI of an MI355X engine for SPARQL basic graph patterns by
 * grouped incident-edge evaluation over a label-carrying sparse RDF matrix
 * (after gSmart, arXiv 2106.14038).
 *
 * Problem statement followed (paper Sections 1, 2.2 and 6.2):
 *  - An RDF dataset is a SET of triples <s,p,o> (Section 2.2.1). It is held as
 *    an N x N sparse matrix A whose nonzero (s,o) carries the label p
 *    (Section 1); subjects and objects are 0-based vertex ids, predicates are
 *    1-based (Section 6.2.1, encoding step). Several labels may sit on one
 *    (s,o) pair: every distinct triple is one labelled nonzero.
 *  - A query is a basic graph pattern given as a query graph (Section 2.2.1):
 *    query vertices are variables or constants, every edge (src, label, dst)
 *    is a triple pattern. Its result is every assignment of data vertices to
 *    the variables under which every pattern is a triple of the dataset
 *    (conjunctive semantics, Section 2.2.3); two variables may take the same
 *    vertex. A result row lists the variables in ascending query-vertex index.
 *  - The engine evaluates the query vertices in the order of the degree-driven
 *    traversal (Section 6.1.2), all unevaluated incident edges of a vertex
 *    together (Section 5, Eq. 17-24), storing bindings in a tree whose level j
 *    holds the bindings of the j-th vertex (Section 7.1).
 *
 * Conventions for every call:
 *  - Every call returns gs_status; GS_OK == 0. No C++ exception crosses the
 *    ABI. On failure gs_last_error() returns a message for the calling thread.
 *  - The caller owns every input buffer; inputs are copied or consumed before
 *    the call returns. Pointers to device memory are accepted where a
 *    mem_kind argument says GS_MEM_DEVICE.
 *  - The library owns engines, results and servers until the matching
 *    destroy/free/stop call. A gs_engine is not re-entrant: calls on one
 *    engine must not overlap, except the gs_server_* calls, which lock.
 *  - Work runs on the stream given in gs_options (NULL: the library's own).
 *    Calls that return host data synchronise that stream. Device inputs are
 *    read in that stream's order: data written on another stream must be
 *    complete (synchronised) before the call.
 */
#ifndef GSMART_H
#define GSMART_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GS_OK = 0,
  GS_EINVAL = 1,        /* malformed argument: NULL pointer, bad endpoint, no edges */
  GS_ERANGE = 2,        /* id out of range: s/o outside [0,N), p outside [1,P], N > 2^31-1 */
  GS_ENOMEM = 3,        /* device or host memory exhausted (one query exceeds the budget) */
  GS_EDEVICE = 4,       /* HIP runtime error or no usable device */
  GS_ESTATE = 5,        /* call out of order: second load, query before load, server stopped */
  GS_EUNSUPPORTED = 6,  /* outside the supported subset (more than 64 edges or 64 variables,
                           rows requested from a count-only result) */
  GS_EAGAIN = 7         /* result not ready yet (gs_poll) */
} gs_status;

typedef struct gs_engine gs_engine;   /* owns the device-resident matrix (both orientations) */
typedef struct gs_result gs_result;   /* owns one query's binding tree and counters */
typedef struct gs_server gs_server;   /* a continuous-batching request loop on one engine */

/* One triple <s,p,o>: s, o in [0, N); p in [1, P]. */
typedef struct { int32_t s, p, o; } gs_triple;

/* One query edge (triple pattern): src and dst are query-vertex indices,
 * label is a predicate id in [1, P]. Predicate variables are not supported. */
typedef struct { int32_t src, label, dst; } gs_edge;

/* A query graph. qv_const[i] == -1 makes query vertex i a variable, any value
 * in [0, N) makes it that constant vertex. 1..64 edges, at most 64 variables.
 * Duplicate edges are ignored (a pattern set). */
typedef struct {
  int32_t n_qv;
  const int32_t *qv_const;   /* length n_qv */
  int32_t n_edges;
  const gs_edge *edges;      /* length n_edges */
} gs_query;

enum { GS_MEM_HOST = 0, GS_MEM_DEVICE = 1 };

/* Query flags (gs_query_run, gs_batch_run, gs_submit). */
enum {
  GS_COUNT_ONLY = 1u,        /* do not store the last tree level: count only, no rows */
  GS_PRUNE = 2u              /* after the last level, prune the tree to nodes with a
                                surviving leaf below them (Section 7.2.2 / 8.1) */
};

/* Frontier-domain mode for edges that close a cycle to already-bound vertices
 * (Eq. 14-16): the vertices reachable from the distinct bindings of the bound
 * end. GS_DOMAIN_AUTO picks per edge between push (sparse-frontier product)
 * and pull (masked product) by estimated work; the other modes force one side,
 * or skip the domain and rely on the exact per-binding check alone. All modes
 * give identical results. */
enum { GS_DOMAIN_AUTO = 0, GS_DOMAIN_PUSH = 1, GS_DOMAIN_PULL = 2, GS_DOMAIN_OFF = 3 };

typedef struct {
  int device;                 /* HIP device ordinal */
  void *hip_stream;           /* hipStream_t to run on; NULL = a stream the engine creates */
  uint64_t tree_bytes;        /* device arena for binding trees; 0 = default (1/4 of free memory) */
  uint64_t scratch_bytes;     /* device arena for per-step temporaries; 0 = default (1/16 of free) */
  /* optional allocator for every device allocation the engine makes (e.g. a
     framework's caching allocator); both NULL = hipMalloc / hipFree */
  void *(*alloc)(void *ctx, size_t bytes);
  void (*free)(void *ctx, void *ptr);
  void *alloc_ctx;
  int32_t domain_mode;        /* GS_DOMAIN_* */
  float push_pull_theta;      /* push when est. push work < theta * est. pull work; 0 = 1.0 */
  int32_t grid_blocks;        /* workgroups of the fixed-grid kernels; 0 = 12 per compute unit */
  int32_t use_graphs;         /* batched form: capture each step's launches in a hipGraph (1) or not (0) */
  int32_t profile_kernels;    /* record HIP events around every kernel launch (gs_kernel_stats) */
  int32_t offset_bytes;       /* stored row offsets: 0 = by size (4 bytes when M < 2^31, else 8), 8 = always 8 */
  const char *autotune_cache; /* optional text file of tuned settings: gs_autotune records its choice for
                                 the loaded graph's sizes there, gs_load_triples applies a recorded one */
  int32_t traversal;          /* GS_TRAVERSAL_*: the planner's traversal for queries without constants */
  int32_t write_block;        /* threads per workgroup of the write pass: 128, 256 or 512; 0 = 256 (a recorded
                                 autotune setting replaces it at load) */
} gs_options;

/* Query-graph traversal that orders the evaluation (Section 6.1): degree-driven
 * (6.1.2, every incident edge of a visited vertex together) or direction-driven
 * (6.1.1, DFS along edge directions from vertices without incoming edges, every
 * outgoing edge of a visited vertex together, several roots). Queries with
 * constants always take the degree-driven traversal with the constants rule. */
enum { GS_TRAVERSAL_DEGREE = 0, GS_TRAVERSAL_DIRECTION = 1, GS_TRAVERSAL_ENGINE = -1 };

/* Per-query counters, filled by gs_result_stats. T counts LSpM nonzeros read
 * by the kernels ("traversed triples"); bytes are algorithmic bytes. */
typedef struct {
  int64_t count;              /* number of result rows */
  int32_t n_levels;           /* tree levels (= variables) */
  int32_t n_domains;          /* cycle-closing edges given a frontier domain */
  int64_t level_nodes[64];    /* nodes per tree level before pruning */
  int64_t t_expand;           /* candidate entries read while growing the tree (a last level that is
                                 only counted and faces no test is summed from segment lengths: its
                                 entries are not read and not counted here) */
  int64_t t_seed;             /* entries read to seed constant filters */
  int64_t t_push;             /* entries read by push domain products */
  int64_t t_pull;             /* entries read by pull domain products */
  int64_t t_probe;            /* entries touched by binary-search membership checks */
  int64_t t_total;            /* sum of the above */
  int64_t bytes_alg;          /* algorithmic bytes: 4 * t_total (int32 ids) + label width * t_label
                                 + 2 * offset width * seg_lookups + 8 * nodes_written + 8 * nodes_read
                                 + 8 * bitmap_words */
  int32_t domain_push;        /* domains evaluated by push */
  int32_t domain_pull;        /* domains evaluated by pull */
  double gpu_ms;              /* device time of the evaluation (events around its launches) */
  double latency_ms;          /* served form: submission to rows on the host; else 0 */
  int64_t t_label;            /* label entries read while locating label sub-segments (not in t_total) */
  int64_t seg_lookups;        /* segment lookups: row or column offset pairs read */
  int64_t bitmap_words;       /* 64-bit bitmap words read or written (filters, lists, seeds, domains) */
  int64_t nodes_written;      /* binding-tree nodes written (a count-only last level is not) */
  int64_t nodes_read;         /* binding-tree nodes read by a later step */
} gs_query_stats;

/* ---- engine ---------------------------------------------------------------- */

/* Create an engine on options->device (NULL options: defaults, device 0).
 * Allocates the two device arenas. Errors: GS_EDEVICE, GS_ENOMEM, GS_EINVAL. */
gs_status gs_engine_create(const gs_options *options, gs_engine **out);

/* Release every device allocation and the engine. NULL is ignored. Results
 * created by the engine must be freed before. */
void gs_engine_destroy(gs_engine *engine);

/* Load the dataset: m triples (host or device memory per mem_kind), n vertices,
 * n_labels predicates. Builds the light-weight sparse matrix of Section 6.2 in
 * both orientations on the device — row-wise (pointer, column, label arrays;
 * each row sorted by (label, column)) and column-wise (pointer, row, label
 * arrays; each column sorted by (label, row)) — after removing duplicate
 * triples (a dataset is a set), plus the label-existence vectors of Eq. (4)
 * and (5) for every label. Only once per engine (GS_ESTATE otherwise).
 * Errors: GS_ERANGE (ids), GS_EINVAL, GS_ENOMEM, GS_EDEVICE. */
gs_status gs_load_triples(gs_engine *engine, int64_t n_vertices, int32_t n_labels,
                          const gs_triple *triples, int64_t m, int mem_kind);

/* One-shot load for one query (Section 6.2.1 and 6.2.2, step 1: only the
 * triples whose predicate the query names): as gs_load_triples, but the
 * triples whose predicate is not among labels[0, n_keep) (1-based) are
 * dropped on the device before the matrix is built, so a query that reads
 * only those predicates evaluates as on the whole dataset, with the device
 * holding and sorting only its part. Every triple is still range-checked.
 * Errors: as gs_load_triples; GS_ERANGE also for a label outside [1, n_labels]. */
gs_status gs_load_triples_labels(gs_engine *engine, int64_t n_vertices, int32_t n_labels,
                                 const gs_triple *triples, int64_t m, int mem_kind, const int32_t *labels,
                                 int32_t n_keep);

/* Sizes after loading: vertices, labels, distinct triples, device bytes held. */
gs_status gs_graph_info(const gs_engine *engine, int64_t *n, int32_t *n_labels, int64_t *m_distinct,
                        uint64_t *device_bytes);

/* Copy one orientation of the stored matrix to host buffers: orientation 0 =
 * row-wise (ptr[n+1], idx = column of each nonzero, label), 1 = column-wise
 * (ptr[n+1], idx = row, label). Labels come back 1-based. Buffers sized n+1
 * and m_distinct. Section 6.2. */
gs_status gs_lspm_export(gs_engine *engine, int orientation, int64_t *ptr, int32_t *idx, int32_t *label);

/* Per-label statistics: nonzeros, rows holding the label, columns holding it.
 * Each array has n_labels entries (index p-1). */
gs_status gs_label_stats(gs_engine *engine, int64_t *nnz, int64_t *rows, int64_t *cols);

/* ---- matrix-algebra primitives (Section 2.1) --------------------------------- */

/* Eq. (4) (direction 0) or Eq. (5) (direction 1): bit i of the result is set
 * iff row (column) i of A holds label p. Bitmap of ceil(n/64) 64-bit words,
 * bit i = word i/64, bit i%64; written to host_words. */
gs_status gs_label_exists(gs_engine *engine, int32_t label, int direction, uint64_t *host_words);

/* Eq. (14)-(16) / (22): the vertices reachable from the frontier F along
 * label p — direction 0: objects of (b,p,*) for b in F (rows of diag(F) A);
 * direction 1: subjects of (*,p,b) (columns of A diag(F)). mode is
 * GS_DOMAIN_PUSH or GS_DOMAIN_PULL; with pull, only candidates in mask are
 * tested (mask NULL = all vertices) and the result is restricted to mask.
 * Bitmaps as in gs_label_exists, host memory. */
gs_status gs_frontier_domain(gs_engine *engine, const uint64_t *frontier_words, int32_t label,
                             int direction, int mode, const uint64_t *mask_words, uint64_t *out_words);

/* Eq. (10) with compaction: the ascending ids of the bits set in every one of
 * the k host bitmaps. out (capacity n ids) receives *count ids. */
gs_status gs_bitmap_and_compact(gs_engine *engine, const uint64_t *const *bitmaps, int32_t k, int32_t *out,
                                int64_t *count);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): gs_bitmap_and_compact
 * over device memory, allocating nothing and copying nothing from the host.
 * dev_bitmaps: host array of k device pointers, each to ceil(n/64) words;
 * k <= 64 (GS_EINVAL above). dev_out: device buffer of capacity n int32
 * (n = the loaded vertex count) that receives the ascending ids; dev_count: a
 * device int64 that receives their number. Stream-ordered on the engine's
 * stream and not synchronised: read the outputs after that stream. Temporaries
 * live in one fixed device workspace per GPU (about 272 KiB, a static device
 * array held until the process ends, located when an engine is created on
 * that GPU); every call on a GPU uses the same workspace, so calls that overlap
 * on one GPU (other streams, other engines, other threads) race. Each call
 * clears what it accumulates. Errors: GS_EINVAL, GS_ESTATE (no data, or a
 * server running), GS_EDEVICE (launch failure). */
gs_status gs_bitmap_and_compact_noalloc(gs_engine *engine, const uint64_t *const *dev_bitmaps, int32_t k,
                                        int32_t *dev_out, int64_t *dev_count);

/* ---- planner (Section 6.1.2, host only, no device needed) -------------------- */

typedef struct {
  int32_t n_vars;             /* variables (tree levels) */
  int32_t order[64];          /* query vertices in binding order (tree level j -> query vertex) */
  int32_t parent_edge[64];    /* per level: index of the edge that generates its candidates,
                                 -1 = none (a new component: candidates independent of level j-1) */
  int32_t n_groups;           /* edge groups, one per popped vertex that evaluated edges */
  int32_t group_vertex[64];   /* popped query vertex of each group */
  int32_t edge_group[64];     /* per input edge: group that evaluates it, -1 = duplicate edge */
  int32_t n_roots;            /* traversal roots (Section 6.1, step 2) */
  int32_t roots[64];
} gs_plan_info;

/* Degree-driven traversal with the constants rule (Section 6.1.2): the roots,
 * the groups of edges evaluated at each visited vertex, and the tree level of
 * each query vertex (order[]: a vertex follows the one that discovered it;
 * among the vertices that may come next, the smallest estimated fan-out goes
 * first, ties in pop order). engine: optional; with an engine that holds a
 * matrix the plan is the one its evaluation uses (label statistics, id and
 * label ranges checked); NULL plans without statistics (levels in pop order).
 * Errors: GS_EINVAL, GS_ERANGE, GS_EUNSUPPORTED. */
gs_status gs_plan_query(gs_engine *engine, const gs_query *query, gs_plan_info *out);

/* As gs_plan_query with the traversal chosen explicitly (GS_TRAVERSAL_ENGINE:
 * the engine's option; degree-driven without an engine). */
gs_status gs_plan_query_ex(gs_engine *engine, const gs_query *query, int32_t traversal, gs_plan_info *out);

/* ---- per-query reduced matrix (Section 6.2.1, 6.2.2; Ex. 6.3, 6.4) ------------ */

typedef struct gs_reduced gs_reduced;   /* device arrays of one query's reduced matrix */

typedef struct {
  int64_t n;                 /* vertices: M has n + 1 entries per part */
  int64_t rows[2];           /* kept rows (part 0, row-wise) and kept columns (part 1, column-wise) */
  int64_t nnz[2];            /* nonzeros of each part */
  int32_t n_labels[2];       /* predicates each part keeps (0: the part is empty) */
  int32_t labels[2][64];     /* those predicates, 1-based, ascending */
} gs_reduced_info;

/* The reduced matrix of one query, built on the device from the resident one.
 * The predicates of each part follow the traversal's edge groups (see
 * gs_plan_query_ex; traversal as there): with the direction-driven traversal
 * and no constant, one row-wise part with every predicate of the query
 * (Section 6.2.1); otherwise (Section 6.2.2) an edge evaluated in the group of
 * its subject puts its predicate in the row-wise part and one evaluated in the
 * group of its object in the column-wise part, an edge out of a constant in
 * the row-wise part and an edge into a constant in the column-wise part. Each
 * part keeps the nonzeros of its predicates, drops the rows (columns) left
 * empty and numbers the kept ones in order. *out is freed with
 * gs_reduced_free (its device memory comes from hipMalloc on the engine's
 * device; it does not depend on the engine afterwards). Errors: GS_ESTATE (no
 * data, or a server running), GS_EINVAL, GS_EUNSUPPORTED (more than 64
 * predicates in a part), GS_ENOMEM, GS_EDEVICE. */
gs_status gs_lspm_reduce(gs_engine *engine, const gs_query *query, int32_t traversal, gs_reduced **out);

gs_status gs_reduced_get_info(const gs_reduced *reduced, gs_reduced_info *out);

/* Copy part `part` (0 row-wise, 1 column-wise) to host buffers: M (n + 1
 * int64: M[i + 1] - M[i] == 1 exactly when row i is kept, and then M[i] is
 * its index among the kept rows), P (rows + 1 int64 offsets into val / idx per
 * kept row), val (nnz int32, the 1-based predicates) and idx (nnz int32, the
 * other endpoint: column for part 0, row for part 1); a kept row's entries in
 * ascending (predicate, endpoint) order. Any pointer may be NULL to skip that
 * array. Errors: GS_EINVAL, GS_EDEVICE. */
gs_status gs_reduced_export(const gs_reduced *reduced, int32_t part, int64_t *M, int64_t *P, int32_t *val,
                            int32_t *idx);

/* Release the reduced matrix. NULL is ignored. */
gs_status gs_reduced_free(gs_reduced *reduced);

/* ---- N-Triples dictionary encoding (Section 6.2.1, step 2) ------------------- */

typedef struct gs_dict gs_dict;   /* integer triples and the dictionaries that decode them */

/* Encode N-Triples text (len bytes, lines separated by LF or CRLF; blank lines
 * and # comments skipped): each line "subject predicate object ." becomes one
 * int32 triple. Subjects and objects share one dictionary numbered from 0,
 * predicates have their own numbered from 1, each in order of first
 * appearance (a line's subject before its object). A term is keyed by its
 * bytes as written: an IRI <...>, a blank node _:label (ASCII letters, digits,
 * "_" and "-"), a literal "..." with its escapes and an optional @tag (ASCII
 * letters, digits and "-") or ^^<datatype>. Repeated lines stay repeated (the
 * loaders remove repeats). The text is copied. Errors: GS_EINVAL (malformed
 * line; the message names it), GS_ERANGE (more than 2^31 vertices), GS_ENOMEM. */
gs_status gs_encode_ntriples(const char *text, int64_t len, gs_dict **out);

/* Sizes: triples (lines), distinct subjects and objects, distinct predicates. */
gs_status gs_dict_info(const gs_dict *dict, int64_t *n_triples, int64_t *n_vertices, int32_t *n_labels);

/* The triples, n_triples * 3 int32 (s, p, o) into host memory, in line order. */
gs_status gs_dict_triples(const gs_dict *dict, int32_t *out);

/* The term of a vertex id / 1-based predicate: *len gets its length; up to
 * cap - 1 bytes and a terminating zero go to buf (buf may be NULL to ask for
 * the length). Errors: GS_ERANGE. */
gs_status gs_dict_vertex(const gs_dict *dict, int64_t id, char *buf, int64_t cap, int64_t *len);
gs_status gs_dict_label(const gs_dict *dict, int32_t label, char *buf, int64_t cap, int64_t *len);

/* Ids of a term: *id = -1 (*label = 0) when the text has no such term. */
gs_status gs_dict_find_vertex(const gs_dict *dict, const char *term, int64_t len, int64_t *id);
gs_status gs_dict_find_label(const gs_dict *dict, const char *term, int64_t len, int32_t *label);

/* Release the dictionary. NULL is ignored. */
gs_status gs_dict_free(gs_dict *dict);

/* ---- plain and batched evaluation ------------------------------------------- */

/* Evaluate one query (one at a time). *out receives a result to be freed with
 * gs_result_free. Errors: GS_ESTATE (no data, or a server running on the
 * engine), GS_EINVAL, GS_ERANGE, GS_EUNSUPPORTED, GS_ENOMEM (tree exceeds the
 * tree arena, or a level's temporaries exceed the scratch arena), GS_EDEVICE
 * (HIP error, or an internal inconsistency between the count and write passes
 * detected on the device). */
gs_status gs_query_run(gs_engine *engine, const gs_query *query, uint32_t flags, gs_result **out);

/* Evaluate nq queries together: each vertex step of every query runs in the
 * same launches (one launch sequence per step for the whole batch). outs[i]
 * receives query i's result; results are identical to gs_query_run's. On
 * error no result is returned (all outs[i] = NULL). */
gs_status gs_batch_run(gs_engine *engine, const gs_query *queries, int32_t nq, uint32_t flags,
                       gs_result **outs);

/* Number of result rows (bindings). */
gs_status gs_result_count(const gs_result *result, int64_t *count);

/* Row width: number of variables of the query. */
gs_status gs_result_width(const gs_result *result, int32_t *n_vars);

/* Copy rows [first, first+n) to dst (host or device per mem_kind), each row
 * n_vars int32 in ascending query-vertex order of the variables. Row order is
 * unspecified but fixed for one result. *n_written = rows copied.
 * Errors: GS_EUNSUPPORTED for count-only results, GS_ERANGE for first > count. */
gs_status gs_result_rows(gs_result *result, int64_t first, int64_t n, void *dst, int mem_kind,
                         int64_t *n_written);

/* Order-independent digest of the result rows, computed on the device without
 * copying rows out: each row (v_0..v_{k-1}, the variables in ascending
 * query-vertex order) hashes to h_k, where h_0 = k and
 * h_{i+1} = mix64(h_i + 0x9E3779B97F4A7C15 + (uint32_t)v_i), mix64 being the
 * output function of the splitmix64 generator (Steele, Lea and Flood, OOPSLA
 * 2014); *hash_sum = sum of the row hashes mod 2^64, *hash_xor = their XOR,
 * *count = rows. Equal results have equal digests; a differing digest proves
 * the row multisets differ (the converse holds only with high probability).
 * Errors: GS_EUNSUPPORTED for count-only results. */
gs_status gs_result_digest(gs_result *result, int64_t *count, uint64_t *hash_sum, uint64_t *hash_xor);

/* Counters of the evaluation (size = sizeof(gs_query_stats)). */
gs_status gs_result_stats(const gs_result *result, gs_query_stats *stats);

/* Copy tree level j to host: parent index into level j-1 (0 at level 0) and
 * the bound vertex of level j's query vertex; *n = nodes. With par/vid NULL
 * only *n is returned. Section 7.1. */
gs_status gs_result_level(gs_result *result, int32_t level, int32_t *par, int32_t *vid, int64_t *n);

/* Kernel timing, available when gs_options.profile_kernels was set: per
 * kernel of the evaluation, launches, device milliseconds (HIP events on the
 * engine's stream around each launch) and bytes moved by two models: the
 * method's own (expansion write pass: a candidate id read per entry and a tree
 * node of parent and vertex written per child) and the implementation's (ids,
 * carried columns, staged node records, validity bits, offsets, as the kernels
 * touch them). Fills up to cap entries, *n = kernels with at least one launch;
 * reset != 0 clears the counters after reading. */
typedef struct {
  const char *name;           /* static string */
  int64_t launches;
  double ms;
  double bytes_alg;           /* the method's bytes; 0 where the kernel has no such model */
  double bytes_impl;          /* the implementation's bytes; 0 where no model is kept */
} gs_kernel_stat;
gs_status gs_kernel_stats(gs_engine *engine, gs_kernel_stat *out, int32_t cap, int32_t *n, int reset);

/* Autotuner: evaluates the given queries (count only, batched) under every
 * candidate workgroup count of the fixed-grid kernels (2, 4, 8, 12 and 16 per
 * compute unit) and push/pull threshold (0.25, 1, 4), then, with the fastest
 * pair, under every workgroup size of the write pass (128, 256 or 512 threads,
 * as many workgroups as the device holds at once); keeps the fastest setting
 * for this engine's later calls, and reports it; with gs_options.autotune_cache
 * set, the setting is also recorded there for the loaded graph's sizes (n, m,
 * P), and a later engine loading a graph of those sizes starts from it.
 * Results are unchanged by the choice. Errors as gs_batch_run. */
typedef struct {
  int32_t grid_blocks;
  float push_pull_theta;
  double best_ms;             /* device time of the calibration batch with the chosen setting */
  double default_ms;          /* same with the engine's settings before tuning */
  int32_t n_tried;
  int32_t write_block;        /* threads per workgroup of the write pass */
} gs_tune_result;
gs_status gs_autotune(gs_engine *engine, const gs_query *queries, int32_t nq, gs_tune_result *out);

/* Free a result. NULL is ignored. */
void gs_result_free(gs_result *result);

/* ---- served form -------------------------------------------------------------- */

typedef struct {
  int32_t max_active;         /* queries evaluated together at most; 0 = 1024 */
  uint64_t tree_budget_bytes; /* admit while the sum of estimated tree bytes fits; 0 = arena size */
  uint32_t flags;             /* GS_COUNT_ONLY applies to every request when set */
} gs_server_options;

typedef struct {
  int64_t submitted, completed, iterations;
  int64_t max_active_seen;
  int64_t rejected;           /* requests failed with an error (e.g. GS_ENOMEM) */
  int64_t requeued;           /* requests re-run after an arena overflow */
} gs_server_stats;

/* Start the request loop on its own host thread. The engine must be loaded, and
 * every result of its direct evaluation freed (the loop uses the whole tree
 * arena). Until gs_server_stop, direct evaluation on the engine (gs_query_run,
 * gs_batch_run, gs_autotune, gs_frontier_domain, gs_bitmap_and_compact) returns
 * GS_ESTATE. Errors: GS_ESTATE (no data, live results, a server already
 * running), GS_ENOMEM. */
gs_status gs_server_start(gs_engine *engine, const gs_server_options *options, gs_server **out);

/* Enqueue a request; *ticket identifies it. Thread-safe. */
gs_status gs_submit(gs_server *server, const gs_query *query, uint32_t flags, uint64_t *ticket);

/* GS_EAGAIN while the request is pending; GS_OK with *out (caller frees) when
 * done, or the request's own error status. Each ticket is returned once. */
gs_status gs_poll(gs_server *server, uint64_t ticket, gs_result **out);

/* Drain finished requests: up to cap of them, in no particular order, each
 * returned once. tickets[i], statuses[i] and results[i] (NULL on error) describe
 * request i; *n = number returned (0 when none is ready). */
gs_status gs_poll_ready(gs_server *server, uint64_t *tickets, int32_t *statuses, gs_result **results, int32_t cap,
                        int32_t *n);

/* Wait until every submitted request is done, then stop the loop. Results not
 * polled yet are freed. */
gs_status gs_server_stop(gs_server *server, gs_server_stats *stats);

/* Thread-local message of the last failing call ("" if none). */
const char *gs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GSMART_H */
