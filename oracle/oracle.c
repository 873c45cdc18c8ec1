/*
 * ORACLE — test infrastructure only.
 *
 * A plain, slow, obviously correct CPU evaluator of SPARQL basic graph
 * patterns over an RDF triple set, and of the matrix-algebra primitives the
 * method is built from. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it. It shares no code with the HIP
 * engine and reads nothing the engine writes.
 *
 * Definitions followed (gSmart, arXiv 2106.14038):
 *  - Data (Section 2.2.1): a dataset is a SET of triples <s,p,o>; the RDF
 *    matrix A is N x N with A(s,o) carrying label p (Section 1), subjects and
 *    objects 0-based, predicates 1-based (Section 6.2.1, encoding step).
 *    Several labels may sit on the same (s,o) pair; each distinct triple is
 *    one labelled nonzero.
 *  - Query (Section 2.2.1): a basic graph pattern, i.e. a set of triple
 *    patterns over variables and constants; its result is every assignment of
 *    data vertices to the variables under which every pattern is a triple of
 *    the dataset (conjunctive semantics, Section 2.2.3). Two variables may take
 *    the same vertex (homomorphism). Output rows list the variables in
 *    ascending query-vertex index.
 *  - Eq. (4)/(5): y = A (x) u_p and y = A^T (x) u_p, the rows / columns of A
 *    holding label p, with (x) the boolean semiring product.
 *  - Eq. (14)-(16): the binding vector of y is the OR of the rows of M_xy, and
 *    M_yz keeps label-p entries of the rows of A selected by it; the vector of
 *    reachable z is therefore OR over selected rows i of [A(i,j) == p].
 *  - LSpM (Section 6.2): row-wise storage with a pointer array, a value
 *    (label) array and a column array; here the full matrix, rows sorted by
 *    (label, column).
 *
 * Algorithms (plain, written from the definitions, not from the paper's
 * parallel executor):
 *  - or_eval: backtracking over variables in a fixed order. A variable's
 *    candidates are the label-p neighbours of an already-bound endpoint of
 *    its first such edge (else every vertex); every edge whose endpoints are
 *    all bound is checked by set membership.
 *  - or_eval_digest: the same backtracking, keeping only the count and an
 *    order-independent digest of the rows; optionally on several threads,
 *    each taking chunks of the first variable's candidates (the timing mode
 *    "on all host cores").
 *  - or_count_acyclic: exact counting by message passing over the query
 *    forest (parallel edges between two variables bundled into one pairwise
 *    constraint). Unsigned 128-bit arithmetic, saturating.
 *
 * Parity pins for every function live in the CPU test suite (brute force,
 * closed forms, the paper's worked examples, invariants).
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The triple set in both orientations. Row v of orientation 0 lists the
 * triples (v, p, o) as keys p << 32 | o, row v of orientation 1 the triples
 * (s, p, v) as keys p << 32 | s; each row sorted ascending, without repeats.
 * A key's neighbour is its low 32 bits, its label the high 32 bits. */
typedef uint64_t okey;
static inline okey mkkey(int32_t p, int32_t v) { return ((uint64_t)(uint32_t)p << 32) | (uint32_t)v; }
static inline int32_t key_nbr(okey k) { return (int32_t)(uint32_t)k; }
static inline int32_t key_lab(okey k) { return (int32_t)(k >> 32); }

typedef struct {
  int64_t n; int32_t P; int64_t m;
  int64_t *ptr[2];    /* n + 1 row offsets per orientation */
  okey *key[2];       /* m keys per orientation */
  int64_t *cur[2];    /* build only: fill cursors */
  int64_t cap;        /* build only: triples counted (repeats included) */
} oracle_graph;

/* Streamed build: count every triple (validating ids), allocate, place every
 * triple again, then sort and deduplicate each row. The same triples must be
 * passed to the count and the fill step. */
oracle_graph *or_graph_begin(int64_t n, int32_t P) {
  if (n < 0 || P < 0) return NULL;
  oracle_graph *g = (oracle_graph *)calloc(1, sizeof *g);
  if (!g) return NULL;
  g->n = n; g->P = P;
  for (int d = 0; d < 2; ++d) {
    g->ptr[d] = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!g->ptr[d]) return NULL;
  }
  return g;
}

/* Returns 0, or -2 when a triple has s/o outside [0, n) or p outside [1, P]. */
int or_graph_count(oracle_graph *g, const int32_t *triples, int64_t m) {
  for (int64_t i = 0; i < m; ++i) {
    int32_t s = triples[3 * i], p = triples[3 * i + 1], o = triples[3 * i + 2];
    if (s < 0 || s >= g->n || o < 0 || o >= g->n || p < 1 || p > g->P) return -2;
  }
  for (int64_t i = 0; i < m; ++i) { g->ptr[0][triples[3 * i] + 1]++; g->ptr[1][triples[3 * i + 2] + 1]++; }
  g->cap += m;
  return 0;
}

int or_graph_alloc(oracle_graph *g) {
  for (int d = 0; d < 2; ++d) {
    for (int64_t v = 0; v < g->n; ++v) g->ptr[d][v + 1] += g->ptr[d][v];
    g->key[d] = (okey *)malloc(sizeof(okey) * (size_t)(g->cap ? g->cap : 1));
    g->cur[d] = (int64_t *)malloc(sizeof(int64_t) * ((size_t)g->n + 1));
    if (!g->key[d] || !g->cur[d]) return -1;
    memcpy(g->cur[d], g->ptr[d], sizeof(int64_t) * ((size_t)g->n + 1));
  }
  return 0;
}

void or_graph_fill(oracle_graph *g, const int32_t *triples, int64_t m) {
  for (int64_t i = 0; i < m; ++i) {
    int32_t s = triples[3 * i], p = triples[3 * i + 1], o = triples[3 * i + 2];
    g->key[0][g->cur[0][s]++] = mkkey(p, o);
    g->key[1][g->cur[1][o]++] = mkkey(p, s);
  }
}

static int cmp_key(const void *x, const void *y) {
  okey a = *(const okey *)x, b = *(const okey *)y;
  return a < b ? -1 : a > b;
}

typedef struct { oracle_graph *g; int d; int64_t v0, v1; int64_t *kept; } sort_job;

/* Sort rows [v0, v1) and drop repeats; each row's distinct keys stay at its start. */
static void *sort_rows_job(void *arg) {
  sort_job *j = (sort_job *)arg;
  const int64_t *ptr = j->g->ptr[j->d];
  okey *key = j->g->key[j->d];
  for (int64_t v = j->v0; v < j->v1; ++v) {
    int64_t a = ptr[v], e = ptr[v + 1], k = a;
    qsort(key + a, (size_t)(e - a), sizeof(okey), cmp_key);
    for (int64_t i = a; i < e; ++i)
      if (k == a || key[k - 1] != key[i]) key[k++] = key[i];
    j->kept[v] = k - a;
  }
  return NULL;
}

/* Returns 0, or -1 when the orientations disagree (cannot happen for equal inputs). */
int or_graph_finish(oracle_graph *g, int32_t nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  int64_t *kept = (int64_t *)malloc(sizeof(int64_t) * ((size_t)g->n + 1));
  int64_t mm[2] = {0, 0};
  for (int d = 0; d < 2; ++d) {
    free(g->cur[d]); g->cur[d] = NULL;
    sort_job jobs[64];
    pthread_t th[64];
    int running[64] = {0};
    for (int t = 0; t < nthreads; ++t) {
      jobs[t].g = g; jobs[t].d = d; jobs[t].kept = kept;
      jobs[t].v0 = g->n * t / nthreads; jobs[t].v1 = g->n * (t + 1) / nthreads;
      running[t] = nthreads > 1 && pthread_create(&th[t], NULL, sort_rows_job, &jobs[t]) == 0;
      if (!running[t]) sort_rows_job(&jobs[t]);   /* this thread takes the job itself */
    }
    for (int t = 0; t < nthreads; ++t) if (running[t]) pthread_join(th[t], NULL);
    /* compact the rows to the front, in order */
    int64_t w = 0;
    for (int64_t v = 0; v < g->n; ++v) {
      const int64_t a = g->ptr[d][v];
      g->ptr[d][v] = w;
      memmove(g->key[d] + w, g->key[d] + a, sizeof(okey) * (size_t)kept[v]);
      w += kept[v];
    }
    g->ptr[d][g->n] = w;
    mm[d] = w;
    okey *shrunk = (okey *)realloc(g->key[d], sizeof(okey) * (size_t)(w ? w : 1));   /* return the repeats' room */
    if (shrunk) g->key[d] = shrunk;
  }
  free(kept);
  g->m = mm[0];
  return mm[0] == mm[1] ? 0 : -1;
}

/* Build the triple set from one array. Returns NULL on bad ids (s/o outside [0,n), p outside [1,P]). */
oracle_graph *or_graph_new(const int32_t *triples, int64_t m, int64_t n, int32_t P) {
  if (m < 0) return NULL;
  oracle_graph *g = or_graph_begin(n, P);
  if (!g) return NULL;
  if (or_graph_count(g, triples, m) != 0 || or_graph_alloc(g) != 0) {
    for (int d = 0; d < 2; ++d) { free(g->ptr[d]); free(g->key[d]); free(g->cur[d]); }
    free(g);
    return NULL;
  }
  or_graph_fill(g, triples, m);
  or_graph_finish(g, 1);
  return g;
}

void or_graph_free(oracle_graph *g) {
  if (!g) return;
  for (int d = 0; d < 2; ++d) { free(g->ptr[d]); free(g->key[d]); free(g->cur[d]); }
  free(g);
}
int64_t or_graph_m(const oracle_graph *g) { return g->m; }

/* first index in key[lo, hi) not less than k */
static int64_t lower_key(const okey *key, int64_t lo, int64_t hi, okey k) {
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (key[mid] < k) lo = mid + 1; else hi = mid;
  }
  return lo;
}

/* Is (s, p, o) in the set? */
static int has_triple(const oracle_graph *g, int32_t s, int32_t p, int32_t o) {
  const okey k = mkkey(p, o);
  const int64_t a = g->ptr[0][s], e = g->ptr[0][s + 1];
  const int64_t i = lower_key(g->key[0], a, e, k);
  return i < e && g->key[0][i] == k;
}

/* Neighbours of v along label p: dir 0 = objects of (v, p, *), dir 1 = subjects of (*, p, v);
 * *cnt keys, each neighbour = key_nbr(key). */
static const okey *adj(const oracle_graph *g, int32_t v, int32_t p, int dir, int64_t *cnt) {
  const int64_t a = g->ptr[dir][v], e = g->ptr[dir][v + 1];
  const int64_t lo = lower_key(g->key[dir], a, e, mkkey(p, 0));
  const int64_t hi = lower_key(g->key[dir], lo, e, mkkey(p + 1, 0));
  *cnt = hi - lo;
  return g->key[dir] + lo;
}

/* ---------------------------------------------------- LSpM (Section 6.2) */
/* Row-wise storage of the whole matrix: row_ptr[n+1], col[m], lab[m] (1-based
 * labels), each row's entries in (label, column) order. */
void or_csr(const oracle_graph *g, int64_t *row_ptr, int32_t *col, int32_t *lab) {
  memcpy(row_ptr, g->ptr[0], sizeof(int64_t) * ((size_t)g->n + 1));
  for (int64_t i = 0; i < g->m; ++i) { col[i] = key_nbr(g->key[0][i]); lab[i] = key_lab(g->key[0][i]); }
}
/* Column-wise storage: col_ptr[n+1], row[m], lab[m], each column in (label, row) order. */
void or_csc(const oracle_graph *g, int64_t *col_ptr, int32_t *row, int32_t *lab) {
  memcpy(col_ptr, g->ptr[1], sizeof(int64_t) * ((size_t)g->n + 1));
  for (int64_t i = 0; i < g->m; ++i) { row[i] = key_nbr(g->key[1][i]); lab[i] = key_lab(g->key[1][i]); }
}

/* ---------------------------------------------- algebra (Section 2.1) */
/* Eq. (4) (dir 0): y(i) = OR_j [A(i,j) == p]; Eq. (5) (dir 1): y(j) = OR_i [A(i,j) == p].
 * Written as the definition: one pass over every nonzero (i, j) of the row-wise storage. */
void or_label_exists(const oracle_graph *g, int32_t p, int dir, uint8_t *y) {
  memset(y, 0, (size_t)g->n);
  for (int64_t i = 0; i < g->n; ++i)
    for (int64_t k = g->ptr[0][i]; k < g->ptr[0][i + 1]; ++k)
      if (key_lab(g->key[0][k]) == p) y[dir ? key_nbr(g->key[0][k]) : i] = 1;
}

/* Eq. (14)-(16): the binding vector reachable from the selected rows F along label p.
 * dir 0: y(j) = OR_i F(i) and A(i,j) == p   (rows of diag(F) A)
 * dir 1: y(i) = OR_j F(j) and A(i,j) == p   (columns of A diag(F)) */
void or_frontier_domain(const oracle_graph *g, const uint8_t *F, int32_t p, int dir, uint8_t *y) {
  memset(y, 0, (size_t)g->n);
  for (int64_t i = 0; i < g->n; ++i)
    for (int64_t k = g->ptr[0][i]; k < g->ptr[0][i + 1]; ++k) {
      if (key_lab(g->key[0][k]) != p) continue;
      const int32_t j = key_nbr(g->key[0][k]);
      if (dir == 0 && F[i]) y[j] = 1;
      if (dir == 1 && F[j]) y[i] = 1;
    }
}

/* ------------------------------------------------ query normalisation */
#define OR_MAXQV 128
#define OR_MAXE 128

typedef struct {
  int32_t n_qv, n_edges;
  int32_t cst[OR_MAXQV];          /* -1 variable, else constant vertex */
  int32_t e[OR_MAXE][3];          /* (src, label, dst), duplicates removed */
  int32_t nvar, var_of[OR_MAXQV]; /* query vertex -> variable rank (ascending index) or -1 */
  int32_t qv_of[OR_MAXQV];        /* variable rank -> query vertex */
} nq_t;

/* Returns 0 ok, -1 malformed, -2 label or constant out of range. */
static int normalise(const oracle_graph *g, int32_t n_qv, const int32_t *qv_const, int32_t n_edges,
                     const int32_t *edges, nq_t *q) {
  if (n_qv < 0 || n_qv > OR_MAXQV || n_edges < 1 || n_edges > OR_MAXE) return -1;
  memset(q, 0, sizeof *q);
  q->n_qv = n_qv;
  for (int i = 0; i < n_qv; ++i) {
    q->cst[i] = qv_const ? qv_const[i] : -1;
    if (q->cst[i] < -1 || q->cst[i] >= g->n) return -2;
  }
  for (int k = 0; k < n_edges; ++k) {
    int32_t s = edges[3 * k], p = edges[3 * k + 1], o = edges[3 * k + 2];
    if (s < 0 || s >= n_qv || o < 0 || o >= n_qv) return -1;
    if (p < 1 || p > g->P) return -2;
    int dup = 0;
    for (int j = 0; j < q->n_edges; ++j) dup |= (q->e[j][0] == s && q->e[j][1] == p && q->e[j][2] == o);
    if (!dup) { q->e[q->n_edges][0] = s; q->e[q->n_edges][1] = p; q->e[q->n_edges][2] = o; q->n_edges++; }
  }
  q->nvar = 0;
  for (int i = 0; i < n_qv; ++i) {
    q->var_of[i] = -1;
    if (q->cst[i] < 0) { q->var_of[i] = q->nvar; q->qv_of[q->nvar++] = i; }
  }
  return 0;
}

/* Edges between two constants hold? */
static int constant_edges_hold(const oracle_graph *g, const nq_t *q) {
  for (int k = 0; k < q->n_edges; ++k) {
    int32_t s = q->e[k][0], o = q->e[k][2];
    if (q->cst[s] >= 0 && q->cst[o] >= 0 && !has_triple(g, q->cst[s], q->e[k][1], q->cst[o])) return 0;
  }
  return 1;
}

/* ------------------------------------------------ backtracking evaluator */
/* Row digest: an order-independent summary of a bag of rows, for comparing
 * results too large to store. A row (v_0..v_{k-1}) of width k hashes to
 *   h_0 = k,  h_{i+1} = mix64(h_i + 0x9E3779B97F4A7C15 + (uint32)v_i),  hash = h_k,
 * where mix64 is the output function of the splitmix64 generator (Steele, Lea
 * and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).
 * The digest of a bag is (count, sum of hashes mod 2^64, XOR of hashes). */
static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* State shared by the workers of one evaluation (several threads: timing mode). */
typedef struct {
  atomic_llong work;              /* candidate visits, flushed in batches of 4096 */
  atomic_int abort;
  atomic_llong next;              /* next root-candidate chunk */
  int64_t work_cap;               /* 0 = unlimited */
} shared_t;

typedef struct {
  const oracle_graph *g; const nq_t *q; shared_t *sh;
  int32_t order[OR_MAXQV];        /* query vertices (variables) in binding order */
  int32_t val[OR_MAXQV];          /* current value per query vertex (constants preset) */
  uint8_t bound[OR_MAXQV];
  int32_t restrict_qv; const uint8_t *restrict_mask;
  int64_t count; int32_t *rows; int64_t rows_cap;
  int digest; uint64_t hsum, hxor;
  const uint8_t *dom;             /* support-filter domains (NULL: none) */
  int64_t work; int aborted;
} bt_t;

static int edges_hold_at(bt_t *B, int32_t x) {
  const nq_t *q = B->q;
  for (int k = 0; k < q->n_edges; ++k) {
    int32_t s = q->e[k][0], o = q->e[k][2];
    if (s != x && o != x) continue;
    if (!B->bound[s] || !B->bound[o]) continue;
    if (!has_triple(B->g, B->val[s], q->e[k][1], B->val[o])) return 0;
  }
  return 1;
}

static void emit(bt_t *B) {
  const nq_t *q = B->q;
  if (B->rows && B->count < B->rows_cap) {
    int32_t *r = B->rows + (size_t)B->count * q->nvar;
    for (int v = 0; v < q->nvar; ++v) r[v] = B->val[q->qv_of[v]];
  }
  if (B->digest) {
    uint64_t h = (uint64_t)q->nvar;
    for (int v = 0; v < q->nvar; ++v) h = mix64(h + 0x9E3779B97F4A7C15ull + (uint64_t)(uint32_t)B->val[q->qv_of[v]]);
    B->hsum += h;
    B->hxor ^= h;
  }
  B->count++;
}

/* One candidate visit against the work cap; returns 1 when the evaluation must stop. */
static int tick(bt_t *B) {
  shared_t *sh = B->sh;
  if (sh->work_cap && (++B->work & 4095) == 0 && atomic_fetch_add(&sh->work, 4096) + 4096 > sh->work_cap)
    atomic_store(&sh->abort, 1);
  if (atomic_load_explicit(&sh->abort, memory_order_relaxed)) { B->aborted = 1; return 1; }
  return 0;
}

/* Candidates of variable x: the label-p neighbours of the bound endpoint of its
 * first edge to a bound query vertex (a constant or an earlier variable); NULL
 * with *cnt = N when no such edge exists (every vertex is a candidate). */
static const okey *candidates(const bt_t *B, int32_t x, int64_t *cnt) {
  const nq_t *q = B->q;
  for (int k = 0; k < q->n_edges; ++k) {
    int32_t s = q->e[k][0], o = q->e[k][2];
    if (s == x && o != x && B->bound[o]) return adj(B->g, B->val[o], q->e[k][1], 1, cnt);
    if (o == x && s != x && B->bound[s]) return adj(B->g, B->val[s], q->e[k][1], 0, cnt);
  }
  *cnt = B->g->n;
  return NULL;
}

static void assign(bt_t *B, int i);

/* Bind order[i] to candidates [lo, hi) of its candidate list in turn, check every
 * edge that becomes fully bound, and go on with the next variable. */
static void assign_range(bt_t *B, int i, const okey *nb, int64_t lo, int64_t hi) {
  int32_t x = B->order[i];
  B->bound[x] = 1;
  for (int64_t t = lo; t < hi; ++t) {
    if (tick(B)) break;
    int32_t c = nb ? key_nbr(nb[t]) : (int32_t)t;
    if (x == B->restrict_qv && !B->restrict_mask[c]) continue;
    if (B->dom && !B->dom[(size_t)B->q->var_of[x] * (size_t)B->g->n + (size_t)c]) continue;
    B->val[x] = c;
    if (edges_hold_at(B, x)) assign(B, i + 1);
  }
  B->bound[x] = 0;
}

static void assign(bt_t *B, int i) {
  if (B->aborted) return;
  if (i == B->q->nvar) { emit(B); return; }
  int64_t cnt;
  const okey *nb = candidates(B, B->order[i], &cnt);
  assign_range(B, i, nb, 0, cnt);
}

/* Default order: breadth-first over the undirected query graph, starting from
 * the lowest-index variable adjacent to a constant (else the lowest-index
 * variable), restarting from the lowest unvisited variable for each further
 * component. */
static void default_order(const nq_t *q, int32_t *order) {
  uint8_t seen[OR_MAXQV] = {0};
  int head = 0, tail = 0;
  int32_t start = -1;
  for (int v = 0; v < q->n_qv && start < 0; ++v) {
    if (q->cst[v] >= 0) continue;
    for (int k = 0; k < q->n_edges; ++k) {
      int32_t s = q->e[k][0], o = q->e[k][2];
      if ((s == v && q->cst[o] >= 0) || (o == v && q->cst[s] >= 0)) { start = v; break; }
    }
  }
  for (;;) {
    if (start < 0) for (int v = 0; v < q->n_qv; ++v) if (q->cst[v] < 0 && !seen[v]) { start = v; break; }
    if (start < 0) break;
    seen[start] = 1; order[tail++] = start; start = -1;
    while (head < tail) {
      int32_t v = order[head++];
      for (int k = 0; k < q->n_edges; ++k) {
        int32_t s = q->e[k][0], o = q->e[k][2], w = -1;
        if (s == v) w = o; else if (o == v) w = s;
        if (w >= 0 && q->cst[w] < 0 && !seen[w]) { seen[w] = 1; order[tail++] = w; }
      }
    }
  }
}

static int cmp_rows_k;
static int cmp_rows(const void *x, const void *y) {
  const int32_t *a = (const int32_t *)x, *b = (const int32_t *)y;
  for (int i = 0; i < cmp_rows_k; ++i) if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return 0;
}

/* Common set-up of an evaluation: normalised query, binding order, constants. */
static int setup(const oracle_graph *g, int32_t n_qv, const int32_t *qv_const, int32_t n_edges, const int32_t *edges,
                 const int32_t *order, nq_t *q, bt_t *B) {
  int rc = normalise(g, n_qv, qv_const, n_edges, edges, q);
  if (rc) return rc;
  memset(B, 0, sizeof *B);
  B->g = g; B->q = q; B->restrict_qv = -1;
  if (order) {
    uint8_t seen[OR_MAXQV] = {0};
    for (int i = 0; i < q->nvar; ++i) {
      int32_t v = order[i];
      if (v < 0 || v >= n_qv || q->cst[v] >= 0 || seen[v]) return -3;
      seen[v] = 1; B->order[i] = v;
    }
  } else {
    default_order(q, B->order);
  }
  for (int v = 0; v < n_qv; ++v) if (q->cst[v] >= 0) { B->bound[v] = 1; B->val[v] = q->cst[v]; }
  return 0;
}

/* Evaluate a query.
 *  order: binding order as query-vertex indices of every variable, or NULL for the default.
 *  restrict_qv / restrict_mask: optionally keep only rows whose query vertex restrict_qv takes
 *    a value c with restrict_mask[c] != 0 (restrict_qv < 0: no restriction).
 *  rows: if non-NULL, up to rows_cap rows of width nvar are written, sorted lexicographically.
 *  work_cap: 0 = unlimited; else abort after about that many candidate visits (returns -4).
 * Returns 0 ok, -1 malformed query, -2 out of range, -3 bad order, -4 aborted on work cap. */
int or_eval(const oracle_graph *g, int32_t n_qv, const int32_t *qv_const, int32_t n_edges, const int32_t *edges,
            const int32_t *order, int32_t restrict_qv, const uint8_t *restrict_mask,
            int64_t *count, int32_t *rows, int64_t rows_cap, int64_t work_cap, int32_t *n_vars_out) {
  nq_t q; bt_t B; shared_t sh;
  int rc = setup(g, n_qv, qv_const, n_edges, edges, order, &q, &B);
  if (rc) return rc;
  if (n_vars_out) *n_vars_out = q.nvar;
  atomic_init(&sh.work, 0); atomic_init(&sh.abort, 0); atomic_init(&sh.next, 0); sh.work_cap = work_cap;
  B.sh = &sh; B.rows = rows; B.rows_cap = rows_cap;
  B.restrict_qv = (restrict_qv >= 0 && restrict_mask) ? restrict_qv : -1; B.restrict_mask = restrict_mask;
  *count = 0;
  if (!constant_edges_hold(g, &q)) return 0;
  assign(&B, 0);
  if (B.aborted) return -4;
  *count = B.count;
  if (rows && q.nvar > 0) {
    int64_t nr = B.count < rows_cap ? B.count : rows_cap;
    cmp_rows_k = q.nvar;
    qsort(rows, (size_t)nr, sizeof(int32_t) * q.nvar, cmp_rows);
  }
  return 0;
}

/* ------------------------------------------------ support filter */
static void par_for(int64_t n, int nthreads, void (*fn)(void *, int64_t, int64_t), void *ctx);
/* Arc consistency (Mackworth, "Consistency in networks of relations", 1977):
 * every variable x gets a domain D(x), initially every vertex; for each edge
 * (a, p, b) a value v stays in D(a) only if some triple (v, p, u) has u in D(b)
 * (u = the constant when b is one; u = v for a self loop), and symmetrically
 * for D(b); the edges are swept until no domain changes. A row is an
 * assignment under which every edge is a triple, so each of its values has
 * that support in every sweep: no row is lost, and none is added (the domains
 * only restrict candidates that the backtracking still checks edge by edge).
 * The filter saves search work only: on acyclic queries nearly every partial
 * assignment then extends to a row. */
/* One narrowing pass of D(mine) by the edge (a, p, b); side 0 along the out-rows
 * (a, p, .), side 1 along the in-rows (., p, b). Each v is decided alone (the
 * other end's domain is not written in the pass), so the vertices may be split
 * over threads. */
typedef struct {
  const oracle_graph *g; const nq_t *q; int32_t a, p, b, side;
  uint8_t *d; const uint8_t *dother; int32_t other_const; atomic_int changed;
} sf_pass;

static void sf_run(void *arg, int64_t lo, int64_t hi) {
  sf_pass *S = (sf_pass *)arg;
  int changed = 0;
  for (int64_t v = lo; v < hi; ++v) {
    if (!S->d[v]) continue;
    int64_t cnt;
    const okey *nb = adj(S->g, (int32_t)v, S->p, S->side, &cnt);
    int ok = 0;
    for (int64_t t = 0; t < cnt && !ok; ++t) {
      const int32_t u = key_nbr(nb[t]);
      if (S->a == S->b) ok = (u == v);
      else ok = S->dother ? S->dother[u] : (u == S->other_const);
    }
    if (!ok) { S->d[v] = 0; changed = 1; }
  }
  if (changed) atomic_store(&S->changed, 1);
}

/* dom[var * n + v]: 1 while v may still take variable rank var. */
static uint8_t *support_filter(const oracle_graph *g, const nq_t *q, int nthreads) {
  const int64_t n = g->n;
  uint8_t *dom = (uint8_t *)malloc((size_t)(q->nvar ? q->nvar : 1) * (size_t)(n ? n : 1));
  memset(dom, 1, (size_t)q->nvar * (size_t)n);
  int changed = 1;
  while (changed) {
    changed = 0;
    for (int k = 0; k < q->n_edges; ++k) {
      const int32_t a = q->e[k][0], p = q->e[k][1], b = q->e[k][2];
      for (int side = 0; side < 2; ++side) {
        const int32_t mine = side ? b : a, other = side ? a : b;
        if (q->cst[mine] >= 0 || (side && a == b)) continue;
        sf_pass S;
        S.g = g; S.q = q; S.a = a; S.p = p; S.b = b; S.side = side;
        S.d = dom + (size_t)q->var_of[mine] * n;
        S.dother = (q->cst[other] >= 0 || mine == other) ? NULL : dom + (size_t)q->var_of[other] * n;
        S.other_const = q->cst[other];
        atomic_init(&S.changed, 0);
        par_for(n, nthreads, sf_run, &S);
        changed |= atomic_load(&S.changed);
      }
    }
  }
  return dom;
}

/* ------------------------------------------------ digest, on all host cores */
typedef struct { bt_t B; const okey *nb; int64_t ncand, chunk; } worker_t;

static void *worker_main(void *arg) {
  worker_t *w = (worker_t *)arg;
  bt_t *B = &w->B;
  for (;;) {
    int64_t c = atomic_fetch_add(&B->sh->next, 1);
    int64_t lo = c * w->chunk;
    if (lo >= w->ncand || B->aborted) break;
    int64_t hi = lo + w->chunk < w->ncand ? lo + w->chunk : w->ncand;
    assign_range(B, 0, w->nb, lo, hi);
  }
  return NULL;
}

/* Count and row digest of a query without storing rows. The first variable's
 * candidates are split into chunks that nthreads threads take in turn, each
 * running the same backtracking below its chunk (nthreads <= 1: the calling
 * thread alone, the plain evaluation). filter != 0 first narrows every
 * variable's candidates by the support filter above. work_cap bounds the
 * candidate visits of all threads together (0 = unlimited). Returns as or_eval. */
int or_eval_digest(oracle_graph *g, int32_t n_qv, const int32_t *qv_const, int32_t n_edges,
                   const int32_t *edges, const int32_t *order, int32_t nthreads, int32_t filter, int64_t work_cap,
                   int64_t *count, uint64_t *hsum, uint64_t *hxor) {
  nq_t q; bt_t B; shared_t sh;
  int rc = setup(g, n_qv, qv_const, n_edges, edges, order, &q, &B);
  if (rc) return rc;
  atomic_init(&sh.work, 0); atomic_init(&sh.abort, 0); atomic_init(&sh.next, 0); sh.work_cap = work_cap;
  B.sh = &sh; B.digest = 1;
  *count = 0; *hsum = 0; *hxor = 0;
  if (!constant_edges_hold(g, &q)) return 0;
  uint8_t *dom = (filter && q.nvar > 0) ? support_filter(g, &q, nthreads) : NULL;
  B.dom = dom;
  if (q.nvar == 0 || nthreads <= 1) {
    assign(&B, 0);
    free(dom);
    if (B.aborted) return -4;
    *count = B.count; *hsum = B.hsum; *hxor = B.hxor;
    return 0;
  }
  int64_t ncand;
  const okey *nb = candidates(&B, B.order[0], &ncand);
  if (nthreads > 256) nthreads = 256;
  worker_t *w = (worker_t *)calloc((size_t)nthreads, sizeof(worker_t));
  pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
  int64_t chunk = ncand / ((int64_t)nthreads * 64);
  if (chunk < 1) chunk = 1;
  int started = 0;
  for (int t = 0; t < nthreads; ++t) {
    w[t].B = B; w[t].nb = nb; w[t].ncand = ncand; w[t].chunk = chunk;
    if (pthread_create(&th[t], NULL, worker_main, &w[t]) != 0) break;
    started++;
  }
  if (started == 0) worker_main(&w[0]);   /* no thread could be started: run the chunks here */
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  int aborted = atomic_load(&sh.abort);
  for (int t = 0; t < (started ? started : 1); ++t) {
    aborted |= w[t].B.aborted;
    *count += w[t].B.count; *hsum += w[t].B.hsum; *hxor ^= w[t].B.hxor;
  }
  free(w); free(th); free(dom);
  if (aborted) { *count = 0; *hsum = 0; *hxor = 0; return -4; }
  return 0;
}

/* ------------------------------------------------ exact counting (acyclic) */
typedef unsigned __int128 u128;
#define U128_CAP (((u128)1) << 120)
static u128 sat_add(u128 a, u128 b) { u128 s = a + b; return s > U128_CAP ? U128_CAP : s; }
static u128 sat_mul(u128 a, u128 b) {
  if (a == 0 || b == 0) return 0;
  if (a > U128_CAP / b) return U128_CAP;
  return a * b;
}

/* pair constraint between variables u and v: list of (label, dir) where dir 0 means (u, p, v), 1 means (v, p, u) */
typedef struct { int32_t u, v, n; int32_t lab[OR_MAXE], dir[OR_MAXE]; } bundle_t;

/* does value cu of u and cv of v satisfy every edge of the bundle? */
static int bundle_holds(const oracle_graph *g, const bundle_t *b, int32_t cu, int32_t cv) {
  for (int i = 0; i < b->n; ++i) {
    int ok = b->dir[i] == 0 ? has_triple(g, cu, b->lab[i], cv) : has_triple(g, cv, b->lab[i], cu);
    if (!ok) return 0;
  }
  return 1;
}

/* unary constraints of query vertex x: self loops and edges to constants */
static int unary_holds(const oracle_graph *g, const nq_t *q, int32_t x, int32_t c) {
  for (int k = 0; k < q->n_edges; ++k) {
    int32_t s = q->e[k][0], p = q->e[k][1], o = q->e[k][2];
    if (s == x && o == x) { if (!has_triple(g, c, p, c)) return 0; }
    else if (s == x && q->cst[o] >= 0) { if (!has_triple(g, c, p, q->cst[o])) return 0; }
    else if (o == x && q->cst[s] >= 0) { if (!has_triple(g, q->cst[s], p, c)) return 0; }
  }
  return 1;
}

typedef struct { const oracle_graph *g; const nq_t *q; bundle_t *B; int nb; uint8_t *done; int nthreads; } dp_t;

/* The vertex loops below are independent per vertex c; with several threads
 * each takes a contiguous range of c (same values, any thread count). */
typedef struct { void (*fn)(void *, int64_t, int64_t); void *ctx; int64_t lo, hi; } par_job;
static void *par_main(void *a) { par_job *j = (par_job *)a; j->fn(j->ctx, j->lo, j->hi); return NULL; }
static void par_for(int64_t n, int nthreads, void (*fn)(void *, int64_t, int64_t), void *ctx) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  par_job jobs[64];
  pthread_t th[64];
  int running[64] = {0};
  for (int t = 0; t < nthreads; ++t) {
    jobs[t].fn = fn; jobs[t].ctx = ctx; jobs[t].lo = n * t / nthreads; jobs[t].hi = n * (t + 1) / nthreads;
    running[t] = nthreads > 1 && pthread_create(&th[t], NULL, par_main, &jobs[t]) == 0;
    if (!running[t]) par_main(&jobs[t]);
  }
  for (int t = 0; t < nthreads; ++t) if (running[t]) pthread_join(th[t], NULL);
}

typedef struct { dp_t *D; int32_t x; u128 *msg; const u128 *cm; const bundle_t *b; int x_is_u, out_from_x; } dp_step;

static void dp_unary(void *a, int64_t lo, int64_t hi) {
  dp_step *S = (dp_step *)a;
  for (int64_t c = lo; c < hi; ++c) S->msg[c] = unary_holds(S->D->g, S->D->q, S->x, (int32_t)c) ? 1 : 0;
}

/* msg[c] *= sum over values d of the child w adjacent to c through the bundle's first
 * edge (oriented from x) that satisfy the bundle's other edges, of cm[d] */
static void dp_combine(void *a, int64_t lo, int64_t hi) {
  dp_step *S = (dp_step *)a;
  const oracle_graph *g = S->D->g;
  const bundle_t *b = S->b;
  const int32_t p0 = b->lab[0];
  for (int64_t c = lo; c < hi; ++c) {
    if (!S->msg[c]) continue;
    u128 s = 0;
    int64_t cnt;
    const okey *nb = adj(g, (int32_t)c, p0, S->out_from_x ? 0 : 1, &cnt);
    for (int64_t t = 0; t < cnt; ++t) {
      int32_t d = key_nbr(nb[t]);
      if (!S->cm[d]) continue;
      int ok = S->x_is_u ? bundle_holds(g, b, (int32_t)c, d) : bundle_holds(g, b, d, (int32_t)c);
      if (ok) s = sat_add(s, S->cm[d]);
    }
    S->msg[c] = sat_mul(S->msg[c], s);
  }
}

/* message of subtree rooted at x (entered from parent bundle pb, -1 for root): msg[c] for all c */
static u128 *dp_message(dp_t *D, int32_t x, int pb) {
  const oracle_graph *g = D->g;
  u128 *msg = (u128 *)malloc(sizeof(u128) * (size_t)g->n);
  dp_step S = {D, x, msg, NULL, NULL, 0, 0};
  par_for(g->n, D->nthreads, dp_unary, &S);
  D->done[x] = 1;
  for (int bi = 0; bi < D->nb; ++bi) {
    if (bi == pb) continue;
    bundle_t *b = &D->B[bi];
    int32_t w;
    if (b->u == x) w = b->v; else if (b->v == x) w = b->u; else continue;
    u128 *cm = dp_message(D, w, bi);
    /* first edge, oriented from x: dir 0 with x == u means (x, p, w): neighbours of c along out-edges */
    S.cm = cm;
    S.b = b;
    S.x_is_u = (b->u == x);
    S.out_from_x = S.x_is_u ? (b->dir[0] == 0) : (b->dir[0] == 1);
    par_for(g->n, D->nthreads, dp_combine, &S);
    free(cm);
  }
  return msg;
}

/* Exact count of an acyclic query (the variable graph, after bundling parallel
 * edges, is a forest). Returns 0 ok, -1 malformed, -2 out of range, -5 cyclic.
 * *saturated is set when the count exceeds 2^63-1 (then *count = INT64_MAX). */
int or_count_acyclic(const oracle_graph *g, int32_t n_qv, const int32_t *qv_const, int32_t n_edges,
                     const int32_t *edges, int32_t nthreads, int64_t *count, int32_t *saturated) {
  nq_t q;
  int rc = normalise(g, n_qv, qv_const, n_edges, edges, &q);
  if (rc) return rc;
  *count = 0; if (saturated) *saturated = 0;
  if (!constant_edges_hold(g, &q)) return 0;
  bundle_t *B = (bundle_t *)calloc(OR_MAXE, sizeof(bundle_t));
  int nb = 0;
  for (int k = 0; k < q.n_edges; ++k) {
    int32_t s = q.e[k][0], p = q.e[k][1], o = q.e[k][2];
    if (s == o || q.cst[s] >= 0 || q.cst[o] >= 0) continue;   /* unary */
    int found = -1;
    for (int j = 0; j < nb; ++j)
      if ((B[j].u == s && B[j].v == o) || (B[j].u == o && B[j].v == s)) found = j;
    if (found < 0) { found = nb++; B[found].u = s; B[found].v = o; }
    bundle_t *b = &B[found];
    b->lab[b->n] = p; b->dir[b->n] = (b->u == s) ? 0 : 1; b->n++;
  }
  /* forest test: union-find over variables */
  int32_t parent[OR_MAXQV];
  for (int i = 0; i < n_qv; ++i) parent[i] = i;
  for (int j = 0; j < nb; ++j) {
    int32_t a = B[j].u, b = B[j].v;
    while (parent[a] != a) a = parent[a];
    while (parent[b] != b) b = parent[b];
    if (a == b) { free(B); return -5; }
    parent[a] = b;
  }
  uint8_t done[OR_MAXQV] = {0};
  dp_t D = {g, &q, B, nb, done, nthreads};
  u128 total = 1;
  for (int x = 0; x < n_qv; ++x) {
    if (q.cst[x] >= 0 || done[x]) continue;
    u128 *msg = dp_message(&D, x, -1);
    u128 s = 0;
    for (int64_t c = 0; c < g->n; ++c) s = sat_add(s, msg[c]);
    free(msg);
    total = sat_mul(total, s);
  }
  free(B);
  if (total > (u128)INT64_MAX) { *count = INT64_MAX; if (saturated) *saturated = 1; }
  else *count = (int64_t)total;
  return 0;
}
