/*
 * Seeded synthetic RDF workloads: graphs, query graphs and arrival traces.
 *
 * This module only draws inputs. It evaluates no query and holds none of the
 * engine's or the oracle's arithmetic; both sides read the arrays it writes.
 *
 * Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), counter = (draw index lo, draw index
 * hi, stream tag, block), key = (seed lo, seed hi). Every draw is a pure
 * function of (seed, tag, index), so results do not depend on thread count.
 *
 * Triples are int32 (s, p, o) with s, o in [0, n) and p in [1, P]: subjects and
 * objects are 0-based and predicates 1-based, as in the paper's encoding step
 * of the LSpM storage (Section 6.2.1). A dataset is a set of triples
 * (Section 2.2.1), so every generator removes duplicates, keeping first
 * occurrences in draw order, until exactly m distinct triples exist.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- Philox */
#define PH_M0 0xD2511F53u
#define PH_M1 0xCD9E8D57u
#define PH_W0 0x9E3779B9u
#define PH_W1 0xBB67AE85u

void gsw_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += PH_W0; k1 += PH_W1; }
    uint64_t p0 = (uint64_t)PH_M0 * c0;
    uint64_t p1 = (uint64_t)PH_M1 * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static inline void ph_block(uint64_t seed, uint32_t tag, uint64_t idx, uint32_t blk, uint32_t out[4]) {
  uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), tag, blk};
  uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  gsw_philox4x32_10(c, k, out);
}

/* A sequential stream of 32-bit words: block after block of one counter. */
typedef struct { uint64_t seed, idx; uint32_t tag, blk, pos, buf[4]; } ph_stream;

static void ps_init(ph_stream *s, uint64_t seed, uint32_t tag, uint64_t idx) {
  s->seed = seed; s->tag = tag; s->idx = idx; s->blk = 0; s->pos = 4;
}
static uint32_t ps_next(ph_stream *s) {
  if (s->pos == 4) { ph_block(s->seed, s->tag, s->idx, s->blk++, s->buf); s->pos = 0; }
  return s->buf[s->pos++];
}
/* Lemire's multiply-shift map of a 32-bit word onto [0, n), n <= 2^32. */
static inline uint64_t bounded(uint32_t r, uint64_t n) { return ((uint64_t)r * n) >> 32; }
static uint64_t ps_below(ph_stream *s, uint64_t n) { return bounded(ps_next(s), n); }
static double ps_unit(ph_stream *s) {               /* uniform in [0, 1) with 53 bits */
  uint64_t a = ps_next(s) >> 5, b = ps_next(s) >> 6;
  return (double)(a * 67108864.0 + b) * (1.0 / 9007199254740992.0);
}

/* splitmix64 finaliser (Steele, Lea, Flood 2014): a fixed 64-bit mixer. */
static inline uint64_t mix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

enum { TAG_UNIFORM = 1, TAG_CL = 2, TAG_PERM = 3, TAG_QUERY = 16, TAG_ARRIVAL = 64 };

/* --------------------------------------------------- alias tables (Vose) */
typedef struct { int64_t n; uint32_t *thr; int32_t *alias; } alias_t;

static int alias_build(alias_t *a, const double *w, int64_t n) {
  a->n = n;
  a->thr = (uint32_t *)malloc(sizeof(uint32_t) * n);
  a->alias = (int32_t *)malloc(sizeof(int32_t) * n);
  double *q = (double *)malloc(sizeof(double) * n);
  int32_t *small = (int32_t *)malloc(sizeof(int32_t) * n), *large = (int32_t *)malloc(sizeof(int32_t) * n);
  if (!a->thr || !a->alias || !q || !small || !large) return -1;
  double sum = 0; for (int64_t i = 0; i < n; ++i) sum += w[i];
  int64_t ns = 0, nl = 0;
  for (int64_t i = 0; i < n; ++i) {
    q[i] = w[i] * (double)n / sum;
    if (q[i] < 1.0) small[ns++] = (int32_t)i; else large[nl++] = (int32_t)i;
  }
  while (ns && nl) {
    int32_t s = small[--ns], l = large[nl - 1];
    a->alias[s] = l;
    a->thr[s] = q[s] >= 1.0 ? 0xFFFFFFFFu : (uint32_t)(q[s] * 4294967296.0);
    q[l] = (q[l] + q[s]) - 1.0;
    if (q[l] < 1.0) { --nl; small[ns++] = l; }
  }
  while (nl) { int32_t l = large[--nl]; a->thr[l] = 0xFFFFFFFFu; a->alias[l] = l; }
  while (ns) { int32_t s = small[--ns]; a->thr[s] = 0xFFFFFFFFu; a->alias[s] = s; }
  free(q); free(small); free(large);
  return 0;
}
static void alias_free(alias_t *a) { free(a->thr); free(a->alias); }
static inline int64_t alias_draw(const alias_t *a, uint32_t r_idx, uint32_t r_coin) {
  int64_t i = (int64_t)bounded(r_idx, (uint64_t)a->n);
  return r_coin < a->thr[i] ? i : a->alias[i];
}

/* ------------------------------------------- arrival-order deduplication */
/* Open addressing over 64 slot ranges ("partitions"), each probed linearly
 * inside its own range. A triple goes to one partition by its hash, and each
 * partition sees the draws in draw order, so the first occurrence of every
 * triple is the one kept however the partitions are spread over threads. */
#define NPART 64
typedef struct { uint32_t s, p, o; } trip_t;
typedef struct { trip_t *slot; uint64_t part_slots; } tset_t;

static inline uint64_t trip_hash(uint32_t s, uint32_t p, uint32_t o) {
  return mix64(((uint64_t)s << 32 | o) ^ mix64((uint64_t)p + 0x51ED27ull));
}
/* A round inserts at most its draws, and only the last round keeps fewer
 * than it inserts, so 2m + 8192 entries bound the set; slots are twice that. */
static int tset_init(tset_t *t, int64_t m) {
  uint64_t per = 64; while (per < (uint64_t)(2 * (2 * m + 8192) / NPART + 64)) per <<= 1;
  t->part_slots = per;
  t->slot = (trip_t *)malloc(sizeof(trip_t) * per * NPART);
  if (!t->slot) return -1;
  memset(t->slot, 0xFF, sizeof(trip_t) * per * NPART);
  return 0;
}
/* returns 1 if inserted (new), 0 if present */
static int tset_insert(tset_t *t, uint64_t h, uint32_t s, uint32_t p, uint32_t o) {
  uint64_t part = h % NPART, mask = t->part_slots - 1, i = (h >> 8) & mask;
  trip_t *base = t->slot + part * t->part_slots;
  for (uint64_t probes = 0; probes < t->part_slots; ++probes) {
    trip_t *e = base + i;
    if (e->s == 0xFFFFFFFFu) { e->s = s; e->p = p; e->o = o; return 1; }
    if (e->s == s && e->p == p && e->o == o) return 0;
    i = (i + 1) & mask;
  }
  return -1;   /* partition full */
}

typedef void (*draw_fn)(const void *ctx, uint64_t idx, int32_t out[3]);

/* Draw triples idx = 0, 1, 2, ... with fn until m distinct ones exist.
 * A draw that returns s < 0 is skipped (rejection failure). */
static int draw_distinct(const void *ctx, draw_fn fn, int64_t m, int32_t *out) {
  tset_t set;
  if (tset_init(&set, m)) return -1;
  int64_t have = 0; uint64_t next = 0;
  while (have < m) {
    int64_t need = m - have, D = need + need / 8 + 4096;
    int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * 3 * D);
    uint64_t *hv = (uint64_t *)malloc(sizeof(uint64_t) * D);
    uint8_t *isnew = (uint8_t *)calloc(D, 1);
    if (!buf || !hv || !isnew) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < D; ++i) {
      fn(ctx, next + (uint64_t)i, buf + 3 * i);
      if (buf[3 * i] >= 0) hv[i] = trip_hash((uint32_t)buf[3 * i], (uint32_t)buf[3 * i + 1], (uint32_t)buf[3 * i + 2]);
    }
    int full = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : full)
    for (int part = 0; part < NPART; ++part)
      for (int64_t i = 0; i < D; ++i)
        if (buf[3 * i] >= 0 && hv[i] % NPART == (uint64_t)part) {
          int r = tset_insert(&set, hv[i], (uint32_t)buf[3 * i], (uint32_t)buf[3 * i + 1], (uint32_t)buf[3 * i + 2]);
          if (r < 0) { full = 1; r = 0; }
          isnew[i] = (uint8_t)r;
        }
    if (full) { free(buf); free(hv); free(isnew); free(set.slot); return -4; }
    for (int64_t i = 0; i < D && have < m; ++i)
      if (isnew[i]) { memcpy(out + 3 * have, buf + 3 * i, 12); ++have; }
    next += (uint64_t)D;
    free(buf); free(hv); free(isnew);
  }
  free(set.slot);
  return 0;
}

/* ------------------------------------------------------- uniform graphs */
typedef struct { uint64_t seed; int64_t n; int32_t P; } uni_ctx;
static void uni_draw(const void *c, uint64_t idx, int32_t out[3]) {
  const uni_ctx *u = (const uni_ctx *)c;
  uint32_t r[4]; ph_block(u->seed, TAG_UNIFORM, idx, 0, r);
  out[0] = (int32_t)bounded(r[0], (uint64_t)u->n);
  out[1] = 1 + (int32_t)bounded(r[2], (uint64_t)u->P);
  out[2] = (int32_t)bounded(r[1], (uint64_t)u->n);
}

/* Subjects and objects uniform over [0, n), predicates uniform over [1, P]. */
int gsw_uniform_graph(uint64_t seed, int64_t n, int32_t P, int64_t m, int32_t *out) {
  if (n <= 0 || n > 2147483647LL || P <= 0 || m < 0) return -2;
  if ((double)m > (double)n * (double)n * (double)P) return -3;
  uni_ctx c = {seed, n, P};
  return draw_distinct(&c, uni_draw, m, out);
}

/* ------------------------------------------------ Chung-Lu power law graphs */
typedef struct {
  uint64_t seed; int64_t n; int32_t P, dom_mod;
  alias_t vw, lab; const int32_t *perm;
} cl_ctx;

static inline int in_domain(uint64_t seed, int32_t p, int32_t v, int32_t mod) {
  if (mod <= 1) return 1;
  return mix64(seed * 0x2545F4914F6CDD1Dull + (uint64_t)p * 0x100000001B3ull + (uint64_t)(uint32_t)v) % (uint64_t)mod == 0;
}

static void cl_draw(const void *c, uint64_t idx, int32_t out[3]) {
  const cl_ctx *g = (const cl_ctx *)c;
  uint32_t r[4]; ph_block(g->seed, TAG_CL, idx, 0, r);
  int32_t s = g->perm[alias_draw(&g->vw, r[0], r[1])];
  int32_t p = 1 + (int32_t)alias_draw(&g->lab, r[2], r[3]);
  for (uint32_t blk = 1; blk <= 48; ++blk) {          /* up to 96 object attempts */
    ph_block(g->seed, TAG_CL, idx, blk, r);
    for (int t = 0; t < 2; ++t) {
      int32_t o = g->perm[alias_draw(&g->vw, r[2 * t], r[2 * t + 1])];
      if (in_domain(g->seed, p, o, g->dom_mod)) { out[0] = s; out[1] = p; out[2] = o; return; }
    }
  }
  out[0] = -1; out[1] = -1; out[2] = -1;
}

/* Tables of a Chung-Lu generator: vertex weight w_i = (i+1)^(-1/(beta-1)),
 * subject and object drawn proportional to weight, vertex ids then shuffled
 * (Fisher-Yates) so that the heavy vertices are spread over the id range.
 * Predicates Zipf(zipf_s) over [1, P]. Each predicate's objects are restricted
 * to the typed domain {v : mix(seed, p, v) mod dom_mod == 0} by rejection
 * (dom_mod = 5 keeps 20%). */
static int cl_init(cl_ctx *c, uint64_t seed, int64_t n, int32_t P, double beta, double zipf_s, int32_t dom_mod) {
  memset(c, 0, sizeof *c);
  double *w = (double *)malloc(sizeof(double) * (size_t)(n > P ? n : P));
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * n);
  if (!w || !perm) { free(w); free(perm); return -1; }
  c->seed = seed; c->n = n; c->P = P; c->dom_mod = dom_mod;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) w[i] = pow((double)(i + 1), -1.0 / (beta - 1.0));
  if (alias_build(&c->vw, w, n)) { free(w); free(perm); return -1; }
  for (int32_t k = 0; k < P; ++k) w[k] = pow((double)(k + 1), -zipf_s);
  if (alias_build(&c->lab, w, P)) { free(w); free(perm); return -1; }
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    uint32_t r[4]; ph_block(seed, TAG_PERM, (uint64_t)i, 0, r);
    int64_t j = (int64_t)((((uint64_t)r[0] << 32) | r[1]) % (uint64_t)(i + 1));
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
  c->perm = perm;
  free(w);
  return 0;
}
static void cl_free(cl_ctx *c) { alias_free(&c->vw); alias_free(&c->lab); free((void *)c->perm); }

/* m distinct Chung-Lu triples: the first distinct ones in draw order. */
int gsw_chunglu_graph(uint64_t seed, int64_t n, int32_t P, int64_t m, double beta, double zipf_s,
                      int32_t dom_mod, int32_t *out) {
  if (n <= 1 || n > 2147483647LL || P <= 0 || m < 0 || beta <= 1.0) return -2;
  cl_ctx c;
  if (cl_init(&c, seed, n, P, beta, zipf_s, dom_mod)) return -1;
  int rc = draw_distinct(&c, cl_draw, m, out);
  cl_free(&c);
  return rc;
}

/* The same draws as a stream, for graphs defined as the distinct triples among
 * a fixed number of draws (too many to deduplicate on the host): a generator
 * holds the tables, gsw_cl_draws writes draws [idx0, idx0 + count) in draw
 * order, leaving out the (rare) draws whose object rejection failed, and
 * returns how many it wrote. */
void *gsw_cl_new(uint64_t seed, int64_t n, int32_t P, double beta, double zipf_s, int32_t dom_mod) {
  if (n <= 1 || n > 2147483647LL || P <= 0 || beta <= 1.0) return NULL;
  cl_ctx *c = (cl_ctx *)malloc(sizeof(cl_ctx));
  if (!c || cl_init(c, seed, n, P, beta, zipf_s, dom_mod)) { free(c); return NULL; }
  return c;
}
void gsw_cl_free(void *h) { if (h) { cl_free((cl_ctx *)h); free(h); } }
/* The generator's tables, for a device twin of cl_draw (gen_dev.hip) that reads
 * copies of them: vertex alias (n thresholds, n aliases), label alias (P, P),
 * vertex permutation (n). */
void gsw_cl_tables(const void *h, const uint32_t **vthr, const int32_t **valias, const uint32_t **lthr,
                   const int32_t **lalias, const int32_t **perm) {
  const cl_ctx *c = (const cl_ctx *)h;
  *vthr = c->vw.thr; *valias = c->vw.alias; *lthr = c->lab.thr; *lalias = c->lab.alias; *perm = c->perm;
}
int64_t gsw_cl_draws(const void *h, uint64_t idx0, int64_t count, int32_t *out) {
  const cl_ctx *c = (const cl_ctx *)h;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i) cl_draw(c, idx0 + (uint64_t)i, out + 3 * i);
  int64_t k = 0;
  for (int64_t i = 0; i < count; ++i)
    if (out[3 * i] >= 0) {
      if (k != i) memcpy(out + 3 * k, out + 3 * i, 12);
      ++k;
    }
  return k;
}

/* --------------------------------------------------------- query graphs */
/* A query record is GSW_QREC int32 words:
 *   [0] n_qv, [1] n_edges, [2 .. 2+GSW_MAXQV) qv_const (-1 = variable),
 *   then GSW_MAXE edges of (src, label, dst) over query-vertex indices. */
#define GSW_MAXQV 16
#define GSW_MAXE 16
#define GSW_QREC (2 + GSW_MAXQV + 3 * GSW_MAXE)
int gsw_query_record_words(void) { return GSW_QREC; }

enum { SHAPE_CHAIN4 = 0, SHAPE_STAR5 = 1, SHAPE_SNOW8 = 2, SHAPE_TRI = 3, SHAPE_C0STAR = 4, SHAPE_MIXED = 5 };

typedef struct {
  int64_t n, m; const int32_t *t;
  int64_t *off;      /* incidence offsets, n+1 */
  int64_t *inc;      /* triple ids incident to each vertex (twice for self loops) */
  int64_t *outoff;   /* out-incidence: ids with s == v */
  int64_t *outinc;
} inc_t;

static int inc_build(inc_t *I, const int32_t *t, int64_t m, int64_t n) {
  I->n = n; I->m = m; I->t = t;
  I->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  I->outoff = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  I->inc = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)(m ? m : 1));
  I->outinc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
  if (!I->off || !I->outoff || !I->inc || !I->outinc) return -1;
  for (int64_t e = 0; e < m; ++e) { I->off[t[3 * e] + 1]++; I->off[t[3 * e + 2] + 1]++; I->outoff[t[3 * e] + 1]++; }
  for (int64_t v = 0; v < n; ++v) { I->off[v + 1] += I->off[v]; I->outoff[v + 1] += I->outoff[v]; }
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n), *ocur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  if (!cur || !ocur) return -1;
  memcpy(cur, I->off, sizeof(int64_t) * n); memcpy(ocur, I->outoff, sizeof(int64_t) * n);
  for (int64_t e = 0; e < m; ++e) {
    I->inc[cur[t[3 * e]]++] = e; I->inc[cur[t[3 * e + 2]]++] = e; I->outinc[ocur[t[3 * e]]++] = e;
  }
  free(cur); free(ocur);
  return 0;
}
static void inc_free(inc_t *I) { free(I->off); free(I->inc); free(I->outoff); free(I->outinc); }

typedef struct {            /* query under construction: query vertices carry a data vertex */
  int nqv, ne; int32_t dv[GSW_MAXQV]; int32_t e[GSW_MAXE][3]; int64_t tid[GSW_MAXE];
} qb_t;

static int qb_add_vertex(qb_t *q, int32_t data_v) { if (q->nqv >= GSW_MAXQV) return -1; q->dv[q->nqv] = data_v; return q->nqv++; }
static int qb_used(const qb_t *q, int64_t tid) { for (int i = 0; i < q->ne; ++i) if (q->tid[i] == tid) return 1; return 0; }
/* add edge for triple `tid`, with query vertex a standing for data vertex dv[a] at one end;
 * the other end becomes query vertex b (new when b < 0). Returns the other query vertex. */
static int qb_add_edge(qb_t *q, const inc_t *I, int64_t tid, int a, int b) {
  const int32_t *tr = I->t + 3 * tid;
  if (q->ne >= GSW_MAXE) return -1;
  int a_is_subj = (tr[0] == q->dv[a]);
  int32_t other = a_is_subj ? tr[2] : tr[0];
  if (b < 0) { b = qb_add_vertex(q, other); if (b < 0) return -1; }
  if (a_is_subj) { q->e[q->ne][0] = a; q->e[q->ne][2] = b; } else { q->e[q->ne][0] = b; q->e[q->ne][2] = a; }
  q->e[q->ne][1] = tr[1]; q->tid[q->ne] = tid; q->ne++;
  return b;
}
static int64_t pick_incident(ph_stream *rs, const inc_t *I, int32_t v) {
  int64_t d = I->off[v + 1] - I->off[v];
  if (d <= 0) return -1;
  return I->inc[I->off[v] + (int64_t)ps_below(rs, (uint64_t)d)];
}
/* a fresh incident triple of query vertex a, not already used by the query */
static int64_t pick_fresh(ph_stream *rs, const inc_t *I, const qb_t *q, int a) {
  for (int tries = 0; tries < 32; ++tries) {
    int64_t t = pick_incident(rs, I, q->dv[a]);
    if (t < 0) return -1;
    if (!qb_used(q, t)) return t;
  }
  return -1;
}
static int32_t start_vertex(ph_stream *rs, const inc_t *I) {   /* endpoint of a uniform triple */
  int64_t e = (int64_t)ps_below(rs, (uint64_t)I->m);
  return I->t[3 * e + (ps_below(rs, 2) ? 2 : 0)];
}

static int gen_shape(ph_stream *rs, const inc_t *I, int shape, qb_t *q) {
  memset(q, 0, sizeof *q);
  if (shape == SHAPE_CHAIN4) {
    int cur = qb_add_vertex(q, start_vertex(rs, I));
    for (int k = 0; k < 4; ++k) {
      int64_t t = pick_fresh(rs, I, q, cur); if (t < 0) return -1;
      cur = qb_add_edge(q, I, t, cur, -1); if (cur < 0) return -1;
    }
    return 0;
  }
  if (shape == SHAPE_STAR5) {
    int c = qb_add_vertex(q, start_vertex(rs, I));
    for (int k = 0; k < 5; ++k) { int64_t t = pick_fresh(rs, I, q, c); if (t < 0 || qb_add_edge(q, I, t, c, -1) < 0) return -1; }
    return 0;
  }
  if (shape == SHAPE_SNOW8) {   /* centre with 3 spokes; spoke ends carry 2, 2 and 1 more edges */
    int c = qb_add_vertex(q, start_vertex(rs, I)), sp[3];
    for (int k = 0; k < 3; ++k) { int64_t t = pick_fresh(rs, I, q, c); if (t < 0) return -1; sp[k] = qb_add_edge(q, I, t, c, -1); if (sp[k] < 0) return -1; }
    static const int fan[3] = {2, 2, 1};
    for (int k = 0; k < 3; ++k)
      for (int f = 0; f < fan[k]; ++f) { int64_t t = pick_fresh(rs, I, q, sp[k]); if (t < 0 || qb_add_edge(q, I, t, sp[k], -1) < 0) return -1; }
    return 0;
  }
  if (shape == SHAPE_TRI) {     /* walk a -> b -> c on distinct data vertices, close with a triple c - a */
    int a = qb_add_vertex(q, start_vertex(rs, I));
    int64_t t = pick_fresh(rs, I, q, a); if (t < 0) return -1;
    int b = qb_add_edge(q, I, t, a, -1);
    t = pick_fresh(rs, I, q, b); if (t < 0) return -1;
    int c = qb_add_edge(q, I, t, b, -1);
    if (q->dv[a] == q->dv[b] || q->dv[b] == q->dv[c] || q->dv[a] == q->dv[c]) return -1;
    int32_t vc = q->dv[c], va = q->dv[a];
    int64_t lo = I->off[vc], hi = I->off[vc + 1], nmatch = 0;
    for (int64_t i = lo; i < hi; ++i) { const int32_t *tr = I->t + 3 * I->inc[i]; if ((tr[0] == vc && tr[2] == va) || (tr[2] == vc && tr[0] == va)) ++nmatch; }
    if (!nmatch) return -1;
    int64_t pick = (int64_t)ps_below(rs, (uint64_t)nmatch);
    for (int64_t i = lo; i < hi; ++i) {
      const int32_t *tr = I->t + 3 * I->inc[i];
      if ((tr[0] == vc && tr[2] == va) || (tr[2] == vc && tr[0] == va)) {
        if (pick-- == 0) {
          if (q->ne >= GSW_MAXE) return -1;
          if (tr[0] == vc) { q->e[q->ne][0] = c; q->e[q->ne][2] = a; } else { q->e[q->ne][0] = a; q->e[q->ne][2] = c; }
          q->e[q->ne][1] = tr[1]; q->tid[q->ne] = I->inc[i]; q->ne++;
          return 0;
        }
      }
    }
    return -1;
  }
  if (shape == SHAPE_C0STAR) {  /* centre with out-degree >= 3, three distinct out-triples */
    for (int tries = 0; tries < 64; ++tries) {
      int32_t v = start_vertex(rs, I);
      int64_t lo = I->outoff[v], d = I->outoff[v + 1] - lo;
      if (d < 3) continue;
      int64_t pick[3]; int k = 0;
      while (k < 3) {
        int64_t j = lo + (int64_t)ps_below(rs, (uint64_t)d), dup = 0;
        for (int z = 0; z < k; ++z) dup |= (pick[z] == j);
        if (!dup) pick[k++] = j;
      }
      memset(q, 0, sizeof *q);
      int c = qb_add_vertex(q, v);
      for (k = 0; k < 3; ++k) qb_add_edge(q, I, I->outinc[pick[k]], c, -1);
      return 0;
    }
    return -1;
  }
  if (shape == SHAPE_MIXED) {   /* random tree of 1..12 edges grown from walk vertices; may close cycles */
    int ne = 1 + (int)ps_below(rs, 12);
    qb_add_vertex(q, start_vertex(rs, I));
    while (q->ne < ne) {
      int a = (int)ps_below(rs, (uint64_t)q->nqv);
      int64_t t = pick_fresh(rs, I, q, a); if (t < 0) return -1;
      const int32_t *tr = I->t + 3 * t;
      int32_t other = (tr[0] == q->dv[a]) ? tr[2] : tr[0];
      int b = -1;
      if (ps_below(rs, 4) == 0)            /* close a cycle when the other end is already a query vertex */
        for (int z = 0; z < q->nqv; ++z) if (z != a && q->dv[z] == other) { b = z; break; }
      if (b < 0 && q->nqv >= GSW_MAXQV) return -1;
      if (qb_add_edge(q, I, t, a, b) < 0) return -1;
    }
    return 0;
  }
  return -1;
}

static void qb_emit(const qb_t *q, const int32_t *is_const, int32_t *rec) {
  memset(rec, 0, sizeof(int32_t) * GSW_QREC);
  rec[0] = q->nqv; rec[1] = q->ne;
  for (int i = 0; i < GSW_MAXQV; ++i) rec[2 + i] = (i < q->nqv && is_const[i]) ? q->dv[i] : -1;
  for (int k = 0; k < q->ne; ++k) for (int z = 0; z < 3; ++z) rec[2 + GSW_MAXQV + 3 * k + z] = q->e[k][z];
}

/* Query graphs from seeded walks on the undirected view of the data graph.
 * Walk positions become distinct query vertices; each edge keeps its triple's
 * label and direction, so every generated query has at least one binding
 * (the walk itself). Constants: for shapes 0-3, with probability const_prob one
 * position other than the centre (the first vertex) is made a constant; shape 4
 * (3-edge star) always makes the third edge's object a constant; shape 5
 * (mixed) makes between 0 and max_consts vertices constants, uniformly.
 * Candidate i is drawn from counter stream (seed, TAG_QUERY + shape, first + i);
 * the walk is retried within that stream until it succeeds. Returns the number
 * of records written (nq unless a stream failed 10000 times). */
/* Non-centre walk positions whose vertex has at most max_deg incident triples
 * (max_deg <= 0: every non-centre position). */
static int light_positions(const inc_t *I, const qb_t *q, int64_t max_deg, int *pos) {
  int k = 0;
  for (int i = 1; i < q->nqv; ++i)
    if (max_deg <= 0 || I->off[q->dv[i] + 1] - I->off[q->dv[i]] <= max_deg) pos[k++] = i;
  return k;
}

/* As gsw_walk_queries, with two more knobs for shapes 0-3: n_consts >= 0 makes
 * exactly that many distinct non-centre positions constants (instead of one
 * with probability const_prob), chosen among the positions whose vertex has at
 * most const_max_deg incident triples when const_max_deg > 0 (a walk with too
 * few such positions is retried): constants of low degree make selective queries. */
int gsw_walk_queries_ex(const int32_t *triples, int64_t m, int64_t n, uint64_t seed, int32_t shape, int64_t first,
                        int32_t nq, double const_prob, int32_t max_consts, int32_t n_consts, int64_t const_max_deg,
                        int32_t *out) {
  if (m <= 0 || n <= 0 || nq < 0) return -2;
  inc_t I;
  if (inc_build(&I, triples, m, n)) return -1;
  int written = 0;
  for (int i = 0; i < nq; ++i) {
    ph_stream rs; ps_init(&rs, seed, (uint32_t)(TAG_QUERY + shape), (uint64_t)(first + i));
    const int exact = n_consts >= 0 && shape != SHAPE_C0STAR && shape != SHAPE_MIXED;
    qb_t q; int ok = 0, pos[GSW_MAXQV], npos = 0;
    for (int tries = 0; tries < 10000 && !ok; ++tries) {
      ok = gen_shape(&rs, &I, shape, &q) == 0;
      if (ok && exact) {
        npos = light_positions(&I, &q, const_max_deg, pos);
        ok = npos >= (n_consts < q.nqv - 1 ? n_consts : q.nqv - 1);
      }
    }
    if (!ok) break;
    int32_t isc[GSW_MAXQV] = {0};
    if (exact) {   /* n_consts distinct positions drawn from the light ones */
      int nc = n_consts < npos ? n_consts : npos;
      for (int k = 0; k < nc; ++k) {
        int z = k + (int)ps_below(&rs, (uint64_t)(npos - k));
        int t = pos[k]; pos[k] = pos[z]; pos[z] = t;
        isc[pos[k]] = 1;
      }
    } else if (shape == SHAPE_C0STAR) {
      isc[q.e[2][2]] = 1;
    } else if (shape == SHAPE_MIXED) {
      int nc = (int)ps_below(&rs, (uint64_t)max_consts + 1);
      if (nc >= q.nqv) nc = q.nqv - 1;
      for (int k = 0; k < nc; ++k) {
        int z = (int)ps_below(&rs, (uint64_t)q.nqv);
        for (int t = 0; t < q.nqv && isc[z]; ++t) z = (z + 1) % q.nqv;
        isc[z] = 1;
      }
    } else if (ps_unit(&rs) < const_prob && q.nqv > 1) {
      isc[1 + (int)ps_below(&rs, (uint64_t)(q.nqv - 1))] = 1;
    }
    qb_emit(&q, isc, out + (size_t)written * GSW_QREC);
    ++written;
  }
  inc_free(&I);
  return written;
}

int gsw_walk_queries(const int32_t *triples, int64_t m, int64_t n, uint64_t seed, int32_t shape,
                     int64_t first, int32_t nq, double const_prob, int32_t max_consts, int32_t *out) {
  return gsw_walk_queries_ex(triples, m, n, seed, shape, first, nq, const_prob, max_consts, -1, 0, out);
}

/* Open-loop Poisson arrival times (seconds from 0) at `rate` per second:
 * exponential gaps by inversion, -ln(1-u)/rate. Returns the count written. */
int64_t gsw_poisson_arrivals(uint64_t seed, double rate, double duration, int64_t cap, double *out) {
  ph_stream rs; ps_init(&rs, seed, TAG_ARRIVAL, 0);
  double t = 0; int64_t k = 0;
  while (k < cap) {
    t += -log(1.0 - ps_unit(&rs)) / rate;
    if (t >= duration) break;
    out[k++] = t;
  }
  return k;
}
