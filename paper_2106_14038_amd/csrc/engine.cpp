// Host engine: loads the light-weight sparse matrix, plans queries, compiles
// their step programs into device tables and drives the per-level launch
// sequence for a whole batch of queries.
#include "engine.hpp"

#include <algorithm>
#include <cstring>

#include "kernels_common.hpp"
#include "lspm.hpp"
#include "query.hpp"

namespace gs {

thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error() { return g_last_error.c_str(); }

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess) {                                                           \
      set_error(std::string("HIP error: ") + hipGetErrorString(_e) + " at " #expr);   \
      return GS_EDEVICE;                                                              \
    }                                                                                 \
  } while (0)

static uint64_t align256(uint64_t x) { return (x + 255ull) & ~255ull; }

void *Engine::dmalloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (opt.alloc) return opt.alloc(opt.alloc_ctx, bytes);
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  return p;
}

void Engine::dfree(void *p) {
  if (!p) return;
  if (opt.free) opt.free(opt.alloc_ctx, p);
  else (void)hipFree(p);
}

void *Engine::pinned(void *&buf, size_t &cap, size_t bytes) {
  if (bytes <= cap && buf) return buf;
  if (buf) (void)hipHostFree(buf);
  buf = nullptr;
  cap = 0;
  size_t want = 1 << 16;
  while (want < bytes) want <<= 1;
  if (hipHostMalloc(&buf, want, hipHostMallocDefault) != hipSuccess) { buf = nullptr; return nullptr; }
  cap = want;
  return buf;
}

Engine::~Engine() {
  (void)hipSetDevice(device);
  if (stream) (void)hipStreamSynchronize(stream);
  if (pin_up) (void)hipHostFree(pin_up);
  if (pin_down) (void)hipHostFree(pin_down);
  for (hipEvent_t e : run_ev) if (e) (void)hipEventDestroy(e);
  for (int o = 0; o < 2; ++o) { dfree(d_ptr[o]); dfree(d_idx[o]); dfree(d_lab[o]); dfree(d_bm[o]); }
  dfree(tree_base);
  dfree(scratch_base);
  dfree(seed_pool);
  dfree(d_arenas);
  for (hipEvent_t e : events) (void)hipEventDestroy(e);
  for (GraphEntry &g : graphs) { (void)hipGraphExecDestroy(g.exec); (void)hipGraphDestroy(g.graph); }
  if (own_stream && stream) (void)hipStreamDestroy(stream);
}

// ------------------------------------------------------------------ loading
// Bytes allocated after the last label: the short-row label search reads the aligned words
// around a row's first eight entries, up to 32 bytes past the row's start.
constexpr size_t kLabelPad = 32;

struct LoadCtx { Engine *E; int64_t n; int32_t P; int64_t words; };

static hipError_t alloc_orientation(void *vctx, int orient, int64_t m2, LspmOut &out) {
  LoadCtx *c = (LoadCtx *)vctx;
  Engine &E = *c->E;
  out.words = c->words;
  E.d_ptr[orient] = E.dmalloc(sizeof(int64_t) * (c->n + 1));
  E.d_idx[orient] = (int32_t *)E.dmalloc(sizeof(int32_t) * std::max<int64_t>(m2, 1));
  E.d_lab[orient] = E.dmalloc(sizeof(uint16_t) * std::max<int64_t>(m2, 1) + kLabelPad);
  E.d_bm[orient] = (uint64_t *)E.dmalloc(sizeof(uint64_t) * c->words * c->P);
  if (!E.d_ptr[orient] || !E.d_idx[orient] || !E.d_lab[orient] || !E.d_bm[orient]) return hipErrorOutOfMemory;
  out.ptr = (int64_t *)E.d_ptr[orient];
  out.idx = E.d_idx[orient];
  out.lab = (uint16_t *)E.d_lab[orient];
  out.bm = E.d_bm[orient];
  return hipSuccess;
}

int load_triples(Engine &E, int64_t n, int32_t P, const gs_triple *t, int64_t m, int mem_kind, const int32_t *keep,
                 int32_t n_keep) {
  if (E.loaded) { set_error("dataset already loaded"); return GS_ESTATE; }
  if (n <= 0 || n > 2147483647LL) { set_error("vertex count must be in [1, 2^31-1]"); return GS_ERANGE; }
  if (P <= 0 || P > 65536) { set_error("label count must be in [1, 65536]"); return GS_ERANGE; }
  if (m < 0 || (m > 0 && !t)) { set_error("bad triple buffer"); return GS_EINVAL; }
  // expansion tiles stage segment positions in 32 bits (see WaveTile)
  if (m > (1ll << 32) - 4096) { set_error("more than 2^32 - 4096 triples"); return GS_EUNSUPPORTED; }
  HIPCHK(hipSetDevice(E.device));
  hipStream_t s = E.stream;
  const int64_t words = (n + 63) / 64;
  const int G = E.grid;
  // temporaries
  std::vector<void *> tmp;
  auto take = [&](size_t bytes) { void *p = E.dmalloc(bytes); tmp.push_back(p); return p; };
  auto release = [&]() { for (void *p : tmp) E.dfree(p); tmp.clear(); };
  const int64_t mm = std::max<int64_t>(m, 1);
  const int32_t *d_trip = (const int32_t *)t;
  if (mem_kind == GS_MEM_HOST && m > 0) {
    int32_t *d = (int32_t *)take(sizeof(gs_triple) * mm);
    if (!d) { release(); set_error("out of device memory for the triples"); return GS_ENOMEM; }
    hipError_t e = hipMemcpyAsync(d, t, sizeof(gs_triple) * m, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) { release(); set_error(hipGetErrorString(e)); return GS_EDEVICE; }
    d_trip = d;
  }
  if (keep && m > 0) {   // only the listed predicates (Section 6.2.1 / 6.2.2, step 1)
    std::vector<uint32_t> km((size_t)P / 32 + 2, 0u);
    for (int32_t k = 0; k < n_keep; ++k) {
      if (keep[k] < 1 || keep[k] > P) { release(); set_error("a kept label is outside [1, n_labels]"); return GS_ERANGE; }
      km[(size_t)keep[k] >> 5] |= 1u << (keep[k] & 31);
    }
    uint32_t *d_keep = (uint32_t *)take(4 * km.size());
    int64_t *parts = (int64_t *)take(8 * (size_t)G + 64);
    int32_t *ferr = (int32_t *)take(64);
    if (!d_keep || !parts || !ferr) { release(); set_error("out of device memory while loading"); return GS_ENOMEM; }
    HIPCHK(hipMemcpyAsync(d_keep, km.data(), 4 * km.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(ferr, 0, 4, s));
    int64_t *d_kept = parts + G;
    HIPCHK(filter_triples(d_trip, m, n, P, d_keep, parts, G, d_kept, ferr, nullptr, s));
    int64_t kept = 0;
    int32_t bad = 0;
    HIPCHK(hipMemcpyAsync(&kept, d_kept, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&bad, ferr, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (bad) { release(); set_error("a triple has s/o outside [0, n) or p outside [1, P]"); return GS_ERANGE; }
    int32_t *d_f = (int32_t *)take(sizeof(gs_triple) * (size_t)std::max<int64_t>(kept, 1));
    if (!d_f) { release(); set_error("out of device memory for the kept triples"); return GS_ENOMEM; }
    HIPCHK(filter_triples(d_trip, m, n, P, d_keep, parts, G, d_kept, ferr, d_f, s));
    d_trip = d_f;
    m = kept;
  }
  const int64_t mk = std::max<int64_t>(m, 1);
  LspmBuildArgs a{};
  a.triples = d_trip; a.m = m; a.n = n; a.P = P; a.grid = G; a.stream = s;
  a.hi0 = (uint64_t *)take(8 * mk); a.hi1 = (uint64_t *)take(8 * mk);
  a.lo0 = (uint32_t *)take(4 * mk); a.lo1 = (uint32_t *)take(4 * mk);
  a.row = (int32_t *)take(4 * mk);
  a.hist = (uint32_t *)take(4 * 256 * (size_t)G);
  a.off = (int64_t *)take(8 * 256 * (size_t)G);
  a.blk = (int64_t *)take(8 * (size_t)G);
  a.total = (int64_t *)take(64);
  a.err = (int32_t *)take(64);
  a.nnz = (int64_t *)take(8 * (size_t)P);
  int64_t *holders0 = (int64_t *)take(8 * (size_t)P), *holders1 = (int64_t *)take(8 * (size_t)P);
  for (void *p : tmp) if (!p) { release(); set_error("out of device memory while loading"); return GS_ENOMEM; }
  HIPCHK(hipMemsetAsync(a.err, 0, 4, s));
  HIPCHK(hipMemsetAsync(a.nnz, 0, 8 * (size_t)P, s));
  LoadCtx ctx{&E, n, P, words};
  a.alloc_out = alloc_orientation;
  a.alloc_ctx = &ctx;
  int64_t m2[2] = {0, 0};
  for (int o = 0; o < 2; ++o) {
    LspmOut out;
    out.holders = o == 0 ? holders0 : holders1;
    hipError_t e = lspm_build_orientation(a, o, out, &m2[o]);
    if (e != hipSuccess) {
      release();
      set_error(e == hipErrorOutOfMemory ? "out of device memory for the matrix" : hipGetErrorString(e));
      return e == hipErrorOutOfMemory ? GS_ENOMEM : GS_EDEVICE;
    }
    if (o == 0) {   // stop early on bad ids
      int32_t err = 0;
      HIPCHK(hipMemcpyAsync(&err, a.err, 4, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (err) {
        release();
        for (int k = 0; k < 2; ++k) {
          E.dfree(E.d_ptr[k]); E.dfree(E.d_idx[k]); E.dfree(E.d_lab[k]); E.dfree(E.d_bm[k]);
          E.d_ptr[k] = nullptr; E.d_idx[k] = nullptr; E.d_lab[k] = nullptr; E.d_bm[k] = nullptr;
        }
        set_error("a triple has s/o outside [0, n) or p outside [1, P]");
        return GS_ERANGE;
      }
    }
  }
  E.stats.n = n;
  E.stats.nnz.assign(P, 0);
  E.stats.rows.assign(P, 0);
  E.stats.cols.assign(P, 0);
  HIPCHK(hipMemcpyAsync(E.stats.nnz.data(), a.nnz, 8 * (size_t)P, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(E.stats.rows.data(), holders0, 8 * (size_t)P, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(E.stats.cols.data(), holders1, 8 * (size_t)P, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  release();
  if (m2[0] != m2[1]) { set_error("orientations disagree on the distinct count"); return GS_EDEVICE; }
  // stored widths: labels in one byte when P <= 256, offsets in four when M < 2^31 (unless wide offsets
  // are asked for); the arrays were built wide and are copied down
  const bool lab8 = P <= 256;
  const bool off32 = m2[0] < (1ll << 31) && E.opt.offset_bytes != 8;
  for (int o = 0; o < 2; ++o) {
    if (off32) {
      int32_t *p32 = (int32_t *)E.dmalloc(sizeof(int32_t) * (n + 1));
      if (!p32) { set_error("out of device memory for the row offsets"); return GS_ENOMEM; }
      HIPCHK(narrow_offsets((const int64_t *)E.d_ptr[o], p32, n + 1, s));
      HIPCHK(hipStreamSynchronize(s));
      E.dfree(E.d_ptr[o]);
      E.d_ptr[o] = p32;
    }
    if (lab8) {
      uint8_t *l8 = (uint8_t *)E.dmalloc(std::max<int64_t>(m2[o], 1) + kLabelPad);
      if (!l8) { set_error("out of device memory for the labels"); return GS_ENOMEM; }
      HIPCHK(narrow_labels((const uint16_t *)E.d_lab[o], l8, m2[o], s));
      HIPCHK(hipStreamSynchronize(s));
      E.dfree(E.d_lab[o]);
      E.d_lab[o] = l8;
    }
  }
  E.lab_bytes = lab8 ? 1 : 2;
  E.off_bytes = off32 ? 4 : 8;
  DevGraph g;
  g.n = n; g.m = m2[0]; g.words = words; g.P = P;
  g.lab8 = lab8 ? 1 : 0;
  g.off32 = off32 ? 1 : 0;
  for (int o = 0; o < 2; ++o) { g.ptr[o] = E.d_ptr[o]; g.idx[o] = E.d_idx[o]; g.lab[o] = E.d_lab[o]; g.bm[o] = E.d_bm[o]; }
  E.g = g;
  E.graph_bytes = 2 * ((uint64_t)(n + 1) * E.off_bytes + (uint64_t)g.m * (4 + E.lab_bytes) +
                       (uint64_t)words * 8 * P);
  E.loaded = true;
  return GS_OK;
}

// ------------------------------------------------------------------ batches
template <class T>
static uint64_t push_bytes(std::vector<char> &buf, const std::vector<T> &v) {
  uint64_t off = align256(buf.size());
  buf.resize(off + sizeof(T) * v.size());
  if (!v.empty()) memcpy(buf.data() + off, v.data(), sizeof(T) * v.size());
  return off;
}

__global__ void k_zero_words(uint64_t *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

__global__ void k_const_only(DevGraph g, const DConst *cc, int n, int64_t *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int64_t ok = 1;
    for (int k = 0; k < n && ok; ++k) {
      int probes = 0;
      ok = seg_has(g, 0, cc[k].a, cc[k].label, cc[k].b, probes);
    }
    *out = ok;
  }
}

hipError_t zero_words(uint64_t *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_words, dim3(64), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_const_only(const DevGraph &g, const DConst *cc, int n, int64_t *out, hipStream_t s) {
  hipLaunchKernelGGL(k_const_only, dim3(1), dim3(64), 0, s, g, cc, n, out);
  return hipGetLastError();
}

static double est_holders(const Engine &E, const FilterRef &f, const std::vector<SeedSpec> &seeds) {
  const LabelStats &st = E.stats;
  if (f.kind == F_LABEL_OUT) return (double)st.rows[f.arg];
  if (f.kind == F_LABEL_IN) return (double)st.cols[f.arg];
  if (f.kind == F_SEED) {
    const SeedSpec &s = seeds[f.arg];
    double h = (double)(s.dir == 0 ? st.rows[s.label] : st.cols[s.label]);
    return h > 0 ? (double)st.nnz[s.label] / h : 0.0;
  }
  return (double)E.g.n;
}

static double avg_seg(const Engine &E, int label, int dir) {
  double h = (double)(dir == 0 ? E.stats.rows[label] : E.stats.cols[label]);
  return h > 0 ? (double)E.stats.nnz[label] / h : 0.0;
}

int plan_query(const Engine &E, const gs_query &q, QInfo &qi, std::string &msg) {
  std::vector<int32_t> e3(3 * (size_t)std::max(q.n_edges, 0));
  if (q.n_edges > 0 && !q.edges) { msg = "query edges missing"; return GS_EINVAL; }
  for (int k = 0; k < q.n_edges; ++k) {
    e3[3 * k] = q.edges[k].src; e3[3 * k + 1] = q.edges[k].label; e3[3 * k + 2] = q.edges[k].dst;
  }
  int rc = normalise_query(q.n_qv, q.qv_const, q.n_edges, e3.data(), E.g.n, E.g.P, qi.nq, msg);
  if (rc == GS_OK)
    rc = build_plan(qi.nq, &E.stats, E.opt.domain_mode != GS_DOMAIN_OFF, qi.plan, msg,
                    E.opt.traversal == GS_TRAVERSAL_DIRECTION);
  qi.zero = rc == GS_OK && qi.plan.n_vars == 0;
  return rc;
}

// Append query qi's step programs to T; its counters and tree levels use slot `slot`.
void compile_query(const Engine &E, QInfo &qi, bool count_only, int slot, Tables &T,
                   const std::function<uint64_t *(bool)> &next_bitmap) {
  const Plan &P = qi.plan;
  const int64_t words = E.g.words;
  qi.slot = slot;
  qi.vr0 = (int32_t)T.var_rank.size();
  T.var_rank.insert(T.var_rank.end(), P.var_rank.begin(), P.var_rank.end());
  qi.step0 = (int32_t)T.steps.size();
  qi.seed0 = (int32_t)T.seeds.size();
  std::vector<int32_t> seed_at(P.seeds.size());
  for (size_t k = 0; k < P.seeds.size(); ++k) {
    seed_at[k] = (int32_t)T.seeds.size();
    T.seeds.push_back({next_bitmap(true), P.seeds[k].c, P.seeds[k].label, P.seeds[k].dir, slot});
  }
  qi.nseed = (int32_t)P.seeds.size();
  qi.dom0 = (int32_t)T.doms.size();
  qi.ndom = (int32_t)P.domains.size();
  std::vector<DDomain> qd(P.domains.size());
  for (size_t k = 0; k < P.domains.size(); ++k) { qd[k].F = next_bitmap(false); qd[k].D = next_bitmap(false); }
  auto filter_ptr = [&](const FilterRef &f) -> const uint64_t * {
    switch (f.kind) {
      case F_LABEL_OUT: return E.g.bm[0] + (int64_t)f.arg * words;
      case F_LABEL_IN: return E.g.bm[1] + (int64_t)f.arg * words;
      case F_SEED: return T.seeds[seed_at[f.arg]].bm;
      default: return qd[f.arg].D;
    }
  };
  auto col_of = [&](int level, int at) {
    if (level == at) return 1;
    const std::vector<int32_t> &c = P.steps[at].carried;
    return 2 + (int)(std::find(c.begin(), c.end(), level) - c.begin());
  };
  // Factorised count (the per-path trees of Section 7.1, Example 7.1, in counting form): when
  // only the count is asked for, trailing levels that are independent leaves (each generated
  // from the segment of an earlier, non-trailing binding and facing no test) are not built:
  // every node of the level before them contributes the product of their segment lengths.
  int j0 = P.n_vars;
  if (count_only) {
    auto leaf = [&](int j, int first) {
      const PlanStep &ps = P.steps[j];
      return ps.kind == STEP_SEG && ps.filters.empty() && ps.checks.empty() && ps.self_labels.empty() &&
             ps.src_level < first;
    };
    for (int f = P.n_vars - 1; f >= 1; --f) {   // the longest suffix [f, n_vars) of such leaves
      bool ok = true;
      for (int j = f; j < P.n_vars && ok; ++j) ok = leaf(j, f);
      if (ok) j0 = f;
    }
    if (P.n_vars - j0 < 2) j0 = P.n_vars;      // one trailing leaf: the last level's own counted form
  }
  qi.nlev = j0 < P.n_vars ? j0 + 1 : P.n_vars;
  qi.factor_lvl = j0 < P.n_vars ? j0 : -1;
  for (int j = 0; j < qi.nlev; ++j) {
    const PlanStep &ps = P.steps[j];
    DStep d{};
    d.kind = ps.kind;
    d.label = ps.label;
    d.dir = ps.dir;
    d.src = ps.kind == STEP_SEG ? col_of(ps.src_level, j - 1) : (ps.kind == STEP_SEG_CONST ? ps.src_const : 0);
    d.filt0 = (int32_t)T.filt.size();
    for (const FilterRef &f : ps.filters) T.filt.push_back(filter_ptr(f));
    d.nfilt = (int32_t)ps.filters.size();
    d.list_nfilt = ps.kind == STEP_LIST ? d.nfilt : 0;
    d.chk0 = (int32_t)T.checks.size();
    for (const CheckRef &c : ps.checks) T.checks.push_back({col_of(c.level, j - 1), c.label, c.dir, 0});
    d.nchk = (int32_t)ps.checks.size();
    d.self0 = (int32_t)T.ints.size();
    for (int32_t l : ps.self_labels) T.ints.push_back(l);
    d.nself = (int32_t)ps.self_labels.size();
    d.copy0 = (int32_t)T.ints.size();
    for (int32_t l : ps.carried) T.ints.push_back(col_of(l, j - 1));
    d.ncopy = (int32_t)ps.carried.size();
    d.ncols_out = (count_only && j == qi.nlev - 1) ? 0 : 2 + d.ncopy;
    if (j == j0 && j0 < P.n_vars) {   // the factor level: this leaf and the ones after it
      d.chk0 = (int32_t)T.checks.size();
      for (int l = j0 + 1; l < P.n_vars; ++l) {
        const PlanStep &pl = P.steps[l];
        T.checks.push_back({col_of(pl.src_level, j0 - 1), pl.label, pl.dir, 0});
      }
      d.nfactor = P.n_vars - 1 - j0;
      d.ncopy = 0;
    }
    d.ncols_prev = j == 0 ? 0 : 2 + (int32_t)P.steps[j - 1].carried.size();
    if (j == 0) {
      d.cc0 = (int32_t)T.cconst.size();
      for (const ConstCheck &c : P.cchecks) T.cconst.push_back({c.a, c.label, c.b, 0});
      d.ncc = (int32_t)P.cchecks.size();
    }
    T.steps.push_back(d);
  }
  for (size_t k = 0; k < P.domains.size(); ++k) {
    const DomainSpec &ds = P.domains[k];
    DDomain &dd = qd[k];
    dd.col = col_of(ds.level, ds.step - 1);
    dd.label = ds.label;
    dd.dir = ds.dir;
    dd.filt0 = (int32_t)T.filt.size();
    double mask = (double)E.g.n;
    for (const FilterRef &f : ds.mask) { T.filt.push_back(filter_ptr(f)); mask = std::min(mask, est_holders(E, f, P.seeds)); }
    dd.nfilt = (int32_t)ds.mask.size();
    dd.mode = E.opt.domain_mode == GS_DOMAIN_PUSH ? 1 : (E.opt.domain_mode == GS_DOMAIN_PULL ? 2 : 0);
    dd.q = slot;
    dd.deg_push = (float)avg_seg(E, ds.label, ds.dir);
    dd.deg_pull = (float)avg_seg(E, ds.label, 1 - ds.dir);
    dd.mask_est = (float)mask;
    dd.theta = E.opt.push_pull_theta > 0 ? E.opt.push_pull_theta : 1.0f;
    T.doms.push_back(dd);
    T.dom_step.push_back(ds.step);
  }
}

// Work lists of one iteration: query qs[i] produces its level `level[i]`.
void build_iteration(const Tables &T, const std::vector<const QInfo *> &qs, const std::vector<int> &level,
                     IterLists &L) {
  L.ents.clear(); L.doms.clear(); L.clears.clear(); L.seeds.clear(); L.has_list = 0; L.has_tested = 0; L.has_checks = 0; L.has_factor = 0; L.has_exact = 0;
  for (size_t i = 0; i < qs.size(); ++i) {
    const QInfo &qi = *qs[i];
    const int t = level[i];
    if (t == 0)
      for (int k = 0; k < qi.nseed; ++k) {
        L.seeds.push_back(T.seeds[qi.seed0 + k]);
        if (!T.seeds_zeroed) L.clears.push_back(T.seeds[qi.seed0 + k].bm);
      }
    DEntry e{qi.slot, t, qi.step0 + t, (int32_t)L.doms.size(), 0, 0};
    for (int k = 0; k < qi.ndom; ++k) {
      if (T.dom_step[qi.dom0 + k] != t) continue;
      L.doms.push_back(T.doms[qi.dom0 + k]);
      L.clears.push_back(T.doms[qi.dom0 + k].F);
      L.clears.push_back(T.doms[qi.dom0 + k].D);
      e.ndom++;
    }
    if (qi.plan.steps[t].kind == STEP_LIST) L.has_list = 1;
    if (t == qi.factor_lvl) L.has_factor = 1;
    {   // the device's test-free rule (no filter beyond a list's own, no check, no self loop), from the plan
      const PlanStep &ps = qi.plan.steps[t];
      const bool filtered = ps.kind == STEP_LIST ? false : !ps.filters.empty();
      if (filtered || !ps.checks.empty() || !ps.self_labels.empty()) L.has_tested = 1;
      if (!ps.checks.empty()) L.has_checks = 1;
      if (!ps.checks.empty() || !ps.self_labels.empty()) L.has_exact = 1;
    }
    L.ents.push_back(e);
  }
}

// Accumulate per-kernel times and algorithmic bytes of one iteration (profiling).
void account_iteration(Engine &E, const hipEvent_t *ev, const IterScalars &I, const IterLists &L, double write_bytes,
                       double children) {
  bool ran[KS_N];
  for (int k = 0; k < KS_N; ++k) ran[k] = true;
  ran[KS_CLEAR] = !L.clears.empty();
  ran[KS_SEED] = !L.seeds.empty();
  ran[KS_LIST_COUNT] = ran[KS_LIST_SCAN] = ran[KS_LIST_WRITE] = L.has_list != 0;
  ran[KS_DOM_FRONTIER] = ran[KS_DOM_PUSH] = ran[KS_DOM_PULL] = !L.doms.empty();
  ran[KS_EXPAND_COUNT] = ran[KS_TILE_OFFSETS] = L.has_tested != 0;
  for (int k = 0; k < KS_N; ++k) {
    if (!ran[k]) continue;
    float kms = 0;
    if (hipEventElapsedTime(&kms, ev[2 * k], ev[2 * k + 1]) != hipSuccess) continue;
    double b = 0, alg = 0;
    const double W = (double)I.w_total, nz = (double)I.nz_total;
    switch (k) {
      case KS_EXPAND_COUNT: {  // tested levels only: ids, staged node records, filter words, parent bindings,
        const double Wt = (double)I.w_tested;   // probes, valid bits
        b = 4 * Wt + 20 * nz * (W > 0 ? Wt / W : 0) + 8.0 * I.ftests + 4.0 * I.ctests + 4.0 * I.probes + Wt / 8;
        // the method's own: each candidate id of a tested level read once, the filter words it tests,
        // the entries the exact checks' searches read
        alg = 4 * Wt + 8.0 * I.ftests + 4.0 * I.probes;
        break;
      }
      case KS_EXPAND_WRITE:   // valid bits, staged node records, candidate ids + copies read + columns written;
                              // the method's own bytes: a candidate id read per entry of an untested level
                              // (a tested level's were read by the count pass) and a tree node (parent,
                              // vertex) written per child
        b = W / 8 + 20 * nz + write_bytes;
        alg = 4 * (W - (double)I.w_tested) + 8 * children;
        break;
      case KS_LOOKUP:         // parent binding, offset pair, segment written (the lookups of cycle-closing
                              // segments at cyclic levels are not counted); the method's own: a tree node
                              // read per parent, the label entries and offset pairs of the segment lookups
        b = 36.0 * I.nodes_total;
        alg = 8.0 * I.nodes_total + (double)E.lab_bytes * I.lk_labels + 2.0 * E.off_bytes * I.lk_lookups;
        break;
      case KS_NZ_WRITE:
        b = 16.0 * I.nodes_total + 20 * nz; break;
      default: break;
    }
    E.kstat[k].launches += 1;
    E.kstat[k].ms += kms;
    E.kstat[k].bytes += b;
    E.kstat[k].alg += alg;
  }
}

int run_batch(Engine &E, const gs_query *qs, int nq, uint32_t flags, std::vector<Result *> &out, double *ms_out) {
  if (!E.loaded) { set_error("no dataset loaded"); return GS_ESTATE; }
  if (E.serving) { set_error("a server is running on this engine"); return GS_ESTATE; }
  if (nq <= 0 || !qs) { set_error("empty batch"); return GS_EINVAL; }
  HIPCHK(hipSetDevice(E.device));
  hipStream_t s = E.stream;
  const bool count_only = flags & GS_COUNT_ONLY;
  const int64_t words = E.g.words;

  // 1. plan every query
  std::vector<QInfo> Q(nq);
  int maxk = 0;
  for (int i = 0; i < nq; ++i) {
    std::string msg;
    int rc = plan_query(E, qs[i], Q[i], msg);
    if (rc != GS_OK) { set_error("query " + std::to_string(i) + ": " + msg); return rc; }
  }

  // 2. compile step programs; domain bitmaps at the front of this run's arena block, seed
  // bitmaps from the engine's zeroed seed pool
  int64_t n_bitmaps = 0, n_seed_bm = 0;
  for (int i = 0; i < nq; ++i) {
    n_bitmaps += 2 * (int64_t)Q[i].plan.domains.size();
    n_seed_bm += (int64_t)Q[i].plan.seeds.size();
  }
  if (n_seed_bm > E.seed_pool_cap || (E.seed_pool_dirty && E.seed_pool)) {
    if (n_seed_bm > E.seed_pool_cap) {
      const int64_t cap = std::max<int64_t>(n_seed_bm, 2 * E.seed_pool_cap);
      E.dfree(E.seed_pool);
      E.seed_pool = nullptr;
      E.seed_pool_cap = 0;
      E.seed_pool = (uint64_t *)E.dmalloc(sizeof(uint64_t) * (size_t)words * (size_t)cap);
      if (!E.seed_pool) { set_error("out of device memory for seed bitmaps"); return GS_ENOMEM; }
      E.seed_pool_cap = cap;
    }
    HIPCHK(hipMemsetAsync(E.seed_pool, 0, sizeof(uint64_t) * (size_t)words * (size_t)E.seed_pool_cap, s));
    E.seed_pool_dirty = false;
  }
  uint64_t off = align256(E.tree_top);
  const uint64_t bm_off = off;
  off += align256((uint64_t)n_bitmaps * words * 8);
  int64_t next_bm = 0, next_seed = 0;
  auto next_bitmap = [&](bool seed) {
    if (seed) return E.seed_pool + (uint64_t)(next_seed++) * words;
    return (uint64_t *)(E.tree_base + bm_off + (uint64_t)(next_bm++) * words * 8);
  };
  Tables T;
  T.seeds_zeroed = true;
  for (int i = 0; i < nq; ++i) {
    compile_query(E, Q[i], count_only, i, T, next_bitmap);
    maxk = std::max(maxk, Q[i].nlev);
  }

  // 3. per-iteration work lists (every query advances one level per iteration)
  std::vector<IterLists> its(maxk);
  std::vector<DEntry> ents;
  std::vector<DDomain> doms;
  std::vector<uint64_t *> clears;
  std::vector<DSeed> seeds;
  std::vector<int32_t> ent_off(maxk + 1, 0), dom_off(maxk + 1, 0), clr_off(maxk + 1, 0), seed_off(maxk + 1, 0);
  int max_e = 1, max_d = 1;
  for (int t = 0; t < maxk; ++t) {
    std::vector<const QInfo *> act;
    std::vector<int> lev;
    for (int i = 0; i < nq; ++i) if (Q[i].nlev > t) { act.push_back(&Q[i]); lev.push_back(t); }
    build_iteration(T, act, lev, its[t]);
    ent_off[t] = (int32_t)ents.size(); dom_off[t] = (int32_t)doms.size();
    clr_off[t] = (int32_t)clears.size(); seed_off[t] = (int32_t)seeds.size();
    ents.insert(ents.end(), its[t].ents.begin(), its[t].ents.end());
    doms.insert(doms.end(), its[t].doms.begin(), its[t].doms.end());
    clears.insert(clears.end(), its[t].clears.begin(), its[t].clears.end());
    seeds.insert(seeds.end(), its[t].seeds.begin(), its[t].seeds.end());
    max_e = std::max(max_e, (int)its[t].ents.size());
    max_d = std::max(max_d, (int)its[t].doms.size());
  }
  ent_off[maxk] = (int32_t)ents.size(); dom_off[maxk] = (int32_t)doms.size();
  clr_off[maxk] = (int32_t)clears.size(); seed_off[maxk] = (int32_t)seeds.size();

  // 4. pack the constant tables
  std::vector<char> buf;
  const uint64_t o_steps = push_bytes(buf, T.steps), o_filt = push_bytes(buf, T.filt), o_chk = push_bytes(buf, T.checks);
  const uint64_t o_ints = push_bytes(buf, T.ints), o_cc = push_bytes(buf, T.cconst), o_seeds = push_bytes(buf, seeds);
  const uint64_t o_doms = push_bytes(buf, doms), o_ents = push_bytes(buf, ents), o_clr = push_bytes(buf, clears);
  const uint64_t o_vr = push_bytes(buf, T.var_rank);
  const uint64_t tab_off = align256(off);
  off = tab_off + align256(buf.size());
  // device-written tables
  const uint64_t o_lvlp = off; off += align256(sizeof(int32_t *) * kMaxLevels * (uint64_t)nq);
  const uint64_t o_lvlc = off; off += align256(sizeof(int32_t *) * kMaxLevels * (uint64_t)nq);
  const uint64_t o_lvln = off; off += align256(sizeof(int64_t) * kMaxLevels * (uint64_t)nq);
  const uint64_t o_qs = off; off += align256(sizeof(int64_t) * QS_N * (uint64_t)nq);
  const uint64_t o_zero = off; off += align256(sizeof(int64_t) * (uint64_t)nq);
  const uint64_t o_flags = off; off += align256(sizeof(int32_t) * RF_N);
  const uint64_t zero_end = off;
  const uint64_t o_fc = off; off += align256(sizeof(int64_t) * max_d);
  const uint64_t o_es = off; off += align256(sizeof(EState) * max_e);
  const uint64_t o_it = off; off += align256(sizeof(IterScalars) * (uint64_t)std::max(maxk, 1));
  const uint64_t o_blk = off; off += align256(sizeof(int64_t) * 4 * (uint64_t)E.grid);
  if (off > E.tree_cap) { set_error("tree arena too small for the batch tables"); return GS_ENOMEM; }
  char *base = E.tree_base;
  auto dp = [&](uint64_t o) { return (void *)(base + o); };
  // the tables and the arena tops go up in one copy each from pinned staging
  DArena ar[2];
  ar[0] = {off, E.tree_cap, 0, 0};
  ar[1] = {0, E.scratch_cap, 0, 0};
  char *up = (char *)E.pinned(E.pin_up, E.pin_up_bytes, align256(buf.size()) + sizeof ar);
  if (!up) { set_error("cannot allocate pinned host staging"); return GS_ENOMEM; }
  memcpy(up, buf.data(), buf.size());
  memcpy(up + align256(buf.size()), ar, sizeof ar);
  HIPCHK(hipMemcpyAsync(base + tab_off, up, buf.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(E.d_arenas, up + align256(buf.size()), sizeof(ar), hipMemcpyHostToDevice, s));

  for (hipEvent_t &e : E.run_ev) if (!e) HIPCHK(hipEventCreate(&e));
  hipEvent_t ev0 = E.run_ev[0], ev1 = E.run_ev[1];

  // 5. iterations
  const bool prof = E.opt.profile_kernels != 0;
  const bool graphs = E.opt.use_graphs != 0 && !prof;
  if (prof) {
    const size_t need = (size_t)2 * KS_N * std::max(maxk, 1);
    while (E.events.size() < need) {
      hipEvent_t ev;
      HIPCHK(hipEventCreate(&ev));
      E.events.push_back(ev);
    }
  }
  std::vector<IterArgs> iargs(maxk);
  for (int t = 0; t < maxk; ++t) {
    IterArgs &A = iargs[t];
    A = IterArgs{};
    A.g = E.g;
    A.ent = (const DEntry *)dp(tab_off + o_ents) + ent_off[t];
    A.E = ent_off[t + 1] - ent_off[t];
    A.S = seed_off[t + 1] - seed_off[t];
    A.D = dom_off[t + 1] - dom_off[t];
    A.nclear = clr_off[t + 1] - clr_off[t];
    A.has_list = its[t].has_list;
    A.has_tested = its[t].has_tested;
    A.has_checks = its[t].has_checks;
    A.has_factor = its[t].has_factor;
    A.has_exact = its[t].has_exact;
    A.grid = E.grid;
    A.wgrid = E.wgrid;
    A.wwaves = E.wwaves;
    A.steps = (const DStep *)dp(tab_off + o_steps);
    A.filt = (const uint64_t *const *)dp(tab_off + o_filt);
    A.checks = (const DCheck *)dp(tab_off + o_chk);
    A.ints = (const int32_t *)dp(tab_off + o_ints);
    A.cconst = (const DConst *)dp(tab_off + o_cc);
    A.seeds = (const DSeed *)dp(tab_off + o_seeds) + seed_off[t];
    A.doms = (const DDomain *)dp(tab_off + o_doms) + dom_off[t];
    A.fcount = (int64_t *)dp(o_fc);
    A.clear = (uint64_t *const *)dp(tab_off + o_clr) + clr_off[t];
    A.es = (EState *)dp(o_es);
    A.it = (IterScalars *)dp(o_it) + t;
    A.lvl_ptr = (int32_t **)dp(o_lvlp);
    A.lvl_cptr = (int32_t **)dp(o_lvlc);
    A.lvl_n = (int64_t *)dp(o_lvln);
    A.qstats = (int64_t *)dp(o_qs);
    A.scratch = E.d_arenas + 1;
    A.scratch_base = E.scratch_base;
    A.tree = E.d_arenas + 0;
    A.tree_base = E.tree_base;
    int64_t *blk = (int64_t *)dp(o_blk);
    A.blk_a = blk; A.blk_b = blk + E.grid; A.blk_off_a = blk + 2 * E.grid; A.blk_off_b = blk + 3 * E.grid;
    A.flags = (int32_t *)dp(o_flags);
  }
  uint64_t *zero_p = (uint64_t *)dp(o_lvlp);
  const int64_t zero_n = (int64_t)((zero_end - o_lvlp) / 8);
  const DSeed *all_seeds = (const DSeed *)dp(tab_off + o_seeds);
  const int32_t n_seeds = (int32_t)seeds.size();
  auto launch_all = [&]() -> hipError_t {
    hipError_t e = zero_words(zero_p, zero_n, s);
    for (int t = 0; t < maxk && e == hipSuccess; ++t)
      e = launch_iteration(iargs[t], s, prof ? &E.events[(size_t)2 * KS_N * t] : nullptr);
    // the seed bitmaps go back to zero: the words the seeds set (after an abort too)
    if (e == hipSuccess && n_seeds > 0) e = launch_unseed(E.g, all_seeds, n_seeds, E.grid, s);
    return e;
  };
  E.seed_pool_dirty = n_seeds > 0;   // until the run has finished: a failure leaves set bits behind
  HIPCHK(hipEventRecord(ev0, s));
  if (graphs) {
    // FNV-1a over every launch argument: equal keys launch identical kernels with identical arguments
    uint64_t key = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
      const unsigned char *c = (const unsigned char *)p;
      for (size_t i = 0; i < n; ++i) { key ^= c[i]; key *= 1099511628211ull; }
    };
    mix(&zero_p, sizeof zero_p); mix(&zero_n, sizeof zero_n); mix(&maxk, sizeof maxk);
    mix(&all_seeds, sizeof all_seeds); mix(&n_seeds, sizeof n_seeds);
    for (const IterArgs &A : iargs) mix(&A, sizeof A);
    Engine::GraphEntry *ge = nullptr;
    for (Engine::GraphEntry &g : E.graphs) if (g.key == key) ge = &g;
    if (!ge) {
      if (E.graphs.size() >= 64) {   // evict the least recently used
        auto it = std::min_element(E.graphs.begin(), E.graphs.end(),
                                   [](const Engine::GraphEntry &a, const Engine::GraphEntry &b) { return a.last_use < b.last_use; });
        (void)hipGraphExecDestroy(it->exec);
        (void)hipGraphDestroy(it->graph);
        E.graphs.erase(it);
      }
      Engine::GraphEntry g{key, nullptr, nullptr, 0};
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      hipError_t e = launch_all();
      hipError_t e2 = hipStreamEndCapture(s, &g.graph);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g.graph) (void)hipGraphDestroy(g.graph);
        set_error(std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        return GS_EDEVICE;
      }
      HIPCHK(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
      E.graphs.push_back(g);
      ge = &E.graphs.back();
      E.graph_builds++;
    } else {
      E.graph_hits++;
    }
    ge->last_use = ++E.graph_clock;
    HIPCHK(hipGraphLaunch(ge->exec, s));
  } else {
    hipError_t e = launch_all();
    if (e != hipSuccess) { set_error(std::string("launch: ") + hipGetErrorString(e)); return GS_EDEVICE; }
  }
  // constant-only queries (no variable): every pattern between constants must hold
  for (int i = 0; i < nq; ++i) {
    if (!Q[i].zero) continue;
    const int ncc = (int)Q[i].plan.cchecks.size();
    std::vector<DConst> cc;
    for (const ConstCheck &c : Q[i].plan.cchecks) cc.push_back({c.a, c.label, c.b, 0});
    DConst *d_cc = (DConst *)E.dmalloc(sizeof(DConst) * std::max(ncc, 1));
    if (!d_cc) { set_error("out of device memory"); return GS_ENOMEM; }
    hipError_t e = hipMemcpyAsync(d_cc, cc.data(), sizeof(DConst) * ncc, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_const_only(E.g, d_cc, ncc, (int64_t *)dp(o_zero) + i, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    E.dfree(d_cc);
    if (e != hipSuccess) { set_error(hipGetErrorString(e)); return GS_EDEVICE; }
  }
  HIPCHK(hipEventRecord(ev1, s));

  // 6. read back sizes and counters: the device-written tables are one contiguous block, copied
  // with the arena tops into pinned staging
  const size_t blk_bytes = zero_end - o_lvlp;
  char *down = (char *)E.pinned(E.pin_down, E.pin_down_bytes, blk_bytes + sizeof ar);
  if (!down) { set_error("cannot allocate pinned host staging"); return GS_ENOMEM; }
  HIPCHK(hipMemcpyAsync(down, dp(o_lvlp), blk_bytes, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(down + blk_bytes, E.d_arenas, sizeof(ar), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  E.seed_pool_dirty = false;
  auto hp = [&](uint64_t o) { return (const void *)(down + (o - o_lvlp)); };
  std::vector<int64_t> lvl_n((size_t)nq * kMaxLevels), qst((size_t)nq * QS_N), zero_res(nq);
  int32_t rflags[RF_N] = {0, 0};
  std::vector<int32_t *> lvl_p((size_t)nq * kMaxLevels), lvl_c((size_t)nq * kMaxLevels);
  memcpy(lvl_n.data(), hp(o_lvln), 8 * lvl_n.size());
  memcpy(lvl_p.data(), hp(o_lvlp), 8 * lvl_p.size());
  memcpy(lvl_c.data(), hp(o_lvlc), 8 * lvl_c.size());
  memcpy(qst.data(), hp(o_qs), 8 * qst.size());
  memcpy(zero_res.data(), hp(o_zero), 8 * zero_res.size());
  memcpy(rflags, hp(o_flags), sizeof(rflags));
  memcpy(ar, down + blk_bytes, sizeof(ar));
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
  if (ms_out) *ms_out = ms;
  if (prof) {
    std::vector<IterScalars> iv(std::max(maxk, 1));
    HIPCHK(hipMemcpy(iv.data(), dp(o_it), sizeof(IterScalars) * iv.size(), hipMemcpyDeviceToHost));
    for (int t = 0; t < maxk; ++t) {
      double wbytes = 0, children = 0;   // rows written this iteration, weighted by the columns each query writes
      for (int i = 0; i < nq; ++i) {
        if (Q[i].nlev <= t) continue;
        const DStep &d = T.steps[Q[i].step0 + t];
        const int64_t c = std::max<int64_t>(lvl_n[(size_t)i * kMaxLevels + t], 0);
        // columns written + copies read + candidate read; CSR levels write no parent column
        const int cols = d.ncols_out - (lvl_c[(size_t)i * kMaxLevels + t] ? 1 : 0);
        if (d.ncols_out > 0) {
          wbytes += (double)c * (4.0 * cols + 4.0 * d.ncopy + 4.0);
          children += (double)c;
        }
      }
      account_iteration(E, &E.events[(size_t)2 * KS_N * t], iv[t], its[t], wbytes, children);
    }
  }
  if (rflags[RF_WRITE]) {
    set_error("device inconsistency: the write pass met output positions beyond a level's count");
    return GS_EDEVICE;
  }
  if (rflags[RF_SCRATCH] || ar[1].overflow) {
    set_error("scratch arena overflow: a level's temporaries exceed the scratch arena");
    return GS_ENOMEM;
  }
  for (int i = 0; i < nq; ++i)
    if (qst[(size_t)i * QS_N + QS_OVERFLOW] == 3) {
      set_error("query " + std::to_string(i) + ": a node's product of leaf segments exceeds 2^50 (count-only factor)");
      return GS_ERANGE;
    }
  for (int i = 0; i < nq; ++i)
    for (int j = 0; j < Q[i].nlev; ++j)
      if (lvl_n[(size_t)i * kMaxLevels + j] < 0) {
        set_error("query " + std::to_string(i) + ": binding tree exceeds the tree arena (level " + std::to_string(j) + ")");
        return GS_ENOMEM;
      }

  // 7. results
  const int run_id = ++E.run_counter;
  for (int i = 0; i < nq; ++i) {
    Result *R = new Result();
    R->eng = &E;
    R->run_id = run_id;
    fill_result(*R, Q[i], count_only, &lvl_p[(size_t)i * kMaxLevels], &lvl_c[(size_t)i * kMaxLevels],
                &lvl_n[(size_t)i * kMaxLevels], &qst[(size_t)i * QS_N], zero_res[i], ms);
    R->d_lvl_ptr = (int32_t **)dp(o_lvlp) + (size_t)i * kMaxLevels;
    R->d_lvl_cptr = (int32_t **)dp(o_lvlc) + (size_t)i * kMaxLevels;
    R->d_lvl_n = (int64_t *)dp(o_lvln) + (size_t)i * kMaxLevels;
    R->d_var_rank = (int32_t *)dp(tab_off + o_vr) + Q[i].vr0;
    out.push_back(R);
  }
  E.tree_top = ar[0].top;
  E.live_results += nq;
  return GS_OK;
}

void fill_result(Result &R, const QInfo &qi, bool count_only, int32_t *const *lvl_p, int32_t *const *lvl_c,
                 const int64_t *lvl_n, const int64_t *c, int64_t zero_res, double ms) {
  const Plan &P = qi.plan;
  R.k = qi.nlev;
  R.n_vars = P.n_vars;
  R.count_only = count_only;
  R.zero_vars = qi.zero;
  R.var_rank = P.var_rank;
  if (qi.zero) {
    R.count = zero_res;
  } else {
    for (int j = 0; j < qi.nlev; ++j) {
      R.lvl_ptr.push_back(lvl_p[j]);
      R.lvl_cptr.push_back(lvl_c[j]);
      R.lvl_n.push_back(lvl_n[j]);
      R.ncols_extra.push_back((int32_t)P.steps[j].carried.size());
    }
    R.count = R.lvl_n.back();
  }
  gs_query_stats &st = R.stats;
  memset(&st, 0, sizeof st);
  st.count = R.count;
  st.n_levels = R.k;
  st.n_domains = (int32_t)P.domains.size();
  for (int j = 0; j < R.k && j < 64; ++j) st.level_nodes[j] = R.lvl_n[j];
  st.t_expand = c[QS_EXPAND];
  st.t_seed = c[QS_SEED];
  st.t_push = c[QS_PUSH];
  st.t_pull = c[QS_PULL];
  st.t_probe = c[QS_PROBE];
  st.t_total = st.t_expand + st.t_seed + st.t_push + st.t_pull + st.t_probe;
  st.domain_push = (int32_t)c[QS_DOMPUSH];
  st.domain_pull = (int32_t)c[QS_DOMPULL];
  // Algorithmic bytes, the method's own traffic: 4 B per traversed entry (int32 id), the label
  // entries read to locate label sub-segments, an offset pair per segment lookup, 8 B per tree
  // node written (parent, vertex) and per node read by a later step, 8 B per bitmap word.
  const int64_t W = R.eng ? R.eng->g.words : 0;
  int64_t nodes_written = 0, nodes_read = 0, bm_words = c[QS_BMWORDS];
  for (int j = 0; j < R.k; ++j) {
    const PlanStep &ps = P.steps[j];
    const int64_t prev = j ? R.lvl_n[j - 1] : 1;
    if (!(count_only && j == R.k - 1)) nodes_written += R.lvl_n[j];
    if (j + 1 < R.k) nodes_read += R.lvl_n[j];
    if (ps.kind == STEP_LIST && prev > 0) bm_words += W * (int64_t)ps.filters.size();   // the AND of the filters
  }
  for (const DomainSpec &d : P.domains) {   // frontier and result bitmaps cleared, one frontier bit set per node
    const int64_t prev = d.step > 0 && d.step <= R.k ? R.lvl_n[d.step - 1] : (d.step == 0 ? 1 : 0);
    bm_words += 2 * W + prev;
    nodes_read += prev;
  }
  bm_words += W * (int64_t)P.seeds.size();   // seed bitmaps cleared
  const int64_t lab_bytes = R.eng ? R.eng->lab_bytes : 2, off_bytes = R.eng ? R.eng->off_bytes : 8;
  st.t_label = c[QS_LABEL];
  st.seg_lookups = c[QS_LOOKUP];
  st.bitmap_words = bm_words;
  st.nodes_written = nodes_written;
  st.nodes_read = nodes_read;
  st.bytes_alg = 4 * st.t_total + lab_bytes * st.t_label + 2 * off_bytes * st.seg_lookups + 8 * nodes_written +
                 8 * nodes_read + 8 * bm_words;
  st.gpu_ms = ms;
}

int result_rows(Result &R, int64_t first, int64_t n, void *dst, int mem_kind, int64_t *written) {
  if (written) *written = 0;
  if (R.count_only && !R.zero_vars) { set_error("rows of a count-only result"); return GS_EUNSUPPORTED; }
  if (first < 0 || n < 0 || first > R.count) { set_error("row range outside the result"); return GS_ERANGE; }
  n = std::min(n, R.count - first);
  if (n == 0 || R.n_vars == 0) { if (written) *written = n; return GS_OK; }
  if (!dst) { set_error("null destination"); return GS_EINVAL; }
  if (R.host_owned) {
    const size_t bytes = sizeof(int32_t) * (size_t)n * R.k;
    const int32_t *src = R.host_rows.data() + (size_t)first * R.k;
    if (mem_kind == GS_MEM_DEVICE) HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
    else memcpy(dst, src, bytes);
    if (written) *written = n;
    return GS_OK;
  }
  Engine &E = *R.eng;
  if (E.serving) { set_error("a server is running on this engine"); return GS_ESTATE; }
  HIPCHK(hipSetDevice(E.device));
  hipStream_t s = E.stream;
  const int k = R.k;
  if (mem_kind == GS_MEM_DEVICE) {
    hipError_t e = launch_enumerate(R.d_lvl_ptr, R.d_lvl_cptr, R.d_lvl_n, k, R.d_var_rank, first, n, (int32_t *)dst, s);
    if (e != hipSuccess) { set_error(hipGetErrorString(e)); return GS_EDEVICE; }
    HIPCHK(hipStreamSynchronize(s));
  } else {
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(n, (int64_t)(64ll << 20) / (4 * k)));
    int32_t *tmp = (int32_t *)E.dmalloc(sizeof(int32_t) * (size_t)chunk * k);
    if (!tmp) { set_error("out of device memory for rows"); return GS_ENOMEM; }
    for (int64_t r = 0; r < n; r += chunk) {
      const int64_t c = std::min(chunk, n - r);
      hipError_t e = launch_enumerate(R.d_lvl_ptr, R.d_lvl_cptr, R.d_lvl_n, k, R.d_var_rank, first + r, c, tmp, s);
      if (e == hipSuccess) e = hipMemcpyAsync((int32_t *)dst + r * k, tmp, sizeof(int32_t) * c * k, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) { E.dfree(tmp); set_error(hipGetErrorString(e)); return GS_EDEVICE; }
    }
    E.dfree(tmp);
  }
  if (written) *written = n;
  return GS_OK;
}

static uint64_t host_row_hash(const int32_t *row, int k) {
  uint64_t h = (uint64_t)k;
  for (int i = 0; i < k; ++i) {
    uint64_t z = h + 0x9E3779B97F4A7C15ull + (uint64_t)(uint32_t)row[i];
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    h = z ^ (z >> 31);
  }
  return h;
}

int result_digest(Result &R, uint64_t *hsum, uint64_t *hxor) {
  *hsum = 0;
  *hxor = 0;
  if (R.count_only && !R.zero_vars) { set_error("digest of a count-only result"); return GS_EUNSUPPORTED; }
  if (R.count == 0) return GS_OK;
  if (R.n_vars == 0) {   // rows of width 0 all hash to 0
    return GS_OK;
  }
  if (R.host_owned) {
    for (int64_t r = 0; r < R.count; ++r) {
      const uint64_t h = host_row_hash(R.host_rows.data() + (size_t)r * R.k, R.k);
      *hsum += h;
      *hxor ^= h;
    }
    return GS_OK;
  }
  Engine &E = *R.eng;
  if (E.serving) { set_error("a server is running on this engine"); return GS_ESTATE; }
  HIPCHK(hipSetDevice(E.device));
  hipStream_t s = E.stream;
  uint64_t *d = (uint64_t *)E.dmalloc(2 * sizeof(uint64_t));
  if (!d) { set_error("out of device memory for the digest"); return GS_ENOMEM; }
  uint64_t h[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(d, h, sizeof h, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_row_digest(R.d_lvl_ptr, R.d_lvl_cptr, R.d_lvl_n, R.k, R.d_var_rank, R.count, d, s);
  if (e == hipSuccess) e = hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  E.dfree(d);
  if (e != hipSuccess) { set_error(hipGetErrorString(e)); return GS_EDEVICE; }
  *hsum = h[0];
  *hxor = h[1];
  return GS_OK;
}

int result_prune(Result &R) {
  if (R.count_only || R.zero_vars || R.host_owned || R.k <= 1) return GS_OK;
  Engine &E = *R.eng;
  if (E.serving) { set_error("a server is running on this engine"); return GS_ESTATE; }
  HIPCHK(hipSetDevice(E.device));
  hipStream_t s = E.stream;
  const int k = R.k;
  int64_t tot = 0;
  for (int j = 0; j < k; ++j) tot += R.lvl_n[j];
  uint8_t *alive = (uint8_t *)E.dmalloc((size_t)tot + 64);
  int32_t *newidx = (int32_t *)E.dmalloc(sizeof(int32_t) * ((size_t)tot + 16));
  int64_t *blk = (int64_t *)E.dmalloc(sizeof(int64_t) * (2 * (size_t)E.grid + 2));
  auto cleanup = [&]() { E.dfree(alive); E.dfree(newidx); E.dfree(blk); };
  if (!alive || !newidx || !blk) { cleanup(); set_error("out of device memory for pruning"); return GS_ENOMEM; }
  std::vector<int64_t> off(k + 1, 0);
  for (int j = 0; j < k; ++j) off[j + 1] = off[j] + R.lvl_n[j];
  hipError_t e = hipMemsetAsync(alive, 0, (size_t)tot, s);
  if (e == hipSuccess) e = hipMemsetAsync(alive + off[k - 1], 1, (size_t)R.lvl_n[k - 1], s);
  for (int j = k - 1; j >= 1 && e == hipSuccess; --j)   // a node survives when one of its children does
    e = launch_prune_mark(R.lvl_ptr[j], R.lvl_cptr[j], R.lvl_n[j - 1], R.lvl_n[j], alive + off[j], alive + off[j - 1],
                          s);
  std::vector<int32_t *> np(k);
  std::vector<int64_t> nn(k);
  for (int j = 0; j < k && e == hipSuccess; ++j) {
    const int ncols = 2 + (int)R.ncols_extra[j];
    int64_t cnt = 0;
    e = launch_prune_count(alive + off[j], R.lvl_n[j], blk, E.grid, s);
    if (e == hipSuccess) e = scan_i64(blk, E.grid, blk + E.grid, blk + 2 * E.grid, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&cnt, blk + 2 * E.grid, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) break;
    const uint64_t bytes = align256(sizeof(int32_t) * (uint64_t)cnt * ncols);
    const uint64_t at = align256(E.tree_top);
    if (at + bytes > E.tree_cap) { cleanup(); set_error("tree arena too small to prune"); return GS_ENOMEM; }
    E.tree_top = at + bytes;
    np[j] = (int32_t *)(E.tree_base + at);
    nn[j] = cnt;
    e = launch_prune_write(R.lvl_ptr[j], R.lvl_cptr[j], j ? R.lvl_n[j - 1] : 1, R.lvl_n[j], ncols, alive + off[j],
                           blk + E.grid, j ? newidx + off[j - 1] : nullptr, newidx + off[j], np[j], cnt, E.grid, s);
  }
  // pruned levels always carry a parent column
  const std::vector<int32_t *> nc(k, nullptr);
  if (e == hipSuccess) e = hipMemcpyAsync(R.d_lvl_cptr, nc.data(), sizeof(void *) * k, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(R.d_lvl_ptr, np.data(), sizeof(void *) * k, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(R.d_lvl_n, nn.data(), sizeof(int64_t) * k, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) { set_error(hipGetErrorString(e)); return GS_EDEVICE; }
  R.lvl_ptr = np;
  R.lvl_cptr = nc;
  R.lvl_n = nn;
  return GS_OK;
}

void result_free(Result *R) {
  if (!R) return;
  Engine *E = R->eng;
  if (R->own) E->dfree(R->own);
  else if (!R->host_owned && E && E->live_results > 0 && --E->live_results == 0) E->tree_top = 0;
  delete R;
}

}  // namespace gs
