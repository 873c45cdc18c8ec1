// The C ABI (include/gsmart.h) over the host engine.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <new>
#include <vector>

#include "engine.hpp"
#include "gsmart.h"
#include "lspm.hpp"
#include "query.hpp"

namespace gs {
const char *last_error();
int server_start(Engine *E, const gs_server_options *o, gs_server **out);
int server_submit(gs_server *S, const gs_query *q, uint32_t flags, uint64_t *ticket);
int server_poll(gs_server *S, uint64_t ticket, gs_result **out);
int server_stop(gs_server *S, gs_server_stats *st);
int server_poll_ready(gs_server *S, uint64_t *tickets, int32_t *statuses, gs_result **results, int32_t cap, int32_t *n);
}  // namespace gs

using namespace gs;

struct gs_engine { Engine e; };


#define HIPRET(expr)                                                                 \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess) {                                                          \
      set_error(std::string("HIP error: ") + hipGetErrorString(_e));                 \
      return GS_EDEVICE;                                                             \
    }                                                                                \
  } while (0)

namespace {

// Temporary device buffers released on scope exit.
struct Temps {
  Engine &E;
  std::vector<void *> v;
  explicit Temps(Engine &e) : E(e) {}
  void *get(size_t bytes) { void *p = E.dmalloc(bytes); v.push_back(p); return p; }
  bool ok() const { for (void *p : v) if (!p) return false; return true; }
  ~Temps() { for (void *p : v) E.dfree(p); }
};

// Workspace of gs_bitmap_and_compact_noalloc: one fixed-size device array per
// GPU, held until the process ends. Its host-side name is not a device address:
// host code only ever uses the per-device address that hipGetSymbolAddress
// returned, taken once per device when an engine is created on it.
static __device__ __align__(256) char scratch[NoAllocLayout::bytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// With `device` current: the device address of its copy of the workspace.
hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void *scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

// Autotune cache: one line per graph, "n m P grid theta".
// One line per graph size: n m P grid theta write_block (lines of five fields: 256 threads).
static bool tune_line(const char *line, long long &n, long long &m, int &P, int &g, float &th, int &wb) {
  wb = 256;
  const int k = sscanf(line, "%lld %lld %d %d %f %d", &n, &m, &P, &g, &th, &wb);
  return k >= 5;
}

bool tune_cache_lookup(const Engine &E, const char *path, int *grid, float *theta, int *write_block) {
  FILE *f = fopen(path, "r");
  if (!f) return false;
  char line[256];
  long long n, m;
  int P, g, wb;
  float th;
  bool hit = false;
  while (fgets(line, sizeof line, f))
    if (tune_line(line, n, m, P, g, th, wb) && n == E.g.n && m == E.g.m && P == E.g.P && g > 0) {
      *grid = g;
      *theta = th;
      *write_block = wb;
      hit = true;
    }
  fclose(f);
  return hit;
}

bool tune_cache_store(const Engine &E, const char *path, int grid, float theta, int write_block) {
  std::vector<std::string> keep;
  if (FILE *f = fopen(path, "r")) {
    char line[256];
    long long n, m;
    int P, g, wb;
    float th;
    while (fgets(line, sizeof line, f)) {
      if (!tune_line(line, n, m, P, g, th, wb) || (n == E.g.n && m == E.g.m && P == E.g.P)) continue;
      char out[160];
      snprintf(out, sizeof out, "%lld %lld %d %d %g %d\n", n, m, P, g, th, wb);
      keep.push_back(out);
    }
    fclose(f);
  }
  FILE *f = fopen(path, "w");
  if (!f) return false;
  for (const std::string &l : keep) fputs(l.c_str(), f);
  fprintf(f, "%lld %lld %d %d %g %d\n", (long long)E.g.n, (long long)E.g.m, E.g.P, grid, theta, write_block);
  return fclose(f) == 0;
}

gs_result *wrap(Result *r) {
  // gs_result is an opaque handle for a Result
  return reinterpret_cast<gs_result *>(r);
}
Result *unwrap(gs_result *r) { return reinterpret_cast<Result *>(r); }
const Result *unwrap(const gs_result *r) { return reinterpret_cast<const Result *>(r); }

}  // namespace

extern "C" {

const char *gs_last_error(void) { return gs::last_error(); }

gs_status gs_engine_create(const gs_options *options, gs_engine **out) {
  if (!out) { set_error("null output"); return GS_EINVAL; }
  *out = nullptr;
  gs_options o{};
  if (options) o = *options;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) { set_error("no HIP device"); return GS_EDEVICE; }
  if (o.device < 0 || o.device >= ndev) { set_error("device ordinal out of range"); return GS_EINVAL; }
  if (o.write_block != 0 && o.write_block != 128 && o.write_block != 256 && o.write_block != 512) {
    set_error("write_block must be 0, 128, 256 or 512");
    return GS_EINVAL;
  }
  gs_engine *ge = new (std::nothrow) gs_engine();
  if (!ge) return GS_ENOMEM;
  Engine &E = ge->e;
  E.opt = o;
  if (o.autotune_cache) {   // the caller's string need not outlive the call
    E.tune_path = o.autotune_cache;
    E.opt.autotune_cache = E.tune_path.c_str();
  }
  E.device = o.device;
  if (hipSetDevice(E.device) != hipSuccess) { delete ge; set_error("hipSetDevice failed"); return GS_EDEVICE; }
  if (hipError_t se = scratch_setup(E.device); se != hipSuccess) {
    delete ge;
    set_error(std::string("cannot locate the device workspace: ") + hipGetErrorString(se));
    return GS_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, E.device) == hipSuccess) E.cus = prop.multiProcessorCount;
  E.grid = o.grid_blocks > 0 ? o.grid_blocks : 12 * E.cus;
  if (E.grid > 8192) E.grid = 8192;
  E.wwaves = o.write_block ? o.write_block / 64 : 4;
  E.wgrid = expand_write_blocks_per_cu(E.wwaves) * E.cus;
  if (o.hip_stream) {
    E.stream = (hipStream_t)o.hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&E.stream, hipStreamNonBlocking) != hipSuccess) {
      delete ge; set_error("stream creation failed"); return GS_EDEVICE;
    }
    E.own_stream = true;
  }
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  uint64_t tree = o.tree_bytes ? o.tree_bytes : std::min<uint64_t>(64ull << 30, free_b / 4);
  uint64_t scratch = o.scratch_bytes ? o.scratch_bytes : std::min<uint64_t>(16ull << 30, free_b / 16);
  tree = std::max<uint64_t>(tree, 1 << 20);
  scratch = std::max<uint64_t>(scratch, 1 << 20);
  E.tree_base = (char *)E.dmalloc(tree);
  E.scratch_base = (char *)E.dmalloc(scratch);
  E.d_arenas = (DArena *)E.dmalloc(sizeof(DArena) * 2);
  if (!E.tree_base || !E.scratch_base || !E.d_arenas) {
    delete ge; set_error("cannot allocate the device arenas"); return GS_ENOMEM;
  }
  E.tree_cap = tree;
  E.scratch_cap = scratch;
  *out = ge;
  return GS_OK;
}

void gs_engine_destroy(gs_engine *engine) { delete engine; }

gs_status gs_load_triples(gs_engine *engine, int64_t n_vertices, int32_t n_labels, const gs_triple *triples,
                          int64_t m, int mem_kind) {
  if (!engine) { set_error("null engine"); return GS_EINVAL; }
  if (mem_kind != GS_MEM_HOST && mem_kind != GS_MEM_DEVICE) { set_error("bad mem_kind"); return GS_EINVAL; }
  std::lock_guard<std::mutex> lk(engine->e.mu);
  Engine &E = engine->e;
  const int rc = load_triples(E, n_vertices, n_labels, triples, m, mem_kind);
  if (rc == GS_OK && E.opt.autotune_cache) {   // a recorded tuning for a graph of these sizes
    int grid = 0, wb = 256;
    float theta = 0;
    if (tune_cache_lookup(E, E.opt.autotune_cache, &grid, &theta, &wb)) {
      E.grid = std::min(grid, 8192);
      E.opt.push_pull_theta = theta;
      if (wb == 128 || wb == 256 || wb == 512) {
        E.wwaves = wb / 64;
        E.wgrid = expand_write_blocks_per_cu(E.wwaves) * E.cus;
      }
    }
  }
  return (gs_status)rc;
}

gs_status gs_load_triples_labels(gs_engine *engine, int64_t n_vertices, int32_t n_labels, const gs_triple *triples,
                                 int64_t m, int mem_kind, const int32_t *labels, int32_t n_keep) {
  if (!engine) { set_error("null engine"); return GS_EINVAL; }
  if (mem_kind != GS_MEM_HOST && mem_kind != GS_MEM_DEVICE) { set_error("bad mem_kind"); return GS_EINVAL; }
  if (n_keep < 0 || (n_keep > 0 && !labels)) { set_error("bad label list"); return GS_EINVAL; }
  std::lock_guard<std::mutex> lk(engine->e.mu);
  static const int32_t none = 0;
  return (gs_status)load_triples(engine->e, n_vertices, n_labels, triples, m, mem_kind, n_keep ? labels : &none,
                                 n_keep);
}

gs_status gs_graph_info(const gs_engine *engine, int64_t *n, int32_t *n_labels, int64_t *m_distinct,
                        uint64_t *device_bytes) {
  if (!engine) { set_error("null engine"); return GS_EINVAL; }
  const Engine &E = engine->e;
  if (!E.loaded) { set_error("no dataset loaded"); return GS_ESTATE; }
  if (n) *n = E.g.n;
  if (n_labels) *n_labels = E.g.P;
  if (m_distinct) *m_distinct = E.g.m;
  if (device_bytes) *device_bytes = E.graph_bytes;
  return GS_OK;
}

gs_status gs_lspm_export(gs_engine *engine, int orientation, int64_t *ptr, int32_t *idx, int32_t *label) {
  if (!engine || orientation < 0 || orientation > 1) { set_error("bad argument"); return GS_EINVAL; }
  Engine &E = engine->e;
  if (!E.loaded) { set_error("no dataset loaded"); return GS_ESTATE; }
  HIPRET(hipSetDevice(E.device));
  if (ptr) {
    if (E.off_bytes == 8) {
      HIPRET(hipMemcpy(ptr, E.d_ptr[orientation], sizeof(int64_t) * (E.g.n + 1), hipMemcpyDeviceToHost));
    } else {
      std::vector<int32_t> p((size_t)E.g.n + 1);
      HIPRET(hipMemcpy(p.data(), E.d_ptr[orientation], sizeof(int32_t) * (E.g.n + 1), hipMemcpyDeviceToHost));
      for (int64_t i = 0; i <= E.g.n; ++i) ptr[i] = p[i];
    }
  }
  if (idx && E.g.m) HIPRET(hipMemcpy(idx, E.d_idx[orientation], sizeof(int32_t) * E.g.m, hipMemcpyDeviceToHost));
  if (label && E.g.m) {
    if (E.lab_bytes == 2) {
      std::vector<uint16_t> l(E.g.m);
      HIPRET(hipMemcpy(l.data(), E.d_lab[orientation], sizeof(uint16_t) * E.g.m, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < E.g.m; ++i) label[i] = (int32_t)l[i] + 1;
    } else {
      std::vector<uint8_t> l(E.g.m);
      HIPRET(hipMemcpy(l.data(), E.d_lab[orientation], E.g.m, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < E.g.m; ++i) label[i] = (int32_t)l[i] + 1;
    }
  }
  return GS_OK;
}

gs_status gs_label_stats(gs_engine *engine, int64_t *nnz, int64_t *rows, int64_t *cols) {
  if (!engine) { set_error("null engine"); return GS_EINVAL; }
  Engine &E = engine->e;
  if (!E.loaded) { set_error("no dataset loaded"); return GS_ESTATE; }
  const size_t P = E.stats.nnz.size();
  if (nnz) memcpy(nnz, E.stats.nnz.data(), 8 * P);
  if (rows) memcpy(rows, E.stats.rows.data(), 8 * P);
  if (cols) memcpy(cols, E.stats.cols.data(), 8 * P);
  return GS_OK;
}

gs_status gs_label_exists(gs_engine *engine, int32_t label, int direction, uint64_t *host_words) {
  if (!engine || !host_words || direction < 0 || direction > 1) { set_error("bad argument"); return GS_EINVAL; }
  Engine &E = engine->e;
  if (!E.loaded) { set_error("no dataset loaded"); return GS_ESTATE; }
  if (label < 1 || label > E.g.P) { set_error("label out of range"); return GS_ERANGE; }
  HIPRET(hipSetDevice(E.device));
  HIPRET(hipMemcpy(host_words, E.g.bm[direction] + (int64_t)(label - 1) * E.g.words, 8 * E.g.words,
                   hipMemcpyDeviceToHost));
  return GS_OK;
}

gs_status gs_frontier_domain(gs_engine *engine, const uint64_t *frontier_words, int32_t label, int direction,
                             int mode, const uint64_t *mask_words, uint64_t *out_words) {
  if (!engine || !frontier_words || !out_words || direction < 0 || direction > 1 ||
      (mode != GS_DOMAIN_PUSH && mode != GS_DOMAIN_PULL)) { set_error("bad argument"); return GS_EINVAL; }
  Engine &E = engine->e;
  if (!E.loaded) { set_error("no dataset loaded"); return GS_ESTATE; }
  if (label < 1 || label > E.g.P) { set_error("label out of range"); return GS_ERANGE; }
  std::lock_guard<std::mutex> lk(E.mu);
  if (E.serving) { set_error("a server is running on this engine"); return GS_ESTATE; }
  HIPRET(hipSetDevice(E.device));
  hipStream_t s = E.stream;
  const size_t wb = 8 * (size_t)E.g.words;
  Temps T(E);
  uint64_t *F = (uint64_t *)T.get(wb), *D = (uint64_t *)T.get(wb), *M = (uint64_t *)T.get(wb);
  DDomain *dm = (DDomain *)T.get(sizeof(DDomain));
  const uint64_t **ft = (const uint64_t **)T.get(sizeof(void *));
  IterScalars *it = (IterScalars *)T.get(sizeof(IterScalars));
  int64_t *qs = (int64_t *)T.get(8 * QS_N), *fc = (int64_t *)T.get(8);
  if (!T.ok()) { set_error("out of device memory"); return GS_ENOMEM; }
  HIPRET(hipMemcpyAsync(F, frontier_words, wb, hipMemcpyHostToDevice, s));
  HIPRET(hipMemsetAsync(D, 0, wb, s));
  HIPRET(hipMemsetAsync(it, 0, sizeof(IterScalars), s));
  HIPRET(hipMemsetAsync(qs, 0, 8 * QS_N, s));
  HIPRET(hipMemsetAsync(fc, 0, 8, s));
  DDomain h{};
  h.F = F; h.D = D; h.label = label - 1; h.dir = direction; h.mode = mode == GS_DOMAIN_PUSH ? 1 : 2;
  h.filt0 = 0; h.nfilt = 0; h.q = 0; h.theta = 1.0f;
  if (mask_words) {
    HIPRET(hipMemcpyAsync(M, mask_words, wb, hipMemcpyHostToDevice, s));
    const uint64_t *mp = M;
    HIPRET(hipMemcpyAsync(ft, &mp, sizeof(void *), hipMemcpyHostToDevice, s));
    h.nfilt = 1;
  }
  HIPRET(hipMemcpyAsync(dm, &h, sizeof h, hipMemcpyHostToDevice, s));
  IterArgs A{};
  A.g = E.g; A.D = 1; A.doms = dm; A.fcount = fc; A.filt = ft; A.it = it; A.qstats = qs; A.grid = E.grid;
  HIPRET(launch_domain_only(A, s));
  HIPRET(hipMemcpyAsync(out_words, D, wb, hipMemcpyDeviceToHost, s));
  HIPRET(hipStreamSynchronize(s));
  return GS_OK;
}

gs_status gs_bitmap_and_compact(gs_engine *engine, const uint64_t *const *bitmaps, int32_t k, int32_t *out,
                                int64_t *count) {
  if (!engine || k < 0 || (k > 0 && !bitmaps) || !count) { set_error("bad argument"); return GS_EINVAL; }
  Engine &E = engine->e;
  if (!E.loaded) { set_error("no dataset loaded"); return GS_ESTATE; }
  std::lock_guard<std::mutex> lk(E.mu);
  if (E.serving) { set_error("a server is running on this engine"); return GS_ESTATE; }
  HIPRET(hipSetDevice(E.device));
  hipStream_t s = E.stream;
  const size_t wb = 8 * (size_t)E.g.words;
  Temps T(E);
  std::vector<const uint64_t *> dptr(std::max(k, 1));
  for (int i = 0; i < k; ++i) dptr[i] = (const uint64_t *)T.get(wb);
  const uint64_t **ft = (const uint64_t **)T.get(sizeof(void *) * std::max(k, 1));
  DStep *st = (DStep *)T.get(sizeof(DStep));
  DEntry *en = (DEntry *)T.get(sizeof(DEntry));
  EState *es = (EState *)T.get(sizeof(EState));
  IterScalars *it = (IterScalars *)T.get(sizeof(IterScalars));
  int32_t **lp = (int32_t **)T.get(sizeof(void *) * kMaxLevels);
  int64_t *ln = (int64_t *)T.get(8 * kMaxLevels);
  int64_t *blk = (int64_t *)T.get(8 * 4 * (size_t)E.grid);
  int64_t *qs = (int64_t *)T.get(8 * QS_N);
  if (!T.ok()) { set_error("out of device memory"); return GS_ENOMEM; }
  for (int i = 0; i < k; ++i) HIPRET(hipMemcpyAsync((void *)dptr[i], bitmaps[i], wb, hipMemcpyHostToDevice, s));
  HIPRET(hipMemcpyAsync(ft, dptr.data(), sizeof(void *) * k, hipMemcpyHostToDevice, s));
  DStep hs{};
  hs.kind = STEP_LIST; hs.filt0 = 0; hs.nfilt = k; hs.list_nfilt = k;
  DEntry he{0, 0, 0, 0, 0, 0};
  HIPRET(hipMemcpyAsync(st, &hs, sizeof hs, hipMemcpyHostToDevice, s));
  HIPRET(hipMemcpyAsync(en, &he, sizeof he, hipMemcpyHostToDevice, s));
  HIPRET(hipMemsetAsync(lp, 0, sizeof(void *) * kMaxLevels, s));
  HIPRET(hipMemsetAsync(ln, 0, 8 * kMaxLevels, s));
  DArena ar[2];
  ar[0] = {E.tree_cap, E.tree_cap, 0, 0};
  ar[1] = {0, E.scratch_cap, 0, 0};
  HIPRET(hipMemcpyAsync(E.d_arenas, ar, sizeof ar, hipMemcpyHostToDevice, s));
  IterArgs A{};
  A.g = E.g; A.ent = en; A.E = 1; A.grid = E.grid; A.wgrid = E.wgrid; A.wwaves = E.wwaves; A.steps = st; A.filt = ft; A.es = es; A.it = it;
  A.lvl_ptr = lp; A.lvl_n = ln; A.qstats = qs; A.scratch = E.d_arenas + 1; A.scratch_base = E.scratch_base;
  A.tree = E.d_arenas; A.tree_base = E.tree_base; A.has_list = 1;
  A.blk_a = blk; A.blk_b = blk + E.grid; A.blk_off_a = blk + 2 * E.grid; A.blk_off_b = blk + 3 * E.grid;
  HIPRET(launch_list_only(A, s));
  IterScalars h{};
  HIPRET(hipMemcpyAsync(&h, it, sizeof h, hipMemcpyDeviceToHost, s));
  HIPRET(hipStreamSynchronize(s));
  if (h.abort) { set_error("scratch arena overflow"); return GS_ENOMEM; }
  *count = h.list_total;
  if (out && h.list_total) HIPRET(hipMemcpy(out, h.list_buf, 4 * h.list_total, hipMemcpyDeviceToHost));
  return GS_OK;
}

gs_status gs_bitmap_and_compact_noalloc(gs_engine *engine, const uint64_t *const *dev_bitmaps, int32_t k,
                                        int32_t *dev_out, int64_t *dev_count) {
  if (!engine || k < 0 || (k > 0 && !dev_bitmaps) || !dev_out || !dev_count) {
    set_error("bad argument");
    return GS_EINVAL;
  }
  if (k > kNoAllocMaxBitmaps) {
    set_error("gs_bitmap_and_compact_noalloc takes at most " + std::to_string(kNoAllocMaxBitmaps) + " bitmaps");
    return GS_EINVAL;
  }
  Engine &E = engine->e;
  if (!E.loaded) { set_error("no dataset loaded"); return GS_ESTATE; }
  std::lock_guard<std::mutex> lk(E.mu);
  if (E.serving) { set_error("a server is running on this engine"); return GS_ESTATE; }
  for (int i = 0; i < k; ++i)
    if (!dev_bitmaps[i]) { set_error("null bitmap"); return GS_EINVAL; }
  char *ws = (char *)scratch_ptr(E.device);
  if (!ws) { set_error("device workspace not set up"); return GS_ESTATE; }
  const int grid = std::min(E.grid, kNoAllocMaxGrid);
  HIPRET(hipSetDevice(E.device));
  NoAllocInit init{};
  init.k = k;
  for (int i = 0; i < k; ++i) init.bm[i] = dev_bitmaps[i];
  HIPRET(launch_list_noalloc(E.g, init, ws, grid, dev_out, dev_count, E.stream));
  return GS_OK;
}

gs_status gs_plan_query(gs_engine *engine, const gs_query *query, gs_plan_info *out) {
  return gs_plan_query_ex(engine, query, GS_TRAVERSAL_ENGINE, out);
}

gs_status gs_plan_query_ex(gs_engine *engine, const gs_query *query, int32_t traversal, gs_plan_info *out) {
  if (!query || !out) { set_error("null argument"); return GS_EINVAL; }
  if (query->n_edges > 0 && !query->edges) { set_error("query edges missing"); return GS_EINVAL; }
  std::vector<int32_t> e3(3 * (size_t)std::max(query->n_edges, 0));
  for (int k = 0; k < query->n_edges; ++k) {
    e3[3 * k] = query->edges[k].src; e3[3 * k + 1] = query->edges[k].label; e3[3 * k + 2] = query->edges[k].dst;
  }
  QInfo qi;
  std::string msg;
  int rc;
  if (traversal != GS_TRAVERSAL_ENGINE && traversal != GS_TRAVERSAL_DEGREE && traversal != GS_TRAVERSAL_DIRECTION) {
    set_error("unknown traversal");
    return GS_EINVAL;
  }
  if (engine && engine->e.g.n > 0) {   // the plan the engine's evaluation uses
    std::lock_guard<std::mutex> lk(engine->e.mu);
    const int32_t keep = engine->e.opt.traversal;
    if (traversal != GS_TRAVERSAL_ENGINE) engine->e.opt.traversal = traversal;
    rc = plan_query(engine->e, *query, qi, msg);
    engine->e.opt.traversal = keep;
  } else {
    rc = normalise_query(query->n_qv, query->qv_const, query->n_edges, e3.data(), -1, -1, qi.nq, msg);
    if (rc == GS_OK) rc = build_plan(qi.nq, nullptr, false, qi.plan, msg, traversal == GS_TRAVERSAL_DIRECTION);
  }
  if (rc != GS_OK) { set_error(msg); return (gs_status)rc; }
  const NormQuery &q = qi.nq;
  const Plan &P = qi.plan;
  memset(out, 0, sizeof *out);
  out->n_vars = P.n_vars;
  std::vector<int32_t> first_input(q.edges.size(), -1);
  for (size_t k = 0; k < q.edge_map.size(); ++k)
    if (first_input[q.edge_map[k]] < 0) first_input[q.edge_map[k]] = (int32_t)k;
  for (int j = 0; j < P.n_vars && j < 64; ++j) {
    out->order[j] = P.order[j];
    const int pe = P.steps[j].parent_edge;
    out->parent_edge[j] = (pe >= 0 && P.steps[j].kind == STEP_SEG) ? first_input[pe] : -1;
  }
  out->n_groups = (int32_t)std::min<size_t>(P.group_vertex.size(), 64);
  for (int g = 0; g < out->n_groups; ++g) out->group_vertex[g] = P.group_vertex[g];
  for (size_t k = 0; k < q.edge_map.size() && k < 64; ++k)
    out->edge_group[k] = q.edge_first[k] ? P.edge_group[q.edge_map[k]] : -1;
  out->n_roots = (int32_t)std::min<size_t>(P.roots.size(), 64);
  for (int r = 0; r < out->n_roots; ++r) out->roots[r] = P.roots[r];
  return GS_OK;
}

// ---- per-query reduced matrix
}  // extern "C"

struct gs_reduced {
  int device = 0;
  int64_t n = 0, rows[2] = {0, 0}, nnz[2] = {0, 0};
  std::vector<int32_t> labels[2];   // 1-based, ascending
  int64_t *M[2] = {nullptr, nullptr}, *P[2] = {nullptr, nullptr};
  int32_t *val[2] = {nullptr, nullptr}, *idx[2] = {nullptr, nullptr};
  ~gs_reduced() {
    for (int o = 0; o < 2; ++o) {
      (void)hipFree(M[o]);
      (void)hipFree(P[o]);
      (void)hipFree(val[o]);
      (void)hipFree(idx[o]);
    }
  }
};

extern "C" {

gs_status gs_lspm_reduce(gs_engine *engine, const gs_query *query, int32_t traversal, gs_reduced **out) {
  if (!engine || !query || !out) { set_error("null argument"); return GS_EINVAL; }
  *out = nullptr;
  Engine &E = engine->e;
  if (!E.loaded) { set_error("no dataset loaded"); return GS_ESTATE; }
  // the traversal's edge groups (Section 6.1), then each edge's part (Section 6.2.1 / 6.2.2)
  gs_plan_info info;
  gs_status rc = gs_plan_query_ex(engine, query, traversal, &info);
  if (rc != GS_OK) return rc;
  if (query->n_edges > 64) { set_error("more than 64 query edges"); return GS_EUNSUPPORTED; }
  const int32_t trav = traversal == GS_TRAVERSAL_ENGINE ? E.opt.traversal : traversal;
  bool has_const = false;
  for (int v = 0; v < query->n_qv; ++v) has_const |= query->qv_const[v] >= 0;
  std::vector<int32_t> part_labels[2];
  auto add = [&](int o, int32_t p) {
    if (std::find(part_labels[o].begin(), part_labels[o].end(), p) == part_labels[o].end()) part_labels[o].push_back(p);
  };
  for (int k = 0; k < query->n_edges; ++k) {
    const gs_edge &e = query->edges[k];
    if (trav == GS_TRAVERSAL_DIRECTION && !has_const) { add(0, e.label); continue; }
    const bool cs = query->qv_const[e.src] >= 0, co = query->qv_const[e.dst] >= 0;
    if (cs || co) {   // out of a constant: row-wise; into a constant: column-wise
      if (cs) add(0, e.label);
      if (co) add(1, e.label);
      continue;
    }
    const int g = info.edge_group[k];
    if (g < 0) continue;   // a repeated edge: evaluated with its first copy
    add(info.group_vertex[g] == e.src ? 0 : 1, e.label);
  }
  std::lock_guard<std::mutex> lk(E.mu);
  if (E.serving) { set_error("a server is running on this engine"); return GS_ESTATE; }
  HIPRET(hipSetDevice(E.device));
  hipStream_t s = E.stream;
  gs_reduced *r = new (std::nothrow) gs_reduced;
  if (!r) { set_error("out of host memory"); return GS_ENOMEM; }
  r->device = E.device;
  r->n = E.g.n;
  const int64_t n = E.g.n;
  struct Tmp {
    std::vector<void *> p;
    ~Tmp() { for (void *x : p) (void)hipFree(x); }
    void *get(size_t b) { void *x = nullptr; if (hipMalloc(&x, b) != hipSuccess) return nullptr; p.push_back(x); return x; }
  } tmp;
  auto fail = [&](gs_status st, const std::string &msg) { delete r; set_error(msg); return st; };
  for (int o = 0; o < 2; ++o) {
    std::sort(part_labels[o].begin(), part_labels[o].end());
    r->labels[o] = part_labels[o];
    if ((int)part_labels[o].size() > 64) return fail(GS_EUNSUPPORTED, "more than 64 predicates in a part");
    if (hipMalloc((void **)&r->M[o], 8 * (size_t)(n + 1)) != hipSuccess) return fail(GS_ENOMEM, "out of device memory");
    const int nk = (int)part_labels[o].size();
    if (nk == 0) {   // an empty part: no kept row
      if (hipMemsetAsync(r->M[o], 0, 8 * (size_t)(n + 1), s) != hipSuccess) return fail(GS_EDEVICE, "memset");
      if (hipMalloc((void **)&r->P[o], 8) != hipSuccess) return fail(GS_ENOMEM, "out of device memory");
      if (hipMemsetAsync(r->P[o], 0, 8, s) != hipSuccess) return fail(GS_EDEVICE, "memset");
      continue;
    }
    std::vector<int32_t> k0(part_labels[o]);
    for (int32_t &x : k0) x -= 1;   // stored 0-based
    int32_t *klab = (int32_t *)tmp.get(4 * 64);
    uint32_t *cnt = (uint32_t *)tmp.get(4 * (size_t)n), *ne = (uint32_t *)tmp.get(4 * (size_t)n);
    int64_t *pos = (int64_t *)tmp.get(8 * (size_t)(n + 1)), *parts = (int64_t *)tmp.get(8 * 256);
    if (!klab || !cnt || !ne || !pos || !parts) return fail(GS_ENOMEM, "out of device memory");
    if (hipMemcpyAsync(klab, k0.data(), 4 * k0.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        reduce_count(E.g, o, klab, nk, cnt, ne, pos, r->M[o], parts, s) != hipSuccess)
      return fail(GS_EDEVICE, "reduction count pass failed");
    int64_t tot[2] = {0, 0};
    if (hipMemcpyAsync(&tot[0], pos + n, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&tot[1], r->M[o] + n, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(GS_EDEVICE, "reduction sizes");
    r->nnz[o] = tot[0];
    r->rows[o] = tot[1];
    if (hipMalloc((void **)&r->P[o], 8 * (size_t)(tot[1] + 1)) != hipSuccess ||
        hipMalloc((void **)&r->val[o], 4 * (size_t)std::max<int64_t>(tot[0], 1)) != hipSuccess ||
        hipMalloc((void **)&r->idx[o], 4 * (size_t)std::max<int64_t>(tot[0], 1)) != hipSuccess)
      return fail(GS_ENOMEM, "out of device memory for the reduced matrix");
    if (reduce_write(E.g, o, klab, nk, cnt, pos, r->M[o], r->P[o], r->val[o], r->idx[o], s) != hipSuccess ||
        hipMemcpyAsync(r->P[o] + tot[1], &r->nnz[o], 8, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(GS_EDEVICE, "reduction write pass failed");
  }
  *out = r;
  return GS_OK;
}

gs_status gs_reduced_get_info(const gs_reduced *r, gs_reduced_info *out) {
  if (!r || !out) { set_error("null argument"); return GS_EINVAL; }
  memset(out, 0, sizeof *out);
  out->n = r->n;
  for (int o = 0; o < 2; ++o) {
    out->rows[o] = r->rows[o];
    out->nnz[o] = r->nnz[o];
    out->n_labels[o] = (int32_t)r->labels[o].size();
    for (size_t k = 0; k < r->labels[o].size() && k < 64; ++k) out->labels[o][k] = r->labels[o][k];
  }
  return GS_OK;
}

gs_status gs_reduced_export(const gs_reduced *r, int32_t part, int64_t *M, int64_t *P, int32_t *val, int32_t *idx) {
  if (!r || part < 0 || part > 1) { set_error("bad argument"); return GS_EINVAL; }
  HIPRET(hipSetDevice(r->device));
  if (M) HIPRET(hipMemcpy(M, r->M[part], 8 * (size_t)(r->n + 1), hipMemcpyDeviceToHost));
  if (P) HIPRET(hipMemcpy(P, r->P[part], 8 * (size_t)(r->rows[part] + 1), hipMemcpyDeviceToHost));
  if (val && r->nnz[part]) HIPRET(hipMemcpy(val, r->val[part], 4 * (size_t)r->nnz[part], hipMemcpyDeviceToHost));
  if (idx && r->nnz[part]) HIPRET(hipMemcpy(idx, r->idx[part], 4 * (size_t)r->nnz[part], hipMemcpyDeviceToHost));
  return GS_OK;
}

gs_status gs_reduced_free(gs_reduced *r) {
  if (r) {
    (void)hipSetDevice(r->device);
    delete r;
  }
  return GS_OK;
}

gs_status gs_query_run(gs_engine *engine, const gs_query *query, uint32_t flags, gs_result **out) {
  if (!engine || !query || !out) { set_error("null argument"); return GS_EINVAL; }
  *out = nullptr;
  std::lock_guard<std::mutex> lk(engine->e.mu);
  std::vector<Result *> rs;
  double ms = 0;
  if ((flags & GS_PRUNE) && (flags & GS_COUNT_ONLY)) { set_error("pruning needs the last level"); return GS_EINVAL; }
  int rc = run_batch(engine->e, query, 1, flags, rs, &ms);
  if (rc != GS_OK) return (gs_status)rc;
  if (flags & GS_PRUNE) rc = result_prune(*rs[0]);
  if (rc != GS_OK) { result_free(rs[0]); return (gs_status)rc; }
  *out = wrap(rs[0]);
  return GS_OK;
}

gs_status gs_batch_run(gs_engine *engine, const gs_query *queries, int32_t nq, uint32_t flags, gs_result **outs) {
  if (!engine || !queries || !outs || nq <= 0) { set_error("bad argument"); return GS_EINVAL; }
  for (int i = 0; i < nq; ++i) outs[i] = nullptr;
  std::lock_guard<std::mutex> lk(engine->e.mu);
  std::vector<Result *> rs;
  double ms = 0;
  if ((flags & GS_PRUNE) && (flags & GS_COUNT_ONLY)) { set_error("pruning needs the last level"); return GS_EINVAL; }
  int rc = run_batch(engine->e, queries, nq, flags, rs, &ms);
  if (rc != GS_OK) return (gs_status)rc;
  for (int i = 0; i < nq && rc == GS_OK && (flags & GS_PRUNE); ++i) rc = result_prune(*rs[i]);
  if (rc != GS_OK) { for (Result *r : rs) result_free(r); return (gs_status)rc; }
  for (int i = 0; i < nq; ++i) outs[i] = wrap(rs[i]);
  return GS_OK;
}

gs_status gs_autotune(gs_engine *engine, const gs_query *queries, int32_t nq, gs_tune_result *out) {
  if (!engine || !queries || nq <= 0 || !out) { set_error("bad argument"); return GS_EINVAL; }
  Engine &E = engine->e;
  std::lock_guard<std::mutex> lk(E.mu);
  if (E.serving) { set_error("a server is running on this engine"); return GS_ESTATE; }
  const int grid0 = E.grid;
  const float theta0 = E.opt.push_pull_theta;
  const int prof0 = E.opt.profile_kernels;
  E.opt.profile_kernels = 0;
  auto trial = [&](int grid, float theta, double &ms) -> int {
    E.grid = grid;
    E.opt.push_pull_theta = theta;
    double best = 1e300;
    for (int rep = 0; rep < 2; ++rep) {   // first run warms caches and the allocator
      std::vector<Result *> rs;
      double t = 0;
      int rc = run_batch(E, queries, nq, GS_COUNT_ONLY, rs, &t);
      for (Result *r : rs) result_free(r);
      if (rc != GS_OK) return rc;
      if (rep) best = std::min(best, t);
    }
    ms = best;
    return GS_OK;
  };
  double ms0 = 0;
  int rc = trial(grid0, theta0, ms0);
  memset(out, 0, sizeof *out);
  out->grid_blocks = grid0;
  out->push_pull_theta = theta0 > 0 ? theta0 : 1.0f;
  out->best_ms = ms0;
  out->default_ms = ms0;
  const int mults[] = {2, 4, 8, 12, 16};
  const float thetas[] = {0.25f, 1.0f, 4.0f};
  for (int m : mults) {
    for (float th : thetas) {
      if (rc != GS_OK) break;
      const int grid = std::min(8192, m * E.cus);
      double ms = 0;
      rc = trial(grid, th, ms);
      out->n_tried++;
      if (rc == GS_OK && ms < out->best_ms) { out->best_ms = ms; out->grid_blocks = grid; out->push_pull_theta = th; }
    }
  }
  // then the write pass's workgroup size (2, 4 or 8 waves) under the chosen pair
  const int ww0 = E.wwaves, wg0 = E.wgrid;
  out->write_block = 64 * ww0;
  for (int nw : {2, 4, 8}) {
    if (rc != GS_OK || nw == ww0) continue;
    E.wwaves = nw;
    E.wgrid = expand_write_blocks_per_cu(nw) * E.cus;
    double ms = 0;
    rc = trial(out->grid_blocks, out->push_pull_theta, ms);
    out->n_tried++;
    if (rc == GS_OK && ms < out->best_ms) { out->best_ms = ms; out->write_block = 64 * nw; }
  }
  E.opt.profile_kernels = prof0;
  if (rc != GS_OK) { E.grid = grid0; E.opt.push_pull_theta = theta0; E.wwaves = ww0; E.wgrid = wg0; return (gs_status)rc; }
  E.grid = out->grid_blocks;
  E.opt.push_pull_theta = out->push_pull_theta;
  E.wwaves = out->write_block / 64;
  E.wgrid = expand_write_blocks_per_cu(E.wwaves) * E.cus;
  if (E.opt.autotune_cache &&
      !tune_cache_store(E, E.opt.autotune_cache, out->grid_blocks, out->push_pull_theta, out->write_block)) {
    set_error(std::string("cannot write the autotune cache ") + E.opt.autotune_cache);
    return GS_EINVAL;
  }
  return GS_OK;
}

gs_status gs_result_count(const gs_result *result, int64_t *count) {
  if (!result || !count) { set_error("null argument"); return GS_EINVAL; }
  *count = unwrap(result)->count;
  return GS_OK;
}

gs_status gs_result_width(const gs_result *result, int32_t *n_vars) {
  if (!result || !n_vars) { set_error("null argument"); return GS_EINVAL; }
  *n_vars = unwrap(result)->n_vars;
  return GS_OK;
}

gs_status gs_result_rows(gs_result *result, int64_t first, int64_t n, void *dst, int mem_kind,
                         int64_t *n_written) {
  if (!result) { set_error("null result"); return GS_EINVAL; }
  Result &R = *unwrap(result);
  if (R.host_owned) return (gs_status)result_rows(R, first, n, dst, mem_kind, n_written);
  std::lock_guard<std::mutex> lk(R.eng->mu);
  return (gs_status)result_rows(R, first, n, dst, mem_kind, n_written);
}

gs_status gs_result_digest(gs_result *result, int64_t *count, uint64_t *hash_sum, uint64_t *hash_xor) {
  if (!result || !count || !hash_sum || !hash_xor) { set_error("null argument"); return GS_EINVAL; }
  Result &R = *unwrap(result);
  *count = R.count;
  if (R.host_owned || !R.eng) return (gs_status)result_digest(R, hash_sum, hash_xor);
  std::lock_guard<std::mutex> lk(R.eng->mu);
  return (gs_status)result_digest(R, hash_sum, hash_xor);
}

gs_status gs_result_stats(const gs_result *result, gs_query_stats *stats) {
  if (!result || !stats) { set_error("null argument"); return GS_EINVAL; }
  *stats = unwrap(result)->stats;
  return GS_OK;
}

gs_status gs_result_level(gs_result *result, int32_t level, int32_t *par, int32_t *vid, int64_t *n) {
  if (!result || !n) { set_error("null argument"); return GS_EINVAL; }
  Result &R = *unwrap(result);
  if (level < 0 || level >= R.k) { set_error("level out of range"); return GS_ERANGE; }
  *n = R.lvl_n[level];
  if (!par && !vid) return GS_OK;
  if (!R.lvl_ptr[level]) {
    if (R.lvl_n[level] == 0) return GS_OK;
    set_error("level not stored (count-only)");
    return GS_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(R.eng->mu);
  HIPRET(hipSetDevice(R.eng->device));
  const int64_t cnt = R.lvl_n[level];
  if (par && R.lvl_cptr[level]) {   // a level stored as child offsets per parent: expand them
    const int64_t pn = level ? R.lvl_n[level - 1] : 1;
    std::vector<int32_t> off((size_t)pn + 1);
    HIPRET(hipMemcpy(off.data(), R.lvl_cptr[level], 4 * (pn + 1), hipMemcpyDeviceToHost));
    for (int64_t p = 0; p < pn; ++p)
      for (int64_t i = off[p]; i < off[p + 1]; ++i) par[i] = (int32_t)p;
  } else if (par) {
    HIPRET(hipMemcpy(par, R.lvl_ptr[level], 4 * cnt, hipMemcpyDeviceToHost));
  }
  if (vid) HIPRET(hipMemcpy(vid, R.lvl_ptr[level] + cnt, 4 * cnt, hipMemcpyDeviceToHost));
  return GS_OK;
}

void gs_result_free(gs_result *result) {
  if (!result) return;
  Result *R = unwrap(result);
  if (R->eng && !R->host_owned) {
    std::lock_guard<std::mutex> lk(R->eng->mu);
    result_free(R);
  } else if (R->eng) {
    result_free(R);
  } else {
    delete R;
  }
}

static const char *kSlotNames[KS_N] = {"setup", "clear", "seed", "list_count", "list_scan", "list_write",
                                       "dom_frontier", "dom_push", "dom_pull", "lookup", "scan_nodes", "nz_write",
                                       "expand_count", "scan_expand", "tile_offsets", "expand_write"};

gs_status gs_kernel_stats(gs_engine *engine, gs_kernel_stat *out, int32_t cap, int32_t *n, int reset) {
  if (!engine || !n || (cap > 0 && !out)) { set_error("bad argument"); return GS_EINVAL; }
  Engine &E = engine->e;
  std::lock_guard<std::mutex> lk(E.mu);
  int k = 0;
  for (int i = 0; i < KS_N; ++i) {
    if (E.kstat[i].launches == 0) continue;
    if (k < cap) {
      out[k].name = kSlotNames[i];
      out[k].launches = E.kstat[i].launches;
      out[k].ms = E.kstat[i].ms;
      out[k].bytes_alg = E.kstat[i].alg;
      out[k].bytes_impl = E.kstat[i].bytes;
    }
    ++k;
  }
  *n = k;
  if (reset) for (int i = 0; i < KS_N; ++i) E.kstat[i] = Engine::KStat();
  return GS_OK;
}

gs_status gs_server_start(gs_engine *engine, const gs_server_options *options, gs_server **out) {
  if (!engine || !out) { set_error("null argument"); return GS_EINVAL; }
  return (gs_status)server_start(&engine->e, options, out);
}

gs_status gs_submit(gs_server *server, const gs_query *query, uint32_t flags, uint64_t *ticket) {
  if (!server || !query || !ticket) { set_error("null argument"); return GS_EINVAL; }
  return (gs_status)server_submit(server, query, flags, ticket);
}

gs_status gs_poll(gs_server *server, uint64_t ticket, gs_result **out) {
  if (!server || !out) { set_error("null argument"); return GS_EINVAL; }
  return (gs_status)server_poll(server, ticket, out);
}

gs_status gs_poll_ready(gs_server *server, uint64_t *tickets, int32_t *statuses, gs_result **results, int32_t cap,
                        int32_t *n) {
  if (!server || !n || cap < 0 || (cap > 0 && (!tickets || !statuses || !results))) { set_error("bad argument"); return GS_EINVAL; }
  return (gs_status)server_poll_ready(server, tickets, statuses, results, cap, n);
}

gs_status gs_server_stop(gs_server *server, gs_server_stats *stats) {
  if (!server) { set_error("null server"); return GS_EINVAL; }
  return (gs_status)server_stop(server, stats);
}

}  // extern "C"
