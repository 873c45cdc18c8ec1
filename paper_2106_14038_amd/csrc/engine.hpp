// Host engine: device-resident matrix, arenas, batched execution, results.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "gs_device.hpp"
#include "gsmart.h"
#include "planner.hpp"

namespace gs {

void set_error(const std::string &msg);

struct Engine;

struct Result {
  Engine *eng = nullptr;
  int32_t k = 0;                   // levels
  int32_t n_vars = 0;
  int64_t count = 0;
  bool count_only = false;
  bool zero_vars = false;
  std::vector<int32_t *> lvl_ptr;  // device pointers per level
  std::vector<int32_t *> lvl_cptr; // child offsets of CSR levels (device), else null
  std::vector<int64_t> lvl_n;
  std::vector<int32_t> var_rank;
  std::vector<int32_t> ncols_extra;  // carried columns per level
  int32_t **d_lvl_ptr = nullptr;   // device copies for enumeration (in the run's arena block)
  int32_t **d_lvl_cptr = nullptr;
  int64_t *d_lvl_n = nullptr;
  int32_t *d_var_rank = nullptr;
  void *own = nullptr;             // device memory owned by this result, else arena
  bool host_owned = false;         // rows live in host_rows (served results), no arena reference
  std::vector<int32_t> host_rows;
  int run_id = -1;                 // arena run this result lives in
  gs_query_stats stats{};
};

struct Engine {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  gs_options opt{};
  int grid = 3072;    // fixed-grid kernels: 12 workgroups per CU unless the options say otherwise
  int wgrid = 1024;   // write-pass workgroups: as many as the device holds at once
  int wwaves = 4;     // waves per write-pass workgroup (2, 4 or 8; the autotuner may change it)
  int cus = 256;

  // matrix
  bool loaded = false;
  DevGraph g{};
  void *d_ptr[2] = {nullptr, nullptr};    // int32 or int64 row offsets (off_bytes)
  int32_t *d_idx[2] = {nullptr, nullptr};
  void *d_lab[2] = {nullptr, nullptr};    // uint8 or uint16 labels (lab_bytes)
  uint64_t *d_bm[2] = {nullptr, nullptr};
  LabelStats stats;
  uint64_t graph_bytes = 0;
  std::string tune_path;           // copy of gs_options.autotune_cache (the option then points here)
  int32_t lab_bytes = 2;           // stored widths of a label and of a row offset
  int32_t off_bytes = 8;

  // arenas: binding trees (+ per-run tables) and per-iteration scratch
  char *tree_base = nullptr;
  uint64_t tree_cap = 0;
  char *scratch_base = nullptr;
  uint64_t scratch_cap = 0;
  DArena *d_arenas = nullptr;      // [0] tree, [1] scratch
  uint64_t tree_top = 0;           // host view of the tree arena's end
  int live_results = 0;
  int run_counter = 0;
  bool serving = false;            // a server owns the tree arena: direct evaluation is refused

  // seed bitmaps of direct evaluation (grown on demand): all zero between runs, each run
  // clearing after itself only the words its seeds set (a seed of a low-degree constant sets a
  // few bits of an N-bit bitmap; clearing whole bitmaps per run cost more than the seeding)
  uint64_t *seed_pool = nullptr;
  int64_t seed_pool_cap = 0;       // bitmaps
  bool seed_pool_dirty = false;    // a run failed after seeding: zero the pool again first

  // per-run workspaces (grown on demand)
  void *work = nullptr;
  size_t work_bytes = 0;
  // pinned host staging of a run's table upload and result readback (grown on demand), and the
  // run's two timing events (created once)
  void *pin_up = nullptr, *pin_down = nullptr;
  size_t pin_up_bytes = 0, pin_down_bytes = 0;
  hipEvent_t run_ev[2] = {nullptr, nullptr};
  void *pinned(void *&buf, size_t &cap, size_t bytes);

  // optional kernel timing (gs_options.profile_kernels)
  struct KStat { int64_t launches = 0; double ms = 0, bytes = 0, alg = 0; };
  KStat kstat[KS_N];
  std::vector<hipEvent_t> events;  // pool, 2 * KS_N per iteration

  // captured launch sequences of batches (gs_options.use_graphs), keyed by a hash of their launch arguments
  struct GraphEntry { uint64_t key; hipGraph_t graph; hipGraphExec_t exec; uint64_t last_use; };
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
  int64_t graph_hits = 0, graph_builds = 0;

  std::mutex mu;                   // serialises runs (server vs. direct use is documented as exclusive)

  void *dmalloc(size_t bytes);
  void dfree(void *p);
  ~Engine();
};

struct QInfo {                      // one planned query and where its tables sit
  NormQuery nq;
  Plan plan;
  int32_t slot = 0;                  // index of its level / counter tables
  int32_t step0 = 0, seed0 = 0, nseed = 0, dom0 = 0, ndom = 0, vr0 = 0;
  int32_t nlev = 0;                  // tree levels evaluated (fewer than the variables when trailing
                                     // independent leaves of a count-only query are counted as a product)
  int32_t factor_lvl = -1;           // the level that counts those leaves' product (-1: none)
  bool zero = false;                 // no variable: constant patterns only
};

struct Tables {                      // compiled step programs of a set of queries (host copy)
  std::vector<DStep> steps;
  std::vector<const uint64_t *> filt;
  std::vector<DCheck> checks;
  std::vector<int32_t> ints;
  std::vector<DConst> cconst;
  std::vector<DSeed> seeds;
  std::vector<DDomain> doms;
  std::vector<int32_t> dom_step;
  std::vector<int32_t> var_rank;
  bool seeds_zeroed = false;         // seed bitmaps come zeroed (the engine's seed pool): no clear pass
};

struct IterLists {                   // host work lists of one iteration
  std::vector<DEntry> ents;
  std::vector<DDomain> doms;
  std::vector<uint64_t *> clears;
  std::vector<DSeed> seeds;
  int32_t has_list = 0;
  int32_t has_tested = 0;
  int32_t has_checks = 0;
  int32_t has_factor = 0;
  int32_t has_exact = 0;
};

int plan_query(const Engine &E, const gs_query &q, QInfo &qi, std::string &msg);
// next_bitmap(seed): a bitmap for a seed (true) or a domain (false)
void compile_query(const Engine &E, QInfo &qi, bool count_only, int slot, Tables &T,
                   const std::function<uint64_t *(bool)> &next_bitmap);
void build_iteration(const Tables &T, const std::vector<const QInfo *> &qs, const std::vector<int> &level,
                     IterLists &L);
void account_iteration(Engine &E, const hipEvent_t *ev, const IterScalars &I, const IterLists &L, double write_bytes,
                       double children);
void fill_result(Result &R, const QInfo &qi, bool count_only, int32_t *const *lvl_p, int32_t *const *lvl_c,
                 const int64_t *lvl_n,
                 const int64_t *qstats, int64_t zero_res, double ms);
hipError_t zero_words(uint64_t *p, int64_t n, hipStream_t s);
hipError_t launch_const_only(const DevGraph &g, const DConst *cc, int n, int64_t *out, hipStream_t s);

// Plan-compile-run a batch; results appended to out (one per query).
int run_batch(Engine &E, const gs_query *qs, int nq, uint32_t flags, std::vector<Result *> &out, double *ms);
// keep / n_keep: when keep is not NULL, only the triples whose (1-based) predicate is listed
int load_triples(Engine &E, int64_t n, int32_t P, const gs_triple *t, int64_t m, int mem_kind,
                 const int32_t *keep = nullptr, int32_t n_keep = 0);
int result_rows(Result &R, int64_t first, int64_t n, void *dst, int mem_kind, int64_t *written);
int result_prune(Result &R);
int result_digest(Result &R, uint64_t *hsum, uint64_t *hxor);
void result_free(Result *R);

}  // namespace gs
