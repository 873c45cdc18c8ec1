// Host engine: device-resident matrix, arenas, batched execution, results.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
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
  std::vector<int64_t> lvl_n;
  std::vector<int32_t> var_rank;
  int32_t **d_lvl_ptr = nullptr;   // device copies for enumeration (in the run's arena block)
  int64_t *d_lvl_n = nullptr;
  int32_t *d_var_rank = nullptr;
  void *own = nullptr;             // memory owned by this result (server results), else arena
  int run_id = -1;                 // arena run this result lives in
  gs_query_stats stats{};
};

struct Engine {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  gs_options opt{};
  int grid = 2048;
  int cus = 256;

  // matrix
  bool loaded = false;
  DevGraph g{};
  int64_t *d_ptr[2] = {nullptr, nullptr};
  int32_t *d_idx[2] = {nullptr, nullptr};
  uint16_t *d_lab[2] = {nullptr, nullptr};
  uint64_t *d_bm[2] = {nullptr, nullptr};
  LabelStats stats;
  uint64_t graph_bytes = 0;

  // arenas: binding trees (+ per-run tables) and per-iteration scratch
  char *tree_base = nullptr;
  uint64_t tree_cap = 0;
  char *scratch_base = nullptr;
  uint64_t scratch_cap = 0;
  DArena *d_arenas = nullptr;      // [0] tree, [1] scratch
  uint64_t tree_top = 0;           // host view of the tree arena's end
  int live_results = 0;
  int run_counter = 0;

  // per-run workspaces (grown on demand)
  void *work = nullptr;
  size_t work_bytes = 0;

  // optional kernel timing (gs_options.profile_kernels)
  struct KStat { int64_t launches = 0; double ms = 0, bytes = 0; };
  KStat kstat[KS_N];
  std::vector<hipEvent_t> events;  // pool, 2 * KS_N per iteration

  std::mutex mu;                   // serialises runs (server vs. direct use is documented as exclusive)

  void *dmalloc(size_t bytes);
  void dfree(void *p);
  ~Engine();
};

// Plan-compile-run a batch; results appended to out (one per query).
int run_batch(Engine &E, const gs_query *qs, int nq, uint32_t flags, std::vector<Result *> &out, double *ms);
int load_triples(Engine &E, int64_t n, int32_t P, const gs_triple *t, int64_t m, int mem_kind);
int result_rows(Result &R, int64_t first, int64_t n, void *dst, int mem_kind, int64_t *written);
void result_free(Result *R);

}  // namespace gs
