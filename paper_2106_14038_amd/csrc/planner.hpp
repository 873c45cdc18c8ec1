// Host-side query planner: normalisation, the degree-driven traversal of
// Section 6.1.2 (with the constants rule), and the per-level step programs
// the device kernels execute.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace gs {

constexpr int kMaxVars = 64;
constexpr int kMaxEdges = 64;

enum StepKind : int32_t { STEP_SEG = 0, STEP_SEG_CONST = 1, STEP_LIST = 2 };
enum FilterKind : int32_t { F_LABEL_OUT = 0, F_LABEL_IN = 1, F_SEED = 2, F_DOMAIN = 3 };

struct QEdge { int32_t s, p, o; };   // query vertices, label 1-based

struct NormQuery {
  int32_t n_qv = 0;
  std::vector<int32_t> cst;          // -1 variable, else constant
  std::vector<QEdge> edges;          // distinct edges
  std::vector<int32_t> edge_map;     // input edge -> distinct edge index, -1 never (duplicates map to first)
  std::vector<uint8_t> edge_first;   // input edge is the first occurrence
};

struct FilterRef { int32_t kind, arg; };       // LABEL_*: arg = label (0-based); SEED/DOMAIN: index
struct CheckRef { int32_t level, label, dir; }; // bound vertex's level, label (0-based), dir of seg from it

struct PlanStep {
  int32_t qv = -1;                   // query vertex bound at this level
  int32_t kind = STEP_LIST;
  int32_t src_level = -1;            // STEP_SEG: level of the parent vertex
  int32_t src_const = -1;            // STEP_SEG_CONST: constant vertex
  int32_t label = 0, dir = 0;        // label 0-based; dir 0: objects of (src,p,*), 1: subjects of (*,p,src)
  int32_t parent_edge = -1;          // distinct edge generating candidates (-1: LIST)
  std::vector<FilterRef> filters;    // bitmap tests on each candidate
  std::vector<CheckRef> checks;      // exact membership checks against bound vertices
  std::vector<int32_t> self_labels;  // self loops (c, p, c) (0-based labels)
  std::vector<int32_t> carried;      // levels whose bindings this level carries (besides its own)
};

struct SeedSpec { int32_t c, label, dir; };        // bitmap of seg(c, label, dir)
struct DomainSpec {                                 // vertices reachable from F_u along (label, dir)
  int32_t step, level, label, dir;
  std::vector<FilterRef> mask;                      // pull candidates: AND of these (empty = all)
};
struct ConstCheck { int32_t a, label, b; };         // constant-constant edge (a, label+1, b) must exist

struct Plan {
  int32_t n_vars = 0;
  std::vector<int32_t> order;          // level -> query vertex
  std::vector<int32_t> var_rank;       // level -> output column (rank among variables by index)
  std::vector<PlanStep> steps;
  std::vector<SeedSpec> seeds;
  std::vector<DomainSpec> domains;
  std::vector<ConstCheck> cchecks;
  // traversal record (Section 6.1.2), over distinct edges
  std::vector<int32_t> group_vertex;   // popped vertex per group (-1: the constants' group)
  std::vector<int32_t> edge_group;     // per distinct edge
  std::vector<int32_t> roots;
};

// Optional per-label statistics used for tie-breaks and cost estimates.
struct LabelStats {
  int64_t n = 0;
  std::vector<int64_t> nnz, rows, cols;   // index = label-1
};

// Returns 0 and fills q, or a gs_status code with msg.
int normalise_query(int32_t n_qv, const int32_t *qv_const, int32_t n_edges, const int32_t *edges3,
                    int64_t n_vertices, int32_t n_labels, NormQuery &q, std::string &msg);

// Traversal + step programs. domains: whether cycle-closing edges get a
// frontier-domain filter. stats may be null. direction: the direction-driven
// traversal of Section 6.1.1 for queries without constants (with constants the
// degree-driven traversal of Section 6.1.2 applies, as the paper prescribes).
int build_plan(const NormQuery &q, const LabelStats *stats, bool domains, Plan &plan, std::string &msg,
               bool direction = false);

}  // namespace gs
