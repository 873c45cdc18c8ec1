// Query planner: the degree-driven traversal of Section 6.1.2 and the step
// programs of the level-synchronous binding tree (Sections 5 and 7.1).
#include "planner.hpp"

#include <algorithm>
#include <array>
#include <cstdio>

#include "gsmart.h"

namespace gs {

int normalise_query(int32_t n_qv, const int32_t *qv_const, int32_t n_edges, const int32_t *e3,
                    int64_t n_vertices, int32_t n_labels, NormQuery &q, std::string &msg) {
  if (n_qv <= 0 || n_edges <= 0 || !e3) { msg = "query needs at least one vertex and one edge"; return GS_EINVAL; }
  if (n_edges > kMaxEdges) { msg = "more than 64 edges"; return GS_EUNSUPPORTED; }
  if (n_qv > 2 * kMaxEdges + 1) { msg = "too many query vertices"; return GS_EUNSUPPORTED; }
  q = NormQuery();
  q.n_qv = n_qv;
  q.cst.assign(n_qv, -1);
  int nvars = 0;
  for (int i = 0; i < n_qv; ++i) {
    int32_t c = qv_const ? qv_const[i] : -1;
    if (c < -1 || (n_vertices >= 0 && c >= n_vertices)) { msg = "constant vertex id out of range"; return GS_ERANGE; }
    q.cst[i] = c;
    nvars += (c < 0);
  }
  if (nvars > kMaxVars) { msg = "more than 64 variables"; return GS_EUNSUPPORTED; }
  std::vector<int> deg(n_qv, 0);
  for (int k = 0; k < n_edges; ++k) {
    QEdge e{e3[3 * k], e3[3 * k + 1], e3[3 * k + 2]};
    if (e.s < 0 || e.s >= n_qv || e.o < 0 || e.o >= n_qv) { msg = "edge endpoint is not a query vertex"; return GS_EINVAL; }
    if (e.p < 1 || (n_labels >= 0 && e.p > n_labels)) { msg = "edge label out of range"; return GS_ERANGE; }
    int found = -1;
    for (size_t j = 0; j < q.edges.size(); ++j)
      if (q.edges[j].s == e.s && q.edges[j].p == e.p && q.edges[j].o == e.o) found = (int)j;
    if (found < 0) { found = (int)q.edges.size(); q.edges.push_back(e); q.edge_first.push_back(1); }
    else q.edge_first.push_back(0);
    q.edge_map.push_back(found);
    deg[e.s]++; deg[e.o]++;
  }
  for (int i = 0; i < n_qv; ++i)
    if (q.cst[i] < 0 && deg[i] == 0) { msg = "a variable has no incident edge"; return GS_EINVAL; }
  return GS_OK;
}

namespace {

// Estimated size of seg(c, label, dir) from label statistics (average degree).
double est_seg(const LabelStats *st, int32_t label0, int dir) {
  if (!st || st->nnz.empty()) return 1.0;
  double holders = (double)(dir == 0 ? st->rows[label0] : st->cols[label0]);
  return holders > 0 ? (double)st->nnz[label0] / holders : 0.0;
}

}  // namespace

int build_plan(const NormQuery &q, const LabelStats *st, bool want_domains, Plan &P, std::string &msg,
               bool direction) {
  P = Plan();
  const int nv = q.n_qv, ne = (int)q.edges.size();
  std::vector<uint8_t> evaluated(ne, 0), visited(nv, 0);
  std::vector<int32_t> discovered_by_edge(nv, -1);   // edge through which a vertex was first reached
  P.edge_group.assign(ne, -1);

  auto is_var = [&](int v) { return q.cst[v] < 0; };
  auto unev = [&](int v, int &total, int &out) {
    total = out = 0;
    for (int k = 0; k < ne; ++k) {
      if (evaluated[k]) continue;
      const QEdge &e = q.edges[k];
      if (e.s == v || e.o == v) { ++total; if (e.s == v) ++out; }
    }
  };

  // Constants rule, step 1: constants are visited and their incident edges evaluated first.
  bool has_const = false;
  for (int v = 0; v < nv; ++v) if (!is_var(v)) { visited[v] = 1; has_const = true; }
  if (has_const) {
    int g = -1;
    for (int k = 0; k < ne; ++k) {
      const QEdge &e = q.edges[k];
      if (!is_var(e.s) || !is_var(e.o)) {
        if (g < 0) { g = (int)P.group_vertex.size(); P.group_vertex.push_back(-1); }
        evaluated[k] = 1; P.edge_group[k] = g;
      }
    }
  }
  auto adjacent_to_const = [&](int v) {
    for (int k = 0; k < ne; ++k) {
      const QEdge &e = q.edges[k];
      if ((e.s == v && !is_var(e.o)) || (e.o == v && !is_var(e.s))) return true;
    }
    return false;
  };
  // smallest estimated constant-seeded candidate set of v (tie-break of the root choice)
  auto seed_est = [&](int v) {
    double best = 1e300;
    for (int k = 0; k < ne; ++k) {
      const QEdge &e = q.edges[k];
      if (e.s == v && !is_var(e.o)) best = std::min(best, est_seg(st, e.p - 1, 1));
      if (e.o == v && !is_var(e.s)) best = std::min(best, est_seg(st, e.p - 1, 0));
    }
    return best;
  };

  std::vector<int32_t> pop_order;
  if (direction && !has_const) {
    // Direction-driven traversal (Section 6.1.1): DFS along edge directions. A root is an
    // unvisited vertex without unevaluated incoming edges (for cyclic queries, if none has,
    // any unvisited vertex), the one with the most unevaluated outgoing edges; a popped vertex
    // evaluates its unevaluated outgoing edges and pushes the newly reached vertices in
    // ascending order of unevaluated outgoing edges (ties: the lower index pops first).
    auto unev_in = [&](int v) {
      int n = 0;
      for (int k = 0; k < ne; ++k) if (!evaluated[k] && q.edges[k].o == v && q.edges[k].s != v) ++n;
      return n;
    };
    for (;;) {
      bool all_eval = true;
      for (int k = 0; k < ne; ++k) if (!evaluated[k]) all_eval = false;
      bool all_visited = true;
      for (int v = 0; v < nv; ++v) if (!visited[v]) all_visited = false;
      if (all_eval && all_visited) break;
      int root = -1, bo = -1;
      for (int pass = 0; pass < 2 && root < 0; ++pass)
        for (int v = 0; v < nv; ++v) {
          if (visited[v] || (pass == 0 && unev_in(v) > 0)) continue;
          int t, o; unev(v, t, o);
          if (root < 0 || o > bo) { root = v; bo = o; }
        }
      if (root < 0) break;
      P.roots.push_back(root);
      visited[root] = 1;
      std::vector<int32_t> stack{root};
      while (!stack.empty()) {
        int v = stack.back(); stack.pop_back();
        pop_order.push_back(v);
        std::vector<int32_t> found;
        int g = -1;
        for (int k = 0; k < ne; ++k) {
          if (evaluated[k] || q.edges[k].s != v) continue;
          if (g < 0) { g = (int)P.group_vertex.size(); P.group_vertex.push_back(v); }
          evaluated[k] = 1; P.edge_group[k] = g;
          const int w = q.edges[k].o;
          if (w != v && !visited[w]) { visited[w] = 1; discovered_by_edge[w] = k; found.push_back(w); }
        }
        std::vector<std::array<int, 2>> keyed;
        for (int w : found) { int t, o; unev(w, t, o); keyed.push_back({o, -w}); }
        std::sort(keyed.begin(), keyed.end());
        for (auto &kk : keyed) stack.push_back(-kk[1]);
      }
      // edges into vertices that were visited already wait for the next root (Step 5)
    }
  }
  for (;;) {
    if (direction && !has_const) break;
    bool all_visited = true;
    for (int v = 0; v < nv; ++v) if (is_var(v) && !visited[v]) all_visited = false;
    bool all_eval = true;
    for (int k = 0; k < ne; ++k) if (!evaluated[k]) all_eval = false;
    if (all_visited && all_eval) break;
    // Step 2: the root. With constants, prefer unvisited vertices adjacent to a constant.
    int root = -1;
    for (int pass = 0; pass < 2 && root < 0; ++pass) {
      int bt = -1, bo = -1; double bs = 0;
      for (int v = 0; v < nv; ++v) {
        if (!is_var(v) || visited[v]) continue;
        if (pass == 0 && !(has_const && adjacent_to_const(v))) continue;
        int t, o; unev(v, t, o);
        double s = seed_est(v);
        bool better = root < 0 || t > bt || (t == bt && o > bo) || (t == bt && o == bo && s < bs);
        if (better) { root = v; bt = t; bo = o; bs = s; }
      }
    }
    if (root < 0) break;
    P.roots.push_back(root);
    visited[root] = 1;
    std::vector<int32_t> stack{root};
    while (!stack.empty()) {                       // steps 3-4
      int v = stack.back(); stack.pop_back();
      pop_order.push_back(v);
      std::vector<int32_t> found;
      int g = -1;
      for (int k = 0; k < ne; ++k) {
        if (evaluated[k]) continue;
        const QEdge &e = q.edges[k];
        if (e.s != v && e.o != v) continue;
        if (g < 0) { g = (int)P.group_vertex.size(); P.group_vertex.push_back(v); }
        evaluated[k] = 1; P.edge_group[k] = g;
        int w = (e.s == v) ? e.o : e.s;
        if (w != v && is_var(w) && !visited[w]) {
          visited[w] = 1; discovered_by_edge[w] = k; found.push_back(w);
        }
      }
      // push in ascending order of unevaluated edges, then of unevaluated out-edges;
      // equal keys push the higher index first so the lower index pops first
      std::vector<std::array<int, 3>> keyed;
      for (int w : found) { int t, o; unev(w, t, o); keyed.push_back({t, o, -w}); }
      std::sort(keyed.begin(), keyed.end());
      for (auto &kk : keyed) stack.push_back(-kk[2]);
    }
  }

  // Level order. The traversal above (roots, edge groups, pops) is the
  // paper's; it keeps one binding tree per traversal path, where the single
  // tree here interleaves the paths. Every vertex follows the vertex that
  // discovered it; among the vertices that may come next, the one with the
  // smallest estimated fan-out goes first, so that selective vertices
  // (constant seeds, label filters, closed cycles) shrink the tree before
  // wide ones grow it. Ties keep the pop order; a further root is placed
  // when nothing else can be.
  const double nvert = (st && st->n > 0) ? (double)st->n : 1.0;
  std::vector<uint8_t> placed(nv, 0);
  auto fanout = [&](int w) {
    const int k0 = discovered_by_edge[w];
    const QEdge &e0 = q.edges[k0];
    const int u = (e0.s == w) ? e0.o : e0.s;
    double f = est_seg(st, e0.p - 1, e0.s == u ? 0 : 1);
    if (!st || st->nnz.empty()) return f;
    for (int k = 0; k < ne; ++k) {
      const QEdge &e = q.edges[k];
      if (k == k0 || (e.s != w && e.o != w) || e.s == e.o) continue;
      const int x = (e.s == w) ? e.o : e.s;
      if (!is_var(x) || placed[x])   // seed bitmap, or exact check against a bound vertex
        f *= std::min(1.0, est_seg(st, e.p - 1, e.s == x ? 0 : 1) / nvert);
      else                           // label-existence filter (Eq. 4/5)
        f *= (double)(e.s == w ? st->rows[e.p - 1] : st->cols[e.p - 1]) / nvert;
    }
    return f;
  };
  std::vector<int32_t> order;
  size_t next_root = 0;
  while (order.size() < pop_order.size()) {
    int best = -1;
    double bf = 0;
    for (int w : pop_order) {
      if (placed[w] || discovered_by_edge[w] < 0) continue;
      const QEdge &e = q.edges[discovered_by_edge[w]];
      if (!placed[(e.s == w) ? e.o : e.s]) continue;
      const double f = fanout(w);
      if (best < 0 || f < bf) { best = w; bf = f; }
    }
    if (best < 0) {
      if (next_root >= P.roots.size()) { msg = "planner: no vertex can take the next level"; return GS_EINVAL; }
      best = P.roots[next_root++];
      // A further root of the direction-driven traversal can have edges to vertices already
      // placed (v3 -> v2 in Example 6.1); the single binding tree binds it through the one
      // with the smallest estimated segment, read against its direction.
      double bs = 0;
      for (int k = 0; k < ne; ++k) {
        const QEdge &e = q.edges[k];
        if (e.s == e.o || (e.s != best && e.o != best)) continue;
        const int u = (e.s == best) ? e.o : e.s;
        if (!is_var(u) || !placed[u]) continue;
        const double s = est_seg(st, e.p - 1, e.s == u ? 0 : 1);
        if (discovered_by_edge[best] < 0 || s < bs) { discovered_by_edge[best] = k; bs = s; }
      }
    }
    placed[best] = 1;
    order.push_back(best);
  }
  P.n_vars = (int)order.size();
  P.order = order;
  std::vector<int32_t> level_of(nv, -1);
  for (int j = 0; j < P.n_vars; ++j) level_of[order[j]] = j;
  {
    std::vector<int32_t> vars;
    for (int v = 0; v < nv; ++v) if (is_var(v)) vars.push_back(v);
    if ((int)vars.size() != P.n_vars) { msg = "planner did not reach every variable"; return GS_EINVAL; }
    P.var_rank.assign(P.n_vars, 0);
    for (int j = 0; j < P.n_vars; ++j)
      P.var_rank[j] = (int)(std::lower_bound(vars.begin(), vars.end(), order[j]) - vars.begin());
  }
  for (int k = 0; k < ne; ++k) {
    const QEdge &e = q.edges[k];
    if (!is_var(e.s) && !is_var(e.o)) P.cchecks.push_back({q.cst[e.s], e.p - 1, q.cst[e.o]});
  }

  // Step programs.
  P.steps.resize(P.n_vars);
  std::vector<std::vector<int32_t>> refs(P.n_vars);   // levels referenced by each step
  for (int j = 0; j < P.n_vars; ++j) {
    PlanStep &S = P.steps[j];
    int x = order[j];
    S.qv = x;
    int pe = discovered_by_edge[x];
    if (pe >= 0 && level_of[(q.edges[pe].s == x) ? q.edges[pe].o : q.edges[pe].s] >= j) pe = -1;
    if (pe >= 0) {
      const QEdge &e = q.edges[pe];
      int u = (e.s == x) ? e.o : e.s;
      S.kind = STEP_SEG; S.src_level = level_of[u]; S.label = e.p - 1; S.dir = (e.s == u) ? 0 : 1;
      S.parent_edge = pe;
      refs[j].push_back(S.src_level);
    } else {
      // no bound neighbour: seed from the constant edge with the smallest estimated segment, else a list
      int best = -1; double bs = 1e300;
      for (int k = 0; k < ne; ++k) {
        const QEdge &e = q.edges[k];
        double s;
        if (e.o == x && e.s != x && !is_var(e.s)) s = est_seg(st, e.p - 1, 0);
        else if (e.s == x && e.o != x && !is_var(e.o)) s = est_seg(st, e.p - 1, 1);
        else continue;
        if (best < 0 || s < bs) { best = k; bs = s; }
      }
      if (best >= 0) {
        const QEdge &e = q.edges[best];
        S.kind = STEP_SEG_CONST; S.parent_edge = best; S.label = e.p - 1;
        if (e.o == x) { S.src_const = q.cst[e.s]; S.dir = 0; } else { S.src_const = q.cst[e.o]; S.dir = 1; }
      } else {
        S.kind = STEP_LIST;
      }
    }
    if (S.kind == STEP_LIST)
      for (int k = 0; k < ne; ++k) {   // a list level is bound by nothing earlier, so tests nothing earlier
        const QEdge &e = q.edges[k];
        const int w = (e.s == x) ? e.o : (e.o == x ? e.s : -1);
        if (w >= 0 && w != x && is_var(w) && level_of[w] < j) {
          msg = "planner: a list level with an edge to an earlier level";
          return GS_EINVAL;
        }
      }
    for (int k = 0; k < ne; ++k) {
      if (k == S.parent_edge) continue;
      const QEdge &e = q.edges[k];
      if (e.s != x && e.o != x) continue;
      if (e.s == x && e.o == x) { S.self_labels.push_back(e.p - 1); continue; }
      int w = (e.s == x) ? e.o : e.s;
      if (!is_var(w)) {                                   // constant: exact seed bitmap
        SeedSpec sd{q.cst[w], e.p - 1, (e.s == w) ? 0 : 1};
        S.filters.push_back({F_SEED, (int32_t)P.seeds.size()});
        P.seeds.push_back(sd);
        continue;
      }
      int lw = level_of[w];
      if (lw < j) {                                       // bound earlier: exact check (+ domain)
        CheckRef c{lw, e.p - 1, (e.s == w) ? 0 : 1};
        S.checks.push_back(c);
        refs[j].push_back(lw);
      } else {                                            // bound later: label-existence filter (Eq. 4/5)
        S.filters.push_back({e.s == x ? F_LABEL_OUT : F_LABEL_IN, e.p - 1});
      }
    }
    if (want_domains && j > 0) {
      for (const CheckRef &c : S.checks) {
        DomainSpec d{j, c.level, c.label, c.dir, {}};
        for (const FilterRef &f : S.filters) if (f.kind != F_DOMAIN) d.mask.push_back(f);
        S.filters.push_back({F_DOMAIN, (int32_t)P.domains.size()});
        P.domains.push_back(d);
      }
    }
  }
  // Carried bindings: level j keeps every earlier binding referenced by a later step.
  for (int j = 0; j < P.n_vars; ++j) {
    std::vector<uint8_t> need(P.n_vars, 0);
    for (int s = j + 1; s < P.n_vars; ++s)
      for (int32_t l : refs[s]) if (l < j) need[l] = 1;
    for (int l = 0; l < j; ++l) if (need[l]) P.steps[j].carried.push_back(l);
  }
  return GS_OK;
}

}  // namespace gs
