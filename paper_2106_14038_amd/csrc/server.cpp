// Served form: a request loop with iteration-level continuous batching.
//
// Every iteration advances each active query by one tree level in a single
// launch sequence (the same kernels as the batched form), so queries admitted
// between iterations start at their own level 0 while older ones continue.
// Admission is by estimated binding-tree bytes against a budget and by free
// query slots and bitmaps. Tree levels are bump-allocated by the kernels inside
// a window of the tree arena; the arena is used as a ring of per-iteration
// regions, each freed when every query with a level in it has retired. A query
// whose level does not fit its window is restarted later (re-queued); a query
// that does not fit an otherwise empty arena fails with GS_ENOMEM. Finished
// queries copy their rows to host memory owned by the result.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "engine.hpp"
#include "gsmart.h"
#include "query.hpp"

struct gs_server;

namespace gs {

namespace {

constexpr int kSlotSteps = kMaxLevels, kSlotFilt = 1024, kSlotChk = 128, kSlotInts = 512, kSlotCc = 64;
constexpr int kSlotDom = 64, kSlotSeed = 64, kIterDomPerQuery = 16;

using clock_t_ = std::chrono::steady_clock;

double now_ms() {
  return std::chrono::duration<double, std::milli>(clock_t_::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  int32_t n_qv = 0;
  std::vector<int32_t> qv_const;
  std::vector<gs_edge> edges;
  uint32_t flags = 0;
  double t_arrive = 0;
  int attempts = 0;
};

struct Region { uint64_t start, end; int refs; };

struct Active {
  Request req;
  QInfo qi;
  Tables T;                 // slot-rebased tables
  int slot = -1;
  int level = 0;            // next level to produce
  double est_bytes = 0;
  std::vector<int> bitmaps; // pool indices
  std::vector<uint64_t> regions;   // region ids holding its levels
  bool count_only = false;
};

}  // namespace

struct ServerImpl {
  Engine *E = nullptr;
  gs_server_options opt{};
  std::thread th;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  bool stopping = false;
  uint64_t next_ticket = 1;
  std::deque<Request> pending;
  std::unordered_map<uint64_t, std::pair<int, Result *>> done;
  gs_server_stats stats{};

  int cap = 0;
  // device tables (persistent, per slot)
  DStep *d_steps = nullptr;
  const uint64_t **d_filt = nullptr;
  DCheck *d_checks = nullptr;
  int32_t *d_ints = nullptr;
  DConst *d_cc = nullptr;
  int32_t *d_vr = nullptr;
  int32_t **d_lvlp = nullptr;
  int32_t **d_lvlc = nullptr;
  int64_t *d_lvln = nullptr;
  int64_t *d_qs = nullptr;
  // per-iteration
  DEntry *d_ents = nullptr;
  DDomain *d_doms = nullptr;
  uint64_t **d_clear = nullptr;
  DSeed *d_seeds = nullptr;
  int64_t *d_fc = nullptr;
  EState *d_es = nullptr;
  IterScalars *d_it = nullptr;
  int64_t *d_blk = nullptr;
  int64_t *d_zero = nullptr;
  int32_t *d_flags = nullptr;       // run flags (RF_*), cleared before every iteration
  int32_t *d_rows = nullptr;
  size_t rows_cap = 0;
  // bitmap pool
  uint64_t *pool = nullptr;
  std::vector<int> free_bm;
  std::vector<int> free_slots;
  // tree arena ring
  std::list<std::pair<uint64_t, Region>> regions;   // id -> region, oldest first
  uint64_t next_region = 1;
  uint64_t head = 0;
  double est_in_use = 0;
  std::vector<Active *> active;
};

}  // namespace gs

struct gs_server { gs::ServerImpl s; };

namespace gs {

namespace {

double estimate_tree_bytes(const Engine &E, const QInfo &qi) {
  const Plan &P = qi.plan;
  const double N = (double)E.g.n;
  auto holders = [&](const FilterRef &f) -> double {
    if (f.kind == F_LABEL_OUT) return (double)E.stats.rows[f.arg];
    if (f.kind == F_LABEL_IN) return (double)E.stats.cols[f.arg];
    if (f.kind == F_SEED) {
      const SeedSpec &s = P.seeds[f.arg];
      const double h = (double)(s.dir == 0 ? E.stats.rows[s.label] : E.stats.cols[s.label]);
      return h > 0 ? (double)E.stats.nnz[s.label] / h : 0.0;
    }
    return N;
  };
  auto avg = [&](int label, int dir) {
    const double h = (double)(dir == 0 ? E.stats.rows[label] : E.stats.cols[label]);
    return h > 0 ? (double)E.stats.nnz[label] / h : 0.0;
  };
  double L = 1, bytes = 0;
  for (int j = 0; j < P.n_vars; ++j) {
    const PlanStep &ps = P.steps[j];
    double sel = 1;
    for (const FilterRef &f : ps.filters) if (f.kind != F_DOMAIN) sel *= std::min(1.0, holders(f) / N);
    double cand;
    if (ps.kind == STEP_LIST) cand = N;
    else cand = avg(ps.label, ps.dir);
    L = (ps.kind == STEP_LIST ? L * N : L * cand) * sel;
    L = std::min(L, 4e9);
    bytes += L * 4.0 * (2 + ps.carried.size());
  }
  return bytes;
}

// Rebase a query's dense tables onto its slot's fixed regions of the device tables.
bool rebase_tables(QInfo &qi, Tables &T, int slot) {
  if (T.steps.size() > (size_t)kSlotSteps || T.filt.size() > (size_t)kSlotFilt || T.checks.size() > (size_t)kSlotChk ||
      T.ints.size() > (size_t)kSlotInts || T.cconst.size() > (size_t)kSlotCc || T.doms.size() > (size_t)kSlotDom ||
      T.seeds.size() > (size_t)kSlotSeed)
    return false;
  for (DStep &d : T.steps) {
    d.filt0 += slot * kSlotFilt;
    d.chk0 += slot * kSlotChk;
    d.self0 += slot * kSlotInts;
    d.copy0 += slot * kSlotInts;
    d.cc0 += slot * kSlotCc;
  }
  for (DDomain &d : T.doms) d.filt0 += slot * kSlotFilt;
  qi.step0 = slot * kSlotSteps;
  return true;
}

void finish(ServerImpl &S, uint64_t ticket, int status, Result *R) {
  std::lock_guard<std::mutex> lk(S.mu);
  S.done[ticket] = {status, R};
  if (status == GS_OK) S.stats.completed++;
  else S.stats.rejected++;
  S.cv_done.notify_all();
}

void release(ServerImpl &S, Active *a) {
  for (int b : a->bitmaps) S.free_bm.push_back(b);
  a->bitmaps.clear();
  for (uint64_t id : a->regions)
    for (auto &r : S.regions) if (r.first == id) { r.second.refs--; break; }
  a->regions.clear();
  while (!S.regions.empty() && S.regions.front().second.refs <= 0) S.regions.pop_front();
  if (S.regions.empty()) S.head = 0;
  if (a->slot >= 0) S.free_slots.push_back(a->slot);
  a->slot = -1;
  S.est_in_use -= a->est_bytes;
}

// Largest free window of the ring: [head, cap) or [0, tail) when wrapping.
void window(const ServerImpl &S, uint64_t &lo, uint64_t &hi) {
  const uint64_t cap = S.E->tree_cap;
  if (S.regions.empty()) { lo = 0; hi = cap; return; }
  const uint64_t tail = S.regions.front().second.start;
  if (S.head >= tail) {   // live data in [tail, head)
    if (cap - S.head >= tail) { lo = S.head; hi = cap; } else { lo = 0; hi = tail; }
  } else {                // wrapped: live in [tail, cap) and [0, head)
    lo = S.head; hi = tail;
  }
}

// 1: admitted (or finished with an error), -1: no room now (rq is left untouched).
int admit(ServerImpl &S, Request &rq, std::vector<Active *> &fresh) {
  Engine &E = *S.E;
  Active *a = new Active();
  a->req = rq;
  gs_query q{a->req.n_qv, a->req.qv_const.data(), (int32_t)a->req.edges.size(), a->req.edges.data()};
  std::string msg;
  int rc = plan_query(E, q, a->qi, msg);
  if (rc != GS_OK) { set_error(msg); finish(S, a->req.ticket, rc, nullptr); delete a; return 1; }
  a->count_only = ((a->req.flags | S.opt.flags) & GS_COUNT_ONLY) != 0;
  const int need_bm = (int)a->qi.plan.seeds.size() + 2 * (int)a->qi.plan.domains.size();
  if (S.free_slots.empty() || (int)S.free_bm.size() < need_bm) { delete a; return -1; }
  a->est_bytes = estimate_tree_bytes(E, a->qi);
  const double budget = S.opt.tree_budget_bytes ? (double)S.opt.tree_budget_bytes : (double)E.tree_cap;
  if ((!S.active.empty() || !fresh.empty()) && S.est_in_use + a->est_bytes > budget) { delete a; return -1; }
  a->slot = S.free_slots.back();
  S.free_slots.pop_back();
  for (int k = 0; k < need_bm; ++k) { a->bitmaps.push_back(S.free_bm.back()); S.free_bm.pop_back(); }
  int next = 0;
  const int64_t words = E.g.words;
  auto next_bitmap = [&](bool) { return S.pool + (uint64_t)a->bitmaps[next++] * words; };
  compile_query(E, a->qi, a->count_only, a->slot, a->T, next_bitmap);
  if (!rebase_tables(a->qi, a->T, a->slot) ||
      a->T.doms.size() > (size_t)kIterDomPerQuery * std::max<size_t>(1, a->qi.plan.n_vars)) {
    set_error("query too large for a server slot");
    release(S, a);
    finish(S, a->req.ticket, GS_EUNSUPPORTED, nullptr);
    delete a;
    return 1;
  }
  S.est_in_use += a->est_bytes;
  fresh.push_back(a);
  return 1;
}

hipError_t upload_slot(ServerImpl &S, Active *a, hipStream_t s) {
  const int sl = a->slot;
  const Tables &T = a->T;
  hipError_t e = hipSuccess;
  auto cp = [&](void *dst, const void *src, size_t bytes) {
    if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  cp(S.d_steps + (size_t)sl * kSlotSteps, T.steps.data(), sizeof(DStep) * T.steps.size());
  cp(S.d_filt + (size_t)sl * kSlotFilt, T.filt.data(), sizeof(void *) * T.filt.size());
  cp(S.d_checks + (size_t)sl * kSlotChk, T.checks.data(), sizeof(DCheck) * T.checks.size());
  cp(S.d_ints + (size_t)sl * kSlotInts, T.ints.data(), sizeof(int32_t) * T.ints.size());
  cp(S.d_cc + (size_t)sl * kSlotCc, T.cconst.data(), sizeof(DConst) * T.cconst.size());
  cp(S.d_vr + (size_t)sl * kMaxLevels, T.var_rank.data(), sizeof(int32_t) * T.var_rank.size());
  if (e == hipSuccess) e = zero_words((uint64_t *)(S.d_lvlp + (size_t)sl * kMaxLevels), kMaxLevels, s);
  if (e == hipSuccess) e = zero_words((uint64_t *)(S.d_lvlc + (size_t)sl * kMaxLevels), kMaxLevels, s);
  if (e == hipSuccess) e = zero_words((uint64_t *)(S.d_lvln + (size_t)sl * kMaxLevels), kMaxLevels, s);
  if (e == hipSuccess) e = zero_words((uint64_t *)(S.d_qs + (size_t)sl * QS_N), QS_N, s);
  return e;
}

// Copy a finished query out of the ring into a result that owns host memory.
// lp_all, lc_all, qs_all, lvl_n_all: host copies of the slots' level pointers, counters and sizes.
int retire(ServerImpl &S, Active *a, int32_t *const *lp_all, int32_t *const *lc_all, const int64_t *qs_all,
           const int64_t *lvl_n_all, hipStream_t s) {
  Engine &E = *S.E;
  if (qs_all[(size_t)a->slot * QS_N + QS_OVERFLOW] == 3) {
    set_error("a node's product of leaf segments exceeds 2^50 (count-only factor)");
    return GS_ERANGE;
  }
  Result *R = new Result();
  R->eng = &E;
  hipError_t e = hipSuccess;
  const size_t lv = (size_t)a->slot * kMaxLevels;
  fill_result(*R, a->qi, a->count_only, lp_all + lv, lc_all + lv, lvl_n_all + lv, qs_all + (size_t)a->slot * QS_N, 0,
              0);
  R->host_owned = true;
  if (!a->count_only && R->count > 0 && R->k > 0) {
    const int k = R->k;
    R->host_rows.resize((size_t)R->count * k);
    const int64_t chunk = std::max<int64_t>(1, (int64_t)(S.rows_cap / (4 * (size_t)k)));
    for (int64_t r = 0; r < R->count && e == hipSuccess; r += chunk) {
      const int64_t c = std::min(chunk, R->count - r);
      e = launch_enumerate(S.d_lvlp + (size_t)a->slot * kMaxLevels, S.d_lvlc + (size_t)a->slot * kMaxLevels,
                           S.d_lvln + (size_t)a->slot * kMaxLevels, k,
                           S.d_vr + (size_t)a->slot * kMaxLevels, r, c, S.d_rows, s);
      if (e == hipSuccess)
        e = hipMemcpyAsync(R->host_rows.data() + (size_t)r * k, S.d_rows, sizeof(int32_t) * c * k,
                           hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) { delete R; return GS_EDEVICE; }
  }
  R->lvl_ptr.assign(R->lvl_ptr.size(), nullptr);   // the ring space is released below
  R->lvl_cptr.assign(R->lvl_cptr.size(), nullptr);
  const double t = now_ms();
  R->stats.latency_ms = t - a->req.t_arrive;
  finish(S, a->req.ticket, GS_OK, R);
  return GS_OK;
}

void fail_all(ServerImpl &S, int status) {
  for (Active *a : S.active) { release(S, a); finish(S, a->req.ticket, status, nullptr); delete a; }
  S.active.clear();
}

void loop(ServerImpl &S) {
  Engine &E = *S.E;
  hipStream_t s = E.stream;
  (void)hipSetDevice(E.device);
  std::vector<int64_t> lvl_n((size_t)S.cap * kMaxLevels), qs_all((size_t)S.cap * QS_N);
  std::vector<int32_t *> lp_all((size_t)S.cap * kMaxLevels), lc_all((size_t)S.cap * kMaxLevels);
  const bool prof = E.opt.profile_kernels != 0;
  for (;;) {
    std::vector<Active *> fresh;
    std::deque<Request> todo;
    {
      std::unique_lock<std::mutex> lk(S.mu);
      S.cv.wait(lk, [&] { return S.stopping || !S.pending.empty() || !S.active.empty(); });
      if (S.stopping && S.pending.empty() && S.active.empty()) break;
      todo.swap(S.pending);
    }
    while (!todo.empty()) {               // admit in arrival order while there is room
      if (admit(S, todo.front(), fresh) < 0) break;
      todo.pop_front();
    }
    if (!todo.empty()) {                  // the rest waits, ahead of newer arrivals
      std::lock_guard<std::mutex> lk(S.mu);
      while (!todo.empty()) { S.pending.push_front(std::move(todo.back())); todo.pop_back(); }
    }
    std::lock_guard<std::mutex> elk(E.mu);
    for (Active *a : fresh) {
      if (a->qi.zero) {   // constants only: evaluate now
        std::vector<DConst> cc;
        for (const ConstCheck &c : a->qi.plan.cchecks) cc.push_back({c.a, c.label, c.b, 0});
        int64_t ok = 0;
        hipError_t e = hipMemcpyAsync(S.d_cc + (size_t)a->slot * kSlotCc, cc.data(), sizeof(DConst) * cc.size(),
                                      hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = launch_const_only(E.g, S.d_cc + (size_t)a->slot * kSlotCc, (int)cc.size(), S.d_zero, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&ok, S.d_zero, 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        Result *R = new Result();
        R->eng = &E;
        std::vector<int64_t> qs0(QS_N, 0);
        fill_result(*R, a->qi, a->count_only, nullptr, nullptr, nullptr, qs0.data(), ok, 0);
        R->host_owned = true;
        R->stats.latency_ms = now_ms() - a->req.t_arrive;
        release(S, a);
        finish(S, a->req.ticket, e == hipSuccess ? GS_OK : GS_EDEVICE, e == hipSuccess ? R : nullptr);
        if (e != hipSuccess) delete R;
        delete a;
        continue;
      }
      if (upload_slot(S, a, s) != hipSuccess) { release(S, a); finish(S, a->req.ticket, GS_EDEVICE, nullptr); delete a; continue; }
      S.active.push_back(a);
    }
    if (S.active.empty()) continue;
    S.stats.max_active_seen = std::max<int64_t>(S.stats.max_active_seen, (int64_t)S.active.size());

    // this iteration's work lists
    IterLists L;
    IterLists one;
    std::vector<const QInfo *> qv(1);
    std::vector<int> lv(1);
    for (Active *a : S.active) {
      // tables of this query are local: seed0 = dom0 = 0 (set once at admission)
      qv[0] = &a->qi;
      lv[0] = a->level;
      build_iteration(a->T, qv, lv, one);
      for (DEntry e : one.ents) { e.dom0 += (int32_t)L.doms.size(); L.ents.push_back(e); }
      L.doms.insert(L.doms.end(), one.doms.begin(), one.doms.end());
      L.clears.insert(L.clears.end(), one.clears.begin(), one.clears.end());
      L.seeds.insert(L.seeds.end(), one.seeds.begin(), one.seeds.end());
      L.has_list |= one.has_list;
      L.has_tested |= one.has_tested;
      L.has_checks |= one.has_checks;
      L.has_factor |= one.has_factor;
      L.has_exact |= one.has_exact;
    }
    uint64_t wlo, whi;
    window(S, wlo, whi);
    DArena ar[2];
    ar[0] = {wlo, whi, 0, 0};
    ar[1] = {0, E.scratch_cap, 0, 0};
    hipError_t e = hipMemcpyAsync(S.d_ents, L.ents.data(), sizeof(DEntry) * L.ents.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !L.doms.empty())
      e = hipMemcpyAsync(S.d_doms, L.doms.data(), sizeof(DDomain) * L.doms.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !L.clears.empty())
      e = hipMemcpyAsync(S.d_clear, L.clears.data(), sizeof(void *) * L.clears.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !L.seeds.empty())
      e = hipMemcpyAsync(S.d_seeds, L.seeds.data(), sizeof(DSeed) * L.seeds.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(E.d_arenas, ar, sizeof(ar), hipMemcpyHostToDevice, s);
    IterArgs A{};
    A.g = E.g; A.ent = S.d_ents; A.E = (int32_t)L.ents.size(); A.S = (int32_t)L.seeds.size();
    A.D = (int32_t)L.doms.size(); A.nclear = (int32_t)L.clears.size(); A.has_list = L.has_list; A.has_tested = L.has_tested; A.has_checks = L.has_checks; A.has_factor = L.has_factor; A.has_exact = L.has_exact; A.grid = E.grid; A.wgrid = E.wgrid; A.wwaves = E.wwaves;
    A.steps = S.d_steps; A.filt = S.d_filt; A.checks = S.d_checks; A.ints = S.d_ints; A.cconst = S.d_cc;
    A.seeds = S.d_seeds; A.doms = S.d_doms; A.fcount = S.d_fc; A.clear = S.d_clear; A.es = S.d_es; A.it = S.d_it;
    A.lvl_ptr = S.d_lvlp; A.lvl_cptr = S.d_lvlc; A.lvl_n = S.d_lvln; A.qstats = S.d_qs;
    A.scratch = E.d_arenas + 1; A.scratch_base = E.scratch_base; A.tree = E.d_arenas; A.tree_base = E.tree_base;
    A.blk_a = S.d_blk; A.blk_b = S.d_blk + E.grid; A.blk_off_a = S.d_blk + 2 * E.grid; A.blk_off_b = S.d_blk + 3 * E.grid;
    A.flags = S.d_flags;
    if (e == hipSuccess) e = zero_words((uint64_t *)S.d_flags, 1, s);
    if (prof) {
      while (E.events.size() < (size_t)2 * KS_N) { hipEvent_t ev; (void)hipEventCreate(&ev); E.events.push_back(ev); }
    }
    if (e == hipSuccess) e = launch_iteration(A, s, prof ? E.events.data() : nullptr);
    IterScalars I{};
    int32_t rflags[RF_N] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(rflags, S.d_flags, sizeof(rflags), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(lvl_n.data(), S.d_lvln, 8 * lvl_n.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ar, E.d_arenas, sizeof(ar), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&I, S.d_it, sizeof(I), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    S.stats.iterations++;
    if (e != hipSuccess) { set_error(hipGetErrorString(e)); fail_all(S, GS_EDEVICE); continue; }
    if (rflags[RF_WRITE]) {
      set_error("device inconsistency: the write pass met output positions beyond a level's count");
      fail_all(S, GS_EDEVICE);
      continue;
    }
    if (rflags[RF_SCRATCH]) ar[1].overflow = 1;   // the iteration was aborted: restart its queries
    if (prof) account_iteration(E, E.events.data(), I, L, 0, 0);

    // level pointers and counters of every slot, once, when some query finishes now
    bool finishing = false;
    for (Active *a : S.active)
      if (lvl_n[(size_t)a->slot * kMaxLevels + a->level] >= 0 && !ar[1].overflow && a->level + 1 == a->qi.nlev)
        finishing = true;
    if (finishing) {
      e = hipMemcpyAsync(lp_all.data(), S.d_lvlp, sizeof(void *) * lp_all.size(), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipMemcpyAsync(lc_all.data(), S.d_lvlc, sizeof(void *) * lc_all.size(), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipMemcpyAsync(qs_all.data(), S.d_qs, 8 * qs_all.size(), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) { set_error(hipGetErrorString(e)); fail_all(S, GS_EDEVICE); continue; }
    }

    // the iteration's region of the ring
    const uint64_t rid = S.next_region++;
    const uint64_t used_end = std::min<uint64_t>(ar[0].top, whi);
    int refs = 0;
    std::vector<Active *> still;
    for (Active *a : S.active) {
      const int64_t n = lvl_n[(size_t)a->slot * kMaxLevels + a->level];
      if (n < 0 || ar[1].overflow) {   // level did not fit: restart this query later
        const bool alone = S.active.size() == 1 && wlo == 0 && whi == E.tree_cap;
        Request rq = std::move(a->req);
        release(S, a);
        delete a;
        if (alone || rq.attempts >= 8) {
          set_error("binding tree exceeds the tree arena");
          finish(S, rq.ticket, GS_ENOMEM, nullptr);
        } else {
          rq.attempts++;
          std::lock_guard<std::mutex> lk(S.mu);
          S.stats.requeued++;
          S.pending.push_back(std::move(rq));
        }
        continue;
      }
      a->level++;
      if (a->level == a->qi.nlev) {   // rows leave the ring now: the new level needs no reference
        const int rc = retire(S, a, lp_all.data(), lc_all.data(), qs_all.data(), lvl_n.data(), s);
        if (rc != GS_OK) finish(S, a->req.ticket, rc, nullptr);
        release(S, a);
        delete a;
        continue;
      }
      if (n > 0) { a->regions.push_back(rid); ++refs; }
      still.push_back(a);
    }
    S.active.swap(still);
    if (refs > 0 && used_end > wlo) {
      S.regions.push_back({rid, Region{wlo, used_end, refs}});
      S.head = used_end;
    }
    while (!S.regions.empty() && S.regions.front().second.refs <= 0) S.regions.pop_front();
    if (S.regions.empty()) S.head = 0;
  }
}

}  // namespace

int server_start(Engine *E, const gs_server_options *o, gs_server **out) {
  *out = nullptr;
  if (!E->loaded) { set_error("no dataset loaded"); return GS_ESTATE; }
  {   // the server uses the whole tree arena as its ring: no direct result may live in it
    std::lock_guard<std::mutex> lk(E->mu);
    if (E->serving) { set_error("a server is already running on this engine"); return GS_ESTATE; }
    if (E->live_results > 0) { set_error("results of direct evaluation are still live; free them first"); return GS_ESTATE; }
    E->serving = true;
  }
  gs_server *srv = new gs_server();
  ServerImpl &S = srv->s;
  S.E = E;
  if (o) S.opt = *o;
  S.cap = S.opt.max_active > 0 ? S.opt.max_active : 1024;
  const int cap = S.cap;
  (void)hipSetDevice(E->device);
  std::vector<void **> allocs;
  auto take = [&](void **p, size_t bytes) { *p = E->dmalloc(bytes); allocs.push_back(p); };
  take((void **)&S.d_steps, sizeof(DStep) * cap * kSlotSteps);
  take((void **)&S.d_filt, sizeof(void *) * cap * kSlotFilt);
  take((void **)&S.d_checks, sizeof(DCheck) * cap * kSlotChk);
  take((void **)&S.d_ints, sizeof(int32_t) * cap * kSlotInts);
  take((void **)&S.d_cc, sizeof(DConst) * cap * kSlotCc);
  take((void **)&S.d_vr, sizeof(int32_t) * cap * kMaxLevels);
  take((void **)&S.d_lvlp, sizeof(void *) * cap * kMaxLevels);
  take((void **)&S.d_lvlc, sizeof(void *) * cap * kMaxLevels);
  take((void **)&S.d_lvln, sizeof(int64_t) * cap * kMaxLevels);
  take((void **)&S.d_qs, sizeof(int64_t) * cap * QS_N);
  take((void **)&S.d_ents, sizeof(DEntry) * cap);
  take((void **)&S.d_doms, sizeof(DDomain) * cap * kIterDomPerQuery);
  take((void **)&S.d_clear, sizeof(void *) * cap * (kSlotSeed + 2 * kIterDomPerQuery));
  take((void **)&S.d_seeds, sizeof(DSeed) * cap * kSlotSeed);
  take((void **)&S.d_fc, sizeof(int64_t) * cap * kIterDomPerQuery);
  take((void **)&S.d_es, sizeof(EState) * cap);
  take((void **)&S.d_it, sizeof(IterScalars));
  take((void **)&S.d_blk, sizeof(int64_t) * 4 * E->grid);
  take((void **)&S.d_zero, 256);
  take((void **)&S.d_flags, 256);
  S.rows_cap = 64ull << 20;
  take((void **)&S.d_rows, S.rows_cap);
  // bitmap pool: up to 8 bitmaps per slot, bounded by a sixteenth of the tree arena
  const uint64_t bm_bytes = (uint64_t)E->g.words * 8;
  uint64_t nbm = std::min<uint64_t>((uint64_t)cap * 8, std::max<uint64_t>(64, (E->tree_cap / 16) / bm_bytes));
  take((void **)&S.pool, bm_bytes * nbm);
  for (void **p : allocs)
    if (!*p) {
      for (void **q : allocs) E->dfree(*q);
      delete srv;
      { std::lock_guard<std::mutex> lk(E->mu); E->serving = false; }
      set_error("out of device memory for the server tables");
      return GS_ENOMEM;
    }
  for (int i = (int)nbm - 1; i >= 0; --i) S.free_bm.push_back(i);
  for (int i = cap - 1; i >= 0; --i) S.free_slots.push_back(i);
  S.th = std::thread([&S] { loop(S); });
  *out = srv;
  return GS_OK;
}

int server_submit(gs_server *srv, const gs_query *q, uint32_t flags, uint64_t *ticket) {
  ServerImpl &S = srv->s;
  Request r;
  r.n_qv = q->n_qv;
  if (q->n_qv < 0 || q->n_edges < 0 || (q->n_edges > 0 && !q->edges)) { set_error("malformed query"); return GS_EINVAL; }
  if (q->qv_const) r.qv_const.assign(q->qv_const, q->qv_const + q->n_qv);
  else r.qv_const.assign(q->n_qv, -1);
  r.edges.assign(q->edges, q->edges + q->n_edges);
  r.flags = flags;
  r.t_arrive = now_ms();
  {
    std::lock_guard<std::mutex> lk(S.mu);
    if (S.stopping) { set_error("server stopped"); return GS_ESTATE; }
    r.ticket = S.next_ticket++;
    *ticket = r.ticket;
    S.stats.submitted++;
    S.pending.push_back(std::move(r));
  }
  S.cv.notify_one();
  return GS_OK;
}

int server_poll(gs_server *srv, uint64_t ticket, gs_result **out) {
  ServerImpl &S = srv->s;
  *out = nullptr;
  std::lock_guard<std::mutex> lk(S.mu);
  auto it = S.done.find(ticket);
  if (it == S.done.end()) {
    if (ticket == 0 || ticket >= S.next_ticket) { set_error("unknown ticket"); return GS_EINVAL; }
    return GS_EAGAIN;
  }
  const int st = it->second.first;
  *out = reinterpret_cast<gs_result *>(it->second.second);
  S.done.erase(it);
  return st;
}

int server_poll_ready(gs_server *srv, uint64_t *tickets, int32_t *statuses, gs_result **results, int32_t cap,
                      int32_t *n) {
  ServerImpl &S = srv->s;
  *n = 0;
  std::lock_guard<std::mutex> lk(S.mu);
  auto it = S.done.begin();
  while (it != S.done.end() && *n < cap) {
    tickets[*n] = it->first;
    statuses[*n] = it->second.first;
    results[*n] = reinterpret_cast<gs_result *>(it->second.second);
    ++*n;
    it = S.done.erase(it);
  }
  return GS_OK;
}

int server_stop(gs_server *srv, gs_server_stats *st) {
  ServerImpl &S = srv->s;
  {
    std::lock_guard<std::mutex> lk(S.mu);
    S.stopping = true;
  }
  S.cv.notify_all();
  if (S.th.joinable()) S.th.join();
  if (st) *st = S.stats;
  for (auto &d : S.done) if (d.second.second) result_free(d.second.second);
  Engine *E = S.E;
  void *ps[] = {S.d_steps, S.d_filt, S.d_checks, S.d_ints, S.d_cc, S.d_vr, S.d_lvlp, S.d_lvlc, S.d_lvln, S.d_qs, S.d_ents,
                S.d_doms, S.d_clear, S.d_seeds, S.d_fc, S.d_es, S.d_it, S.d_blk, S.d_zero, S.d_flags, S.d_rows, S.pool};
  for (void *p : ps) E->dfree(p);
  delete srv;
  { std::lock_guard<std::mutex> lk(E->mu); E->serving = false; }
  return GS_OK;
}

}  // namespace gs
