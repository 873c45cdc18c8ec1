// Query-evaluation kernels. One launch sequence advances every active query
// of an iteration by one tree level (one query vertex, Section 7.1):
//
//   setup      per-entry previous level, node tiles, scratch reset
//   clear      zero the seed / frontier / domain bitmaps used this iteration
//   seed       constant edges: segment of the constant -> bitmap (light queries)
//   list_*     root or new-component candidates: AND of bitmaps + compaction
//              (Eq. 17 / 21: v_x = AND of the label-existence vectors)
//   dom_*      cycle-closing edges: frontier F of distinct bindings of the bound
//              end, then D = vertices reachable from F (Eq. 14-16 / 22), by push
//              over F or by a masked pull over the candidates
//   lookup     per tree node: the label-p segment of its parent binding
//              (the row or column selection of Eq. 18 / 22)
//   nz_write   compact the nodes with a non-empty segment
//   expand_*   per candidate: bitmap filters, exact checks against bound
//              vertices, self loops; count, scan, write (parent, vertex,
//              carried bindings) in node order (Eq. 19 / 23)
//
// Every kernel runs on a fixed grid and reads its sizes from device memory,
// so an iteration needs no host round trip. Index spaces are cut into tiles
// that never straddle two queries; block g of G takes a contiguous share of
// the tiles, so results come out in a fixed order.
#include "kernels_common.hpp"
#include "planner.hpp"
#include "query.hpp"

namespace gs {

__device__ __forceinline__ void *arena_alloc(DArena *a, char *base, uint64_t bytes) {
  const uint64_t sz = (bytes + 255ull) & ~255ull;
  if (sz == 0) return base;
  const uint64_t at = atomicAdd((unsigned long long *)&a->top, (unsigned long long)sz);
  if (at + sz > a->cap) { atomicOr(&a->overflow, 1); return nullptr; }
  return base + at;
}

// Several arrays from one arena bump (one atomic instead of one per array).
template <int K>
__device__ __forceinline__ void arena_alloc_many(DArena *a, char *base, const uint64_t (&bytes)[K], void *(&out)[K]) {
  uint64_t tot = 0, off[K];
  for (int k = 0; k < K; ++k) { off[k] = tot; tot += (bytes[k] + 255ull) & ~255ull; }
  uint64_t at = 0;
  if (tot) {
    at = atomicAdd((unsigned long long *)&a->top, (unsigned long long)tot);
    if (at + tot > a->cap) {
      atomicOr(&a->overflow, 1);
      for (int k = 0; k < K; ++k) out[k] = nullptr;
      return;
    }
  }
  for (int k = 0; k < K; ++k) out[k] = base + at + off[k];
}

// last entry e with key(e) <= t (key non-decreasing)
template <class Key>
__device__ __forceinline__ int last_le(int E, int64_t t, Key key) {
  int lo = 0, hi = E;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (key(mid) <= t) lo = mid + 1; else hi = mid;
  }
  return lo - 1;
}

__device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// An index read from LDS is the same in every lane; saying so lets the compiler
// load the structs it selects through the scalar unit.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Per-workgroup accumulation of per-entry counters: a workgroup walks a
// contiguous range of tiles, so it meets few entries; adding to the entry's
// counter only when the entry changes keeps global atomics off the per-tile
// path (one counter address would otherwise serialise every tile of a level).
struct EntryAcc {
  int e = -1;
  int64_t v0 = 0, v1 = 0;
  __device__ void add(int en, int64_t a, int64_t b, int64_t *p0, int64_t *p1, int64_t stride) {
    if (en != e) { flush(p0, p1, stride); e = en; }
    v0 += a; v1 += b;
  }
  __device__ void flush(int64_t *p0, int64_t *p1, int64_t stride) {
    if (e >= 0) {
      if (v0 && p0) atomicAdd((unsigned long long *)(p0 + (int64_t)e * stride), (unsigned long long)v0);
      if (v1 && p1) atomicAdd((unsigned long long *)(p1 + (int64_t)e * stride), (unsigned long long)v1);
    }
    v0 = v1 = 0;
  }
};

// A step whose candidates face no test: every candidate entry becomes a child.
__device__ __forceinline__ bool test_free(const DStep &S) { return step_test_free(S); }

// The count-only last level of a query whose candidates face no test: its
// count is the sum of its nodes' segment lengths, known after the node scan;
// it has no tiles, no compacted nodes, no count or write pass, and its entries
// are not read (nor counted as traversed).
__device__ __forceinline__ bool counted_only(const DStep &S) { return test_free(S) && S.ncols_out == 0; }

// Per-node segment reference: the start of the segment the node's candidates
// are read from, the orientation of that segment, and which of the step's
// bound segments it is (0: the parent edge's, k: exact check k - 1). A level
// whose new variable is bound by several edges reads its candidates from the
// shortest of their segments and tests the others; all of them are sorted by
// id, so the children and their order are the same whichever is read.
// A factor level's per-node product of segment lengths is capped here (a tile of 1024
// such products stays far below 2^63); a capped product fails the query with GS_ERANGE.
constexpr int64_t kFactorCap = 1ll << 50;

constexpr int kLoBits = 40;
constexpr int kMaxGen = 63;
__device__ __forceinline__ int64_t seg_ref(int64_t lo, int dir, int gen) {
  return lo | ((int64_t)dir << kLoBits) | ((int64_t)gen << (kLoBits + 1));
}
__device__ __forceinline__ int64_t ref_lo(int64_t r) { return r & ((1ll << kLoBits) - 1); }
__device__ __forceinline__ int ref_dir(int64_t r) { return (int)((r >> kLoBits) & 1); }
__device__ __forceinline__ int ref_gen(int64_t r) { return (int)((r >> (kLoBits + 1)) & kMaxGen); }

static_assert(sizeof(EState) % sizeof(int64_t) == 0, "EState must be a whole number of int64");
constexpr int64_t kEsStride = sizeof(EState) / sizeof(int64_t);

// ------------------------------------------------------------------ setup
// A scratch overflow in any iteration of a run stops the run: the aborted
// level is never published, so no later iteration may read it.
__device__ __forceinline__ void run_abort(const IterArgs &A) {
  A.it->abort = 1;
  if (A.flags) atomicOr(&A.flags[RF_SCRATCH], 1);
}

__global__ __launch_bounds__(1024) void k_it_setup(const IterArgs A) {
  __shared__ int64_t lds[1024];
  IterScalars *it = A.it;
  EState *es = A.es;
  const bool dead = A.flags && gld(&A.flags[RF_SCRATCH]) != 0;   // set by an earlier iteration's kernels only
  if (threadIdx.x == 0) {
    A.scratch->top = 0;
    A.scratch->overflow = 0;
    it->n_entries = A.E;
    it->abort = dead ? 1 : 0;
    it->ftests = 0;
    it->ctests = 0;
    it->probes = 0;
    it->lk_labels = 0;
    it->lk_lookups = 0;
  }
  if (dead) return;
  for (int e = threadIdx.x; e < A.E; e += blockDim.x) {
    const DEntry d = A.ent[e];
    const DStep S = A.steps[d.step];
    EState z{};
    if (d.level == 0) {
      z.prev = nullptr;
      z.prev_n = 1;
    } else {
      const int64_t n = A.lvl_n[(int64_t)d.q * kMaxLevels + d.level - 1];
      z.prev = A.lvl_ptr[(int64_t)d.q * kMaxLevels + d.level - 1];
      z.prev_n = n < 0 ? 0 : n;
    }
    z.list_words = (S.kind == STEP_LIST && z.prev_n > 0) ? A.g.words : 0;
    es[e] = z;
  }
  for (int d = threadIdx.x; d < A.D; d += blockDim.x) A.fcount[d] = 0;
  __syncthreads();
  int64_t tot3[3];   // nodes, node tiles, list tiles
  wg_scan_k<3>(
      A.E,
      [&](int64_t i, int64_t *v) {
        const int64_t pn = es[i].prev_n;
        v[0] = pn;
        v[1] = ceil_div(pn, kTileNodes);
        v[2] = ceil_div(es[i].list_words, kTileWords);
      },
      [&](int64_t i, const int64_t *o) { es[i].node0 = o[0]; es[i].node_tile0 = o[1]; es[i].list_tile0 = o[2]; },
      lds, tot3);
  const int64_t nodes = tot3[0], ntiles = tot3[1], ltiles = tot3[2];
  if (threadIdx.x == 0) {
    it->nodes_total = nodes;
    it->node_tiles = ntiles;
    it->list_tiles = ltiles;
    const uint64_t b8 = sizeof(int64_t) * (uint64_t)nodes;
    const uint64_t sz[4] = {b8, b8, A.has_checks ? b8 : 0, A.has_checks ? b8 : 0};
    void *p[4];
    arena_alloc_many(A.scratch, A.scratch_base, sz, p);
    it->lo = (int64_t *)p[0];
    it->len = (int64_t *)p[1];
    it->chk_lo = (int64_t *)p[2];
    it->chk_hi = (int64_t *)p[3];
    if (A.scratch->overflow) run_abort(A);
  }
}

// Zero every bitmap on the iteration's clear list.
__global__ __launch_bounds__(kBlock) void k_clear(const IterArgs A) {
  const int64_t W = A.g.words, stride = (int64_t)gridDim.x * blockDim.x;
  for (int32_t b = 0; b < A.nclear; ++b) {
    uint64_t *bm = A.clear[b];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < W; i += stride) bm[i] = 0ull;
  }
}

// Constant edges (c, p, x) / (x, p, c): the segment of c -> bitmap of x's candidates.
// Each segment is cut into as many contiguous parts as the grid has workgroups per
// constant edge (a hub constant's segment holds millions of entries). The ids of a
// segment ascend, so lanes whose ids fall in one bitmap word are neighbours: the
// wave ORs their bits together and the first of them sets the word, one atomic per
// word instead of one per entry.
__global__ __launch_bounds__(kBlock) void k_seed(const IterArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t parts = max((int64_t)1, (int64_t)gridDim.x / A.S);
  for (int64_t b = blockIdx.x; b < (int64_t)A.S * parts; b += gridDim.x) {
    const int s = (int)(b / parts);
    const int64_t part = b % parts;
    const DSeed sd = A.seeds[s];
    int64_t lo, hi;
    int probes = 0;
    seg_find(A.g, sd.dir, sd.c, sd.label, lo, hi, probes);
    int64_t words_set = 0;
    const int32_t *idx = sd.dir ? A.g.idx[1] : A.g.idx[0];
    const int64_t per = ceil_div(hi - lo, parts);
    const int64_t a = lo + part * per, e = min(hi, a + per);
    for (int64_t k0 = a + (threadIdx.x & ~63); k0 < e; k0 += blockDim.x) {   // whole waves
      const int64_t k = k0 + lane;
      const bool ok = k < e;
      const int32_t c = ok ? gld(idx + k) : 0;
      const int64_t w = ok ? (int64_t)(c >> 6) : -1;
      uint64_t bits = ok ? (1ull << (c & 63)) : 0ull;
      for (int off = 1; off < 64; off <<= 1) {   // OR over the following lanes of the same word
        const uint64_t ob = __shfl_down(bits, off, 64);
        const int64_t ow = __shfl_down(w, off, 64);
        if (lane + off < 64 && ow == w) bits |= ob;
      }
      const int64_t pw = __shfl_up(w, 1, 64);
      const bool first = ok && (lane == 0 || pw != w);
      if (first) atomicOr((unsigned long long *)&sd.bm[w], (unsigned long long)bits);
      words_set += __popcll(__ballot(first));
    }
    int64_t *qs = A.qstats + (int64_t)sd.q * QS_N;
    if ((threadIdx.x & 63) == 0 && words_set) atomicAdd((unsigned long long *)&qs[QS_BMWORDS], (unsigned long long)words_set);
    if (part == 0 && threadIdx.x == 0) {
      atomicAdd((unsigned long long *)&qs[QS_SEED], (unsigned long long)(hi - lo));
      atomicAdd((unsigned long long *)&qs[QS_LABEL], (unsigned long long)probes);
      atomicAdd((unsigned long long *)&qs[QS_LOOKUP], 1ull);
    }
  }
}

// ------------------------------------------------------------------ lists
__device__ __forceinline__ uint64_t list_word(const IterArgs &A, const DStep &S, int64_t w) {
  uint64_t x = ~0ull;
  for (int f = 0; f < S.list_nfilt; ++f) x &= A.filt[S.filt0 + f][w];
  if (w == A.g.words - 1 && (A.g.n & 63)) x &= (1ull << (A.g.n & 63)) - 1ull;
  return x;
}

__global__ __launch_bounds__(kBlock) void k_list_count(const IterArgs A) {
  __shared__ int64_t lds[kWaves];
  __shared__ int sh_e;
  IterScalars *it = A.it;
  if (it->abort) return;
  EState *es = A.es;
  const int64_t G = active_groups(it->list_tiles, gridDim.x);
  if (blockIdx.x >= G) return;
  int64_t tb, te;
  block_share_g(it->list_tiles, G, tb, te);
  int64_t bsum = 0;
  EntryAcc acc;
  int64_t *p_list_n = &es[0].list_n;
  for (int64_t t = tb; t < te; ++t) {
    if (threadIdx.x == 0) sh_e = last_le(A.E, t, [&](int i) { return es[i].list_tile0; });
    __syncthreads();
    const int e = uniform(sh_e);
    const DStep S = A.steps[A.ent[e].step];
    const int64_t w = (t - es[e].list_tile0) * kTileWords + threadIdx.x;
    int64_t c = 0;
    if (w < es[e].list_words) c = __popcll(list_word(A, S, w));
    c = block_sum_i64(c, lds);
    if (threadIdx.x == 0) acc.add(e, c, 0, p_list_n, nullptr, kEsStride);
    bsum += c;
  }
  if (threadIdx.x == 0) { acc.flush(p_list_n, nullptr, kEsStride); A.blk_a[blockIdx.x] = bsum; }
}

__global__ __launch_bounds__(1024) void k_list_scan(const IterArgs A) {
  __shared__ int64_t lds[1024];
  IterScalars *it = A.it;
  if (it->abort) return;
  EState *es = A.es;
  wg_scan(active_groups(it->list_tiles, A.grid), [&](int64_t i) { return A.blk_a[i]; },
          [&](int64_t i, int64_t v) { A.blk_off_a[i] = v; }, lds);
  const int64_t total = wg_scan(A.E, [&](int64_t i) { return es[i].list_n; },
                                [&](int64_t i, int64_t v) { es[i].list_base = v; }, lds);
  __shared__ int32_t *buf;
  if (threadIdx.x == 0) {
    it->list_total = total;
    buf = A.list_out ? A.list_out : (int32_t *)arena_alloc(A.scratch, A.scratch_base, sizeof(int32_t) * total);
    it->list_buf = buf;
    if (A.scratch->overflow) run_abort(A);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < A.E; e += blockDim.x) es[e].list = buf ? buf + es[e].list_base : nullptr;
}

__global__ __launch_bounds__(kBlock) void k_list_write(const IterArgs A) {
  __shared__ int64_t lds[kWaves];
  __shared__ int sh_e;
  IterScalars *it = A.it;
  if (it->abort) return;
  EState *es = A.es;
  const int64_t G = active_groups(it->list_tiles, gridDim.x);
  if (blockIdx.x >= G) return;
  int64_t tb, te;
  block_share_g(it->list_tiles, G, tb, te);
  int64_t run = A.blk_off_a[blockIdx.x];
  for (int64_t t = tb; t < te; ++t) {
    if (threadIdx.x == 0) sh_e = last_le(A.E, t, [&](int i) { return es[i].list_tile0; });
    __syncthreads();
    const int e = uniform(sh_e);
    const DStep S = A.steps[A.ent[e].step];
    const int64_t w = (t - es[e].list_tile0) * kTileWords + threadIdx.x;
    uint64_t x = 0;
    if (w < es[e].list_words) x = list_word(A, S, w);
    int64_t tot;
    int64_t pos = block_excl_scan_i64(__popcll(x), tot, lds);
    int32_t *out = it->list_buf + (run + pos);
    while (x) {
      const int b = __ffsll((unsigned long long)x) - 1;
      *out++ = (int32_t)(w * 64 + b);
      x &= x - 1;
    }
    run += tot;
  }
}

// ------------------------------------------------------------------ domains
__device__ __forceinline__ int node_entry(const IterArgs &A, int64_t t) {
  return last_le(A.E, t, [&](int i) { return A.es[i].node_tile0; });
}

// Entry of node tile t for a workgroup walking its tiles in increasing order.
struct NodeCursor {
  int e = -1;
  int64_t end = 0;
  __device__ int at(const IterArgs &A, int64_t t) {
    if (e < 0 || t >= end) {
      e = node_entry(A, t);
      end = A.es[e].node_tile0 + ceil_div(A.es[e].prev_n, kTileNodes);
    }
    return e;
  }
};

// F = distinct bindings of the bound end of each cycle-closing edge.
__global__ __launch_bounds__(kBlock) void k_dom_frontier(const IterArgs A) {
  __shared__ int64_t lds[kWaves];
  __shared__ int sh_e;
  IterScalars *it = A.it;
  if (it->abort || A.D == 0) return;
  EState *es = A.es;
  const int64_t G = active_groups(it->node_tiles, gridDim.x);
  if (blockIdx.x >= G) return;
  int64_t tb, te;
  block_share_g(it->node_tiles, G, tb, te);
  NodeCursor ncur;
  for (int64_t t = tb; t < te; ++t) {
    if (threadIdx.x == 0) sh_e = ncur.at(A, t);
    __syncthreads();
    const int e = uniform(sh_e);
    __syncthreads();
    const DEntry d = A.ent[e];
    if (d.ndom == 0) continue;   // uniform across the block
    const int64_t i0 = (t - es[e].node_tile0) * kTileNodes, pn = es[e].prev_n;
    for (int k = 0; k < d.ndom; ++k) {
      const DDomain dm = A.doms[d.dom0 + k];
      int64_t fresh = 0;
      for (int r = 0; r < kTileNodes / kBlock; ++r) {
        const int64_t i = i0 + r * kBlock + threadIdx.x;
        if (i < pn) {
          const int32_t b = es[e].prev[(int64_t)dm.col * pn + i];
          const uint64_t bit = 1ull << (b & 63);
          // bindings repeat (hubs): test before the atomic, which then runs once per distinct word bit
          if (!(gld(dm.F + (b >> 6)) & bit)) {
            const uint64_t old = atomicOr((unsigned long long *)&dm.F[b >> 6], bit);
            fresh += (old & bit) ? 0 : 1;
          }
        }
      }
      fresh = block_sum_i64(fresh, lds);
      if (threadIdx.x == 0 && fresh) atomicAdd((unsigned long long *)&A.fcount[d.dom0 + k], (unsigned long long)fresh);
    }
  }
}

__device__ __forceinline__ int dom_mode(const IterArgs &A, int d) {
  const DDomain &dm = A.doms[d];
  if (dm.mode == 1 || dm.mode == 2) return dm.mode;
  const double push = (double)A.fcount[d] * dm.deg_push;
  const double pull = (double)dm.mask_est * dm.deg_pull;
  return push <= (double)dm.theta * pull ? 1 : 2;
}

constexpr int64_t kCoopSeg = 32;   // push: segments longer than this are walked by a whole wave

// Set bit c of a bitmap that other waves set concurrently; the atomic is
// skipped when the bit is already visible (many segments share targets).
__device__ __forceinline__ void set_bit_once(uint64_t *bm, int32_t c) {
  const uint64_t bit = 1ull << (c & 63);
  if (!(gld(bm + (c >> 6)) & bit)) atomicOr((unsigned long long *)&bm[c >> 6], bit);
}

// Push: for every b in F, OR the label-p segment of b into D (sparse-frontier product).
__global__ __launch_bounds__(kBlock) void k_dom_push(const IterArgs A) {
  __shared__ int64_t lds[2 * kWaves];
  if (A.it->abort || A.D == 0) return;
  const int64_t W = A.g.words, tpd = ceil_div(W, kTileWords);
  const int64_t NT = (int64_t)A.D * tpd;
  for (int64_t t = blockIdx.x; t < NT; t += gridDim.x) {
    const int d = (int)(t / tpd);
    if (dom_mode(A, d) != 1) continue;
    const DDomain dm = A.doms[d];
    const int64_t w = (t % tpd) * kTileWords + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int64_t work = 0, lk = 0, lp = 0, bw = w < W ? 1 : 0;   // bw: frontier words read
    uint64_t x = w < W ? dm.F[w] : 0;
    if (w == W - 1 && (A.g.n & 63)) x &= (1ull << (A.g.n & 63)) - 1ull;   // no vertex ids >= n
    const int32_t *idx = A.g.idx[dm.dir];
    // one set bit per lane per round; short segments are walked by their lane,
    // long ones (hubs) by the whole wave, one after the other
    while (__ballot(x != 0)) {
      int64_t lo = 0, hi = 0;
      bool coop = false;
      if (x) {
        const int b = __ffsll((unsigned long long)x) - 1;
        x &= x - 1;
        int probes = 0;
        seg_find(A.g, dm.dir, (int32_t)(w * 64 + b), dm.label, lo, hi, probes);
        work += hi - lo;
        ++lk;
        lp += probes;
        coop = hi - lo > kCoopSeg;
        if (!coop)
          for (int64_t k = lo; k < hi; ++k) set_bit_once(dm.D, idx[k]);
      }
      for (uint64_t m = __ballot(coop); m; m &= m - 1) {
        const int l = __ffsll((unsigned long long)m) - 1;
        const int64_t L = __shfl(lo, l, 64), H = __shfl(hi, l, 64);
        for (int64_t k = L + lane; k < H; k += 64) set_bit_once(dm.D, idx[k]);
      }
    }
    bw += work;   // one result-bitmap word read per entry
    block_sum2_i64(work, bw, lds);
    block_sum2_i64(lk, lp, lds);
    if (threadIdx.x == 0) {
      int64_t *qs = A.qstats + (int64_t)dm.q * QS_N;
      if (work) atomicAdd((unsigned long long *)&qs[QS_PUSH], (unsigned long long)work);
      if (lk) atomicAdd((unsigned long long *)&qs[QS_LOOKUP], (unsigned long long)lk);
      if (lp) atomicAdd((unsigned long long *)&qs[QS_LABEL], (unsigned long long)lp);
      if (bw) atomicAdd((unsigned long long *)&qs[QS_BMWORDS], (unsigned long long)bw);
      if (t % tpd == 0) atomicAdd((unsigned long long *)&qs[QS_DOMPUSH], 1ull);
    }
  }
}

// Pull: for every candidate c of the mask, D(c) = OR over b in seg(c, p, opposite) of F(b).
__global__ __launch_bounds__(kBlock) void k_dom_pull(const IterArgs A) {
  __shared__ int64_t lds[2 * kWaves];
  if (A.it->abort || A.D == 0) return;
  const int64_t W = A.g.words, tpd = ceil_div(W, kTileWords);
  const int64_t NT = (int64_t)A.D * tpd;
  for (int64_t t = blockIdx.x; t < NT; t += gridDim.x) {
    const int d = (int)(t / tpd);
    if (dom_mode(A, d) != 2) continue;
    const DDomain dm = A.doms[d];
    const int64_t w = (t % tpd) * kTileWords + threadIdx.x;
    int64_t work = 0, lk = 0, lp = 0, bw = 0;
    if (w < W) {
      bw = dm.nfilt + 1;   // mask words read, result word written
      uint64_t x = ~0ull;
      for (int f = 0; f < dm.nfilt; ++f) x &= A.filt[dm.filt0 + f][w];
      if (w == W - 1 && (A.g.n & 63)) x &= (1ull << (A.g.n & 63)) - 1ull;
      const int od = 1 - dm.dir;
      const int32_t *idx = A.g.idx[od];
      uint64_t out = 0;
      while (x) {
        const int b = __ffsll((unsigned long long)x) - 1;
        x &= x - 1;
        int64_t lo, hi;
        int probes = 0;
        seg_find(A.g, od, (int32_t)(w * 64 + b), dm.label, lo, hi, probes);
        ++lk;
        lp += probes;
        int64_t k = lo;
        for (; k < hi; ++k)
          if (bit_test(dm.F, idx[k])) { out |= 1ull << b; ++k; break; }
        work += k - lo;
      }
      dm.D[w] = out;
    }
    bw += work;   // one frontier word read per entry tested
    block_sum2_i64(work, bw, lds);
    block_sum2_i64(lk, lp, lds);
    if (threadIdx.x == 0) {
      int64_t *qs = A.qstats + (int64_t)dm.q * QS_N;
      if (work) atomicAdd((unsigned long long *)&qs[QS_PULL], (unsigned long long)work);
      if (lk) atomicAdd((unsigned long long *)&qs[QS_LOOKUP], (unsigned long long)lk);
      if (lp) atomicAdd((unsigned long long *)&qs[QS_LABEL], (unsigned long long)lp);
      if (bw) atomicAdd((unsigned long long *)&qs[QS_BMWORDS], (unsigned long long)bw);
      if (t % tpd == 0) atomicAdd((unsigned long long *)&qs[QS_DOMPULL], 1ull);
    }
  }
}

// ------------------------------------------------------------------ lookup
__device__ __forceinline__ bool const_checks_hold(const IterArgs &A, const DStep &S) {
  for (int k = 0; k < S.ncc; ++k) {
    const DConst c = A.cconst[S.cc0 + k];
    int probes = 0;
    if (!seg_has(A.g, 0, c.a, c.label, c.b, probes)) return false;
  }
  return true;
}

template <int LB, int OB, bool FACTOR>
__device__ __forceinline__ void lookup_body(const IterArgs &A, int64_t *lds, int &sh_e, int &sh_ok,
                                            unsigned long long *s_cnt) {
  IterScalars *it = A.it;
  if (it->abort) return;
  EState *es = A.es;
  const int64_t G = active_groups(it->node_tiles, gridDim.x);
  if (blockIdx.x >= G) return;
  int64_t tb, te;
  block_share_g(it->node_tiles, G, tb, te);
  NodeCursor ncur;
  int64_t bnz = 0, bw = 0;
  EntryAcc acc;
  // label entries read and segment lookups: per thread over a tile, then in LDS while the
  // entry stays the same, then to the entry's query
  int cur = -1;
  int64_t *p_nz = &es[0].nz, *p_w = &es[0].w;
  for (int64_t t = tb; t < te; ++t) {
    if (threadIdx.x == 0) sh_e = ncur.at(A, t);
    __syncthreads();
    const int e = uniform(sh_e);
    const DEntry d = sld(A.ent + e);
    const DStep S = sld(A.steps + d.step);
    if (threadIdx.x == 0) sh_ok = (d.level == 0 && S.ncc > 0) ? const_checks_hold(A, S) : 1;
    __syncthreads();
    const int64_t i0 = (t - sld(&es[e].node_tile0)) * kTileNodes, pn = sld(&es[e].prev_n);
    const int32_t *const eprev = sld(&es[e].prev);
    const int64_t enode0 = sld(&es[e].node0);
    int64_t cnz = 0, cw = 0;
    uint32_t cnt = 0;   // this thread's label entries read (bits 0-21) and lookups (22-31) in the tile
    bool factor_over = false;
    if (threadIdx.x == 0 && e != cur) {   // the previous entry's counters go to its query
      if (cur >= 0 && (s_cnt[0] | s_cnt[1])) {
        int64_t *qs = A.qstats + (int64_t)A.ent[cur].q * QS_N;
        atomicAdd((unsigned long long *)&qs[QS_LABEL], s_cnt[0]);
        atomicAdd((unsigned long long *)&qs[QS_LOOKUP], s_cnt[1]);
        s_cnt[2] += s_cnt[0];
        s_cnt[3] += s_cnt[1];
      }
      s_cnt[0] = s_cnt[1] = 0;
    }
    cur = e;
    const bool counted = counted_only(S);
    constexpr int RN = kTileNodes / kBlock;
    // the parent bindings, then their rows, of all of the thread's nodes first (independent loads)
    const int32_t *src = eprev + (int64_t)S.src * pn;
    const void *ptr = S.dir ? A.g.ptr[1] : A.g.ptr[0];
    using I = OffT<OB>;   // entry positions at the offsets' width
    I ra[RN];             // row starts, and row lengths (a row holds fewer than 2^31 entries)
    int32_t rn[RN];
    for (int r = 0; r < RN; ++r) {
      const int64_t i = i0 + r * kBlock + threadIdx.x;
      ra[r] = 0;
      rn[r] = 0;
      if (i < pn && S.kind != STEP_LIST) {
        const int32_t b = S.kind == STEP_SEG ? gld(src + i) : S.src;
        ra[r] = off_w<OB>(ptr, b);
        rn[r] = (int32_t)(off_w<OB>(ptr, (int64_t)b + 1) - ra[r]);
      }
    }
    for (int r = 0; r < RN; ++r) {
      const int64_t i = i0 + r * kBlock + threadIdx.x;
      if (i >= pn) break;
      I lo = 0, hi = 0;
      int probes = 0, lookups = 0;   // label entries read, segment lookups of this node
      int dir = S.dir, gen = 0;
      if (S.kind != STEP_LIST) {
        const I re = ra[r] + rn[r];
        label_range_w<LB>(S.dir ? A.g.lab[1] : A.g.lab[0], ra[r], re, S.label, lo, hi, probes);
        probes = label_reads(ra[r], re, lo, hi);
        const I plo = lo, phi = hi;
        I c0lo = 0, c0hi = 0;
        ++lookups;
        for (int k = 0; k < min(S.nchk, kMaxGen) && hi > lo; ++k) {   // read the shortest bound segment
          const DCheck ck = A.checks[S.chk0 + k];
          I clo, chi;
          ++lookups;
          int unused = 0;
          seg_find_w<LB, OB>(A.g, ck.dir, eprev[(int64_t)ck.col * pn + i], ck.label, clo, chi, unused);
          if (k == 0) { c0lo = clo; c0hi = chi; }
          if (chi - clo < hi - lo) { lo = clo; hi = chi; dir = ck.dir; gen = k + 1; }
        }
        if (S.nchk > 0) {   // the first check the count pass makes: the parent's segment when check 0 generates
          const int64_t gn = enode0 + i;
          it->chk_lo[gn] = gen == 1 ? plo : c0lo;
          it->chk_hi[gn] = gen == 1 ? phi : c0hi;
        }
      } else {
        hi = (I)es[e].list_n;
      }
      if (!sh_ok) hi = lo;
      const int64_t gn = enode0 + i;
      cnz += (hi > lo) && !counted;
      int64_t len = hi - lo;
      if (FACTOR && counted && S.nfactor > 0 && len > 0) {   // a factor level: times the further leaves' segments
        for (int k = 0; k < S.nfactor && len > 0; ++k) {
          const DCheck ck = A.checks[S.chk0 + k];
          I clo, chi;
          ++lookups;
          seg_find_w<LB, OB>(A.g, ck.dir, eprev[(int64_t)ck.col * pn + i], ck.label, clo, chi, probes);
          const int64_t f = (int64_t)chi - clo;
          if (f > 0 && len > kFactorCap / f) { len = kFactorCap; factor_over = true; }
          else len *= f;
        }
      }
      cnt += (uint32_t)probes + ((uint32_t)lookups << 22);
      if (!counted) {   // a counted level's nodes take no part in the passes after the scan
        it->lo[gn] = seg_ref(lo, dir, gen);
        it->len[gn] = hi - lo;
      }
      cw += len;
    }
    {   // one reduction for both: entries above bit 11, non-empty nodes (at most kTileNodes) below;
        // a counted level has no non-empty nodes: its sums go unshifted (a factor level's products)
      const int64_t pk = block_sum_i64(counted ? cw : (cw << 11) | cnz, lds);
      cnz = counted ? 0 : pk & 2047;
      cw = counted ? pk : pk >> 11;
      if (threadIdx.x == 0) acc.add(e, cnz, cw, p_nz, p_w, kEsStride);
    }
    {   // the wave's sums (DPP scan, the total in lane 63), one LDS add each per wave
      const int64_t wsum = wave_incl_scan_i64(((int64_t)(cnt >> 22) << 32) | (cnt & ((1u << 22) - 1)));
      if ((threadIdx.x & 63) == 63 && wsum) {
        atomicAdd(&s_cnt[0], (unsigned long long)(wsum & 0xffffffffll));
        atomicAdd(&s_cnt[1], (unsigned long long)(wsum >> 32));
      }
    }
    if (factor_over) A.qstats[(int64_t)d.q * QS_N + QS_OVERFLOW] = 3;
    bnz += cnz;
    bw += counted ? 0 : cw;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    acc.flush(p_nz, p_w, kEsStride);
    if (cur >= 0 && (s_cnt[0] | s_cnt[1])) {
      int64_t *qs = A.qstats + (int64_t)A.ent[cur].q * QS_N;
      atomicAdd((unsigned long long *)&qs[QS_LABEL], s_cnt[0]);
      atomicAdd((unsigned long long *)&qs[QS_LOOKUP], s_cnt[1]);
    }
    // the launch's totals, for per-kernel byte accounting
    if (s_cnt[0] + s_cnt[2]) atomicAdd((unsigned long long *)&it->lk_labels, s_cnt[0] + s_cnt[2]);
    if (s_cnt[1] + s_cnt[3]) atomicAdd((unsigned long long *)&it->lk_lookups, s_cnt[1] + s_cnt[3]);
    A.blk_a[blockIdx.x] = bnz;
    A.blk_b[blockIdx.x] = bw;
  }
}

// FACTOR: the launch holds a count-only factor level (its own variant: the product loop
// costs registers that every other level would pay for in occupancy)
// One instance per stored width pair (labels LB bytes, offsets OB bytes), chosen on the host:
// each carries only its own width's code, and so only its own register count.
template <int LB, int OB, bool FACTOR>
__global__ __launch_bounds__(kBlock) void k_lookup(const IterArgs A) {
  __shared__ int64_t lds[kWaves];
  __shared__ int sh_e, sh_ok;
  __shared__ unsigned long long s_cnt[4];   // this entry's label reads and lookups, then the earlier entries'
  if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = s_cnt[2] = s_cnt[3] = 0;
  lookup_body<LB, OB, FACTOR>(A, lds, sh_e, sh_ok, s_cnt);
}

// Allocate the tree level of entry e (es[e].cnt children) in the tree arena and
// publish it. Levels without tests are stored with child offsets per parent
// instead of a parent column. On overflow the level is recorded as -1 nodes.
__device__ void alloc_level(const IterArgs &A, int e, const DEntry &d, const DStep &S) {
  EState *es = A.es;
  const int64_t cnt = es[e].cnt, pn = es[e].prev_n;
  const bool csr = test_free(S);
  int32_t *out = nullptr, *cptr = nullptr;
  int64_t n_rec = cnt;
  if (cnt > 2147483647LL && S.ncols_out > 0) {   // child positions and parent indices are int32
    n_rec = -1;
    A.qstats[(int64_t)d.q * QS_N + QS_OVERFLOW] = 2;
  } else if (cnt > 0 && S.ncols_out > 0) {
    const uint64_t cols = (uint64_t)cnt * (S.ncols_out - (csr ? 1 : 0));
    const uint64_t offs = csr ? (uint64_t)(pn + 1) : 0;
    int32_t *blk = (int32_t *)arena_alloc(A.tree, A.tree_base, sizeof(int32_t) * (cols + offs));
    if (!blk) {
      n_rec = -1;
      A.qstats[(int64_t)d.q * QS_N + QS_OVERFLOW] = 1;
    } else if (csr) {
      cptr = blk;
      cptr[pn] = (int32_t)cnt;
      out = blk + (pn + 1) - cnt;   // column c >= 1 at out + c * cnt, inside the block
    } else {
      out = blk;
    }
  }
  es[e].out = out;
  es[e].cptr = cptr;
  A.lvl_ptr[(int64_t)d.q * kMaxLevels + d.level] = out;
  A.lvl_cptr[(int64_t)d.q * kMaxLevels + d.level] = cptr;
  A.lvl_n[(int64_t)d.q * kMaxLevels + d.level] = n_rec;
}

__global__ __launch_bounds__(1024) void k_scan_nodes(const IterArgs A) {
  __shared__ int64_t lds[1024];
  IterScalars *it = A.it;
  if (it->abort) return;
  EState *es = A.es;
  const int64_t G = active_groups(it->node_tiles, A.grid);
  int64_t tot2[2], tot3[3];
  wg_scan_k<2>(
      G, [&](int64_t i, int64_t *v) { v[0] = A.blk_a[i]; v[1] = A.blk_b[i]; },
      [&](int64_t i, const int64_t *o) { A.blk_off_a[i] = o[0]; A.blk_off_b[i] = o[1]; }, lds, tot2);
  // entry offsets and the block offsets above leave out counted levels, as the node lengths do
  wg_scan_k<3>(
      A.E,
      [&](int64_t i, int64_t *v) {
        const bool c = counted_only(A.steps[A.ent[i].step]);
        const int64_t ew = es[i].w;
        v[0] = es[i].nz;
        v[1] = c ? 0 : ew;
        v[2] = c ? 0 : ceil_div(ew, kTileWork);
      },
      [&](int64_t i, const int64_t *o) { es[i].nz_base = o[0]; es[i].w_base = o[1]; es[i].w_tile0 = o[2]; }, lds,
      tot3);
  const int64_t nz = tot3[0], w = tot3[1], wt = tot3[2];
  __shared__ int64_t wtest;
  __shared__ int32_t sh_abort;
  if (threadIdx.x == 0) wtest = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < A.E; e += blockDim.x) {
    if (!test_free(A.steps[A.ent[e].step])) {
      if (es[e].w) atomicAdd((unsigned long long *)&wtest, (unsigned long long)es[e].w);
    } else {
      es[e].cnt = es[e].w;   // no test: every candidate entry becomes a child
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) it->w_tested = wtest;
  if (threadIdx.x == 0) {
    it->nz_total = nz;
    it->w_total = w;
    it->work_tiles = wt;
    const uint64_t b8 = sizeof(int64_t) * (uint64_t)nz;
    const uint64_t sz[7] = {sizeof(int32_t) * (uint64_t)nz, b8, b8, (uint64_t)wt * (kTileWork / 8),
                            sizeof(DTile) * (uint64_t)(wt + 1), A.has_checks ? b8 : 0, A.has_checks ? b8 : 0};
    void *p[7];
    arena_alloc_many(A.scratch, A.scratch_base, sz, p);
    it->nz_node = (int32_t *)p[0];
    it->nz_lo = (int64_t *)p[1];
    it->nz_woff = (int64_t *)p[2];
    it->valid = (uint32_t *)p[3];
    it->tiles = (DTile *)p[4];
    it->nz_chk_lo = (int64_t *)p[5];
    it->nz_chk_hi = (int64_t *)p[6];
    if (A.scratch->overflow) {
      run_abort(A);
    } else {
      DTile z{};
      z.k0 = nz;
      z.e = -1;
      it->tiles[wt] = z;
    }
    sh_abort = it->abort;
  }
  __syncthreads();
  if (sh_abort) return;   // no level of an aborted iteration is published
  for (int e = threadIdx.x; e < A.E; e += blockDim.x) {
    const DEntry d = A.ent[e];
    const DStep S = A.steps[d.step];
    if (S.kind != STEP_LIST && es[e].w && !counted_only(S))
      atomicAdd((unsigned long long *)&A.qstats[(int64_t)d.q * QS_N + QS_EXPAND], (unsigned long long)es[e].w);
    if (test_free(S)) alloc_level(A, e, d, S);   // its size is known now: the node pass writes its offsets
  }
}

__global__ __launch_bounds__(kBlock) void k_nz_write(const IterArgs A) {
  constexpr int NPT = kTileNodes / kBlock;   // consecutive nodes per thread
  __shared__ int64_t lds[kWaves];
  __shared__ int64_t s_woff[kTileNodes];     // entry-local first entry of the tile's non-empty nodes
  __shared__ int sh_e;
  IterScalars *it = A.it;
  if (it->abort) return;
  EState *es = A.es;
  const int64_t G = active_groups(it->node_tiles, gridDim.x);
  if (blockIdx.x >= G) return;
  int64_t tb, te;
  block_share_g(it->node_tiles, G, tb, te);
  NodeCursor ncur;
  int64_t run_nz = A.blk_off_a[blockIdx.x], run_w = A.blk_off_b[blockIdx.x];
  for (int64_t t = tb; t < te; ++t) {
    if (threadIdx.x == 0) sh_e = ncur.at(A, t);
    __syncthreads();
    const int e = uniform(sh_e);
    if (counted_only(A.steps[A.ent[e].step])) {   // no segments recorded, no children, no tiles
      __syncthreads();   // sh_e is rewritten for the next tile
      continue;
    }
    const int64_t i0 = (t - es[e].node_tile0) * kTileNodes + (int64_t)NPT * threadIdx.x, pn = es[e].prev_n;
    const int64_t ew = es[e].w, etile0 = es[e].w_tile0, wb = es[e].w_base, n0 = es[e].node0;
    int32_t *const cptr = es[e].cptr;
    const bool checked = A.steps[A.ent[e].step].nchk > 0 && A.steps[A.ent[e].step].kind != STEP_LIST;
    int64_t len[NPT], lo[NPT], ws = 0;
    int nzc = 0;
    for (int k = 0; k < NPT; ++k) {
      len[k] = lo[k] = 0;
      if (i0 + k < pn) {
        len[k] = gld(it->len + n0 + i0 + k);
        lo[k] = gld(it->lo + n0 + i0 + k);
      }
      nzc += len[k] > 0;
      ws += len[k];
    }
    // one scan for both counts: entries above bit 11, non-empty nodes (at most kTileNodes) below
    int64_t tot;
    const int64_t ex = block_excl_scan_i64((ws << 11) | nzc, tot, lds);
    int pos = (int)(ex & 2047);
    int64_t wpos = ex >> 11;
    const int ftot = (int)(tot & 2047);
    const int64_t wtot = tot >> 11;
    for (int k = 0; k < NPT; ++k) {
      const int64_t i = i0 + k;
      const int64_t woff = run_w + wpos - wb;   // entry-local first entry of node i
      if (cptr && i < pn) cptr[i] = (int32_t)woff;
      if (len[k] > 0) {
        const int64_t kk = run_nz + pos;
        it->nz_node[kk] = (int32_t)i;
        it->nz_lo[kk] = lo[k];
        it->nz_woff[kk] = woff;
        if (checked) {
          it->nz_chk_lo[kk] = gld(it->chk_lo + n0 + i);
          it->nz_chk_hi[kk] = gld(it->chk_hi + n0 + i);
        }
        s_woff[pos] = woff;
        ++pos;
      }
      wpos += len[k];
    }
    __syncthreads();
    // the tiles whose first entry lies among this node tile's entries [r0, r0 + wtot):
    // each takes the last of the tile's nodes starting at or before it
    const int64_t r0 = run_w - wb;
    for (int64_t j = ceil_div(r0, kTileWork) + threadIdx.x; j * kTileWork < r0 + wtot; j += blockDim.x) {
      const int64_t a = j * kTileWork;
      int lo_k = 0, hi_k = ftot - 1;   // s_woff[0] == r0 <= a
      while (lo_k < hi_k) {
        const int mid = (lo_k + hi_k + 1) >> 1;
        if (s_woff[mid] <= a) lo_k = mid; else hi_k = mid - 1;
      }
      DTile d;
      d.k0 = run_nz + lo_k;
      d.a = a;
      d.out = 0;
      d.e = e;
      d.n = (int32_t)min((int64_t)kTileWork, ew - a);
      d.cnt = 0;
      d.pad = 0;
      it->tiles[etile0 + j] = d;
    }
    __syncthreads();   // s_woff is refilled by the next tile
    run_nz += ftot;
    run_w += wtot;
  }
}

// ------------------------------------------------------------------ expansion
// Expansion tiles are taken by single waves: each wave stages its tile's nodes
// in its own LDS region and maps items to nodes with wave-wide scans, so no
// workgroup barrier couples the waves of a workgroup.
constexpr int kItemsPerLane = kTileWork / 64;

// Orders the calling wave's LDS accesses (LDS operations of one wave complete
// in order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Staged nodes of one tile. Node i of the tile is non-empty node tiles[t].k0 + i;
// item p (entry a + p) belongs to node kmap[p] and reads entry base[i] + p of
// that node's segment (or list).
struct WaveTile {
  uint32_t base[kTileWork + 2]; // segment start minus the node's first item position in the tile, plus
                                // kTileWork (>= 0; below 2^32 while the matrix has under 2^32 - 4096 entries)
  int32_t node[kTileWork + 2];  // local node index in the previous level
  uint8_t dg[kTileWork + 2];    // orientation | generator << 1 (see seg_ref)
  uint16_t kmap[kTileWork];     // item -> node; all zero between tiles
};

// The first 64 nodes of a tile's window, one per lane (loaded ahead of staging).
struct WinSlot {
  int64_t woff = 0, lo = 0;
  int32_t node = 0;
};

// Nodes k0 .. the node holding the next tile's first entry (when it is the same entry's).
__device__ __forceinline__ int win_nodes(const DTile &d, const DTile &dn) {
  return (int)(dn.k0 - d.k0 + (dn.e == d.e ? 1 : 0));
}

__device__ __forceinline__ WinSlot load_slot(const IterScalars *it, const DTile &d, int nwin) {
  WinSlot w;
  const int lane = threadIdx.x & 63;
  if (lane < nwin) {
    const int64_t k = d.k0 + lane;
    w.woff = gld(it->nz_woff + k);
    w.lo = gld(it->nz_lo + k);
    w.node = gld(it->nz_node + k);
  }
  return w;
}

// Stage tile d (dn: the record after it; s0: its first window slot) into the
// calling wave's region. On return kmap holds the item -> node map (a
// max-scan of node starts); the item pass reads each entry once and clears it.
__device__ __forceinline__ void stage_tile(const IterScalars *it, const DTile &d, int nwin, const WinSlot &s0,
                                           WaveTile &W) {
  const int lane = threadIdx.x & 63;
  bool scat = false;
  for (int i = lane; i < nwin; i += 64) {
    const int64_t k = d.k0 + i;
    int64_t woff, r;
    int32_t nd;
    if (i < 64) {
      woff = s0.woff; r = s0.lo; nd = s0.node;
    } else {
      woff = gld(it->nz_woff + k); r = gld(it->nz_lo + k); nd = gld(it->nz_node + k);
    }
    const int64_t s = woff - d.a;   // first item of the node, relative to the tile
    W.base[i] = (uint32_t)(ref_lo(r) - s + kTileWork);
    W.dg[i] = (uint8_t)(ref_dir(r) | (ref_gen(r) << 1));
    W.node[i] = nd;
    if (i > 0 && s < d.n) { W.kmap[s] = (uint16_t)i; scat = true; }
  }
  wave_lds_sync();
  if (__ballot(scat) == 0) return;   // one node covers the whole tile: the map stays zero
  // forward fill: each item takes the last node start at or before it (node starts ascend)
  int v[kItemsPerLane];
  int mx = 0;
  for (int i = 0; i < kItemsPerLane; ++i) { mx = max(mx, (int)W.kmap[lane * kItemsPerLane + i]); v[i] = mx; }
  // inclusive max-scan over the wave with DPP row shifts and row broadcasts
  // (values are >= 0, so lanes without a source read 0)
  int incl = max(mx, __builtin_amdgcn_update_dpp(0, mx, 0x111, 0xf, 0xf, true));   // row_shr:1
  incl = max(incl, __builtin_amdgcn_update_dpp(0, mx, 0x112, 0xf, 0xf, true));     // row_shr:2
  incl = max(incl, __builtin_amdgcn_update_dpp(0, mx, 0x113, 0xf, 0xf, true));     // row_shr:3
  incl = max(incl, __builtin_amdgcn_update_dpp(0, incl, 0x114, 0xf, 0xe, true));   // row_shr:4, lanes 4-15 of a row
  incl = max(incl, __builtin_amdgcn_update_dpp(0, incl, 0x118, 0xf, 0xc, true));   // row_shr:8, lanes 8-15 of a row
  incl = max(incl, __builtin_amdgcn_update_dpp(0, incl, 0x142, 0xa, 0xf, false));  // row_bcast:15 into rows 1, 3
  incl = max(incl, __builtin_amdgcn_update_dpp(0, incl, 0x143, 0xc, 0xf, false));  // row_bcast:31 into rows 2, 3
  const int pre = __builtin_amdgcn_update_dpp(0, incl, 0x138, 0xf, 0xf, true);    // wave_shr:1 (lane 0 reads 0)
  for (int i = 0; i < kItemsPerLane; ++i) W.kmap[lane * kItemsPerLane + i] = (uint16_t)max(pre, v[i]);
  wave_lds_sync();
}

// Node of item p of the staged tile; clears the map entry for the next tile
// (each entry is read by exactly one lane).
__device__ __forceinline__ int take_node(WaveTile &W, int p) {
  const int k = W.kmap[p];
  W.kmap[p] = 0;
  return k;
}

// The orientation bit of a node selects between the two id arrays with a
// select (indexing A.g.idx by a per-lane value would load the pointer from
// memory for every item).
__device__ __forceinline__ const int32_t *seg_ids(const IterArgs &A, int dg) {
  return (dg & 1) ? A.g.idx[1] : A.g.idx[0];
}

__device__ __forceinline__ int32_t candidate(const IterArgs &A, const EState &E, const DStep &S, const WaveTile &W,
                                             int k, int p) {
  const int32_t *src = S.kind == STEP_LIST ? E.list : seg_ids(A, W.dg[k]);
  return gld(src + ((int64_t)W.base[k] - kTileWork + p));
}

// gen: which bound segment the candidate was read from (see seg_ref); that
// check is replaced by the parent edge's.
// clo/chi: bounds of the first tested segment (found by the lookup), searched
// directly; the others are located by row and label first.
template <int LB, int OB>
__device__ __forceinline__ bool test_candidate(const IterArgs &A, const EState &E, const DStep &S, int32_t node,
                                               int gen, int64_t clo, int64_t chi, int32_t c, int &probes, int &ftests,
                                               int &ctests) {
  for (int f = S.list_nfilt; f < S.nfilt; ++f) {
    ++ftests;
    if (!bit_test(A.filt[S.filt0 + f], c)) return false;
  }
  for (int k = 0; k < S.nchk; ++k) {
    ++ctests;
    if (k == 0) {
      const int dir0 = gen == 1 ? S.dir : A.checks[S.chk0].dir;
      const int32_t *ids = dir0 ? A.g.idx[1] : A.g.idx[0];
      int64_t x = clo, y = chi;
      while (x < y) {
        const int64_t mid = (x + y) >> 1;
        ++probes;
        if (gld(ids + mid) < c) x = mid + 1; else y = mid;
      }
      if (!(x < chi && gld(ids + x) == c)) return false;
      continue;
    }
    int32_t b, label, dir;
    if (k + 1 == gen) {
      b = S.kind == STEP_SEG ? gld(E.prev + (int64_t)S.src * E.prev_n + node) : S.src;
      label = S.label;
      dir = S.dir;
    } else {
      const DCheck ck = A.checks[S.chk0 + k];
      b = gld(E.prev + (int64_t)ck.col * E.prev_n + node);
      label = ck.label;
      dir = ck.dir;
    }
    if (!seg_has_w<LB, OB>(A.g, dir, b, label, c, probes)) return false;
  }
  for (int k = 0; k < S.nself; ++k)
    if (!seg_has_w<LB, OB>(A.g, 0, c, A.ints[S.self0 + k], c, probes)) return false;
  return true;
}

// Count pass over the tiles of tested levels: validity bits per tile, valid
// entries per tile, per entry and per workgroup. A workgroup takes a
// contiguous tile range; test-free entries in it are passed over whole, the
// tiles of tested entries are dealt to its waves.
template <int LB, int OB, bool FILTERS_ONLY>
__device__ __forceinline__ void expand_count_body(const IterArgs &A, WaveTile *Wt, int64_t (*red4)[4]) {
  IterScalars *it = A.it;
  if (it->abort) return;
  EState *es = A.es;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  WaveTile &W = Wt[wv];
  for (int i = lane; i < kTileWork; i += 64) W.kmap[i] = 0;
  wave_lds_sync();
  const int64_t G = active_groups(it->work_tiles, gridDim.x);
  if (blockIdx.x >= G) return;
  int64_t tb, te;
  block_share_g(it->work_tiles, G, tb, te);
  int64_t free_items = 0, w_cnt = 0, w_pr = 0, w_ft = 0, w_ct = 0;
  for (int64_t t = tb; t < te;) {
    const int e = uniform(gld(&it->tiles[t].e));
    const EState E = es[e];
    const DEntry d = A.ent[e];
    const DStep S = A.steps[d.step];
    const int64_t t_end = min(te, E.w_tile0 + ceil_div(E.w, kTileWork));
    if (test_free(S)) {   // every candidate is a child: the entry's count was set by the node scan
      free_items += min((t_end - E.w_tile0) * kTileWork, E.w) - (t - E.w_tile0) * kTileWork;
      t = t_end;
      continue;
    }
    int64_t e_cnt = 0;
    int pr = 0, ft = 0, ct = 0;
    for (int64_t u = t + wv; u < t_end; u += kWaves) {
      const DTile dt = it->tiles[u], dn = it->tiles[u + 1];
      const int nwin = win_nodes(dt, dn);
      stage_tile(it, dt, nwin, load_slot(it, dt, nwin), W);
      uint64_t *vw = (uint64_t *)(it->valid + u * (kTileWork / 32));
      int c_tile = 0;
      if constexpr (FILTERS_ONLY) {
        // bitmap filters only: four of the lane's candidates at a time, then each filter's words
        // for the four, every round a batch of independent loads (instead of two or more
        // dependent round trips per item)
#pragma unroll
        for (int h = 0; h < kItemsPerLane; h += 4) {
          int32_t cv[4];
          uint32_t live = 0;   // bit r: item h + r exists and has passed the filters tested so far
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int p = (h + r) * 64 + lane;
            const int k = take_node(W, p);
            cv[r] = 0;
            if (p < dt.n) {
              cv[r] = candidate(A, E, S, W, k, p);
              live |= 1u << r;
            }
          }
          for (int f = S.list_nfilt; f < S.nfilt && live; ++f) {
            // the 32-bit half of the 64-bit bitmap word that holds each bit (little-endian words)
            const uint32_t *bm = (const uint32_t *)A.filt[S.filt0 + f];
            uint32_t wd[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) wd[r] = gld(bm + (cv[r] >> 5));   // word 0 for absent items
            ft += __popc(live);
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (!((wd[r] >> (cv[r] & 31)) & 1u)) live &= ~(1u << r);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint64_t bal = __ballot((live >> r) & 1u);
            if (lane == 0) gst(vw + h + r, bal);
            c_tile += __popcll(bal);
          }
        }
      } else {
        for (int r = 0; r < kItemsPerLane; ++r) {
          const int p = r * 64 + lane;
          const int k = take_node(W, p);
          bool ok = false;
          if (p < dt.n) {
            const int32_t c = candidate(A, E, S, W, k, p);
            int64_t clo = 0, chi = 0;
            if (S.nchk > 0) { clo = gld(it->nz_chk_lo + dt.k0 + k); chi = gld(it->nz_chk_hi + dt.k0 + k); }
            ok = test_candidate<LB, OB>(A, E, S, W.node[k], W.dg[k] >> 1, clo, chi, c, pr, ft, ct);
          }
          const uint64_t bal = __ballot(ok);
          if (lane == 0) gst(vw + r, bal);
          c_tile += __popcll(bal);
        }
      }
      wave_lds_sync();
      if (lane == 0) it->tiles[u].cnt = c_tile;
      e_cnt += c_tile;
    }
    // this wave's share of the entry and of its query's probes
    const int64_t epr = wave_sum_i64(pr), eft = wave_sum_i64(ft), ect = wave_sum_i64(ct);
    if (lane == 0) {
      if (e_cnt) atomicAdd((unsigned long long *)&es[e].cnt, (unsigned long long)e_cnt);
      if (epr) atomicAdd((unsigned long long *)&A.qstats[(int64_t)d.q * QS_N + QS_PROBE], (unsigned long long)epr);
      if (eft) atomicAdd((unsigned long long *)&A.qstats[(int64_t)d.q * QS_N + QS_BMWORDS], (unsigned long long)eft);
    }
    w_cnt += e_cnt;
    w_pr += epr;
    w_ft += eft;
    w_ct += ect;
    t = t_end;
  }
  if (lane == 0) { red4[wv][0] = w_cnt; red4[wv][1] = w_pr; red4[wv][2] = w_ft; red4[wv][3] = w_ct; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t v4[4] = {0, 0, 0, 0};
    for (int i = 0; i < 4; ++i) for (int w2 = 0; w2 < kWaves; ++w2) v4[i] += red4[w2][i];
    if (v4[1]) atomicAdd((unsigned long long *)&it->probes, (unsigned long long)v4[1]);
    if (v4[2]) atomicAdd((unsigned long long *)&it->ftests, (unsigned long long)v4[2]);
    if (v4[3]) atomicAdd((unsigned long long *)&it->ctests, (unsigned long long)v4[3]);
    A.blk_a[blockIdx.x] = v4[0] + free_items;
  }
}

// One instance per stored width pair, chosen on the host (as the lookup), and one for launches
// whose entries test bitmap filters only: that variant batches the loads of several items, which
// in the general one would cost registers (and spills) that its exact checks need.
template <int LB, int OB, bool FILTERS_ONLY>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_expand_count(const IterArgs A) {
  __shared__ WaveTile Wt[kWaves];
  __shared__ int64_t red4[kWaves][4];
  expand_count_body<LB, OB, FILTERS_ONLY>(A, Wt, red4);
}

__global__ __launch_bounds__(1024) void k_scan_expand(const IterArgs A) {
  __shared__ int64_t lds[1024];
  IterScalars *it = A.it;
  if (it->abort) return;
  EState *es = A.es;
  wg_scan(active_groups(it->work_tiles, A.grid), [&](int64_t i) { return A.blk_a[i]; },
          [&](int64_t i, int64_t v) { A.blk_off_a[i] = v; }, lds);
  // the same sums as the tiles carry (levels counted without tiles take no positions)
  const int64_t tot = wg_scan(A.E, [&](int64_t i) { return counted_only(A.steps[A.ent[i].step]) ? (int64_t)0 : es[i].cnt; },
                              [&](int64_t i, int64_t v) { es[i].out_base = v; }, lds);
  if (threadIdx.x == 0) it->cnt_total = tot;
  for (int e = threadIdx.x; e < A.E; e += blockDim.x) {
    const DEntry d = A.ent[e];
    const DStep S = A.steps[d.step];
    if (!test_free(S)) alloc_level(A, e, d, S);   // levels without tests were allocated by the node scan
    es[e].copies = A.ints + S.copy0;
    es[e].ncopy = S.ncopy;
    es[e].wflags = (test_free(S) ? EW_FREE : 0) | (S.kind == STEP_LIST ? EW_LIST : 0);
  }
}

// Output position of every tile's first child, entry-local: the count pass's
// contiguous tile ranges again, each scanned from its workgroup's offset.
__global__ __launch_bounds__(kBlock) void k_tile_offsets(const IterArgs A) {
  __shared__ int64_t lds[kWaves];
  IterScalars *it = A.it;
  if (it->abort) return;
  EState *es = A.es;
  const int64_t G = active_groups(it->work_tiles, gridDim.x);
  if (blockIdx.x >= G) return;
  int64_t tb, te;
  block_share_g(it->work_tiles, G, tb, te);
  int64_t run = A.blk_off_a[blockIdx.x];
  for (int64_t c0 = tb; c0 < te; c0 += kBlock) {
    const int64_t t = c0 + threadIdx.x;
    int64_t v = 0;
    int e = 0;
    if (t < te) {
      DTile *d = it->tiles + t;
      e = d->e;
      v = test_free(A.steps[A.ent[e].step]) ? d->n : d->cnt;
    }
    int64_t tot;
    const int64_t x = block_excl_scan_i64(v, tot, lds);
    if (t < te) it->tiles[t].out = run + x - es[e].out_base;
    run += tot;
  }
}

// Write pass: tiles dealt round-robin to the waves of a grid of resident
// workgroups (tiles are independent; neighbours run side by side). A wave
// loads its tile records two tiles ahead and the node window one tile ahead,
// so that one round trip to memory (the candidates) remains per tile. Every
// item's output position is ranked first (tile offset + item for test-free
// levels, + rank among the valid items otherwise); then each lane reads the
// nodes and candidates of all its items before it issues their stores.
// NW waves per workgroup (2, 4 or 8): every wave works on its own tiles with its own staging
// slot, so the workgroup size only sets how the waves are grouped onto compute units.
template <int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(6))) void k_expand_write(const IterArgs A) {
  __shared__ WaveTile Wt[NW];
  const IterScalars *it = A.it;
  if (sld(&it->abort)) return;
  const EState *es = A.es;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int R = kItemsPerLane;
  WaveTile &W = Wt[wv];
  for (int i = lane; i < kTileWork; i += 64) W.kmap[i] = 0;
  wave_lds_sync();
  const DTile *tiles = sld(&it->tiles);
  const uint32_t *valid = sld(&it->valid);
  const int64_t ntiles = sld(&it->work_tiles), stride = (int64_t)gridDim.x * NW;
  int64_t t = (int64_t)blockIdx.x * NW + wv;
  if (t >= ntiles) return;
  DTile d1 = sld(tiles + t), d1n = sld(tiles + t + 1), d2{}, d2n{};
  int nw1 = win_nodes(d1, d1n);
  WinSlot s1 = load_slot(it, d1, nw1);
  if (t + stride < ntiles) { d2 = sld(tiles + t + stride); d2n = sld(tiles + t + stride + 1); }
  for (; t < ntiles; t += stride) {
    stage_tile(it, d1, nw1, s1, W);
    const int e = d1.e;
    const int64_t out0 = d1.out, a0 = d1.a;
    const int n = d1.n;
    // next tile: its window loads now (its records arrived during the previous tile), the one after: its records
    const int64_t tn = t + stride;
    if (tn < ntiles) {
      d1 = d2; d1n = d2n;
      nw1 = win_nodes(d1, d1n);
      s1 = load_slot(it, d1, nw1);
      if (tn + stride < ntiles) { d2 = sld(tiles + tn + stride); d2n = sld(tiles + tn + stride + 1); }
    }
    int32_t *out = sld(&es[e].out);
    const int32_t wflags = sld(&es[e].wflags);
    int kk[R];
    for (int r = 0; r < R; ++r) kk[r] = take_node(W, r * 64 + lane);
    int32_t li[R];   // output position of each item, -1: not a child (levels stay below 2^31 nodes)
    int64_t end = a0 + n;   // one past the tile's last output position
    if (wflags & EW_FREE) {   // every entry is a child: a tile's children start at its first entry
      for (int r = 0; r < R; ++r) {
        const int p = r * 64 + lane;
        li[r] = p < n ? (int32_t)(a0 + p) : -1;
      }
    } else {
      const uint64_t *vw = (const uint64_t *)(valid + t * (kTileWork / 32));
      int32_t before = (int32_t)out0;
      for (int r = 0; r < R; ++r) {
        const uint64_t bal = gld(vw + r);
        li[r] = ((bal >> lane) & 1ull) ? before + (int32_t)__popcll(bal & lanemask_lt()) : -1;
        before += (int32_t)__popcll(bal);
      }
      end = __builtin_amdgcn_readfirstlane(before);
    }
    const int64_t cnt = out ? sld(&es[e].cnt) : 0;
    if (out && end > cnt) {   // count and write passes disagree: write nothing, report it
      if (lane == 0 && A.flags) atomicOr(&A.flags[RF_WRITE], 1);
    } else if (out) {
      const int32_t *list = sld(&es[e].list);
      int32_t node[R], c[R];
      for (int r = 0; r < R; ++r) {
        node[r] = 0;
        c[r] = 0;
        if (li[r] >= 0) {
          const int k = kk[r];
          node[r] = W.node[k];
          const int32_t *src = (wflags & EW_LIST) ? list : seg_ids(A, W.dg[k]);
          c[r] = gld(src + ((int64_t)W.base[k] - kTileWork + r * 64 + lane));
        }
      }
      for (int r = 0; r < R; ++r)
        if (li[r] >= 0) {
          if (!(wflags & EW_FREE)) gst_stream(out + li[r], node[r]);   // levels without tests keep offsets instead
          gst_stream(out + cnt + li[r], c[r]);
        }
      const int ncopy = sld(&es[e].ncopy);
      if (ncopy) {
        const int32_t *prev = sld(&es[e].prev), *copies = sld(&es[e].copies);
        const int64_t prev_n = sld(&es[e].prev_n);
        for (int j = 0; j < ncopy; ++j) {
          const int32_t *col = prev + (int64_t)sld(copies + j) * prev_n;
          int32_t v[R];
          for (int r = 0; r < R; ++r) v[r] = li[r] >= 0 ? gld(col + node[r]) : 0;
          for (int r = 0; r < R; ++r)
            if (li[r] >= 0) gst_stream(out + (int64_t)(2 + j) * cnt + li[r], v[r]);
        }
      }
    }
    wave_lds_sync();
  }
}

// ------------------------------------------------------------------ results
// Rows [first, first + n) of one query: walk each leaf's parents to the root.
// Parent of node i of a level: its parent column, or the last parent whose
// first child is at or before i (child offsets ascend).
__device__ __forceinline__ int64_t parent_of(const int32_t *L, const int32_t *cptr, int64_t prev_n, int64_t i) {
  if (!cptr) return L[i];
  int64_t lo = 0, hi = prev_n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (cptr[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Rows [first, first + n) of one query: walk each leaf's parents to the root.
__global__ __launch_bounds__(kBlock) void k_enumerate(int32_t *const *lvl_ptr, int32_t *const *lvl_cptr,
                                                      const int64_t *lvl_n, int k, const int32_t *var_rank,
                                                      int64_t first, int64_t n, int32_t *rows) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    int64_t node = first + r;
    for (int j = k - 1; j >= 0; --j) {
      const int32_t *L = lvl_ptr[j];
      const int64_t nj = lvl_n[j];
      rows[r * k + var_rank[j]] = L[nj + node];
      if (j > 0) node = parent_of(L, lvl_cptr[j], lvl_n[j - 1], node);
    }
  }
}

// Order-independent digest of the rows: each leaf's row (variables in ascending
// query-vertex order, k values) hashes to h_k with h_0 = k and
// h_{i+1} = mix64(h_i + 0x9E3779B97F4A7C15 + (uint32)v_i), mix64 being the output
// function of the splitmix64 generator (Steele, Lea and Flood, OOPSLA 2014);
// the digest is the sum (mod 2^64) and the XOR of the row hashes.
__device__ __forceinline__ uint64_t splitmix_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(kBlock) void k_row_digest(int32_t *const *lvl_ptr, int32_t *const *lvl_cptr,
                                                       const int64_t *lvl_n, int k, const int32_t *var_rank,
                                                       int64_t n, unsigned long long *out) {
  uint64_t hs = 0, hx = 0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    int32_t row[kMaxLevels];
    int64_t node = r;
    for (int j = k - 1; j >= 0; --j) {
      const int32_t *L = lvl_ptr[j];
      const int64_t nj = lvl_n[j];
      row[var_rank[j]] = L[nj + node];
      if (j > 0) node = parent_of(L, lvl_cptr[j], lvl_n[j - 1], node);
    }
    uint64_t h = (uint64_t)k;
    for (int i = 0; i < k; ++i) h = splitmix_out(h + 0x9E3779B97F4A7C15ull + (uint64_t)(uint32_t)row[i]);
    hs += h;
    hx ^= h;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    hs += __shfl_xor(hs, off, 64);
    hx ^= __shfl_xor(hx, off, 64);
  }
  if ((threadIdx.x & 63) == 0 && (hs | hx)) {
    atomicAdd(&out[0], (unsigned long long)hs);
    atomicXor(&out[1], (unsigned long long)hx);
  }
}

// ---------------------------------------------------------------- launchers
int expand_write_blocks_per_cu(int waves) {
  const void *k = waves == 2   ? reinterpret_cast<const void *>(k_expand_write<2>)
                  : waves == 8 ? reinterpret_cast<const void *>(k_expand_write<8>)
                               : reinterpret_cast<const void *>(k_expand_write<4>);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 64 * waves, 0) != hipSuccess || nb < 1)
    nb = 16 / waves;
  return nb;
}

// Seed bitmaps back to zero after a run (they are kept zero between runs): a seed whose
// segment is short clears the words its ids fall in, one with a segment longer than a
// quarter of the bitmap's words clears the whole bitmap. Plain stores of zero: lanes that
// meet in a word write the same value.
__global__ __launch_bounds__(kBlock) void k_unseed(const DevGraph g, const DSeed *seeds, int32_t n) {
  for (int32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const DSeed sd = seeds[i];
    int64_t lo, hi;
    int probes = 0;
    seg_find(g, sd.dir, sd.c, sd.label, lo, hi, probes);
    if (hi - lo > g.words / 4) {
      for (int64_t w = threadIdx.x; w < g.words; w += kBlock) sd.bm[w] = 0ull;
    } else {
      const int32_t *ids = sd.dir ? g.idx[1] : g.idx[0];
      for (int64_t x = lo + threadIdx.x; x < hi; x += kBlock) sd.bm[ids[x] >> 6] = 0ull;
    }
  }
}

hipError_t launch_unseed(const DevGraph &g, const DSeed *seeds, int32_t n, int grid, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unseed, dim3((unsigned)std::min<int64_t>(n, std::max(grid, 1))), dim3(kBlock), 0, s, g,
                     seeds, n);
  return hipGetLastError();
}

hipError_t launch_iteration(const IterArgs &A, hipStream_t s, hipEvent_t *ev) {
  const dim3 G(A.grid), B(kBlock), W1(1024);
  auto mark = [&](int slot, int end) { if (ev) (void)hipEventRecord(ev[2 * slot + end], s); };
#define GS_LAUNCH(slot, kern, grid, block)                          \
  do {                                                              \
    mark(slot, 0);                                                  \
    hipLaunchKernelGGL(kern, grid, block, 0, s, A);                 \
    mark(slot, 1);                                                  \
  } while (0)
  GS_LAUNCH(KS_SETUP, k_it_setup, dim3(1), W1);
  if (A.nclear) GS_LAUNCH(KS_CLEAR, k_clear, G, B);
  if (A.S) GS_LAUNCH(KS_SEED, k_seed, G, B);
  if (A.has_list) {
    GS_LAUNCH(KS_LIST_COUNT, k_list_count, G, B);
    GS_LAUNCH(KS_LIST_SCAN, k_list_scan, dim3(1), W1);
    GS_LAUNCH(KS_LIST_WRITE, k_list_write, G, B);
  }
  if (A.D) {
    GS_LAUNCH(KS_DOM_FRONTIER, k_dom_frontier, G, B);
    GS_LAUNCH(KS_DOM_PUSH, k_dom_push, G, B);
    GS_LAUNCH(KS_DOM_PULL, k_dom_pull, G, B);
  }
  {
    const int w = (A.g.lab8 ? 0 : 2) + (A.g.off32 ? 0 : 1) + (A.has_factor ? 4 : 0);
    switch (w) {
      case 0: GS_LAUNCH(KS_LOOKUP, (k_lookup<1, 4, false>), G, B); break;
      case 1: GS_LAUNCH(KS_LOOKUP, (k_lookup<1, 8, false>), G, B); break;
      case 2: GS_LAUNCH(KS_LOOKUP, (k_lookup<2, 4, false>), G, B); break;
      case 3: GS_LAUNCH(KS_LOOKUP, (k_lookup<2, 8, false>), G, B); break;
      case 4: GS_LAUNCH(KS_LOOKUP, (k_lookup<1, 4, true>), G, B); break;
      case 5: GS_LAUNCH(KS_LOOKUP, (k_lookup<1, 8, true>), G, B); break;
      case 6: GS_LAUNCH(KS_LOOKUP, (k_lookup<2, 4, true>), G, B); break;
      default: GS_LAUNCH(KS_LOOKUP, (k_lookup<2, 8, true>), G, B); break;
    }
  }
  GS_LAUNCH(KS_SCAN_NODES, k_scan_nodes, dim3(1), W1);
  GS_LAUNCH(KS_NZ_WRITE, k_nz_write, G, B);
  if (A.has_tested) {
    switch ((A.g.lab8 ? 0 : 2) + (A.g.off32 ? 0 : 1) + (A.has_exact ? 0 : 4)) {
      case 0: GS_LAUNCH(KS_EXPAND_COUNT, (k_expand_count<1, 4, false>), G, B); break;
      case 1: GS_LAUNCH(KS_EXPAND_COUNT, (k_expand_count<1, 8, false>), G, B); break;
      case 2: GS_LAUNCH(KS_EXPAND_COUNT, (k_expand_count<2, 4, false>), G, B); break;
      case 3: GS_LAUNCH(KS_EXPAND_COUNT, (k_expand_count<2, 8, false>), G, B); break;
      case 4: GS_LAUNCH(KS_EXPAND_COUNT, (k_expand_count<1, 4, true>), G, B); break;
      case 5: GS_LAUNCH(KS_EXPAND_COUNT, (k_expand_count<1, 8, true>), G, B); break;
      case 6: GS_LAUNCH(KS_EXPAND_COUNT, (k_expand_count<2, 4, true>), G, B); break;
      default: GS_LAUNCH(KS_EXPAND_COUNT, (k_expand_count<2, 8, true>), G, B); break;
    }
  }
  GS_LAUNCH(KS_SCAN_EXPAND, k_scan_expand, dim3(1), W1);
  if (A.has_tested) GS_LAUNCH(KS_TILE_OFFSETS, k_tile_offsets, G, B);
  if (A.wwaves == 2) GS_LAUNCH(KS_EXPAND_WRITE, k_expand_write<2>, dim3((unsigned)A.wgrid), dim3(128));
  else if (A.wwaves == 8) GS_LAUNCH(KS_EXPAND_WRITE, k_expand_write<8>, dim3((unsigned)A.wgrid), dim3(512));
  else GS_LAUNCH(KS_EXPAND_WRITE, k_expand_write<4>, dim3((unsigned)A.wgrid), B);
#undef GS_LAUNCH
  return hipGetLastError();
}

hipError_t launch_enumerate(int32_t *const *lvl_ptr, int32_t *const *lvl_cptr, const int64_t *lvl_n, int k,
                            const int32_t *var_rank, int64_t first, int64_t n, int32_t *rows, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_enumerate, dim3((unsigned)g), dim3(kBlock), 0, s, lvl_ptr, lvl_cptr, lvl_n, k, var_rank, first,
                     n, rows);
  return hipGetLastError();
}

hipError_t launch_row_digest(int32_t *const *lvl_ptr, int32_t *const *lvl_cptr, const int64_t *lvl_n, int k,
                             const int32_t *var_rank, int64_t n, uint64_t *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 8192) g = 8192;
  hipLaunchKernelGGL(k_row_digest, dim3((unsigned)g), dim3(kBlock), 0, s, lvl_ptr, lvl_cptr, lvl_n, k, var_rank, n,
                     (unsigned long long *)out);
  return hipGetLastError();
}

}  // namespace gs

namespace gs {

// Standalone pieces of an iteration, used by the matrix-algebra primitives of the ABI.
hipError_t launch_list_only(const IterArgs &A, hipStream_t s) {
  const dim3 G(A.grid), B(kBlock), W1(1024);
  hipLaunchKernelGGL(k_it_setup, dim3(1), W1, 0, s, A);
  hipLaunchKernelGGL(k_list_count, G, B, 0, s, A);
  hipLaunchKernelGGL(k_list_scan, dim3(1), W1, 0, s, A);
  hipLaunchKernelGGL(k_list_write, G, B, 0, s, A);
  return hipGetLastError();
}

static_assert(sizeof(DArena) <= NoAllocLayout::it - NoAllocLayout::arena, "workspace layout");
static_assert(sizeof(IterScalars) <= NoAllocLayout::es - NoAllocLayout::it, "workspace layout");
static_assert(sizeof(EState) <= NoAllocLayout::step - NoAllocLayout::es, "workspace layout");
static_assert(sizeof(DStep) <= NoAllocLayout::ent - NoAllocLayout::step, "workspace layout");
static_assert(sizeof(DEntry) <= NoAllocLayout::filt - NoAllocLayout::ent, "workspace layout");
static_assert(8 * kNoAllocMaxBitmaps <= NoAllocLayout::lvl_ptr - NoAllocLayout::filt, "workspace layout");
static_assert(8 * kMaxLevels <= NoAllocLayout::lvl_n - NoAllocLayout::lvl_ptr, "workspace layout");
static_assert(8 * kMaxLevels <= NoAllocLayout::qstats - NoAllocLayout::lvl_n, "workspace layout");
static_assert(8 * QS_N <= NoAllocLayout::heap - NoAllocLayout::qstats, "workspace layout");
static_assert(NoAllocLayout::heap + NoAllocLayout::heap_bytes <= NoAllocLayout::blk, "workspace layout");

// Writes the tables of a one-entry list iteration into the workspace and zeroes
// what the list kernels accumulate into (the workspace keeps an earlier call's
// contents). One wave.
__global__ __launch_bounds__(64) void k_noalloc_setup(char *ws, const NoAllocInit init) {
  using L = NoAllocLayout;
  const int t = threadIdx.x;
  for (size_t i = t; i < L::heap / 8; i += 64) {   // arena, scalars, entry state, tables, counters
    if (i * 8 >= L::filt && i * 8 < L::lvl_ptr) continue;
    ((int64_t *)ws)[i] = 0;
  }
  if (t < kNoAllocMaxBitmaps) ((const uint64_t **)(ws + L::filt))[t] = t < init.k ? init.bm[t] : nullptr;
  if (t == 0) {
    DArena *a = (DArena *)(ws + L::arena);
    a->top = 0;
    a->cap = L::heap_bytes;
    DStep *st = (DStep *)(ws + L::step);
    st->kind = STEP_LIST;
    st->nfilt = init.k;
    st->list_nfilt = init.k;
  }
}

__global__ __launch_bounds__(64) void k_noalloc_finish(const IterScalars *it, int64_t *count) {
  if (threadIdx.x == 0) *count = it->abort ? -1 : it->list_total;
}

hipError_t launch_list_noalloc(const DevGraph &g, const NoAllocInit &init, char *ws, int grid, int32_t *out,
                               int64_t *count, hipStream_t s) {
  using L = NoAllocLayout;
  if (grid < 1 || grid > kNoAllocMaxGrid || init.k < 0 || init.k > kNoAllocMaxBitmaps) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(64), 0, s, ws, init);
  IterArgs A{};
  A.g = g;
  A.ent = (const DEntry *)(ws + L::ent);
  A.E = 1;
  A.grid = grid;
  A.has_list = 1;
  A.steps = (const DStep *)(ws + L::step);
  A.filt = (const uint64_t *const *)(ws + L::filt);
  A.es = (EState *)(ws + L::es);
  A.it = (IterScalars *)(ws + L::it);
  A.lvl_ptr = (int32_t **)(ws + L::lvl_ptr);
  A.lvl_n = (int64_t *)(ws + L::lvl_n);
  A.qstats = (int64_t *)(ws + L::qstats);
  A.scratch = (DArena *)(ws + L::arena);
  A.scratch_base = ws + L::heap;
  int64_t *blk = (int64_t *)(ws + L::blk);
  A.blk_a = blk;
  A.blk_b = blk + kNoAllocMaxGrid;
  A.blk_off_a = blk + 2 * kNoAllocMaxGrid;
  A.blk_off_b = blk + 3 * kNoAllocMaxGrid;
  A.list_out = out;
  hipError_t e = launch_list_only(A, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_noalloc_finish, dim3(1), dim3(64), 0, s, (const IterScalars *)A.it, count);
  return hipGetLastError();
}

hipError_t launch_domain_only(const IterArgs &A, hipStream_t s) {
  const dim3 G(A.grid), B(kBlock);
  hipLaunchKernelGGL(k_dom_push, G, B, 0, s, A);
  hipLaunchKernelGGL(k_dom_pull, G, B, 0, s, A);
  return hipGetLastError();
}

}  // namespace gs

// ---------------------------------------------------------------- pruning
// Explicit tree pruning (Section 7.2.2 / 8.1): a node is kept when a leaf
// survives below it. Marking runs from the leaves up, compaction from the root
// down, remapping each child's parent index to its parent's new position.
namespace gs {

__global__ __launch_bounds__(kBlock) void k_prune_mark(const int32_t *par, const int32_t *cptr, int64_t prev_n,
                                                       int64_t n, const uint8_t *alive, uint8_t *alive_parent) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!alive || alive[i]) alive_parent[parent_of(par, cptr, prev_n, i)] = 1;
}

__global__ __launch_bounds__(kBlock) void k_prune_count(const uint8_t *alive, int64_t n, int64_t *blk) {
  __shared__ int64_t lds[kWaves];
  int64_t b, e;
  block_share(n, b, e);
  int64_t c = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += kBlock) c += alive[i];
  c = block_sum_i64(c, lds);
  if (threadIdx.x == 0) blk[blockIdx.x] = c;
}

__global__ __launch_bounds__(kBlock) void k_prune_write(const int32_t *L, const int32_t *cptr, int64_t prev_n,
                                                        int64_t n, int ncols, const uint8_t *alive,
                                                        const int64_t *blkoff, const int32_t *parent_newidx,
                                                        int32_t *newidx, int32_t *out, int64_t n_out) {
  __shared__ int lds[kWaves];
  int64_t b, e;
  block_share(n, b, e);
  int64_t run = blkoff[blockIdx.x];
  for (int64_t r = b; r < e; r += kBlock) {
    const int64_t i = r + threadIdx.x;
    const bool f = i < e && alive[i];
    int tot;
    const int pos = block_excl_flag(f, tot, lds);
    if (f) {
      const int64_t k = run + pos;
      newidx[i] = (int32_t)k;
      const int64_t p = parent_of(L, cptr, prev_n, i);
      out[k] = parent_newidx ? parent_newidx[p] : (int32_t)p;
      for (int c = 1; c < ncols; ++c) out[(int64_t)c * n_out + k] = L[(int64_t)c * n + i];
    }
    run += tot;
  }
}

hipError_t launch_prune_mark(const int32_t *par, const int32_t *cptr, int64_t prev_n, int64_t n, const uint8_t *alive,
                             uint8_t *alive_parent, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = std::min<int64_t>((n + kBlock - 1) / kBlock, 8192);
  hipLaunchKernelGGL(k_prune_mark, dim3((unsigned)g), dim3(kBlock), 0, s, par, cptr, prev_n, n, alive, alive_parent);
  return hipGetLastError();
}

hipError_t launch_prune_count(const uint8_t *alive, int64_t n, int64_t *blk, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_prune_count, dim3(grid), dim3(kBlock), 0, s, alive, n, blk);
  return hipGetLastError();
}

hipError_t launch_prune_write(const int32_t *L, const int32_t *cptr, int64_t prev_n, int64_t n, int ncols,
                              const uint8_t *alive, const int64_t *blkoff, const int32_t *parent_newidx,
                              int32_t *newidx, int32_t *out, int64_t n_out, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_prune_write, dim3(grid), dim3(kBlock), 0, s, L, cptr, prev_n, n, ncols, alive, blkoff,
                     parent_newidx, newidx, out, n_out);
  return hipGetLastError();
}

}  // namespace gs
