// Device helpers shared by the engine's kernels (wave64 / workgroup scans,
// reductions, segment lookup in the light-weight sparse matrix).
#pragma once
#include "gs_device.hpp"
#include <type_traits>

namespace gs {

// Workgroup barrier that orders LDS accesses only: outstanding global stores
// are not waited for. For loops whose waves share nothing through global
// memory within the kernel.
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Loads and stores through the global address space (the table pointers live
// in device memory, where the compiler cannot see it and would emit flat
// accesses, which also count against the LDS counter).
template <class T>
__device__ __forceinline__ T gld(const T *p) {
  return *(const __attribute__((address_space(1))) T *)p;
}
// Wave-uniform load through the scalar cache (constant address space): only for
// data no wave writes while the kernel runs.
template <class T>
__device__ __forceinline__ T sld(const T *p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return *(const __attribute__((address_space(4))) T *)p;
#else
  return *p;   // host pass: never executed
#endif
}
template <class T>
__device__ __forceinline__ void gst(T *p, T v) {
  *(__attribute__((address_space(1))) T *)p = v;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return (1ull << lane) - 1ull;
}

// v of the lane that DPP control `ctrl` names, as two 32-bit moves; 0 where the
// control names no lane (bound_ctrl) or the lane is masked off.
template <int ctrl, int row_mask, int bank_mask, bool bound>
__device__ __forceinline__ int64_t dpp_i64(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, ctrl, row_mask, bank_mask, bound);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), ctrl, row_mask, bank_mask, bound);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Inclusive sum over the lanes of a full wave: row shifts by 1, 2, 3 (of the
// input), 4 and 8 (of the partial sums, upper banks only), then the last lane
// of rows 0 and 2 into rows 1 and 3, and lane 31 into rows 2 and 3.
__device__ __forceinline__ int64_t wave_incl_scan_i64(int64_t v) {
  int64_t s = v + dpp_i64<0x111, 0xf, 0xf, true>(v);
  s += dpp_i64<0x112, 0xf, 0xf, true>(v);
  s += dpp_i64<0x113, 0xf, 0xf, true>(v);
  s += dpp_i64<0x114, 0xf, 0xe, true>(s);
  s += dpp_i64<0x118, 0xf, 0xc, true>(s);
  s += dpp_i64<0x142, 0xa, 0xf, false>(s);
  s += dpp_i64<0x143, 0xc, 0xf, false>(s);
  return s;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Exclusive scan of one int64 per thread over a kBlock workgroup. lds holds kWaves entries.
__device__ __forceinline__ int64_t block_excl_scan_i64(int64_t v, int64_t &total, int64_t *lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t inc = wave_incl_scan_i64(v);
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  int64_t off = 0;
  total = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    int64_t c = lds[i];
    if (i < w) off += c;
    total += c;
  }
  __syncthreads();
  return off + inc - v;
}

// Exclusive rank of a flag over a kBlock workgroup (ballot + popcount). lds: kWaves ints.
__device__ __forceinline__ int block_excl_flag(bool f, int &total, int *lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t b = __ballot(f);
  int r = __popcll(b & lanemask_lt());
  if (lane == 0) lds[w] = __popcll(b);
  __syncthreads();
  int off = 0;
  total = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    int c = lds[i];
    if (i < w) off += c;
    total += c;
  }
  __syncthreads();
  return off + r;
}

__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t *lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = wave_sum_i64(v);
  if (lane == 0) lds[w] = v;
  __syncthreads();
  int64_t t = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) t += lds[i];
  __syncthreads();
  return t;
}

// Two sums over a kBlock workgroup with one pair of barriers. lds holds 2 * kWaves entries.
__device__ __forceinline__ void block_sum2_i64(int64_t &a, int64_t &b, int64_t *lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  a = wave_sum_i64(a);
  b = wave_sum_i64(b);
  if (lane == 0) { lds[w] = a; lds[kWaves + w] = b; }
  __syncthreads();
  a = 0;
  b = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) { a += lds[i]; b += lds[kWaves + i]; }
  __syncthreads();
}

// Exclusive scan over an index space [0, L) by one workgroup (size a multiple
// of 64, at most 64 waves). get(i) returns the value, set(i, prefix) stores the
// exclusive prefix. Each thread takes a contiguous chunk; the chunk sums are
// scanned within waves by shuffles and across waves through lds (at least one
// entry per wave). Returns the total.
template <class Get, class Set>
__device__ int64_t wg_scan(int64_t L, Get get, Set set, int64_t *lds) {
  const int t = threadIdx.x, T = blockDim.x;
  const int lane = t & 63, w = t >> 6, nw = T >> 6;
  const int64_t per = (L + T - 1) / T;
  const int64_t b = min(L, (int64_t)t * per), e = min(L, b + per);
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += get(i);
  const int64_t inc = wave_incl_scan_i64(s);
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  int64_t off = 0, total = 0;
  for (int i = 0; i < nw; ++i) {
    const int64_t c = lds[i];
    if (i < w) off += c;
    total += c;
  }
  __syncthreads();
  int64_t run = off + inc - s;
  if (per == 1) {   // one element per thread: its value is s, no second read
    if (b < e) set(b, run);
  } else {
    for (int64_t i = b; i < e; ++i) {
      const int64_t v = get(i);
      set(i, run);
      run += v;
    }
  }
  __syncthreads();
  return total;
}

// K exclusive scans of the same length at once (one pass, one exchange through LDS): get(i, v)
// fills v[0..K) for element i, set(i, off) receives the K offsets. lds holds K * kWaves-of-
// the-workgroup entries. The totals go to total[0..K).
template <int K, class Get, class Set>
__device__ void wg_scan_k(int64_t L, Get get, Set set, int64_t *lds, int64_t (&total)[K]) {
  const int t = threadIdx.x, T = blockDim.x;
  const int lane = t & 63, w = t >> 6, nw = T >> 6;
  const int64_t per = (L + T - 1) / T;
  const int64_t b = min(L, (int64_t)t * per), e = min(L, b + per);
  int64_t s[K], v[K], run[K];
  for (int k = 0; k < K; ++k) s[k] = 0;
  for (int64_t i = b; i < e; ++i) {
    get(i, v);
    for (int k = 0; k < K; ++k) s[k] += v[k];
  }
  for (int k = 0; k < K; ++k) {
    const int64_t inc = wave_incl_scan_i64(s[k]);
    if (lane == 63) lds[k * nw + w] = inc;
    run[k] = inc - s[k];
  }
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    int64_t off = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
      const int64_t c = lds[k * nw + i];
      if (i < w) off += c;
      tot += c;
    }
    run[k] += off;
    total[k] = tot;
  }
  __syncthreads();
  if (per == 1) {   // one element per thread: no second read
    if (b < e) set(b, run);
  } else {
    for (int64_t i = b; i < e; ++i) {
      get(i, v);
      set(i, run);
      for (int k = 0; k < K; ++k) run[k] += v[k];
    }
  }
  __syncthreads();
}

// Block g of gridDim.x takes the contiguous share [lo, hi) of [0, total).
__device__ __forceinline__ void block_share(int64_t total, int64_t &lo, int64_t &hi) {
  const int64_t G = gridDim.x, g = blockIdx.x;
  // index spaces here stay far below 2^63 / 8192
  lo = total * g / G;
  hi = total * (g + 1) / G;
}

// Workgroups that take part in a pass over `units` tiles on a grid of `grid`: all of
// them, or one per tile when there are fewer tiles (a small level then costs a
// small partial-sum scan). The pass's count, scan and write kernels agree on it.
__device__ __forceinline__ int64_t active_groups(int64_t units, int64_t grid) {
  return units < 1 ? 1 : (units < grid ? units : grid);
}
// Block g of G takes the contiguous share [lo, hi) of [0, total).
__device__ __forceinline__ void block_share_g(int64_t total, int64_t G, int64_t &lo, int64_t &hi) {
  const int64_t g = blockIdx.x;
  lo = total * g / G;
  hi = total * (g + 1) / G;
}

// Reads of the stored matrix at its widths: LB bytes per label (1 or 2), OB
// bytes per row offset (4 or 8). The hot kernels are instantiated for the
// loaded widths; the others dispatch once per segment lookup.
template <int LB>
__device__ __forceinline__ uint32_t lab_w(const void *lab, int64_t x) {
  if constexpr (LB == 1) return (uint32_t)gld((const uint8_t *)lab + x);
  else return (uint32_t)gld((const uint16_t *)lab + x);
}
// Positions in the entry arrays at the offsets' width: 32-bit when the offsets are (M < 2^31),
// so that searches keep half the registers.
template <int OB>
using OffT = std::conditional_t<OB == 4, int32_t, int64_t>;
template <int OB>
__device__ __forceinline__ OffT<OB> off_w(const void *ptr, int64_t b) {
  if constexpr (OB == 4) return gld((const int32_t *)ptr + b);
  else return gld((const int64_t *)ptr + b);
}

// Iterations of the halving search over m entries (the label entries it reads).
__device__ __forceinline__ int search_steps(int64_t m) { return m > 0 ? 64 - __clzll((unsigned long long)m) : 0; }

// Short rows (e - a <= 8): the labels of entries [a, a + 8) come from aligned 8-byte loads
// of the words around them (one or two cache lines, no dependent load; the label arrays
// are allocated with 32 bytes to spare after their last entry), and the entries below and
// equal to `label` among the first e - a of them are counted in registers.
template <int LB, class I>
__device__ __forceinline__ void label_range_short(const void *lab, I a, I e, uint32_t label, I &lo, I &hi) {
  const int n = (int)(e - a);
  int less = 0, eq = 0;
  if (n > 0) {
    const I base = a & ~(I)7;   // 8 entries: 8-byte aligned (LB 1), 16-byte aligned (LB 2)
    const int sh = (int)(a - base);
    uint64_t x0, x1 = 0;
    if constexpr (LB == 1) {
      const uint64_t *p = (const uint64_t *)((const uint8_t *)lab + base);
      const uint64_t w0 = gld(p), w1 = gld(p + 1);
      x0 = sh ? (w0 >> (8 * sh)) | (w1 << (64 - 8 * sh)) : w0;   // entries a .. a+7, one byte each
    } else {
      // two 16-byte loads (base is 16-byte aligned)
      typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
      const u64x2 *p = (const u64x2 *)((const uint16_t *)lab + base);
      const u64x2 wa = gld(p), wb = gld(p + 1);
      const uint64_t w0 = wa.x, w1 = wa.y, w2 = wb.x, w3 = wb.y;
      const bool q = sh >= 4;
      const int r = sh & 3;
      uint64_t y0 = q ? w1 : w0, y1 = q ? w2 : w1, y2 = q ? w3 : w2;
      if (r) {
        y0 = (y0 >> (16 * r)) | (y1 << (64 - 16 * r));
        y1 = (y1 >> (16 * r)) | (y2 << (64 - 16 * r));
      }
      x0 = y0;   // entries a .. a+3
      x1 = y1;   // entries a+4 .. a+7
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      uint32_t v;
      if constexpr (LB == 1) v = (uint32_t)(x0 >> (8 * k)) & 0xffu;
      else v = (uint32_t)((k < 4 ? x0 : x1) >> (16 * (k & 3))) & 0xffffu;
      if (k < n) {
        less += v < label;
        eq += v == label;
      }
    }
  }
  lo = a + less;
  hi = lo + eq;
}

// Entries with label `label` among the row entries [a, e) (labels ascend): [lo, hi).
template <int LB, class I>
__device__ __forceinline__ void label_range_w(const void *lab, I a, I e, int32_t label, I &lo, I &hi, int &probes) {
  if (e - a <= 8) {          // short rows: the labels of [a, a + 8) at once, counted in registers
    label_range_short<LB>(lab, a, e, (uint32_t)label, lo, hi);
    probes += (int)(hi - a + (hi < e));   // the entries a linear pass would read
    return;
  }
  // both bounds (first entry >= label, first entry > label) halve the row in lockstep: two
  // independent loads per step instead of one search after the other; positions are
  // 32-bit, relative to the row's first entry (a row holds fewer than 2^31 entries)
  const uint32_t key = (uint32_t)label;
  const void *row = (const char *)lab + (int64_t)a * LB;
  const int32_t n = (int32_t)(e - a);
  // while the two intervals coincide (every probe so far missed the label's entries) the
  // bounds read the same entry: one load serves both
  int32_t l1 = 0, h1 = n, l2 = 0, h2 = n;
  while (l1 < h1 || l2 < h2) {
    const bool s1 = l1 < h1, s2 = l2 < h2, same = l1 == l2 && h1 == h2;
    const int32_t m1 = (l1 + h1) >> 1, m2 = (l2 + h2) >> 1;
    const uint32_t v1 = s1 ? lab_w<LB>(row, m1) : 0u;
    const uint32_t v2 = same ? v1 : s2 ? lab_w<LB>(row, m2) : 0u;
    if (s1) { if (v1 < key) l1 = m1 + 1; else h1 = m1; }
    if (s2) { if (v2 <= key) l2 = m2 + 1; else h2 = m2; }
  }
  lo = a + l1;
  hi = a + l2;
  probes += search_steps(e - a) + search_steps(e - lo);   // as the search of [lo, e) after [a, e) reads
}

// Label entries label_range_w reads to find [lo, hi) in [a, e), counted from the bounds
// (so that the search itself keeps no counter).
__device__ __forceinline__ int label_reads(int64_t a, int64_t e, int64_t lo, int64_t hi) {
  if (e - a <= 8) return (int)(hi - a + (hi < e));
  return search_steps(e - a) + search_steps(e - lo);
}

// Entries of vertex b with label `label` in orientation dir: [lo, hi).
template <int LB, int OB, class I>
__device__ __forceinline__ void seg_find_w(const DevGraph &g, int dir, int32_t b, int32_t label, I &lo, I &hi,
                                           int &probes) {
  // selects, not indexing: dir may differ between lanes, and indexing the
  // pointer arrays by a per-lane value loads the pointers from memory
  const void *ptr = dir ? g.ptr[1] : g.ptr[0];
  const OffT<OB> a = off_w<OB>(ptr, b), e = off_w<OB>(ptr, (int64_t)b + 1);
  OffT<OB> l, h;
  label_range_w<LB>(dir ? g.lab[1] : g.lab[0], a, e, label, l, h, probes);
  lo = (I)l;
  hi = (I)h;
}

template <int LB, int OB>
__device__ __forceinline__ bool seg_has_w(const DevGraph &g, int dir, int32_t b, int32_t label, int32_t c,
                                          int &probes) {
  using I = OffT<OB>;
  I lo, hi;
  seg_find_w<LB, OB>(g, dir, b, label, lo, hi, probes);
  const int32_t *idx = dir ? g.idx[1] : g.idx[0];
  I x = lo, y = hi;
  while (x < y) {
    const I mid = x + ((y - x) >> 1);
    ++probes;
    if (gld(idx + mid) < c) x = mid + 1; else y = mid;
  }
  return x < hi && gld(idx + x) == c;
}

// Runs CALL with constexpr LB and OB set to the loaded widths (one uniform branch).
#define GS_WITH_WIDTHS(g, CALL)                                  \
  do {                                                           \
    if ((g).lab8) {                                              \
      if ((g).off32) { constexpr int LB = 1, OB = 4; CALL; }     \
      else { constexpr int LB = 1, OB = 8; CALL; }               \
    } else {                                                     \
      if ((g).off32) { constexpr int LB = 2, OB = 4; CALL; }     \
      else { constexpr int LB = 2, OB = 8; CALL; }               \
    }                                                            \
  } while (0)

__device__ __forceinline__ void seg_find(const DevGraph &g, int dir, int32_t b, int32_t label, int64_t &lo,
                                         int64_t &hi, int &probes) {
  GS_WITH_WIDTHS(g, (seg_find_w<LB, OB>(g, dir, b, label, lo, hi, probes)));
}

// Is c among the entries of vertex b with label `label` (orientation dir)?
__device__ __forceinline__ bool seg_has(const DevGraph &g, int dir, int32_t b, int32_t label, int32_t c,
                                        int &probes) {
  bool r = false;
  GS_WITH_WIDTHS(g, (r = seg_has_w<LB, OB>(g, dir, b, label, c, probes)));
  return r;
}

// Store that is not kept in the caches (tree levels are written once and read
// back by a later kernel, from HBM).
template <class T>
__device__ __forceinline__ void gst_stream(T *p, T v) {
  __builtin_nontemporal_store(v, p);
}

__device__ __forceinline__ bool bit_test(const uint64_t *bm, int32_t c) {
  return (gld(bm + (c >> 6)) >> (c & 63)) & 1ull;
}

}  // namespace gs
