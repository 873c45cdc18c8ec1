// Device helpers shared by the engine's kernels (wave64 / workgroup scans,
// reductions, segment lookup in the light-weight sparse matrix).
#pragma once
#include "gs_device.hpp"

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
  for (int64_t i = b; i < e; ++i) {
    const int64_t v = get(i);
    set(i, run);
    run += v;
  }
  __syncthreads();
  return total;
}

// Block g of gridDim.x takes the contiguous share [lo, hi) of [0, total).
__device__ __forceinline__ void block_share(int64_t total, int64_t &lo, int64_t &hi) {
  const int64_t G = gridDim.x, g = blockIdx.x;
  // index spaces here stay far below 2^63 / 8192
  lo = total * g / G;
  hi = total * (g + 1) / G;
}

__device__ __forceinline__ int64_t lower_bound_u16(const uint16_t *a, int64_t lo, int64_t hi, uint32_t key,
                                                   int &probes) {
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    ++probes;
    if (gld(a + mid) < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Entries with label `label` among the row entries [a, e) (labels ascend): [lo, hi).
__device__ __forceinline__ void label_range(const uint16_t *lab, int64_t a, int64_t e, int32_t label, int64_t &lo,
                                            int64_t &hi, int &probes) {
  if (e - a <= 8) {          // short rows: one linear pass
    int64_t x = a;
    while (x < e && gld(lab + x) < (uint32_t)label) ++x;
    int64_t y = x;
    while (y < e && gld(lab + y) == (uint32_t)label) ++y;
    probes += (int)(y - a + (y < e));
    lo = x; hi = y;
    return;
  }
  lo = lower_bound_u16(lab, a, e, (uint32_t)label, probes);
  hi = lower_bound_u16(lab, lo, e, (uint32_t)label + 1, probes);
}

// Entries of vertex b with label `label` in orientation dir: [lo, hi).
__device__ __forceinline__ void seg_find(const DevGraph &g, int dir, int32_t b, int32_t label, int64_t &lo,
                                         int64_t &hi, int &probes) {
  // selects, not indexing: dir may differ between lanes, and indexing the
  // pointer arrays by a per-lane value loads the pointers from memory
  const int64_t *ptr = dir ? g.ptr[1] : g.ptr[0];
  const int64_t a = gld(ptr + b), e = gld(ptr + b + 1);
  label_range(dir ? g.lab[1] : g.lab[0], a, e, label, lo, hi, probes);
}

// Is c among the entries of vertex b with label `label` (orientation dir)?
__device__ __forceinline__ bool seg_has(const DevGraph &g, int dir, int32_t b, int32_t label, int32_t c,
                                        int &probes) {
  int64_t lo, hi;
  seg_find(g, dir, b, label, lo, hi, probes);
  const int32_t *idx = dir ? g.idx[1] : g.idx[0];
  int64_t x = lo, y = hi;
  while (x < y) {
    int64_t mid = (x + y) >> 1;
    ++probes;
    if (gld(idx + mid) < c) x = mid + 1; else y = mid;
  }
  return x < hi && gld(idx + x) == c;
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
