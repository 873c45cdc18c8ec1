// Light-weight sparse matrix builder (Section 6.2): the whole dataset in both
// orientations, duplicates removed, each row (column) sorted by (label, id),
// plus the label-existence vectors of Eq. (4)/(5) for every label.
//
// Keys: orientation 0 sorts (s, p, o), orientation 1 sorts (o, p, s). A key is
// held as hi = (a << pbits) | (p - 1) and lo = b, and sorted by (hi, lo) with a
// stable least-significant-digit radix sort, 8-bit digits: first the digits
// of lo, then those of hi.
#include "kernels_common.hpp"
#include "lspm.hpp"

namespace gs {

__global__ __launch_bounds__(kBlock) void k_make_keys(const int32_t *trip, int64_t m, int64_t n, int32_t P,
                                                      int orient, int pbits, uint64_t *hi, uint32_t *lo,
                                                      int32_t *err) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    int32_t s = trip[3 * i], p = trip[3 * i + 1], o = trip[3 * i + 2];
    if (s < 0 || s >= n || o < 0 || o >= n || p < 1 || p > P) {
      atomicOr(err, 1);
      s = 0; o = 0; p = 1;
    }
    const int32_t a = orient ? o : s, b = orient ? s : o;
    hi[i] = ((uint64_t)(uint32_t)a << pbits) | (uint64_t)(uint32_t)(p - 1);
    lo[i] = (uint32_t)b;
  }
}

__device__ __forceinline__ uint32_t digit_of(uint64_t h, uint32_t l, int shift, int use_hi) {
  return use_hi ? (uint32_t)(h >> shift) & 255u : (l >> shift) & 255u;
}

// Per-block digit histogram over the block's contiguous chunk; hist is digit-major.
__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t *hi, const uint32_t *lo, int64_t m,
                                                       int shift, int use_hi, int64_t chunk, uint32_t *hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t b = blockIdx.x * chunk, e = min(m, b + chunk);
  for (int64_t i = b + threadIdx.x; i < e; i += kBlock)
    atomicAdd(&h[use_hi ? (uint32_t)(hi[i] >> shift) & 255u : (lo[i] >> shift) & 255u], 1u);
  __syncthreads();
  hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Multi-workgroup exclusive scan of L uint32 counts into int64 offsets, in three
// launches: chunk sums (one chunk per workgroup, coalesced), a one-workgroup scan
// of the chunk sums, then each chunk rescanned from its offset.
__global__ __launch_bounds__(kBlock) void k_scan_parts(const uint32_t *in, int64_t L, int64_t *parts) {
  __shared__ int64_t lds[kWaves];
  int64_t b, e;
  block_share(L, b, e);
  int64_t v = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += kBlock) v += in[i];
  v = block_sum_i64(v, lds);
  if (threadIdx.x == 0) parts[blockIdx.x] = v;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(const uint32_t *in, int64_t L, const int64_t *parts,
                                                       int64_t *out) {
  __shared__ int64_t lds[kWaves];
  int64_t b, e;
  block_share(L, b, e);
  int64_t carry = parts[blockIdx.x];
  for (int64_t c0 = b; c0 < e; c0 += kBlock) {
    const int64_t i = c0 + threadIdx.x;
    const int64_t v = i < e ? (int64_t)in[i] : 0;
    int64_t tot;
    const int64_t x = block_excl_scan_i64(v, tot, lds);
    if (i < e) out[i] = carry + x;
    carry += tot;
  }
}

// One workgroup: exclusive scan of L int64 values (in place allowed); *total gets the sum.
__global__ __launch_bounds__(1024) void k_scan_i64(const int64_t *in, int64_t L, int64_t *out, int64_t *total) {
  __shared__ int64_t lds[1024];
  int64_t t = wg_scan(L, [&](int64_t i) { return in[i]; }, [&](int64_t i, int64_t v) { out[i] = v; }, lds);
  if (threadIdx.x == 0 && total) *total = t;
}

// Stable scatter: rounds of 256 consecutive keys; within a wave the rank of a
// key among equal digits comes from eight ballots (lanes holding the same
// digit), across the four waves from per-digit counts in LDS.
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint64_t *hi_in, const uint32_t *lo_in,
                                                          uint64_t *hi_out, uint32_t *lo_out, int64_t m,
                                                          int shift, int use_hi, int64_t chunk,
                                                          const int64_t *off) {
  __shared__ int64_t base[256], obase[256];
  __shared__ uint32_t wcnt[kWaves][256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  base[t] = off[(int64_t)t * gridDim.x + blockIdx.x];
  const int64_t b = blockIdx.x * chunk, e = min(m, b + chunk);
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int64_t r = b; r < e; r += kBlock) {
    const int64_t i = r + t;
    const bool valid = i < e;
    uint64_t h = 0;
    uint32_t l = 0, d = 0;
    if (valid) { h = hi_in[i]; l = lo_in[i]; d = digit_of(h, l, shift, use_hi); }
#pragma unroll
    for (int k = 0; k < kWaves; ++k) wcnt[k][t] = 0;
    __syncthreads();
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint64_t bb = __ballot((d >> k) & 1u);
      peers &= ((d >> k) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = __popcll(peers & lt);
    if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    {   // thread t owns digit t
      uint32_t run = 0;
#pragma unroll
      for (int k = 0; k < kWaves; ++k) { uint32_t c = wcnt[k][t]; wcnt[k][t] = run; run += c; }
      obase[t] = base[t];
      base[t] += run;
    }
    __syncthreads();
    if (valid) {
      const int64_t pos = obase[d] + wcnt[w][d] + rank;
      hi_out[pos] = h;
      lo_out[pos] = l;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ bool is_first(const uint64_t *hi, const uint32_t *lo, int64_t i) {
  return i == 0 || hi[i] != hi[i - 1] || lo[i] != lo[i - 1];
}

__global__ __launch_bounds__(kBlock) void k_uniq_count(const uint64_t *hi, const uint32_t *lo, int64_t m,
                                                       int64_t *blk) {
  __shared__ int64_t lds[kWaves];
  int64_t b, e;
  block_share(m, b, e);
  int64_t c = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += kBlock) c += is_first(hi, lo, i);
  c = block_sum_i64(c, lds);
  if (threadIdx.x == 0) blk[blockIdx.x] = c;
}

// Keep the first of every run of equal keys, in order; split into id, label and row.
__global__ __launch_bounds__(kBlock) void k_uniq_write(const uint64_t *hi, const uint32_t *lo, int64_t m,
                                                       const int64_t *blkoff, int pbits, int32_t *idx,
                                                       uint16_t *lab, int32_t *row) {
  __shared__ int lds[kWaves];
  int64_t b, e;
  block_share(m, b, e);
  int64_t run = blkoff[blockIdx.x];
  const uint64_t pmask = (pbits >= 64) ? ~0ull : ((1ull << pbits) - 1ull);
  for (int64_t r = b; r < e; r += kBlock) {
    const int64_t i = r + threadIdx.x;
    const bool f = i < e && is_first(hi, lo, i);
    int tot;
    const int pos = block_excl_flag(f, tot, lds);
    if (f) {
      const uint64_t h = hi[i];
      idx[run + pos] = (int32_t)lo[i];
      lab[run + pos] = (uint16_t)(h & pmask);
      row[run + pos] = (int32_t)(h >> pbits);
    }
    run += tot;
  }
}

// ptr[x] = first entry whose row is >= x, for x in [0, n].
__global__ __launch_bounds__(kBlock) void k_row_ptr(const int32_t *row, int64_t m, int64_t n, int64_t *ptr) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x <= n; x += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if ((int64_t)row[mid] < x) lo = mid + 1; else hi = mid;
    }
    ptr[x] = lo;
  }
}

// Eq. (4)/(5): bit r of bitmap p is set iff row r holds label p (one atomic per (row, label) run).
__global__ __launch_bounds__(kBlock) void k_label_bitmaps(const int32_t *row, const uint16_t *lab, int64_t m,
                                                          int64_t words, uint64_t *bm) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = row[j];
    const uint16_t p = lab[j];
    if (j == 0 || row[j - 1] != r || lab[j - 1] != p)
      atomicOr((unsigned long long *)&bm[(int64_t)p * words + (r >> 6)], 1ull << (r & 63));
  }
}

__global__ __launch_bounds__(kBlock) void k_label_hist(const uint16_t *lab, int64_t m, int32_t P, int64_t *nnz) {
  extern __shared__ unsigned long long hs[];
  const bool local = P <= 4096;
  if (local)
    for (int i = threadIdx.x; i < P; i += kBlock) hs[i] = 0;
  __syncthreads();
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
    if (local) atomicAdd(&hs[lab[j]], 1ull);
    else atomicAdd((unsigned long long *)&nnz[lab[j]], 1ull);
  }
  __syncthreads();
  if (local)
    for (int i = threadIdx.x; i < P; i += kBlock)
      if (hs[i]) atomicAdd((unsigned long long *)&nnz[i], hs[i]);
}

// One block per label: popcount of its bitmap.
__global__ __launch_bounds__(kBlock) void k_bitmap_popcount(const uint64_t *bm, int64_t words, int32_t P,
                                                            int64_t *out) {
  __shared__ int64_t lds[kWaves];
  for (int p = blockIdx.x; p < P; p += gridDim.x) {
    int64_t c = 0;
    for (int64_t w = threadIdx.x; w < words; w += kBlock) c += __popcll(bm[(int64_t)p * words + w]);
    c = block_sum_i64(c, lds);
    if (threadIdx.x == 0) out[p] = c;
  }
}

__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------- host side
static int grid_for(int64_t n, int cap) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

hipError_t fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 4096)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t scan_i64(const int64_t *in, int64_t L, int64_t *out, int64_t *total, hipStream_t s) {
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, s, in, L, out, total);
  return hipGetLastError();
}

// Sort (hi, lo) pairs of length m; the result ends in (hi0, lo0). Temporaries
// hi1/lo1 of the same size; hist of 256 * G uint32 and off of 256 * G int64.
// parts: at least min(G, 256) int64 of scratch for the offset scan.
static hipError_t radix_sort(uint64_t *hi0, uint32_t *lo0, uint64_t *hi1, uint32_t *lo1, int64_t m, int lo_bits,
                             int hi_bits, uint32_t *hist, int64_t *off, int64_t *parts, int G, hipStream_t s) {
  const int np = G < 256 ? G : 256;
  if (m <= 1) return hipSuccess;
  const int64_t chunk = (m + G - 1) / G;
  bool swapped = false;
  for (int pass = 0; pass < 2; ++pass) {
    const int bits = pass == 0 ? lo_bits : hi_bits;
    for (int shift = 0; shift < bits; shift += 8) {
      uint64_t *hs = swapped ? hi1 : hi0, *hd = swapped ? hi0 : hi1;
      uint32_t *ls = swapped ? lo1 : lo0, *ld = swapped ? lo0 : lo1;
      hipLaunchKernelGGL(k_radix_hist, dim3(G), dim3(kBlock), 0, s, hs, ls, m, shift, pass, chunk, hist);
      hipLaunchKernelGGL(k_scan_parts, dim3(np), dim3(kBlock), 0, s, hist, (int64_t)256 * G, parts);
      hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, s, parts, (int64_t)np, parts, nullptr);
      hipLaunchKernelGGL(k_scan_apply, dim3(np), dim3(kBlock), 0, s, hist, (int64_t)256 * G, parts, off);
      hipLaunchKernelGGL(k_radix_scatter, dim3(G), dim3(kBlock), 0, s, hs, ls, hd, ld, m, shift, pass, chunk,
                         (const int64_t *)off);
      swapped = !swapped;
    }
  }
  if (swapped) {
    hipError_t e = hipMemcpyAsync(hi0, hi1, sizeof(uint64_t) * m, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(lo0, lo1, sizeof(uint32_t) * m, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

static int bits_for(uint64_t maxval) {   // bits to hold values in [0, maxval]
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
}

__global__ __launch_bounds__(kBlock) void k_narrow_offsets(const int64_t *in, int32_t *out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (int32_t)in[i];
}
__global__ __launch_bounds__(kBlock) void k_narrow_labels(const uint16_t *in, uint8_t *out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (uint8_t)in[i];
}
hipError_t narrow_offsets(const int64_t *in, int32_t *out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_narrow_offsets, dim3(grid_for(n, 8192)), dim3(kBlock), 0, s, in, out, n);
  return hipGetLastError();
}
hipError_t narrow_labels(const uint16_t *in, uint8_t *out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_narrow_labels, dim3(grid_for(n, 8192)), dim3(kBlock), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t lspm_build_orientation(const LspmBuildArgs &a, int orient, LspmOut &out, int64_t *m_out) {
  hipStream_t s = a.stream;
  const int G = a.grid;
  const int pbits = bits_for((uint64_t)(a.P - 1));
  const int abits = bits_for((uint64_t)(a.n - 1));
  hipLaunchKernelGGL(k_make_keys, dim3(grid_for(a.m, 4096)), dim3(kBlock), 0, s, a.triples, a.m, a.n, a.P, orient,
                     pbits, a.hi0, a.lo0, a.err);
  hipError_t e = radix_sort(a.hi0, a.lo0, a.hi1, a.lo1, a.m, abits, abits + pbits, a.hist, a.off, a.blk, G, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_uniq_count, dim3(G), dim3(kBlock), 0, s, a.hi0, a.lo0, a.m, a.blk);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, s, a.blk, (int64_t)G, a.blk, a.total);
  int64_t m2 = 0;
  e = hipMemcpyAsync(&m2, a.total, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  *m_out = m2;
  // the caller sizes the outputs from m2
  e = a.alloc_out(a.alloc_ctx, orient, m2, out);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_uniq_write, dim3(G), dim3(kBlock), 0, s, a.hi0, a.lo0, a.m, (const int64_t *)a.blk, pbits,
                     out.idx, out.lab, a.row);
  hipLaunchKernelGGL(k_row_ptr, dim3(grid_for(a.n + 1, 8192)), dim3(kBlock), 0, s, (const int32_t *)a.row, m2, a.n,
                     out.ptr);
  e = fill_u64(out.bm, (int64_t)a.P * out.words, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_label_bitmaps, dim3(grid_for(m2, 8192)), dim3(kBlock), 0, s, (const int32_t *)a.row,
                     (const uint16_t *)out.lab, m2, out.words, out.bm);
  hipLaunchKernelGGL(k_bitmap_popcount, dim3(a.P < 4096 ? a.P : 4096), dim3(kBlock), 0, s,
                     (const uint64_t *)out.bm, out.words, a.P, out.holders);
  if (orient == 0) {
    const size_t sh = a.P <= 4096 ? sizeof(unsigned long long) * a.P : 0;
    hipLaunchKernelGGL(k_label_hist, dim3(grid_for(m2, 1024)), dim3(kBlock), sh, s, (const uint16_t *)out.lab, m2,
                       a.P, a.nnz);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ query-driven load
// Step 1 of Section 6.2.1 / 6.2.2: only the triples whose predicate the query
// names. Per-workgroup counts over contiguous chunks, one scan of the counts,
// then each chunk writes its kept triples in input order from its offset.
// keep: bit p for the 1-based predicate p. Ids and labels are range-checked.
__device__ __forceinline__ bool triple_ok(int32_t s, int32_t p, int32_t o, int64_t n, int32_t P) {
  return s >= 0 && s < n && o >= 0 && o < n && p >= 1 && p <= P;
}

__global__ __launch_bounds__(kBlock) void k_filter_count(const int32_t *trip, int64_t m, int64_t n, int32_t P,
                                                         const uint32_t *keep, int64_t *parts, int32_t *err) {
  __shared__ int64_t lds[kWaves];
  int64_t b, e;
  block_share(m, b, e);
  int64_t c = 0;
  bool bad = false;
  for (int64_t i = b + threadIdx.x; i < e; i += kBlock) {
    const int32_t s = trip[3 * i], p = trip[3 * i + 1], o = trip[3 * i + 2];
    if (!triple_ok(s, p, o, n, P)) { bad = true; continue; }
    c += (keep[p >> 5] >> (p & 31)) & 1u;
  }
  if (bad) atomicOr(err, 1);
  c = block_sum_i64(c, lds);
  if (threadIdx.x == 0) parts[blockIdx.x] = c;
}

__global__ __launch_bounds__(kBlock) void k_filter_write(const int32_t *trip, int64_t m, int64_t n, int32_t P,
                                                         const uint32_t *keep, const int64_t *parts, int32_t *out) {
  __shared__ int64_t lds[kWaves];
  int64_t b, e;
  block_share(m, b, e);
  int64_t run = parts[blockIdx.x];
  for (int64_t c0 = b; c0 < e; c0 += kBlock) {
    const int64_t i = c0 + threadIdx.x;
    int32_t s = 0, p = 0, o = 0;
    bool k = false;
    if (i < e) {
      s = trip[3 * i];
      p = trip[3 * i + 1];
      o = trip[3 * i + 2];
      k = triple_ok(s, p, o, n, P) && ((keep[p >> 5] >> (p & 31)) & 1u);
    }
    int64_t tot;
    const int64_t x = block_excl_scan_i64(k ? 1 : 0, tot, lds);
    if (k) {
      int32_t *w = out + 3 * (run + x);
      w[0] = s;
      w[1] = p;
      w[2] = o;
    }
    run += tot;
  }
}

hipError_t filter_triples(const int32_t *trip, int64_t m, int64_t n, int32_t P, const uint32_t *keep,
                          int64_t *parts, int G, int64_t *total, int32_t *err, int32_t *out_or_null,
                          hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (!out_or_null) {   // counting pass: parts scanned in place, the kept count into *total
    hipLaunchKernelGGL(k_filter_count, dim3(G), dim3(kBlock), 0, s, trip, m, n, P, keep, parts, err);
    hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, s, parts, (int64_t)G, parts, total);
  } else {
    hipLaunchKernelGGL(k_filter_write, dim3(G), dim3(kBlock), 0, s, trip, m, n, P, keep, (const int64_t *)parts,
                       out_or_null);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ per-query reduction
// One part of the reduced matrix (Section 6.2.1 step 3-4, Section 6.2.2 steps
// 3-5; Ex. 6.3, 6.4) from the resident one: the entries of each row (column)
// whose label is kept, rows left empty dropped. Rows are sorted by (label, id),
// so a row's kept entries are the sub-segments of the kept labels, which are
// taken in ascending order. klab: kept 0-based labels, ascending (at most 64).
template <int LB, int OB>
__global__ __launch_bounds__(kBlock) void k_red_count(const DevGraph g, int dir, const int32_t *klab, int nk,
                                                      uint32_t *cnt, uint32_t *nonempty) {
  __shared__ int32_t sk[64];
  if (threadIdx.x < nk) sk[threadIdx.x] = klab[threadIdx.x];
  __syncthreads();
  const void *ptr = dir ? g.ptr[1] : g.ptr[0];
  const void *lab = dir ? g.lab[1] : g.lab[0];
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < g.n; i += (int64_t)gridDim.x * kBlock) {
    const OffT<OB> a = off_w<OB>(ptr, i), e = off_w<OB>(ptr, i + 1);
    int64_t c = 0;
    for (int k = 0; k < nk && a < e; ++k) {
      OffT<OB> lo, hi;
      int unused = 0;
      label_range_w<LB>(lab, a, e, sk[k], lo, hi, unused);
      c += hi - lo;
    }
    cnt[i] = (uint32_t)c;
    nonempty[i] = c > 0 ? 1u : 0u;
  }
}

template <int LB, int OB>
__global__ __launch_bounds__(kBlock) void k_red_write(const DevGraph g, int dir, const int32_t *klab, int nk,
                                                      const uint32_t *cnt, const int64_t *pos, const int64_t *M,
                                                      int64_t *P, int32_t *val, int32_t *idx) {
  __shared__ int32_t sk[64];
  if (threadIdx.x < nk) sk[threadIdx.x] = klab[threadIdx.x];
  __syncthreads();
  const void *ptr = dir ? g.ptr[1] : g.ptr[0];
  const void *lab = dir ? g.lab[1] : g.lab[0];
  const int32_t *ids = dir ? g.idx[1] : g.idx[0];
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < g.n; i += (int64_t)gridDim.x * kBlock) {
    if (cnt[i] == 0) continue;
    int64_t w = pos[i];
    P[M[i]] = w;
    const OffT<OB> a = off_w<OB>(ptr, i), e = off_w<OB>(ptr, i + 1);
    for (int k = 0; k < nk; ++k) {
      OffT<OB> lo, hi;
      int unused = 0;
      label_range_w<LB>(lab, a, e, sk[k], lo, hi, unused);
      for (OffT<OB> x = lo; x < hi; ++x, ++w) {
        val[w] = sk[k] + 1;
        idx[w] = ids[x];
      }
    }
  }
}

// Exclusive scan of L uint32 values into out[0, L) and the total into out[L].
static hipError_t scan_u32(const uint32_t *in, int64_t L, int64_t *out, int64_t *parts, hipStream_t s) {
  const int np = 256;
  hipLaunchKernelGGL(k_scan_parts, dim3(np), dim3(kBlock), 0, s, in, L, parts);
  hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, s, parts, (int64_t)np, parts, out + L);
  hipLaunchKernelGGL(k_scan_apply, dim3(np), dim3(kBlock), 0, s, in, L, (const int64_t *)parts, out);
  return hipGetLastError();
}

template <int LB, int OB>
static void launch_red_count(int G, hipStream_t s, const DevGraph &g, int dir, const int32_t *klab, int nk,
                             uint32_t *cnt, uint32_t *nonempty) {
  hipLaunchKernelGGL((k_red_count<LB, OB>), dim3(G), dim3(kBlock), 0, s, g, dir, klab, nk, cnt, nonempty);
}

template <int LB, int OB>
static void launch_red_write(int G, hipStream_t s, const DevGraph &g, int dir, const int32_t *klab, int nk,
                             const uint32_t *cnt, const int64_t *pos, const int64_t *M, int64_t *P, int32_t *val,
                             int32_t *idx) {
  hipLaunchKernelGGL((k_red_write<LB, OB>), dim3(G), dim3(kBlock), 0, s, g, dir, klab, nk, cnt, pos, M, P, val, idx);
}

hipError_t reduce_count(const DevGraph &g, int dir, const int32_t *klab, int nk, uint32_t *cnt, uint32_t *nonempty,
                        int64_t *pos, int64_t *M, int64_t *parts, hipStream_t s) {
  const int G = grid_for(g.n, 4096);
  GS_WITH_WIDTHS(g, (launch_red_count<LB, OB>(G, s, g, dir, klab, nk, cnt, nonempty)));
  hipError_t e = scan_u32(cnt, g.n, pos, parts, s);
  if (e != hipSuccess) return e;
  return scan_u32(nonempty, g.n, M, parts, s);
}

hipError_t reduce_write(const DevGraph &g, int dir, const int32_t *klab, int nk, const uint32_t *cnt,
                        const int64_t *pos, const int64_t *M, int64_t *P, int32_t *val, int32_t *idx, hipStream_t s) {
  const int G = grid_for(g.n, 4096);
  GS_WITH_WIDTHS(g, (launch_red_write<LB, OB>(G, s, g, dir, klab, nk, cnt, pos, M, P, val, idx)));
  return hipGetLastError();
}

}  // namespace gs
