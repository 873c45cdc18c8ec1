// Launchers of the light-weight sparse matrix builder (lspm.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gs_device.hpp"

namespace gs {

struct LspmOut {            // one orientation, allocated by the caller once the distinct count is known
  int64_t *ptr = nullptr;   // n + 1
  int32_t *idx = nullptr;   // m
  uint16_t *lab = nullptr;  // m (0-based labels)
  uint64_t *bm = nullptr;   // P * words label-existence bitmaps
  int64_t *holders = nullptr;  // P: vertices holding each label in this orientation
  int64_t words = 0;
};

struct LspmBuildArgs {
  const int32_t *triples;   // device, m * 3
  int64_t m, n;
  int32_t P;
  int grid;
  hipStream_t stream;
  uint64_t *hi0, *hi1;      // m each
  uint32_t *lo0, *lo1;      // m each
  int32_t *row;             // m
  uint32_t *hist;           // 256 * grid
  int64_t *off;             // 256 * grid
  int64_t *blk;             // grid
  int64_t *total;           // 1
  int32_t *err;             // 1, set to 1 on an out-of-range triple
  int64_t *nnz;             // P, zeroed by the caller, filled by orientation 0
  hipError_t (*alloc_out)(void *ctx, int orient, int64_t m_distinct, LspmOut &out);
  void *alloc_ctx;
};

hipError_t lspm_build_orientation(const LspmBuildArgs &a, int orient, LspmOut &out, int64_t *m_out);
hipError_t fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s);
// Copies into the narrower stored widths (values known to fit): row offsets
// int64 -> int32, labels uint16 -> uint8.
hipError_t narrow_offsets(const int64_t *in, int32_t *out, int64_t n, hipStream_t s);
hipError_t narrow_labels(const uint16_t *in, uint8_t *out, int64_t n, hipStream_t s);
hipError_t scan_i64(const int64_t *in, int64_t L, int64_t *out, int64_t *total, hipStream_t s);

// Triples whose predicate has its bit set in keep, in input order. With out NULL: counts per
// workgroup of a grid of G into parts (G int64, scanned in place) and the kept count into
// *total, with *err set on a triple out of range; with out: writes the kept triples.
hipError_t filter_triples(const int32_t *trip, int64_t m, int64_t n, int32_t P, const uint32_t *keep,
                          int64_t *parts, int G, int64_t *total, int32_t *err, int32_t *out_or_null,
                          hipStream_t s);

// Per-query reduced matrix, one part (dir 0 row-wise, 1 column-wise) over the kept 0-based labels
// klab[0, nk) (device, ascending, nk <= 64): counts and non-empty flags per row, their exclusive
// scans pos and M (n + 1 int64 each, the totals at index n; parts: 256 int64 of scratch), then
// the kept rows' offsets P[M[i]] and their entries (val 1-based labels, idx the other endpoint).
hipError_t reduce_count(const DevGraph &g, int dir, const int32_t *klab, int nk, uint32_t *cnt, uint32_t *nonempty,
                        int64_t *pos, int64_t *M, int64_t *parts, hipStream_t s);
hipError_t reduce_write(const DevGraph &g, int dir, const int32_t *klab, int nk, const uint32_t *cnt,
                        const int64_t *pos, const int64_t *M, int64_t *P, int32_t *val, int32_t *idx, hipStream_t s);

}  // namespace gs
