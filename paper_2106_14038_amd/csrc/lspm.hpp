// Launchers of the light-weight sparse matrix builder (lspm.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

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

}  // namespace gs
