// Launchers and argument block of the query-evaluation kernels (query.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "gs_device.hpp"

namespace gs {

// Everything one iteration's kernels read, passed by value to each kernel.
struct IterArgs {
  DevGraph g;
  const DEntry *ent;
  int32_t E;               // entries (queries advancing this iteration)
  int32_t S;               // seeds to fill
  int32_t D;               // domains
  int32_t nclear;          // bitmaps to zero
  int32_t has_list;        // any LIST step among the entries
  int32_t has_tested;      // any entry whose candidates face a test (else no count and tile-offset passes)
  int32_t has_checks;      // any entry with exact checks (cycle-closing edges)
  int32_t has_factor;      // any entry at a count-only factor level (the lookup variant that multiplies)
  int32_t has_exact;       // any entry whose candidates face exact checks or self loops (else the count
                           // pass variant for bitmap filters only)
  int32_t grid;            // workgroups of the fixed-grid kernels
  int32_t wgrid;           // workgroups of the write pass (as many as are resident at once)
  int32_t wwaves;          // waves per workgroup of the write pass: 2, 4 or 8
  const DStep *steps;
  const uint64_t *const *filt;
  const DCheck *checks;
  const int32_t *ints;     // self-loop labels and copy columns
  const DConst *cconst;
  const DSeed *seeds;
  const DDomain *doms;
  int64_t *fcount;         // per domain: |F|
  uint64_t *const *clear;
  EState *es;
  IterScalars *it;
  int32_t **lvl_ptr;       // [q * kMaxLevels + level]: column c of a level at lvl_ptr + c * n (c >= 1 on CSR levels)
  int32_t **lvl_cptr;      // [q * kMaxLevels + level]: child offsets of a CSR level, else null
  int64_t *lvl_n;          // [q * kMaxLevels + level], -1 = overflow
  int64_t *qstats;         // [q * QS_N + counter]
  DArena *scratch;
  char *scratch_base;
  DArena *tree;
  char *tree_base;
  int64_t *blk_a, *blk_b, *blk_off_a, *blk_off_b;   // grid entries each
  // Run-wide flags, zeroed by the host before the first iteration of a run:
  // [RF_SCRATCH] a level's temporaries overflowed the scratch arena (every later
  // iteration of the run then does nothing); [RF_WRITE] the write pass met a tile
  // whose output positions leave its level (count and write passes disagree).
  // Null only for the standalone list and domain launches.
  int32_t *flags;
  // Standalone list launch only: the caller's output for the compacted ids (null:
  // the ids go to a scratch-arena buffer, it->list_buf).
  int32_t *list_out;
};
enum RunFlag { RF_SCRATCH = 0, RF_WRITE = 1, RF_N = 2 };

// Workgroups of the write pass, with `waves` waves each (2, 4 or 8), that one compute unit holds at once.
int expand_write_blocks_per_cu(int waves);

// ev: null, or 2 * KS_N events recorded around each launch (slot k: ev[2k], ev[2k+1]).
hipError_t launch_iteration(const IterArgs &A, hipStream_t s, hipEvent_t *ev = nullptr);
// After a run: the n seeds' bitmaps back to zero (the words their segments set, or the whole
// bitmap for a long segment); grid: workgroups at most.
hipError_t launch_unseed(const DevGraph &g, const DSeed *seeds, int32_t n, int grid, hipStream_t s);
hipError_t launch_list_only(const IterArgs &A, hipStream_t s);
hipError_t launch_domain_only(const IterArgs &A, hipStream_t s);

// The standalone list launch over caller memory: every table it reads sits in one
// caller-provided workspace (NoAllocLayout), written by a set-up kernel from the
// by-value argument block, so the sequence allocates nothing and copies nothing
// from the host. The count (or -1 when the workspace's arena overflowed) goes to
// a device int64.
constexpr int kNoAllocMaxBitmaps = 64;
constexpr int kNoAllocMaxGrid = 8192;
struct NoAllocInit {
  const uint64_t *bm[kNoAllocMaxBitmaps];
  int32_t k;
};
struct NoAllocLayout {   // byte offsets inside the workspace
  static constexpr size_t arena = 0, it = 256, es = 1024, step = 2048, ent = 2304, filt = 2560,
                          lvl_ptr = 3584, lvl_n = 4096, qstats = 4608, heap = 8192, heap_bytes = 8192,
                          blk = 16384, bytes = blk + 4 * 8 * (size_t)kNoAllocMaxGrid;
};
hipError_t launch_list_noalloc(const DevGraph &g, const NoAllocInit &init, char *ws, int grid, int32_t *out,
                               int64_t *count, hipStream_t s);
// Tree levels come in two forms: a parent column (column 0, one entry per
// node), or, for levels whose candidates face no test, child offsets per
// parent (cptr, prev_n + 1 entries; the children of parent p are
// [cptr[p], cptr[p + 1])) and no column 0. cptr = null selects the first form.
hipError_t launch_prune_mark(const int32_t *par, const int32_t *cptr, int64_t prev_n, int64_t n, const uint8_t *alive,
                             uint8_t *alive_parent, hipStream_t s);
hipError_t launch_prune_count(const uint8_t *alive, int64_t n, int64_t *blk, int grid, hipStream_t s);
hipError_t launch_prune_write(const int32_t *L, const int32_t *cptr, int64_t prev_n, int64_t n, int ncols,
                              const uint8_t *alive, const int64_t *blkoff,
                              const int32_t *parent_newidx, int32_t *newidx, int32_t *out, int64_t n_out, int grid,
                              hipStream_t s);
// Sum (mod 2^64) and XOR of the row hashes of every leaf into out[0], out[1]
// (which the caller zeroes).
hipError_t launch_row_digest(int32_t *const *lvl_ptr, int32_t *const *lvl_cptr, const int64_t *lvl_n, int k,
                             const int32_t *var_rank, int64_t n, uint64_t *out, hipStream_t s);
hipError_t launch_enumerate(int32_t *const *lvl_ptr, int32_t *const *lvl_cptr, const int64_t *lvl_n, int k,
                            const int32_t *var_rank,
                            int64_t first, int64_t n, int32_t *rows, hipStream_t s);

}  // namespace gs
