// Device-side data layout shared by the engine's host code and its kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace gs {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kTileNodes = 1024;     // tree nodes per tile (lookup, frontier, nz pass)
constexpr int kTileWork = 512;       // candidate entries per tile (expansion; one wave's work)
constexpr int kTileWords = 256;      // bitmap words per tile (lists, domains)
constexpr int kMaxLevels = 64;

// The light-weight sparse matrix in both orientations (Section 6.2).
// Orientation 0 (row-wise): for vertex b, entries [ptr[0][b], ptr[0][b+1]) hold
// the objects o of triples (b, p, o), sorted by (p, o). Orientation 1
// (column-wise): entries [ptr[1][b], ptr[1][b+1]) hold the subjects s of
// (s, p, b), sorted by (p, s). Labels are stored 0-based (p - 1).
// bm[d] + p * words: label-existence vector of Eq. (4) (d = 0: rows holding p)
// or Eq. (5) (d = 1: columns holding p), one bit per vertex.
// Storage widths follow the sizes: labels are uint8 when P <= 256 (lab8) and
// uint16 otherwise; row offsets are int32 when M < 2^31 (off32) and int64
// otherwise (or when wide offsets are asked for).
struct DevGraph {
  int64_t n = 0, m = 0, words = 0;
  int32_t P = 0;
  int8_t lab8 = 0, off32 = 0, pad0 = 0, pad1 = 0;
  const void *ptr[2] = {nullptr, nullptr};
  const int32_t *idx[2] = {nullptr, nullptr};
  const void *lab[2] = {nullptr, nullptr};
  const uint64_t *bm[2] = {nullptr, nullptr};
};

// One tree level of one query: how its candidates are generated and tested.
struct DStep {
  int32_t kind;        // STEP_SEG / STEP_SEG_CONST / STEP_LIST
  int32_t src;         // SEG: column of the parent binding in the previous level; SEG_CONST: constant
  int32_t label, dir;  // label 0-based; dir: orientation of the segment read from the parent binding
  int32_t filt0, nfilt;
  int32_t chk0, nchk;
  int32_t self0, nself;
  int32_t copy0, ncopy;
  int32_t ncols_out;   // columns written: parent, vid, carried bindings; 0 = count only
  int32_t ncols_prev;
  int32_t cc0, ncc;    // constant-constant checks (level 0 only)
  int32_t dom0, ndom;  // domains computed before this level
  int32_t list_nfilt;  // LIST: filters ANDed into the list (the first list_nfilt of filt0..)
  int32_t nfactor;     // count-only factor level: further independent leaves, as DCheck records at
                       // chk0.. (column, label, dir), whose segment lengths multiply this one's
};

struct DCheck { int32_t col, label, dir, pad; };   // exact check: c in seg(prev[col], label, dir)
struct DConst { int32_t a, label, b, pad; };       // (a, label, b) must be a triple

struct DSeed { uint64_t *bm; int32_t c, label, dir, q; };

struct DDomain {
  uint64_t *F;         // frontier bitmap: distinct bindings of the bound end
  uint64_t *D;         // result bitmap
  int32_t col;         // column of the bound binding in the previous level
  int32_t label, dir;  // push reads seg(b, label, dir); pull reads seg(c, label, 1 - dir)
  int32_t filt0, nfilt;// pull candidate mask: AND of these bitmaps
  int32_t mode;        // forced mode (0 auto, 1 push, 2 pull)
  int32_t q;
  float deg_push, deg_pull;   // average segment lengths for the cost estimate
  float mask_est, theta;      // estimated pull candidates, switch threshold
  int32_t pad;
};

// A step whose candidates face no test: every candidate entry becomes a child.
__host__ __device__ inline bool step_test_free(const DStep &S) {
  return S.nfilt == S.list_nfilt && S.nchk == 0 && S.nself == 0;
}

// Host-built per-iteration work list entry: query q produces level `level`
// using step program `step`.
struct DEntry { int32_t q, level, step, dom0, ndom, pad; };

// Device-filled per-iteration state of one entry.
struct EState {
  const int32_t *prev;   // previous level's columns: column c at prev + c * prev_n
  int64_t prev_n;        // nodes of the previous level (1 for the virtual root)
  int64_t node0;         // first global node index of this entry
  int64_t node_tile0;    // first node tile
  int64_t nz, nz_base;   // nodes with a non-empty candidate segment; global position of the first
  int64_t w, w_base;     // candidate entries; global position of the first
  int64_t w_tile0;       // first work tile
  int64_t cnt, out_base; // valid candidates; global position of the first
  int32_t *out;          // produced level (columns at out + c * cnt)
  int64_t list_words;    // LIST: bitmap words to scan
  int64_t list_tile0;
  int64_t list_n, list_base;
  int32_t *list;
  const int32_t *copies; // write pass: previous-level columns copied into the new level
  int32_t ncopy;
  int32_t wflags;        // write pass: EW_FREE | EW_LIST
  int32_t *cptr;         // levels without tests: child offsets per parent (prev_n + 1), no parent column
};
enum { EW_FREE = 1, EW_LIST = 2 };

// One work tile of the expansion (kTileWork consecutive candidate entries of
// one entry), written by the non-empty-node pass for the node its first entry
// belongs to, so that any workgroup can take any tile.
struct DTile {
  int64_t k0;    // index (in the non-empty node arrays) of the node holding the first entry
  int64_t a;     // entry-local position of the first entry
  int64_t out;   // entry-local output position of the tile's first child (tile-offset pass)
  int32_t e;     // entry; -1 on the sentinel after the last tile
  int32_t n;     // entries in the tile
  int32_t cnt;   // valid entries (count pass; tested levels)
  int32_t pad;
};

// Per-iteration scalars written by the scan kernels.
struct IterScalars {
  int64_t n_entries;
  int32_t abort, pad;
  int64_t node_tiles, work_tiles, list_tiles;
  int64_t nodes_total, nz_total, w_total, cnt_total, list_total;
  int64_t *lo;             // per node: segment start
  int64_t *len;            // per node: segment length
  int32_t *nz_node;        // compacted non-empty nodes: local node index
  int64_t *nz_lo, *nz_woff;// their segment start and entry-local work offset
  // levels with exact checks: bounds of the first tested segment of each node (the
  // check the count pass makes first), per node and per non-empty node
  int64_t *chk_lo, *chk_hi, *nz_chk_lo, *nz_chk_hi;
  uint32_t *valid;         // expansion validity bits, kTileWork bits per work tile
  DTile *tiles;            // work_tiles + 1 records (the last one a sentinel)
  int32_t *list_buf;
  // work counters of the expansion count pass (for algorithmic-byte accounting)
  int64_t ftests;          // bitmap filter words tested
  int64_t ctests;          // exact checks started (each reads one parent binding)
  int64_t probes;          // label / id entries touched by binary searches
  int64_t w_tested;        // candidate entries of levels that test their candidates
  // work counters of the node pass
  int64_t lk_labels;       // label entries read while locating label sub-segments
  int64_t lk_lookups;      // segment lookups (offset pairs read)
};

// Kernel slots of one iteration, for optional event timing.
enum KSlot { KS_SETUP = 0, KS_CLEAR, KS_SEED, KS_LIST_COUNT, KS_LIST_SCAN, KS_LIST_WRITE, KS_DOM_FRONTIER,
             KS_DOM_PUSH, KS_DOM_PULL, KS_LOOKUP, KS_SCAN_NODES, KS_NZ_WRITE, KS_EXPAND_COUNT, KS_SCAN_EXPAND,
             KS_TILE_OFFSETS, KS_EXPAND_WRITE, KS_N };

// Bump allocator over one device region; top and cap in bytes.
struct DArena {
  uint64_t top, cap;
  int32_t overflow, pad;
};

// Per-query counters (int64 each). QS_LABEL: label entries read while locating
// label sub-segments; QS_LOOKUP: segment lookups (offset pairs read); QS_BMWORDS:
// bitmap words read or written by the candidate filters, seeds and domains.
enum QStat { QS_EXPAND = 0, QS_SEED, QS_PUSH, QS_PULL, QS_PROBE, QS_DOMPUSH, QS_DOMPULL, QS_OVERFLOW, QS_LABEL,
             QS_LOOKUP, QS_BMWORDS, QS_N };

}  // namespace gs
