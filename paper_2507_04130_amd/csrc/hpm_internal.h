// hpm_internal.h -- types shared by the HIP kernels and the host runtime of libhpm.
//
// Nothing here is part of the public ABI (include/hpm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpm {

constexpr int kMaxK = 16;
constexpr int kMaxCols = 4;
constexpr int kBlock = 256;           // threads per block (4 wave64s)
constexpr int kWaves = kBlock / 64;
constexpr int kScanItems = 8;         // arcs per thread per tile in the arc scan
constexpr int kScanTile = kBlock * kScanItems;
constexpr int kExpandItems = 4;       // candidates per thread per tile in the extension
constexpr int kExpandTile = kBlock * kExpandItems;
constexpr int kPivotItems = 4;        // rows per thread in the pivot/length pass
constexpr int kPivotTile = kBlock * kPivotItems;
constexpr int kLdsRowInts = 1024;     // partial-mapping entries staged in LDS per tile
constexpr int kTilePool = 2048;       // LDS entries for staged adjacency lists per block
constexpr int kWaveList = kTilePool / kWaves;  // longest list one wavefront stages
constexpr int kMaxCons = 2 * kMaxK;   // checked relations of one new position
constexpr int kFilterMinLen = 32;     // pivot lists at least this long are pre-filtered
constexpr int kFilterPiece = kExpandTile;  // list entries per block of the filter
constexpr int kAssignItems = 16;     // hash slots per thread and step when numbering groups
constexpr int kAssignTile = kBlock * kAssignItems;
constexpr int kMergePieces = 64;     // filter pieces per block when closing the gaps
constexpr int kCountStage = 2048;    // filtered-list entries a wavefront stages in the count pass
constexpr int kCountNbrMax = 2048;   // neighbours a wavefront walks for one row in the count pass
constexpr int kTailWords = 1024;      // tail-flag bitmap words a scan tile stages in LDS
constexpr int kValidatorSpan = 256;   // consecutive vertices a wavefront validates per step
constexpr int kAlignMin = 512;        // rows with this many candidates get tiles of their own
constexpr int kMarkEntries = 4 * kExpandTile;  // longest list window marked into a tile
constexpr uint32_t kDonePivot = 1u << 31;  // filtered rows: the pivot position's relations done

// Graph as the kernels see it.  m < 2^31, so offsets and arc ids are int32.
struct DevGraph {
  int32_t n;
  int32_t m;
  const int32_t* out_off;   // [n+1]
  const int32_t* out_nbrs;  // [m]   heads, rows ascending
  const int32_t* in_off;    // [n+1]
  const int32_t* in_nbrs;   // [m]   tails, rows ascending
  const int32_t* src;       // [m]   tail of out-CSR arc e (edge-to-source index)
  const int32_t* in_eid;    // [m]   out-CSR arc id of in-CSR position j
  const int32_t* rev_eid;   // [m]   out-CSR id of the reverse of arc e, or -1
  int32_t n_vcols, n_ecols;
  const int32_t* vcol[kMaxCols];  // [n] each
  const int32_t* ecol[kMaxCols];  // [m] each, out-CSR order
  const int32_t* ecol_in[kMaxCols];  // [m] each, the same columns in in-CSR order
};

// Matching plan in "position" space: position p holds original pattern vertex
// orig[p]; positions are filled in increasing order.  Predicates are stored as
// inclusive int32 ranges per column (ANY = full range, EQ v = [v,v],
// GE v = [v, INT32_MAX]); a mask bit says which columns need reading at all.
struct DevPlan {
  int32_t k;
  int32_t mode;          // 0 induced isomorphism, 1 monomorphism
  int32_t mve_forward;   // 1: scanned arc x->y binds pos0=x, pos1=y; 0: pos1=x, pos0=y
  int32_t rev_rule;      // reverse of the scanned arc: 0 ignore, 1 required (+pred 1->0), 2 forbidden
  int32_t pin[kMaxK];    // pattern in-degree per position
  int32_t pout[kMaxK];   // pattern out-degree per position
  uint32_t vmask[kMaxK];
  int32_t vlo[kMaxK][kMaxCols];
  int32_t vhi[kMaxK][kMaxCols];
  uint32_t fwd[kMaxK];   // bit b of fwd[a]: arc (pos b -> pos a) in the pattern, b < a
  uint32_t bwd[kMaxK];   // bit b of bwd[a]: arc (pos a -> pos b) in the pattern, b < a
  uint32_t amask[kMaxK][kMaxK];  // columns constrained on arc (p -> q)
  int32_t alo[kMaxK][kMaxK][kMaxCols];
  int32_t ahi[kMaxK][kMaxK][kMaxCols];
  int32_t orig[kMaxK];
};

// Error bits raised by the graph-checking kernels.
enum : uint32_t {
  kErrRange = 1u,        // neighbour id outside [0, n)
  kErrSelfLoop = 2u,
  kErrUnsorted = 4u,     // row not strictly ascending (covers repeats)
  kErrTranspose = 8u,    // in-CSR is not the transpose of the out-CSR
};

// ---- persistent batched matcher (hpm_persist.hip) ---------------------------------

enum : int32_t { kTaskScan = 2, kTaskExpand = 3 };
// launch state bits: queue full, a block left after waiting idle, arena
// full, a descriptor outside the batch's bounds
enum : uint32_t { kPErrQueueFull = 1u, kPErrIdleExit = 2u, kPErrArenaFull = 4u,
                  kPErrBadTask = 8u };
enum : uint32_t { kPatFailed = 1u, kPatOverflow = 2u };  // per-pattern flags
enum : int32_t { kStratMapped = 0, kStratShorter = 1 };  // arc lookups of the extension

// One work-queue slot.  ready is set last, after the descriptor is visible.
struct alignas(64) PTask {
  int32_t ready;
  int32_t type;
  int32_t q;      // pattern index in the batch
  int32_t d;      // EXPAND: positions mapped in each row (the row width)
  int32_t nrows;  // EXPAND: rows of the chunk
  int32_t pad;
  int64_t a;      // SCAN: first arc; EXPAND: arena offset of the rows
  int64_t b;      // SCAN: end of the arc range
  int64_t w0, w1; // EXPAND: candidate range of the chunk; w1 < 0: all of them
};

// Queue and arena state; the hot words sit on separate 128-byte lines.
struct PState {
  unsigned long long head;
  unsigned long long pad0[15];
  unsigned long long tail;
  unsigned long long pad1[15];
  unsigned long long pending;   // tasks queued or running
  unsigned long long pad2[15];
  unsigned long long arena_top; // int32 entries handed out
  unsigned long long pad3[15];
  uint32_t error;               // kPErr* bits
  uint32_t pad4;
  unsigned long long tasks[4];  // tasks run, by type
};

struct PParams {
  DevGraph g;
  const DevPlan* plans;       // [patterns]
  uint32_t* bits;             // validator bitmaps: pattern q position p at bits + bit_base[q] + p * words
  const int64_t* bit_base;    // [patterns]
  int64_t words;              // uint32 words per bitmap
  PTask* queue;
  int64_t qcap;               // slots
  int32_t* arena;
  int64_t arena_cap;          // int32 entries
  PState* st;
  unsigned long long* counts; // [patterns]
  uint32_t* pflags;           // [patterns] kPat* bits
  int32_t n_pat;              // patterns of the batch
  int32_t chunk_rows;         // rows per output chunk (at most 1024)
  int64_t task_work;          // candidates per EXPAND task before the chunk is split
  int32_t strategy;           // kStrat*
  int64_t idle_ticks;         // wall-clock ticks a block waits for a task before it leaves
};

// Resident blocks per CU of the persistent kernel with `items` candidates per
// lane (1, 2 or 4), 0 on error.
int persist_blocks_per_cu(int items);
hipError_t launch_persist(const PParams& P, int items, int grid, hipStream_t stream);
// Validator bitmaps of every position of every pattern of a batch (pattern q
// position p at bits + bit_base[q] + p * words; a plan with k = 0 writes none).
hipError_t launch_batch_validate(const DevGraph& g, const DevPlan* plans, uint32_t* bits,
                                 const int64_t* bit_base, int64_t words, int32_t n_pat,
                                 hipStream_t stream);

// ---- launchers (hpm_kernels.hip) -------------------------------------------------
// Every launcher enqueues on `stream` and returns the launch status.

hipError_t launch_derive_rows(const int32_t* off, int32_t n, int32_t m, int32_t* row_of,
                              hipStream_t stream);
hipError_t launch_check_rows(const int32_t* off, const int32_t* nbrs, const int32_t* row_of,
                             int32_t n, int32_t m, uint32_t* err, hipStream_t stream);
hipError_t launch_transpose_ids(const int32_t* in_off, const int32_t* in_nbrs,
                                const int32_t* in_row, const int32_t* out_off,
                                const int32_t* out_nbrs, int32_t n, int32_t m, int32_t* in_eid,
                                uint32_t* err, hipStream_t stream);
// rev_eid[e] = out-CSR id of arc (head -> tail) for out-CSR arc e, or -1.
hipError_t launch_reverse_ids(const int32_t* out_off, const int32_t* out_nbrs, const int32_t* src,
                              int32_t m, int32_t* rev_eid, hipStream_t stream);

// col_in[j] = col[in_eid[j]]: an arc column copied into in-CSR order.
hipError_t launch_columns_in_order(const int32_t* col, const int32_t* in_eid, int32_t m,
                                   int32_t* col_in, hipStream_t stream);
// vbits: one bitmap per pattern position (position p at vbits + p * words,
// words = 2 * ceil(n / 64)); bit v set when v passes that position's validator.
hipError_t launch_vertex_validator(const DevGraph& g, const DevPlan* plan, uint32_t* vbits,
                                   int64_t words, hipStream_t stream);
// out_mode 0: depth-2 rows [.][2] in position order, written into per-block
//   regions of `out` (rows indexed like the chunk's arcs), per-block counts to
//   blk_count[grid]; compact them with launch_rows2_compact + _gather.
// out_mode 1: count only, per-block counts to blk_count[grid].
// out_mode 2: final rows [.][2] in original pattern order (two-vertex
//   patterns) into out[out_cap], slots reserved on *cursor.
hipError_t launch_edge_scan(const DevGraph& g, const DevPlan* plan, const uint32_t* bits0,
                            const uint32_t* bits1, int32_t e_begin, int32_t e_end, int out_mode,
                            int32_t* out, unsigned long long* cursor, unsigned long long out_cap,
                            unsigned long long* blk_count, int grid, hipStream_t stream);
// In place: blk_count[0..nb) -> exclusive prefix sums, blk_count[nb] = total.
// blk_count must have nb + 1 entries; bsum ceil(nb / kPivotTile) + 1.
hipError_t launch_rows2_compact(int64_t* blk_count, int32_t nb, int64_t* bsum,
                                hipStream_t stream);
// dense[0..s2) = the rows of the per-tile regions of a scan over [e_begin, e_end)
// launched with nb = edge_scan_blocks(e_end - e_begin) blocks.
hipError_t launch_rows2_gather(const int32_t* sparse, const int64_t* prefix, int32_t nb,
                               int32_t e_begin, int32_t e_end, int32_t* dense, int64_t s2,
                               hipStream_t stream);
// Neighbour-overlap test on n depth-2 rows: the rows whose endpoints share at
// least `need` neighbours go to out (unspecified order), *cursor += their
// number (zero it first).
hipError_t launch_overlap_filter(const DevGraph& g, const int32_t* rows, int64_t n, int32_t need,
                                 int32_t* out, unsigned long long* cursor, hipStream_t stream);
// Frontier look-ahead on n rows of d mapped positions: a row is kept (copied
// to out, unspecified order, *cursor += kept; zero it first) when every
// position in fmask that is adjacent to a mapped position has at least one
// candidate consistent with all its mapped neighbours.  vbits: the call's
// validator bitmaps (position p at vbits + p * words).
hipError_t launch_lookahead_filter(const DevGraph& g, const DevPlan* plan, const uint32_t* vbits,
                                   int64_t words, const int32_t* rows, int64_t n, int32_t d,
                                   uint32_t fmask, int32_t* out, unsigned long long* cursor,
                                   hipStream_t stream);
// Arc-predicate index: adjacency restricted to the arcs whose columns in
// cmask lie in [lo[c], hi[c]], built for both CSR sides at once (s[0] the
// out side, s[1] the in side).  Per side: mask and wpre hold
// arc_index_words(m) entries, bsum arc_index_tiles(m) + 1.
struct ArcIndexSide {
  const int32_t* off;                // n + 1 row offsets
  const int32_t* nbrs;               // m targets
  const int32_t* cols[kMaxCols];     // m values per column
  uint64_t* mask;                    // pass bits, 64 arcs per word
  int32_t* wpre;                     // passing arcs before each word
  int64_t* bsum;                     // per-tile counts, then their prefix
  int32_t* off_out;                  // n + 1
  int32_t* nbrs_out;                 // cap
  int32_t* cols_out[kMaxCols];       // cap each (the first ncols)
};
struct ArcIndexSides {
  ArcIndexSide s[2];
};
int64_t arc_index_tiles(int64_t m);
int64_t arc_index_words(int64_t m);
// count: pass bits and tile prefixes of both sides; totals[side] = the number
// of passing arcs (equal for a consistent graph).
hipError_t launch_arc_index_count(const ArcIndexSides& S, const int32_t* lo, const int32_t* hi,
                                  uint32_t cmask, int64_t m, int64_t* totals, hipStream_t stream);
// fill: off_out[0..n] and the passing arcs' targets and first ncols columns,
// in arc order (rows stay sorted); ranks at or past cap are dropped.
hipError_t launch_arc_index_fill(const ArcIndexSides& S, int32_t n, int32_t ncols, int64_t m,
                                 int64_t cap, hipStream_t stream);
// Blocks for an arc scan over `arcs` arcs with out_mode 0 or 1 (one per tile).
int64_t edge_scan_blocks(int64_t arcs);
// Pivot choice and candidate-list length of every row at depth d; writes piv[r]
// ({code, list start}), len into off[0..r) and per-block sums into
// bsum[ceil(r / kPivotTile)].
hipError_t launch_row_pivot(const DevGraph& g, const DevPlan* plan, int32_t d,
                            const int32_t* rows, int32_t r, int2* piv, int64_t* off,
                            int64_t* bsum, hipStream_t stream);
// Turns the lengths in off[0..r) into exclusive prefix sums; off[r] = total.
hipError_t launch_scan_lengths(int64_t* off, int32_t r, int64_t* bsum, hipStream_t stream);
// out_mode: 0 write depth d+1 rows; 1 count only; 2 count and write final rows.
// fpool: pre-filtered candidate lists (rows whose pivot code has bit 1 set).
// abits: the validator bitmap of position d.
// toff NULL: packed tiles over work items [w_begin, w_end) of the prefix sums
// off.  toff non-NULL: w_end tiles of long rows (toff = their tile prefix sums
// from launch_split_rows, off = the full length prefix sums).
// done: positions whose relations with position d the pre-filtered lists
// already enforce (rows with pivot code bit 1 skip them); kDonePivot stands
// for each row's own pivot position.
hipError_t launch_expand(const DevGraph& g, const DevPlan* plan, const uint32_t* abits, int32_t d,
                         const int32_t* rows, const int64_t* off, const int2* piv,
                         const int32_t* fpool, int32_t r, int64_t w_begin, int64_t w_end,
                         const int64_t* toff, uint32_t done, int out_mode, int32_t* out,
                         unsigned long long* cursor, unsigned long long out_cap,
                         unsigned long long* partials, int grid, hipStream_t stream);
// Last-level count of r rows whose filtered lists enforce every arc-related
// position: filtered rows are counted as list length minus the list members
// that are the row's own images or (umask != 0, induced isomorphism)
// neighbours of its images at the positions in umask; other rows check every
// candidate; per-block sums into partials[grid].  With umask != 0, rest[0..r)
// receives the list length of each filtered row left to the tiled extension
// (its images in umask have more than kCountNbrMax neighbours), else 0.
hipError_t launch_count_rows(const DevGraph& g, const DevPlan* plan, const uint32_t* abits,
                             int32_t d, const int32_t* rows, const int64_t* off, const int2* piv,
                             const int32_t* fpool, int32_t r, uint32_t umask, int64_t* rest,
                             unsigned long long* partials, int grid, hipStream_t stream);
// Split rows by list length (prefix sums off[0..r]): soff[0..r] = prefix sums
// of the lengths of rows shorter than kAlignMin (long rows count 0), toff[0..r]
// = prefix sums of the tile counts of long rows; sbsum/tbsum as for
// launch_scan_lengths.
hipError_t launch_split_rows(const int64_t* off, int32_t r, int64_t* soff, int64_t* toff,
                             int64_t* sbsum, int64_t* tbsum, hipStream_t stream);
// Pivot-list filter.  off: the rows' exclusive length prefix sums.  Rows with
// a list of >= min_len entries are grouped by key: table 0 by pivot list;
// tables 1 and 2 (when mask1 / mask2 != 0) by the images of the positions in
// that mask, which must contain every position tied to the new one by a
// pattern arc (so equal keys give equal pivots).  Each table has H slots (a
// power of two above the number of such rows), table t at keys + t * H; keys
// must hold ~0 (empty) on entry.  Only the tables whose bit is set in
// `tables` are filled; distinct[t] += keys of table t.
hipError_t launch_filter_insert(const int32_t* rows, int32_t r, int32_t d, const int2* piv,
                                const int64_t* off, int32_t min_len, uint32_t mask1,
                                uint32_t mask2, uint32_t tables, unsigned long long* keys,
                                uint32_t H, unsigned long long* distinct, hipStream_t stream);
// Number the groups of one table (keys[H]; rmask 0 for table 0, else the
// table-1 mask with rep[H] holding INT32_MAX on entry): dense[H] maps slots to
// groups, slot_key (table 0) or slot_rep (table 1, the group's smallest row)
// and slot_region describe each group; counters[0] += groups, counters[1] +=
// pool entries reserved (raw list lengths).
hipError_t launch_filter_groups(const DevGraph& g, const int32_t* rows, int32_t r, int32_t d,
                                const int2* piv, const int64_t* off, int32_t min_len,
                                uint32_t rmask, const unsigned long long* keys, uint32_t H,
                                int32_t* rep, int32_t* dense, unsigned long long* slot_key,
                                int32_t* slot_rep, int64_t* slot_region,
                                unsigned long long* counters, hipStream_t stream);
// Pieces per group (raw list length split into runs of plen entries):
// pbase[0..nslots] = their exclusive prefix sums, pbase[nslots] = total;
// bsum as for launch_scan_lengths; pslot[piece] = its group and pdesc[piece]
// = {list start, end, pivot code, representative row or pivot vertex}
// (total entries each).
hipError_t launch_filter_pieces(const DevGraph& g, const int32_t* rows, int32_t d,
                                const int2* piv, int32_t nslots,
                                const unsigned long long* slot_key, const int32_t* slot_rep,
                                int32_t plen, int64_t* pbase, int64_t* bsum, int32_t* pslot,
                                int4* pdesc, hipStream_t stream);
// One block per piece (grid >= pbase[nslots]; the blocks past it exit): the
// filtered list of each group into pool + slot_region[s], its length into
// fcount[s].  Groups of two or more pieces go through tmp (pool's size) and
// a second kernel that closes the gaps; tmp may be NULL only when every group
// is one piece.  pcnt / pslot / pdesc hold grid entries (pslot and pdesc
// from launch_filter_pieces).
hipError_t launch_filter_lists(const DevGraph& g, const DevPlan* plan, const uint32_t* abits,
                               int32_t a, const int32_t* rows, uint32_t rmask, int32_t nslots,
                               const int64_t* pbase, int32_t plen, int32_t grid,
                               const int64_t* slot_region, int32_t* pool, int32_t* fcount,
                               int32_t* tmp, int32_t* pcnt, const int32_t* pslot,
                               const int4* pdesc, hipStream_t stream);
// New list lengths into len[0..r) (+ block sums), grouped rows redirected in
// piv (code bit 1); a row whose images differ from its group's representative
// stays as it is.
hipError_t launch_filter_apply(const int32_t* rows, int32_t r, int32_t d, int2* piv,
                               const int64_t* off, int64_t* len, int32_t min_len, uint32_t rmask,
                               const unsigned long long* keys, uint32_t H, const int32_t* dense,
                               const int32_t* slot_rep, const int64_t* slot_region,
                               const int32_t* fcount, int64_t* bsum, hipStream_t stream);
// total[0] += sum(partials[0..nparts)); overflow[0] |= 1 on uint64 wrap.
hipError_t launch_reduce_counts(const unsigned long long* partials, int32_t nparts,
                                unsigned long long* total, uint32_t* overflow, hipStream_t stream);

}  // namespace hpm
