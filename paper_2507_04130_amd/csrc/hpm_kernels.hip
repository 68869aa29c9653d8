// hpm_kernels.hip -- device side of libhpm (gfx950, wave64).
//
// Kernels, in the order a match runs them:
//   k_vertex_validator  vertex validator (Sec. III-B, Alg. 2) evaluated for
//                       every pattern position: one flag word per vertex
//   k_edge_scan         every target arc as a candidate image of pattern arc
//                       (0,1): vertex flags, arc attributes, reverse arc
//                       (Sec. III-B, Alg. 3; Sec. III-C, Alg. 4), compacted
//                       into depth-2 partial mappings (state injection)
//   k_row_pivot         per partial mapping: the shortest adjacency list of a
//                       mapped neighbour of the next position (candidate source)
//   k_scan_*            exclusive prefix sums of the list lengths
//   k_expand            one candidate per thread, load-balanced over the
//                       prefix sums; full feasibility of the new vertex against
//                       every mapped one (Sec. II-A, Eq. (1)-(3)); writes the
//                       extended rows, or counts (and emits) at the last level
//   k_reduce_counts     per-block uint64 partial counts -> total
// plus the graph checks run once by hpm_graph_create.
//
// Wave-level compaction: a thread evaluates several items, a block-wide
// exclusive scan (wave shuffles + LDS across the 4 waves) ranks the survivors,
// and one atomicAdd per block tile reserves the output slots.
#include "hpm_internal.h"
#include "hpm_device.h"

#include <climits>

namespace hpm {
namespace {

// ------------------------------------------------------------ graph checks

__global__ __launch_bounds__(kBlock) void k_derive_rows(const int32_t* __restrict__ off, int32_t n,
                                                        int32_t m, int32_t* __restrict__ row_of) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * kBlock) {
    int32_t lo = 0, hi = n - 1;  // last u with off[u] <= e
    while (lo < hi) {
      const int32_t mid = lo + ((hi - lo + 1) >> 1);
      if (off[mid] <= e)
        lo = mid;
      else
        hi = mid - 1;
    }
    row_of[e] = lo;
  }
}

__global__ __launch_bounds__(kBlock) void k_check_rows(const int32_t* __restrict__ off,
                                                       const int32_t* __restrict__ nbrs,
                                                       const int32_t* __restrict__ row_of,
                                                       int32_t n, int32_t m,
                                                       uint32_t* __restrict__ err) {
  uint32_t bits = 0;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * kBlock) {
    const int32_t v = nbrs[e];
    const int32_t u = row_of[e];
    if (v < 0 || v >= n)
      bits |= kErrRange;
    else if (v == u)
      bits |= kErrSelfLoop;
    if (e > off[u] && nbrs[e - 1] >= v) bits |= kErrUnsorted;
  }
  if (bits) atomicOr(err, bits);
}

__global__ __launch_bounds__(kBlock) void k_transpose_ids(
    const int32_t* __restrict__ in_off, const int32_t* __restrict__ in_nbrs,
    const int32_t* __restrict__ in_row, const int32_t* __restrict__ out_off,
    const int32_t* __restrict__ out_nbrs, int32_t n, int32_t m, int32_t* __restrict__ in_eid,
    uint32_t* __restrict__ err) {
  (void)in_off;
  uint32_t bits = 0;
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < m;
       j += (int64_t)gridDim.x * kBlock) {
    const int32_t v = in_row[j];
    const int32_t u = in_nbrs[j];
    int32_t pos = -1;
    if (u >= 0 && u < n) {
      pos = find_in(out_nbrs, out_off[u], out_off[u + 1], v);
      if (pos < 0) bits |= kErrTranspose;
    }
    in_eid[j] = pos;
  }
  if (bits) atomicOr(err, bits);
}

__global__ __launch_bounds__(kBlock) void k_reverse_ids(const int32_t* __restrict__ out_off,
                                                        const int32_t* __restrict__ out_nbrs,
                                                        const int32_t* __restrict__ src, int32_t m,
                                                        int32_t* __restrict__ rev_eid) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * kBlock) {
    const int32_t v = out_nbrs[e];
    rev_eid[e] = find_in(out_nbrs, out_off[v], out_off[v + 1], src[e]);
  }
}

__global__ __launch_bounds__(kBlock) void k_columns_in_order(const int32_t* __restrict__ col,
                                                             const int32_t* __restrict__ in_eid,
                                                             int32_t m, int32_t* __restrict__ col_in) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < m;
       j += (int64_t)gridDim.x * kBlock)
    col_in[j] = col[in_eid[j]];
}

// ------------------------------------------------------------ vertex validator

typedef int32_t v4i __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_vertex_validator(DevGraph g,
                                                             const DevPlan* __restrict__ P,
                                                             uint32_t* __restrict__ vbits,
                                                             int64_t words) {
  // Bit v of bitmap p (vbits + p * words): v passes the vertex validator for
  // pattern position p (predicates and in/out degree at least the pattern's).
  // Alg. 2 states it for position 0 and Alg. 3 applies it to position 1; the
  // same test is a sound filter for every later position, so it is computed
  // once per vertex.  One bit per vertex keeps each position's flags small
  // enough (n/8 bytes) to stay in L2 while kernels test random vertices.
  // Each wavefront takes 256 consecutive vertices per step, four per lane, so
  // every array is read with 16-byte loads; a lane's four flag bits per
  // position are merged across 8 lanes into one 32-bit bitmap word.
  const int32_t k = P->k;
  uint32_t cols = 0;
  for (int p = 0; p < k; ++p) cols |= P->vmask[p];
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  const int64_t n = g.n;
  for (int64_t base = wave * kValidatorSpan; base < n; base += nwaves * kValidatorSpan) {
    const int64_t v0 = base + 4 * lane;
    int32_t oo[5], io[5], x[kMaxCols][4];
    if (v0 + 4 <= n) {
      const v4i a = *reinterpret_cast<const v4i*>(g.out_off + v0);
      const v4i c = *reinterpret_cast<const v4i*>(g.in_off + v0);
      oo[0] = a.x; oo[1] = a.y; oo[2] = a.z; oo[3] = a.w; oo[4] = g.out_off[v0 + 4];
      io[0] = c.x; io[1] = c.y; io[2] = c.z; io[3] = c.w; io[4] = g.in_off[v0 + 4];
#pragma unroll
      for (int col = 0; col < kMaxCols; ++col) {
        v4i w = {0, 0, 0, 0};
        if ((cols >> col) & 1u) w = *reinterpret_cast<const v4i*>(g.vcol[col] + v0);
        x[col][0] = w.x; x[col][1] = w.y; x[col][2] = w.z; x[col][3] = w.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const bool in = v0 + j <= n;
        oo[j] = in ? g.out_off[v0 + j] : 0;
        io[j] = in ? g.in_off[v0 + j] : 0;
      }
#pragma unroll
      for (int col = 0; col < kMaxCols; ++col)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          x[col][j] = (v0 + j < n && ((cols >> col) & 1u)) ? g.vcol[col][v0 + j] : 0;
    }
    int32_t dout[4], din[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      dout[j] = oo[j + 1] - oo[j];
      din[j] = io[j + 1] - io[j];
    }
    for (int p = 0; p < k; ++p) {
      // the position's plan entries once per step, then this lane's 4 bits at
      // (lane % 8) * 4, OR-merged over the 8 lanes of a bitmap word
      const int32_t pin = P->pin[p], pout = P->pout[p];
      const uint32_t mask = P->vmask[p];
      uint32_t w = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bool ok = v0 + j < n && din[j] >= pin && dout[j] >= pout;
#pragma unroll
        for (int col = 0; col < kMaxCols; ++col)
          if ((mask >> col) & 1u) ok = ok && x[col][j] >= P->vlo[p][col] && x[col][j] <= P->vhi[p][col];
        w |= (uint32_t)ok << ((lane & 7) * 4 + j);
      }
      w |= __shfl_xor(w, 1);
      w |= __shfl_xor(w, 2);
      w |= __shfl_xor(w, 4);
      if ((lane & 7) == 0 && v0 < n) vbits[p * words + ((base + 4 * lane) >> 5)] = w;
    }
  }
}


// ------------------------------------------------------------ arc scan

template <int OUT, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_edge_scan(DevGraph g, const DevPlan* __restrict__ P,
                                                      const uint32_t* __restrict__ bits0,
                                                      const uint32_t* __restrict__ bits1,
                                                      int32_t e_begin, int32_t e_end,
                                                      int32_t* __restrict__ out,
                                                      unsigned long long* __restrict__ cursor,
                                                      unsigned long long out_cap,
                                                      unsigned long long* __restrict__ blk_count) {
  // OUT 0 (depth-2 rows) and 1 (count only): block b scans a contiguous range
  // of tiles and keeps a running count; rows go to the block's own region of
  // `out` (the rows of its arcs' positions), to be gathered densely later, and
  // blk_count[b] receives its total -- no global atomics.  OUT 2 (final rows
  // into the caller's buffer) reserves slots with one atomic per tile.
  __shared__ unsigned long long s_scan[kWaves + 1];
  __shared__ unsigned long long s_base;
  __shared__ uint32_t s_tw[kTailWords];
  __shared__ int32_t s_tw0, s_tw1;
  const int fwd = P->mve_forward;
  const int rev = P->rev_rule;
  const int ps = fwd ? 0 : 1;  // the scanned arc is the image of pattern arc (ps -> pd)
  const int pd = fwd ? 1 : 0;
  const int32_t o0 = P->orig[0], o1 = P->orig[1];
  // first constrained column of the scanned arc's predicate (streamed); others gathered
  const uint32_t emask = P->amask[ps][pd];
  const int ec0 = emask ? __builtin_ctz(emask) : -1;
  const int32_t* ecol0 = g.ecol[ec0 >= 0 ? ec0 : 0];
  const int32_t elo0 = ec0 >= 0 ? P->alo[ps][pd][ec0] : 0;
  const int32_t ehi0 = ec0 >= 0 ? P->ahi[ps][pd][ec0] : 0;
  constexpr int64_t kTile = kBlock * ITEMS;
  const int64_t ntiles = ((int64_t)e_end - e_begin + kTile - 1) / kTile;
  int64_t t_begin, t_end, t_step;
  if (OUT == 2) {
    t_begin = xcd_block_id();
    t_end = ntiles;
    t_step = gridDim.x;
  } else {
    t_begin = (int64_t)blockIdx.x * ntiles / gridDim.x;
    t_end = (int64_t)(blockIdx.x + 1) * ntiles / gridDim.x;
    t_step = 1;
  }
  unsigned long long running = 0;
  for (int64_t t = t_begin; t < t_end; t += t_step) {
    const int64_t tb = e_begin + t * kTile;
    // All streamed arrays of the tile (tails, heads, the first constrained arc
    // column) are loaded before the first barrier, so the tile pays one HBM
    // round trip; the flag tests follow from LDS and L2.  Reverse-arc ids are
    // gathered for the arcs that pass every other test only.
    int32_t v0s[ITEMS], v1s[ITEMS], ev[ITEMS];
    uint32_t valid = 0;
#pragma unroll
    for (int iv = 0; iv < ITEMS / 4; ++iv) {
      const int64_t e0 = tb + ((int64_t)iv * kBlock + threadIdx.x) * 4;
      int32_t xs[4], ys[4], es[4];
      if (e0 + 4 <= e_end) {
        // streamed once: non-temporal, so the flag bitmaps stay in L2
        const v4i a = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(g.src + e0));
        const v4i b = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(g.out_nbrs + e0));
        v4i c = {0, 0, 0, 0};
        if (ec0 >= 0) c = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(ecol0 + e0));
        xs[0] = a.x; xs[1] = a.y; xs[2] = a.z; xs[3] = a.w;
        ys[0] = b.x; ys[1] = b.y; ys[2] = b.z; ys[3] = b.w;
        es[0] = c.x; es[1] = c.y; es[2] = c.z; es[3] = c.w;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool in = e0 + j < e_end;
          xs[j] = in ? g.src[e0 + j] : g.src[tb];  // padding stays in the tail window
          ys[j] = in ? g.out_nbrs[e0 + j] : 0;
          es[j] = (in && ec0 >= 0) ? ecol0[e0 + j] : 0;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v0s[iv * 4 + j] = fwd ? xs[j] : ys[j];
        v1s[iv * 4 + j] = fwd ? ys[j] : xs[j];
        ev[iv * 4 + j] = es[j];
        valid |= (uint32_t)(e0 + j < e_end) << (iv * 4 + j);
      }
    }
    // Tails are sorted, so their flags lie in a few contiguous bitmap words:
    // the tile's window is staged in LDS.  Heads are random; their words are
    // fetched only for arcs whose tail passed, all before any is used.
    const uint32_t* tbits = fwd ? bits0 : bits1;  // position of the tail x
    const uint32_t* hbits = fwd ? bits1 : bits0;  // position of the head y
    {
      // first and last tail of the tile, from the threads that loaded them
      const int64_t last = (tb + kTile < e_end ? tb + kTile : e_end) - 1 - tb;
      const int64_t owner = (last % (4 * kBlock)) >> 2;
      const int lit = (int)(last / (4 * kBlock)) * 4 + (int)(last & 3);
      if (threadIdx.x == 0) s_tw0 = (fwd ? v0s[0] : v1s[0]) >> 5;
      if (threadIdx.x == owner) {
        int32_t xl = 0;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
          if (i == lit) xl = fwd ? v0s[i] : v1s[i];
        s_tw1 = xl >> 5;
      }
    }
    __syncthreads();
    const int32_t tw0 = s_tw0, twn = s_tw1 - s_tw0 + 1;
    const bool tail_lds = twn <= kTailWords;
    if (tail_lds)
      for (int32_t i = threadIdx.x; i < twn; i += kBlock) s_tw[i] = tbits[tw0 + i];
    __syncthreads();
    uint32_t keep = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int32_t x = fwd ? v0s[i] : v1s[i];
      const uint32_t w = tail_lds ? s_tw[(x >> 5) - tw0] : tbits[x >> 5];
      bool ok = ((w >> (x & 31)) & 1u) != 0;
      if (ec0 >= 0) ok = ok && ev[i] >= elo0 && ev[i] <= ehi0;
      keep |= (uint32_t)ok << i;
    }
    keep &= valid;
    uint32_t hw[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int32_t y = fwd ? v1s[i] : v0s[i];
      hw[i] = ((keep >> i) & 1u) ? hbits[y >> 5] : 0u;
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int32_t y = fwd ? v1s[i] : v0s[i];
      if (!((hw[i] >> (y & 31)) & 1u)) keep &= ~(1u << i);
    }
    // further constrained arc columns (rare): gathered for survivors only
    for (int c = ec0 + 1; c < kMaxCols && keep; ++c) {
      if (!((emask >> c) & 1u)) continue;
      const int32_t lo = P->alo[ps][pd][c], hi = P->ahi[ps][pd][c];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        if (!((keep >> i) & 1u)) continue;
        const int64_t e = tb + ((int64_t)(i >> 2) * kBlock + threadIdx.x) * 4 + (i & 3);
        const int32_t w = g.ecol[c][e];
        if (w < lo || w > hi) keep &= ~(1u << i);
      }
    }
    if (rev && keep) {
      // the reverse arc y -> x of each surviving arc: its id gathered from the
      // reverse-arc index (all loads issued before any is used)
      int32_t rv[ITEMS];
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        const int64_t e = tb + ((int64_t)(i >> 2) * kBlock + threadIdx.x) * 4 + (i & 3);
        rv[i] = ((keep >> i) & 1u) ? g.rev_eid[e] : -1;
      }
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        if (!((keep >> i) & 1u)) continue;
        const bool ok = (rev == 1) ? (rv[i] >= 0 && arc_ok(g, P, 1, 0, rv[i])) : (rv[i] < 0);
        if (!ok) keep &= ~(1u << i);
      }
    }
    const unsigned long long cnt = __popc(keep);
    unsigned long long total;
    const unsigned long long excl = block_exclusive_scan<unsigned long long>(cnt, s_scan, &total);
    unsigned long long first;
    if (OUT == 2) {
      if (threadIdx.x == 0) s_base = total ? atomicAdd(cursor, total) : 0ull;
      __syncthreads();
      first = s_base;
    } else {
      first = (unsigned long long)(t_begin * kTile) + running;
    }
    running += total;
    if (OUT != 1 && keep) {
      unsigned long long slot = first + excl;
#pragma unroll
      for (int i = 0; i < ITEMS; ++i) {
        if (keep & (1u << i)) {
          if (slot < out_cap) {
            if (OUT == 0) {
              out[slot * 2 + 0] = v0s[i];
              out[slot * 2 + 1] = v1s[i];
            } else {
              out[slot * 2 + o0] = v0s[i];
              out[slot * 2 + o1] = v1s[i];
            }
          }
          ++slot;
        }
      }
    }
  }
  if (OUT != 2 && threadIdx.x == 0) blk_count[blockIdx.x] = running;
}

// Per-block sums (blocks of kPivotTile entries) of the per-tile survivor counts,
// for launch_scan_lengths.
__global__ __launch_bounds__(kBlock) void k_count_sums(const int64_t* __restrict__ cnt, int32_t nb,
                                                       int64_t* __restrict__ bsum) {
  __shared__ int64_t s_scan[kWaves + 1];
  int64_t sum = 0;
#pragma unroll
  for (int it = 0; it < kPivotItems; ++it) {
    const int64_t i = (int64_t)blockIdx.x * kPivotTile + it * kBlock + threadIdx.x;
    if (i < nb) sum += cnt[i];
  }
  const int64_t tot = block_sum<int64_t>(sum, s_scan);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Dense depth-2 rows from the per-tile regions written by k_edge_scan (one
// block per tile there and here): tile b's rows start at row b * tile of
// `sparse` and go to [prefix[b], prefix[b+1]) of `dense`.
__global__ __launch_bounds__(kBlock) void k_gather_rows2(const int2* __restrict__ sparse,
                                                         const int64_t* __restrict__ prefix,
                                                         int64_t tile, int2* __restrict__ dense) {
  const int64_t b = blockIdx.x;
  const int64_t lo = prefix[b], n = prefix[b + 1] - lo;
  const int2* src = sparse + b * tile;
  for (int64_t i = threadIdx.x; i < n; i += kBlock) dense[lo + i] = src[i];
}

// ------------------------------------------------------------ neighbour overlap
//
// The edge validator's neighbour-overlap test (Sec. III-B, Alg. 3): in any
// embedding the images of the common neighbours of pattern positions 0 and 1
// are distinct common neighbours of their images, so a depth-2 row (u, v)
// whose u and v share fewer neighbours (either direction, u and v excluded)
// than positions 0 and 1 share in the pattern (need) extends to nothing.  One
// wavefront per row walks the out- and then in-list of the endpoint with the
// smaller degree, 64 entries per step, and probes each entry in both lists of
// the other endpoint; an in-neighbour that is also an out-neighbour is counted
// once.  The walk stops as soon as `need` common neighbours are found, or as
// soon as the entries left cannot reach `need`.  Rows that pass go to out
// (unspecified order, one atomic per row kept).
__device__ __forceinline__ bool adjacent_either(const DevGraph& g, int32_t y, int32_t w) {
  return find_in(g.out_nbrs, g.out_off[y], g.out_off[y + 1], w) >= 0 ||
         find_in(g.in_nbrs, g.in_off[y], g.in_off[y + 1], w) >= 0;
}

__global__ __launch_bounds__(kBlock) void k_overlap_filter(DevGraph g, const int2* __restrict__ rows,
                                                           int64_t n, int32_t need,
                                                           int2* __restrict__ out,
                                                           unsigned long long* __restrict__ cursor) {
  const int lane = threadIdx.x & 63;
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  for (int64_t i = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); i < n; i += nwaves) {
    const int2 rw = rows[i];
    int32_t x = rw.x, y = rw.y;
    const int32_t dx = (g.out_off[x + 1] - g.out_off[x]) + (g.in_off[x + 1] - g.in_off[x]);
    const int32_t dy = (g.out_off[y + 1] - g.out_off[y]) + (g.in_off[y + 1] - g.in_off[y]);
    if (dy < dx) {
      const int32_t t = x;
      x = y;
      y = t;
    }
    const int32_t olo = g.out_off[x], ohi = g.out_off[x + 1];
    const int32_t ilo = g.in_off[x], ihi = g.in_off[x + 1];
    const int32_t nout = ohi - olo, total = nout + (ihi - ilo);
    int32_t cnt = 0;
    for (int32_t base = 0; base < total; base += 64) {
      const int32_t j = base + lane;
      bool hit = false;
      if (j < total) {
        const bool from_out = j < nout;
        const int32_t w = from_out ? g.out_nbrs[olo + j] : g.in_nbrs[ilo + j - nout];
        hit = w != y && adjacent_either(g, y, w);
        // a reciprocal neighbour was already counted from the out-list
        if (hit && !from_out) hit = find_in(g.out_nbrs, olo, ohi, w) < 0;
      }
      cnt += __popcll(__ballot(hit));
      const int32_t left = total - (base + 64);
      if (cnt >= need || cnt + (left > 0 ? left : 0) < need) break;  // wave-uniform
    }
    if (lane == 0 && cnt >= need) out[atomicAdd(cursor, 1ull)] = rw;
  }
}

// ------------------------------------------------------------ frontier look-ahead
//
// VF2's look-ahead on the frontier sets (Sec. II-C; the T sets Alg. 3 builds
// for the injected state): a pattern position b beyond the next one that is
// adjacent to a mapped position lies in the pattern's frontier, and in any
// embedding its image is an unmapped target vertex that passes b's vertex
// validator and is joined to the image of every mapped position related to b
// by a target arc in the same direction with that arc's predicate (and, for
// induced isomorphism, to no other mapped image).  A row for which some such
// b has no candidate at all extends to nothing.  A group of G lanes takes one
// row (64 / G rows per wavefront): for each frontier position b (mask
// fmask), the shortest list among the mapped positions related to b is
// walked G entries per step until one entry satisfies every condition; a row
// with a position that has none is dropped.  Rows kept go to out
// (unspecified order).
template <int G>
__global__ __launch_bounds__(kBlock) void k_lookahead_filter(
    DevGraph g, const DevPlan* __restrict__ P, const uint32_t* __restrict__ vbits, int64_t words,
    const int32_t* __restrict__ rows, int64_t n, int32_t d, uint32_t fmask,
    int32_t* __restrict__ out, unsigned long long* __restrict__ cursor) {
  constexpr int kRowsPerWave = 64 / G;
  const int lane = threadIdx.x & 63;
  const int grp = lane / G, gl = lane % G;
  const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1ull)) << (grp * G);
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  const bool iso = P->mode == 0;
  const int32_t k = P->k;
  const uint32_t mapped = (1u << d) - 1u;
  for (int64_t base = ((int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6)) * kRowsPerWave;
       base < n; base += nwaves * kRowsPerWave) {
    const int64_t i = base + grp;
    const int32_t* row = rows + (i < n ? i : 0) * d;
    bool keep = i < n;
    for (int b = 0; b < k; ++b) {  // wave-uniform loop
      if (!((fmask >> b) & 1u)) continue;
      const uint32_t fw = P->fwd[b] & mapped, bw = P->bwd[b] & mapped;
      if ((fw | bw) == 0) continue;
      // pivot: the shortest list of a related mapped position
      int32_t best = 0, pq = 0, plo = 0;
      bool pout = false;
      if (keep) {
        best = INT32_MAX;
        for (int q = 0; q < d; ++q) {
          const int32_t fq = row[q];
          if ((fw >> q) & 1u) {
            const int32_t L = g.out_off[fq + 1] - g.out_off[fq];
            if (L < best) { best = L; pq = q; pout = true; plo = g.out_off[fq]; }
          }
          if ((bw >> q) & 1u) {
            const int32_t L = g.in_off[fq + 1] - g.in_off[fq];
            if (L < best) { best = L; pq = q; pout = false; plo = g.in_off[fq]; }
          }
        }
      }
      const uint32_t* bbits = vbits + (int64_t)b * words;
      bool found = !keep;  // dropped rows take no further steps
      for (int32_t at = 0;; at += G) {
        const bool walking = !found && at < best;
        if (!__any(walking)) break;  // wave-uniform
        bool ok = walking && at + gl < best;
        if (ok) {
          const int32_t pos = plo + at + gl;
          const int32_t c = pout ? g.out_nbrs[pos] : g.in_nbrs[pos];
          ok = test_bit(bbits, c);
          if (ok) ok = pout ? arc_ok(g, P, pq, b, pos) : arc_ok_in(g, P, b, pq, pos);
          for (int q = 0; q < d && ok; ++q) ok = row[q] != c;
          for (int q = 0; q < d && ok; ++q) {
            const int32_t fq = row[q];
            const bool arc_in = (fw >> q) & 1u, arc_out = (bw >> q) & 1u;
            if ((arc_in && !(q == pq && pout)) || (!arc_in && iso)) {
              const int32_t e = find_in(g.out_nbrs, g.out_off[fq], g.out_off[fq + 1], c);
              ok = arc_in ? (e >= 0 && arc_ok(g, P, q, b, e)) : e < 0;
            }
            if (ok && ((arc_out && !(q == pq && !pout)) || (!arc_out && iso))) {
              const int32_t e = find_in(g.in_nbrs, g.in_off[fq], g.in_off[fq + 1], c);
              ok = arc_out ? (e >= 0 && arc_ok_in(g, P, b, q, e)) : e < 0;
            }
          }
        }
        found = found || (__ballot(ok) & gmask) != 0;
      }
      keep = keep && found && best > 0;
    }
    const uint64_t kept = __ballot(keep && gl == 0);
    unsigned long long slot0 = 0;
    if (lane == 0 && kept) slot0 = atomicAdd(cursor, (unsigned long long)__popcll(kept));
    slot0 = __shfl(slot0, 0);
    if (keep) {
      const unsigned long long slot = slot0 + __popcll(kept & ((1ull << (grp * G)) - 1ull));
      for (int x = gl; x < d; x += G) out[slot * d + x] = row[x];
    }
  }
}

// ------------------------------------------------------------ extension

__global__ __launch_bounds__(kBlock) void k_row_pivot(DevGraph g, const DevPlan* __restrict__ P,
                                                      int32_t d, const int32_t* __restrict__ rows,
                                                      int32_t r, int2* __restrict__ piv,
                                                      int64_t* __restrict__ len,
                                                      int64_t* __restrict__ bsum) {
  // For row i (a partial mapping of positions 0..d-1) pick, among the mapped
  // pattern neighbours b of position d, the adjacency list of f(b) in the
  // arc's direction with the fewest entries: every image of position d lies in
  // it.  piv[i] = {(b << 2) | via_out, first index of that list}; bit 1 of the
  // code is set later when the row is redirected to a pre-filtered list.
  __shared__ int64_t s_scan[kWaves + 1];
  const uint32_t fw = P->fwd[d], bw = P->bwd[d];
  int64_t sum = 0;
#pragma unroll
  for (int it = 0; it < kPivotItems; ++it) {
    const int64_t i = (int64_t)blockIdx.x * kPivotTile + it * kBlock + threadIdx.x;
    if (i < r) {
      int32_t best = INT32_MAX, code = 0, base = 0;
      for (int b = 0; b < d; ++b) {
        if (((fw | bw) >> b) & 1u) {
          const int32_t fb = rows[i * d + b];
          if ((fw >> b) & 1u) {
            const int32_t lo = g.out_off[fb];
            const int32_t L = g.out_off[fb + 1] - lo;
            if (L < best) { best = L; code = (b << 2) | 1; base = lo; }
          }
          if ((bw >> b) & 1u) {
            const int32_t lo = g.in_off[fb];
            const int32_t L = g.in_off[fb + 1] - lo;
            if (L < best) { best = L; code = b << 2; base = lo; }
          }
        }
      }
      if (best == INT32_MAX) best = 0;  // cannot happen: every position has an earlier neighbour
      piv[i] = make_int2(code, base);
      len[i] = best;
      sum += best;
    }
  }
  const int64_t tot = block_sum<int64_t>(sum, s_scan);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Exclusive scan of bsum[0..nb) in place by one block; bsum[nb] = off[r] = total.
__global__ __launch_bounds__(kBlock) void k_scan_bsum(int64_t* __restrict__ bsum, int32_t nb,
                                                      int64_t* __restrict__ off, int32_t r) {
  // thread t owns the contiguous run [t * per, (t + 1) * per): its sum, one
  // block scan of the sums, then the run rewritten with running prefixes
  __shared__ int64_t s_scan[kWaves + 1];
  const int32_t per = (nb + kBlock - 1) / kBlock;
  const int32_t i0 = (int32_t)threadIdx.x * per;
  const int32_t i1 = i0 + per < nb ? i0 + per : nb;
  int64_t sum = 0;
  for (int32_t i = i0; i < i1; ++i) sum += bsum[i];
  int64_t tot;
  int64_t run = block_exclusive_scan<int64_t>(sum, s_scan, &tot);
  for (int32_t i = i0; i < i1; ++i) {
    const int64_t x = bsum[i];
    bsum[i] = run;
    run += x;
  }
  if (threadIdx.x == 0) {
    bsum[nb] = tot;
    off[r] = tot;
  }
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(int64_t* __restrict__ off, int32_t r,
                                                       const int64_t* __restrict__ bsum) {
  __shared__ int64_t s_scan[kWaves + 1];
  // thread t owns rows blockIdx*tile + t*kPivotItems .. +kPivotItems-1 (contiguous)
  const int64_t base = (int64_t)blockIdx.x * kPivotTile + (int64_t)threadIdx.x * kPivotItems;
  int64_t v[kPivotItems];
  int64_t s = 0;
#pragma unroll
  for (int it = 0; it < kPivotItems; ++it) {
    v[it] = (base + it < r) ? off[base + it] : 0;
    s += v[it];
  }
  int64_t tot;
  int64_t run = block_exclusive_scan<int64_t>(s, s_scan, &tot) + bsum[blockIdx.x];
#pragma unroll
  for (int it = 0; it < kPivotItems; ++it) {
    if (base + it < r) off[base + it] = run;
    run += v[it];
  }
}

// One checked relation of the position being filled, packed as
// q | dir << 5 | required << 6: dir 0 is the pattern arc q -> a (target arc
// f(q) -> c, looked up in out(f(q))), dir 1 the arc a -> q (c -> f(q), looked
// up in in(f(q))); required 0 means the arc is absent in the pattern and must
// be absent in the target (induced isomorphism only).
__device__ __forceinline__ int32_t pack_cons(int q, int dir, int req) {
  return q | (dir << 5) | (req << 6);
}

// Positions whose relations with the new one a pre-filtered list already
// enforces: the mask of a grouping by related images, or (kDonePivot) the
// row's own pivot position b for a grouping by pivot list.
__device__ __forceinline__ uint32_t done_mask(uint32_t done, int32_t b) {
  return (done & ~kDonePivot) | ((done & kDonePivot) ? (1u << b) : 0u);
}

// A single-row tile whose candidate ids lie in [cmin, cmax] checks relations
// through an LDS bitmap when that range fits in the tile pool.
__device__ __forceinline__ bool tile_bitmap(int32_t cmin, int32_t cmax) {
  return (((int64_t)cmax - cmin) >> 5) < kTilePool;
}

template <int OUT, bool LONG>
__global__ __launch_bounds__(kBlock) void k_expand(
    DevGraph g, const DevPlan* __restrict__ P, const uint32_t* __restrict__ abits, int32_t d,
    const int32_t* __restrict__ rows, const int64_t* __restrict__ off,
    const int2* __restrict__ piv, const int32_t* __restrict__ fpool, int32_t r, int64_t w_begin,
    int64_t w_end, const int64_t* __restrict__ toff, uint32_t done, int32_t* __restrict__ out,
    unsigned long long* __restrict__ cursor, unsigned long long out_cap,
    unsigned long long* __restrict__ partials) {
  // Packed tiles (LONG false): work item w in [w_begin, w_end) is candidate
  // j = w - off[i] of the row i with off[i] <= w < off[i+1] (entry j of that
  // row's pivot list); a tile of kExpandTile consecutive items covers rows
  // [r_lo, r_hi], whose prefix sums, pivots and (if small) the rows themselves
  // are staged in LDS.  Rows of zero length are never selected.
  // Row tiles (LONG true): w_end tiles; tile t is segment s = t - toff[i] of the
  // row i with toff[i] <= t < toff[i+1], i.e. entries [s, s+1) * kExpandTile
  // (cut at the row's length off[i+1] - off[i]) of that row's list.
  // done: positions whose relations with the new one a pre-filtered list
  // (pivot code bit 1) has already checked.
  //
  // Membership tests (is f(q) -> c an arc?) go three ways:
  //  * tile inside one row (every row tile; packed tiles of long lists): the
  //    tile's candidates are the sorted run [cmin, cmax] of one list, so every
  //    checked list is cut to that window once per tile; the window becomes an
  //    LDS bitmap over [cmin, cmax] when that id range is narrow, else each
  //    entry of a short enough window is looked up among the tile's staged
  //    candidates and marks its position, else candidates binary-search the
  //    cut window;
  //  * wavefront inside one row: checked lists of at most kWaveList entries
  //    are staged in the wavefront's LDS slice;
  //  * otherwise each lane binary-searches the list of the mapped vertex.
  // s_off: the tile's row offsets relative to its first item (clamped; the
  // first row's true offset is off[r_lo])
  __shared__ int32_t s_off[kExpandTile + 2];
  __shared__ int2 s_piv[kExpandTile];
  __shared__ int32_t s_rows[kLdsRowInts];
  __shared__ int32_t s_pool[kTilePool];
  __shared__ int32_t s_cons[kMaxCons], s_wlo[kMaxCons], s_whi[kMaxCons];
  __shared__ int32_t s_misc[5];
  __shared__ unsigned long long s_scan[kWaves + 1];
  __shared__ unsigned long long s_base;
  // Single-row tiles leave most of s_off and s_piv unused: the tile's
  // candidates (in order) and their hit mask live there.
  int32_t* s_cand = reinterpret_cast<int32_t*>(s_off + 2);
  uint32_t* s_mark = reinterpret_cast<uint32_t*>(s_piv + 1);
  const int32_t a = d;
  const uint32_t fw = P->fwd[a], bw = P->bwd[a];
  const bool iso = P->mode == 0;
  const int32_t k = P->k;
  const int lane = threadIdx.x & 63;
  int32_t* wl = s_pool + (threadIdx.x >> 6) * kWaveList;
  unsigned long long my_count = 0;
  const int64_t ntiles = LONG ? w_end : (w_end - w_begin + kExpandTile - 1) / kExpandTile;
  for (int64_t t = xcd_block_id(); t < ntiles; t += gridDim.x) {
    int64_t tb, te;  // packed: work items [tb, te); row tiles: list entries [tb, te)
    int32_t r_lo, r_hi;
    if (LONG) {
      if (threadIdx.x < 64) {
        const int32_t x = wave_bound<int64_t>(toff, 0, r, t, true) - 1;
        if (lane == 0) s_misc[0] = x;
      }
      __syncthreads();
      r_lo = r_hi = s_misc[0];
      const int64_t len = off[r_lo + 1] - off[r_lo];
      tb = (t - toff[r_lo]) * kExpandTile;
      te = tb + kExpandTile < len ? tb + kExpandTile : len;
    } else {
      tb = w_begin + t * kExpandTile;
      te = (tb + kExpandTile < w_end) ? tb + kExpandTile : w_end;
      if (threadIdx.x < 128) {
        // wave 0: first row of the tile, wave 1: last row (last i with off[i] <= key)
        const int64_t key = threadIdx.x < 64 ? tb : te - 1;
        const int32_t x = wave_bound<int64_t>(off, 0, r, key, true) - 1;
        if (lane == 0) s_misc[threadIdx.x >> 6] = x;
      }
      __syncthreads();
      r_lo = s_misc[0];
      r_hi = s_misc[1];
    }
    const int32_t nrow = r_hi - r_lo + 1;
    const bool single = nrow == 1;
    const bool use_lds = nrow <= kExpandTile;
    const bool rows_lds = use_lds && nrow * d <= kLdsRowInts;
    if (use_lds) {
      if (!LONG)
        for (int32_t i = threadIdx.x; i <= nrow; i += kBlock) {
          const int64_t rel = off[r_lo + i] - tb;
          s_off[i] = (int32_t)(rel < -1 ? -1 : (rel > kExpandTile + 1 ? kExpandTile + 1 : rel));
        }
      for (int32_t i = threadIdx.x; i < nrow; i += kBlock) s_piv[i] = piv[r_lo + i];
      if (rows_lds)
        for (int32_t i = threadIdx.x; i < nrow * d; i += kBlock)
          s_rows[i] = rows[(int64_t)r_lo * d + i];
    }
    // first and last list entry of the tile (single-row tiles)
    const int64_t jb = LONG ? tb : tb - off[r_lo];
    const int32_t nt = (int32_t)(te - tb);
    if (single && threadIdx.x == 0) {
      const int2 pv = piv[r_lo];
      const int32_t b = pv.x >> 2;
      const bool vo = (pv.x & 1) != 0;
      const uint32_t skip = (pv.x & 2) ? done_mask(done, b) : 0u;
      int32_t n = 0;
      for (int q = 0; q < d; ++q) {
        if ((skip >> q) & 1u) continue;
        const bool arc_in = (fw >> q) & 1u, arc_out = (bw >> q) & 1u;
        if (arc_in ? !(q == b && vo) : iso) s_cons[n++] = pack_cons(q, 0, arc_in);
        if (arc_out ? !(q == b && !vo) : iso) s_cons[n++] = pack_cons(q, 1, arc_out);
      }
      s_misc[2] = n;
      const int32_t* list = (pv.x & 2) ? fpool : (vo ? g.out_nbrs : g.in_nbrs);
      s_misc[3] = list[pv.y + (int32_t)jb];
      s_misc[4] = list[pv.y + (int32_t)jb + nt - 1];
    }
    __syncthreads();
    int32_t ncons = 0;
    bool bitmap = false;
    if (single) {
      ncons = s_misc[2];
      bitmap = tile_bitmap(s_misc[3], s_misc[4]);
      // each wavefront cuts the lists of some relations to [cmin, cmax]
      for (int32_t ci = threadIdx.x >> 6; ci < ncons; ci += kWaves) {
        const int32_t desc = s_cons[ci];
        const int32_t fq = rows[(int64_t)r_lo * d + (desc & 31)];
        const bool in_dir = ((desc >> 5) & 1) != 0;
        const int32_t* lst = in_dir ? g.in_nbrs : g.out_nbrs;
        const int32_t l = in_dir ? g.in_off[fq] : g.out_off[fq];
        const int32_t h = in_dir ? g.in_off[fq + 1] : g.out_off[fq + 1];
        const int32_t wlo = wave_bound<int32_t>(lst, l, h, s_misc[3], false);
        const int32_t whi = wave_bound<int32_t>(lst, wlo, h, s_misc[4], true);
        if (lane == 0) {
          s_wlo[ci] = wlo;
          s_whi[ci] = whi;
        }
      }
      if (!bitmap && ncons > 0) {
        // the tile's candidates, in list order, for marking
        const int2 pv = s_piv[0];
        const int32_t* list = (pv.x & 2) ? fpool : ((pv.x & 1) ? g.out_nbrs : g.in_nbrs);
        for (int32_t x = threadIdx.x; x < nt; x += kBlock) s_cand[x] = list[pv.y + (int32_t)jb + x];
      }
      __syncthreads();
    }

    int32_t cand[kExpandItems], crow[kExpandItems];
    uint32_t keep = 0;
#pragma unroll
    for (int it = 0; it < kExpandItems; ++it) {
      // Items of one wavefront are 64 consecutive w, so valid lanes form a prefix.
      const int64_t w = tb + it * kBlock + threadIdx.x;
      const bool valid = w < te;
      int32_t i = r_lo, li = 0, c = 0, b = 0, pos = 0;
      bool via_out = false, filtered = false;
      if (valid) {
        int64_t j;
        int2 pv;
        if (LONG) {
          j = w;
          pv = s_piv[0];
        } else if (use_lds) {
          const int32_t wr = (int32_t)(w - tb);
          int32_t lo = 0, hi = nrow - 1;
          while (lo < hi) {
            const int32_t mid = lo + ((hi - lo + 1) >> 1);
            if (s_off[mid] <= wr)
              lo = mid;
            else
              hi = mid - 1;
          }
          li = lo;
          i = r_lo + lo;
          j = lo ? (int64_t)(wr - s_off[lo]) : w - off[r_lo];
          pv = s_piv[lo];
        } else {
          int32_t lo = r_lo, hi = r_hi;
          while (lo < hi) {
            const int32_t mid = lo + ((hi - lo + 1) >> 1);
            if (off[mid] <= w)
              lo = mid;
            else
              hi = mid - 1;
          }
          i = lo;
          j = w - off[lo];
          pv = piv[lo];
        }
        b = pv.x >> 2;
        via_out = (pv.x & 1) != 0;
        filtered = (pv.x & 2) != 0;
        pos = pv.y + (int32_t)j;
        c = filtered ? fpool[pos] : (via_out ? g.out_nbrs[pos] : g.in_nbrs[pos]);
      }
      cand[it] = c;
      crow[it] = i;
      const uint64_t vmask = __ballot(valid);
      if (vmask == 0) continue;  // wave-uniform
      const int32_t* grow = rows + (int64_t)i * d;
      const int32_t* lrow = s_rows + li * d;
      auto rowv = [&](int q) -> int32_t { return rows_lds ? lrow[q] : grow[q]; };

      // vertex validator for position a (predicates, degrees); a pre-filtered
      // list holds only candidates that passed it and the pivot-arc predicate
      bool ok = valid && (filtered || ((abits[c >> 5] >> (c & 31)) & 1u) != 0);
      // predicate of the pivot arc itself
      if (ok && !filtered) {
        if (via_out) {
          if (P->amask[b][a]) ok = arc_ok(g, P, b, a, pos);
        } else if (P->amask[a][b]) {
          ok = arc_ok_in(g, P, a, b, pos);
        }
      }
      for (int q = 0; q < d && ok; ++q) ok = rowv(q) != c;  // injectivity

      if (!single) {
        // Does the whole wavefront extend one row?  Then all lanes probe the
        // same lists, and short ones are staged once in LDS (wave_member).
        const int32_t i0 = __shfl(i, 0);
        const bool same_row = __ballot(valid && i == i0) == vmask;
        if (same_row) {
          const int32_t b0 = __shfl(b, 0);
          const bool vo0 = __shfl((int)via_out, 0) != 0;
          const uint32_t skip0 = __shfl((int)filtered, 0) ? done_mask(done, b0) : 0u;
          const int32_t cmin = __shfl(c, 0);
          const int32_t cmax = __shfl(c, 63 - __clzll((long long)vmask));
          for (int q = 0; q < d; ++q) {
            if (!__any(ok)) break;  // wave-uniform
            if ((skip0 >> q) & 1u) continue;
            const int32_t fq = __shfl(rowv(q), 0);
            const bool arc_in = (fw >> q) & 1u;   // pattern arc q -> a
            const bool arc_out = (bw >> q) & 1u;  // pattern arc a -> q
            if (arc_in ? !(q == b0 && vo0) : iso) {
              const int32_t e = wave_member(g.out_nbrs, g.out_off[fq], g.out_off[fq + 1], c,
                                            cmin, cmax, ok, wl, lane);
              if (ok) ok = arc_in ? (e >= 0 && arc_ok(g, P, q, a, e)) : e < 0;
            }
            if (arc_out ? !(q == b0 && !vo0) : iso) {
              const int32_t e = wave_member(g.in_nbrs, g.in_off[fq], g.in_off[fq + 1], c,
                                            cmin, cmax, ok, wl, lane);
              if (ok) ok = arc_out ? (e >= 0 && arc_ok_in(g, P, a, q, e)) : e < 0;
            }
          }
        } else {
          const uint32_t skip = filtered ? done_mask(done, b) : 0u;
          for (int q = 0; q < d && ok; ++q) {
            if ((skip >> q) & 1u) continue;
            const int32_t fq = rowv(q);
            // pattern arc q -> a  <=>  target arc f(q) -> c  (=> only, for monomorphism)
            if ((fw >> q) & 1u) {
              if (!(q == b && via_out)) {
                const int32_t e = find_in(g.out_nbrs, g.out_off[fq], g.out_off[fq + 1], c);
                ok = e >= 0 && arc_ok(g, P, q, a, e);
              }
            } else if (iso) {
              ok = find_in(g.out_nbrs, g.out_off[fq], g.out_off[fq + 1], c) < 0;
            }
            if (!ok) break;
            // pattern arc a -> q  <=>  target arc c -> f(q)
            if ((bw >> q) & 1u) {
              if (!(q == b && !via_out)) {
                const int32_t e = find_in(g.in_nbrs, g.in_off[fq], g.in_off[fq + 1], c);
                ok = e >= 0 && arc_ok_in(g, P, a, q, e);
              }
            } else if (iso) {
              ok = find_in(g.in_nbrs, g.in_off[fq], g.in_off[fq + 1], c) < 0;
            }
          }
        }
      }
      keep |= (uint32_t)ok << it;
    }

    if (single) {
      // Relations of the new position, one at a time for the whole tile.  A
      // hit is an arc that exists and passes its predicate; required arcs
      // keep the hits, absent ones (induced isomorphism) drop them.  With the
      // candidate ids spanning at most 32*kTilePool values the window of the
      // list becomes an LDS bitmap over [cmin, cmax]; else a window of at most
      // kMarkEntries entries marks the tile positions of its entries among the
      // staged candidates; else candidates binary-search the window.
      const int32_t cmin = s_misc[3];
      const int32_t words = (int32_t)(((int64_t)s_misc[4] - cmin) >> 5) + 1;
      uint32_t* bm = reinterpret_cast<uint32_t*>(s_pool);
      for (int32_t ci = 0; ci < ncons; ++ci) {
        if (!__syncthreads_or(keep != 0)) break;  // also orders reuse of the bitmaps
        const int32_t desc = s_cons[ci];
        const int q = desc & 31;
        const bool in_dir = ((desc >> 5) & 1) != 0;
        const bool req = ((desc >> 6) & 1) != 0;
        const int32_t wlo = s_wlo[ci], whi = s_whi[ci];
        const int32_t* lst = in_dir ? g.in_nbrs : g.out_nbrs;
        const bool need = req && (in_dir ? P->amask[a][q] : P->amask[q][a]) != 0;
        if (bitmap || whi - wlo <= kMarkEntries) {
          const int32_t nw = bitmap ? words : (kExpandTile >> 5);
          uint32_t* mk = bitmap ? bm : s_mark;
          for (int32_t x = threadIdx.x; x < nw; x += kBlock) mk[x] = 0u;
          __syncthreads();
          for (int32_t x = wlo + threadIdx.x; x < whi; x += kBlock) {
            const int32_t e = lst[x];
            const int32_t o = bitmap ? e - cmin : lds_find(s_cand, nt, e);
            if (o < 0) continue;
            bool pass = true;
            if (need) pass = in_dir ? arc_ok_in(g, P, a, q, x) : arc_ok(g, P, q, a, x);
            if (pass) atomicOr(&mk[o >> 5], 1u << (o & 31));
          }
          __syncthreads();
#pragma unroll
          for (int it = 0; it < kExpandItems; ++it) {
            if ((keep >> it) & 1u) {
              const int32_t o = bitmap ? cand[it] - cmin : it * kBlock + (int32_t)threadIdx.x;
              const bool hit = ((mk[o >> 5] >> (o & 31)) & 1u) != 0;
              if (hit != req) keep &= ~(1u << it);
            }
          }
        } else {
#pragma unroll
          for (int it = 0; it < kExpandItems; ++it) {
            if ((keep >> it) & 1u) {
              const int32_t pos = find_in(lst, wlo, whi, cand[it]);
              bool ok;
              if (!req)
                ok = pos < 0;
              else if (!need)
                ok = pos >= 0;
              else
                ok = pos >= 0 && (in_dir ? arc_ok_in(g, P, a, q, pos) : arc_ok(g, P, q, a, pos));
              if (!ok) keep &= ~(1u << it);
            }
          }
        }
      }
    }

    const unsigned long long cnt = __popc(keep);
    if (OUT == 1) {
      my_count += cnt;
    } else {
      unsigned long long total;
      const unsigned long long excl = block_exclusive_scan<unsigned long long>(cnt, s_scan, &total);
      if (threadIdx.x == 0) s_base = total ? atomicAdd(cursor, total) : 0ull;
      __syncthreads();
      unsigned long long slot = s_base + excl;
#pragma unroll
      for (int it = 0; it < kExpandItems; ++it) {
        if (keep & (1u << it)) {
          if (slot < out_cap) {
            const int32_t* row = rows + (int64_t)crow[it] * d;
            if (OUT == 0) {
              int32_t* o = out + slot * (unsigned long long)(d + 1);
              for (int q = 0; q < d; ++q) o[q] = row[q];
              o[d] = cand[it];
            } else {
              int32_t* o = out + slot * (unsigned long long)k;
              for (int q = 0; q < d; ++q) o[P->orig[q]] = row[q];
              o[P->orig[a]] = cand[it];
            }
          }
          ++slot;
        }
      }
      if (OUT == 2) my_count += cnt;
    }
    __syncthreads();  // LDS staging and s_base are rewritten by the next tile
  }
  if (OUT != 0) {
    const unsigned long long tot = block_sum<unsigned long long>(my_count, s_scan);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
  }
}

constexpr int kCountBatch = 4;  // candidates of an unfiltered row checked together (count pass)

// Last level, count only, after a filter that enforced every condition
// between the new position and the mapped positions it is tied to by a
// pattern arc.  What a filtered row still has to check is injectivity and,
// for induced isomorphism, the absence of arcs (either direction) between
// the new vertex and the images of the positions in umask.  Its count is
// therefore its filtered list's length minus the list members that are the
// row's own images or neighbours of an image in umask:
//  * umask == 0 (SUB false): d binary searches in the list, one lane per row;
//  * else (SUB true), when those images have at most kCountNbrMax neighbours in all,
//    the block queues the row and a wavefront walks the neighbours, looking
//    each up in the list (staged in LDS when it has at most kCountStage
//    entries; neighbouring rows often share one list, staged once).  A
//    neighbour is taken off once: not if it is an image, nor if an earlier
//    list (by position, out before in) holds it too.  Rows with more
//    neighbours are not counted here: rest[i] = their list length (0 for
//    every other row) for the tiled extension.
// Rows left unfiltered (short lists, or a group-key collision) check their
// candidates one by one in their lane.  Per-block sums go to
// partials[blockIdx].
template <bool SUB>
__global__ __launch_bounds__(kBlock) void k_count_rows(DevGraph g, const DevPlan* __restrict__ P,
                                                       const uint32_t* __restrict__ abits,
                                                       int32_t d, const int32_t* __restrict__ rows,
                                                       const int64_t* __restrict__ off,
                                                       const int2* __restrict__ piv,
                                                       const int32_t* __restrict__ fpool,
                                                       int32_t r, uint32_t umask,
                                                       int64_t* __restrict__ rest,
                                                       unsigned long long* __restrict__ partials) {
  __shared__ long long s_scan[kWaves + 1];
  __shared__ int32_t s_iscan[kWaves + 1];
  __shared__ int32_t s_q[kBlock];
  __shared__ int32_t s_len[kBlock], s_lst[kBlock];  // queued rows: list length and start
  __shared__ int4 s_rng[kBlock];  // queued rows, one position in umask: its out / in ranges
  __shared__ int32_t s_list[kWaves * kCountStage];
  const int32_t a = d;
  const uint32_t fw = P->fwd[a], bw = P->bwd[a];
  const bool iso = P->mode == 0;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int32_t* wl = s_list + wave * kCountStage;
  long long acc = 0;
  for (int64_t i0 = (int64_t)blockIdx.x * kBlock; i0 < r; i0 += (int64_t)gridDim.x * kBlock) {
    const int64_t i = i0 + threadIdx.x;
    bool queue = false;
    if (i < r) {
      int64_t left = 0;
      const int64_t o = off[i];
      const int32_t len = (int32_t)(off[i + 1] - o);
      const int2 pv = len > 0 ? piv[i] : make_int2(0, 0);
      const int32_t* row = rows + i * d;
      if (len > 0 && (pv.x & 2)) {
        if (!SUB) {
          int32_t cnt = len;
          for (int q = 0; q < d; ++q)
            if (find_in(fpool, pv.y, pv.y + len, row[q]) >= 0) --cnt;
          acc += cnt;
        } else {
          int64_t nbrs = 0;
          int4 rng = make_int4(0, 0, 0, 0);
          for (int q = 0; q < d; ++q)
            if ((umask >> q) & 1u) {
              const int32_t f = row[q];
              rng = make_int4(g.out_off[f], g.out_off[f + 1], g.in_off[f], g.in_off[f + 1]);
              nbrs += (int64_t)(rng.y - rng.x) + (rng.w - rng.z);
            }
          if (nbrs <= kCountNbrMax) {
            queue = true;
            s_len[threadIdx.x] = len;
            s_lst[threadIdx.x] = pv.y;
            s_rng[threadIdx.x] = rng;  // used when umask has one position
          } else {
            left = len;
          }
        }
      } else if (len > 0) {
        // Four candidates at a time: their ids, flags and pivot-arc columns
        // are loaded together, and each relation's binary searches (one list,
        // four keys) advance in step, so the lane keeps four loads in flight.
        const int32_t b = pv.x >> 2;
        const bool via_out = (pv.x & 1) != 0;
        const int32_t* __restrict__ plist = via_out ? g.out_nbrs : g.in_nbrs;
        for (int32_t j0 = 0; j0 < len; j0 += kCountBatch) {
          int32_t c[kCountBatch];
          uint32_t ok = 0;
#pragma unroll
          for (int j = 0; j < kCountBatch; ++j) {
            c[j] = j0 + j < len ? plist[pv.y + j0 + j] : 0;
            ok |= (uint32_t)(j0 + j < len) << j;
          }
          uint32_t w[kCountBatch];
#pragma unroll
          for (int j = 0; j < kCountBatch; ++j) w[j] = ((ok >> j) & 1u) ? abits[c[j] >> 5] : 0u;
#pragma unroll
          for (int j = 0; j < kCountBatch; ++j) {
            if (!((ok >> j) & 1u)) continue;
            bool okj = ((w[j] >> (c[j] & 31)) & 1u) != 0;
            const int32_t pos = pv.y + j0 + j;
            if (okj) {
              if (via_out) {
                if (P->amask[b][a]) okj = arc_ok(g, P, b, a, pos);
              } else if (P->amask[a][b]) {
                okj = arc_ok_in(g, P, a, b, pos);
              }
            }
            for (int q = 0; q < d && okj; ++q) okj = row[q] != c[j];
            if (!okj) ok &= ~(1u << j);
          }
          for (int q = 0; q < d && ok; ++q) {
            const int32_t fq = row[q];
            for (int dir = 0; dir < 2 && ok; ++dir) {
              // dir 0: pattern arc q -> a <=> target arc f(q) -> c, in out(f(q));
              // dir 1: pattern arc a -> q <=> target arc c -> f(q), in in(f(q))
              const bool req = dir ? ((bw >> q) & 1u) != 0 : ((fw >> q) & 1u) != 0;
              if (req ? (q == b && via_out == (dir == 0)) : !iso) continue;
              const int32_t* __restrict__ cl = dir ? g.in_nbrs : g.out_nbrs;
              const int32_t lo = dir ? g.in_off[fq] : g.out_off[fq];
              const int32_t hi = dir ? g.in_off[fq + 1] : g.out_off[fq + 1];
              int32_t l[kCountBatch], h[kCountBatch];
#pragma unroll
              for (int j = 0; j < kCountBatch; ++j) {
                l[j] = lo;
                h[j] = ((ok >> j) & 1u) ? hi : lo;
              }
              for (;;) {
                int32_t mid[kCountBatch], v[kCountBatch];
                uint32_t go = 0;
#pragma unroll
                for (int j = 0; j < kCountBatch; ++j) {
                  const bool gj = l[j] < h[j];
                  mid[j] = gj ? l[j] + ((h[j] - l[j]) >> 1) : 0;
                  go |= (uint32_t)gj << j;
                }
                if (!go) break;
#pragma unroll
                for (int j = 0; j < kCountBatch; ++j) v[j] = ((go >> j) & 1u) ? cl[mid[j]] : 0;
#pragma unroll
                for (int j = 0; j < kCountBatch; ++j) {
                  if (!((go >> j) & 1u)) continue;
                  if (v[j] < c[j])
                    l[j] = mid[j] + 1;
                  else
                    h[j] = mid[j];
                }
              }
#pragma unroll
              for (int j = 0; j < kCountBatch; ++j) {
                if (!((ok >> j) & 1u)) continue;
                const bool found = l[j] < hi && cl[l[j]] == c[j];
                bool okj;
                if (!req)
                  okj = !found;
                else if (dir == 0)
                  okj = found && arc_ok(g, P, q, a, l[j]);
                else
                  okj = found && arc_ok_in(g, P, a, q, l[j]);
                if (!okj) ok &= ~(1u << j);
              }
            }
          }
          acc += __popc(ok);
        }
      }
      if (rest) rest[i] = left;
    }
    if (!SUB) continue;  // no queue
    int32_t nq;
    const int32_t qpos = block_exclusive_scan<int32_t>(queue ? 1 : 0, s_iscan, &nq);
    if (queue) s_q[qpos] = threadIdx.x;
    __syncthreads();
    // each wavefront takes a contiguous share of the queue, in row order
    const int32_t qb = wave * nq / kWaves, qe = (wave + 1) * nq / kWaves;
    int32_t st_at = -1, st_len = -1;
    for (int32_t qi = qb; qi < qe; ++qi) {
      const int32_t t = s_q[qi];
      const int64_t ri = i0 + t;
      const int32_t len = s_len[t];
      const int32_t lst = s_lst[t];
      const int32_t* row = rows + ri * d;
      const bool staged = len <= kCountStage;
      if (staged && (lst != st_at || len != st_len)) {
        wave_sync();  // earlier readers of wl are done
        for (int32_t x = lane; x < len; x += 64) wl[x] = fpool[lst + x];
        wave_sync();
        st_at = lst;
        st_len = len;
      }
      int32_t hits = 0;
      if (lane < d) {
        const int32_t y = row[lane];
        if (staged ? lds_find(wl, len, y) >= 0 : find_in(fpool, lst, lst + len, y) >= 0) ++hits;
      }
      const bool one = (umask & (umask - 1u)) == 0;
      const int4 rng1 = s_rng[t];
      for (int q = 0; q < d; ++q) {
        if (!((umask >> q) & 1u)) continue;
        const int32_t fq = one ? 0 : row[q];
        const int4 rq = one ? rng1
                            : make_int4(g.out_off[fq], g.out_off[fq + 1], g.in_off[fq],
                                        g.in_off[fq + 1]);
        for (int dir = 0; dir < 2; ++dir) {
          const int32_t* nb = dir ? g.in_nbrs : g.out_nbrs;
          const int32_t lo = dir ? rq.z : rq.x;
          const int32_t hi = dir ? rq.w : rq.y;
          for (int32_t x = lo + lane; x < hi; x += 64) {
            const int32_t y = nb[x];
            bool hit = staged ? lds_find(wl, len, y) >= 0 : find_in(fpool, lst, lst + len, y) >= 0;
            for (int p = 0; p < d && hit; ++p) hit = row[p] != y;
            if (hit && dir) hit = find_in(g.out_nbrs, rq.x, rq.y, y) < 0;
            for (int q2 = 0; q2 < q && hit; ++q2) {
              if (!((umask >> q2) & 1u)) continue;
              const int32_t f2 = row[q2];
              hit = find_in(g.out_nbrs, g.out_off[f2], g.out_off[f2 + 1], y) < 0 &&
                    find_in(g.in_nbrs, g.in_off[f2], g.in_off[f2 + 1], y) < 0;
            }
            hits += hit ? 1 : 0;
          }
        }
      }
      acc -= hits;
      if (lane == 0) acc += len;
    }
    __syncthreads();  // s_q is rewritten by the next step
  }
  const long long tot = block_sum<long long>(acc, s_scan);
  if (threadIdx.x == 0) partials[blockIdx.x] = (unsigned long long)tot;
}

// Rows with at least kAlignMin candidates get tiles of their own: soff[i] is
// the length of a shorter row (0 for a long one), toff[i] the tile count of a
// long row (0 for a short one); per-block sums go to sbsum / tbsum for
// launch_scan_lengths (same tiling as k_row_pivot).
__global__ __launch_bounds__(kBlock) void k_split_rows(const int64_t* __restrict__ off, int32_t r,
                                                       int64_t* __restrict__ soff,
                                                       int64_t* __restrict__ toff,
                                                       int64_t* __restrict__ sbsum,
                                                       int64_t* __restrict__ tbsum) {
  __shared__ int64_t s_scan[kWaves + 1];
  int64_t ss = 0, ts = 0;
#pragma unroll
  for (int it = 0; it < kPivotItems; ++it) {
    const int64_t i = (int64_t)blockIdx.x * kPivotTile + it * kBlock + threadIdx.x;
    if (i < r) {
      const int64_t len = off[i + 1] - off[i];
      const bool lng = len >= kAlignMin;
      const int64_t sl = lng ? 0 : len;
      const int64_t tl = lng ? (len + kExpandTile - 1) / kExpandTile : 0;
      soff[i] = sl;
      toff[i] = tl;
      ss += sl;
      ts += tl;
    }
  }
  const int64_t a = block_sum<int64_t>(ss, s_scan);
  const int64_t b = block_sum<int64_t>(ts, s_scan);
  if (threadIdx.x == 0) {
    sbsum[blockIdx.x] = a;
    tbsum[blockIdx.x] = b;
  }
}

// ------------------------------------------------------------ pivot-list filter
//
// Rows of one depth often share a long pivot list (many partial mappings
// extend the same hub).  Rows are grouped by a key and each group's list is
// filtered once; the candidates that pass, in list order, go to a pool and
// the rows are pointed at their filtered list.
//  * rmask == 0: the key is the pivot list itself (vertex, direction, pivot
//    position); the filter applies the vertex validator of the new position
//    and the predicate of the pivot arc.
//  * rmask != 0: the key is the images of the positions in rmask, which are
//    all the mapped positions related to the new one by a pattern arc (the
//    pivot is one of them and is chosen from them alone, so equal keys give
//    equal pivots).  The filter applies, besides, every condition between the
//    new position and those positions (Eq. (1)-(3) for that pair), so the
//    extension of such a row only checks injectivity and, for induced
//    isomorphism, non-arcs to the other positions.
// Keys of the second kind are 64-bit hashes; each group keeps its smallest
// row as representative and a row whose images differ from its group's
// representative (a hash collision) is simply left unfiltered.

__device__ __forceinline__ uint64_t pivot_key(int32_t v, int32_t code) {
  // vertex | direction bit | pivot position
  return (uint64_t)(uint32_t)v | ((uint64_t)(code & 1) << 32) | ((uint64_t)(code >> 2) << 33);
}

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

__device__ __forceinline__ uint32_t key_hash(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  return (uint32_t)x;
}

constexpr unsigned long long kEmptyKey = ~0ull;
constexpr int kInsertItems = 4;  // rows per thread and step of the hash insert

// The value of lane - 1 (lane 0 gets its own).
__device__ __forceinline__ unsigned long long shfl_up_u64(unsigned long long x) {
  const int lo = __shfl_up((int)(uint32_t)x, 1, 64);
  const int hi = __shfl_up((int)(uint32_t)(x >> 32), 1, 64);
  return (unsigned long long)(uint32_t)lo | ((unsigned long long)(uint32_t)hi << 32);
}

// Group key of row i (see above).
__device__ __forceinline__ unsigned long long row_key(const int32_t* __restrict__ rows, int64_t i,
                                                      int32_t d, int32_t code, uint32_t rmask) {
  if (rmask == 0) return pivot_key(rows[i * d + (code >> 2)], code);
  uint64_t h = 0x243f6a8885a308d3ull;
  for (int q = 0; q < d; ++q)
    if ((rmask >> q) & 1u) h = mix64(h ^ ((uint64_t)(uint32_t)rows[i * d + q] + ((uint64_t)q << 32)));
  return h == kEmptyKey ? kEmptyKey - 1 : h;
}

// Slot of key in the open-addressing table (keys[H], H a power of two).
__device__ __forceinline__ uint32_t table_find(const unsigned long long* __restrict__ keys,
                                               uint32_t H, unsigned long long key) {
  uint32_t h = key_hash(key) & (H - 1);
  while (keys[h] != key) h = (h + 1) & (H - 1);
  return h;
}

// off: exclusive prefix sums of the rows' list lengths (off[r] = total).
// Table 0 (keys[0..H)) groups by pivot list; table t = 1, 2 (keys[t*H ..)),
// when masks[t-1] != 0, groups by the images of the positions in that mask.
// Only the tables with their bit in `tables` are filled; distinct[t] counts
// the keys of table t.
__global__ __launch_bounds__(kBlock) void k_filter_insert(const int32_t* __restrict__ rows,
                                                          int32_t r, int32_t d,
                                                          const int2* __restrict__ piv,
                                                          const int64_t* __restrict__ off,
                                                          int32_t min_len, uint32_t mask1,
                                                          uint32_t mask2, uint32_t tables,
                                                          unsigned long long* __restrict__ keys,
                                                          uint32_t H,
                                                          unsigned long long* __restrict__ distinct) {
  // kInsertItems rows per thread and step (row i0 + j * kBlock + thread):
  // their keys and first probes are loaded before any is resolved, so a
  // thread has that many table reads in flight.
  const int lane = threadIdx.x & 63;
  for (int64_t i0 = (int64_t)blockIdx.x * kBlock * kInsertItems; i0 < r;
       i0 += (int64_t)gridDim.x * kBlock * kInsertItems) {
    bool ins[kInsertItems];
#pragma unroll
    for (int j = 0; j < kInsertItems; ++j) {
      const int64_t i = i0 + j * kBlock + threadIdx.x;
      ins[j] = i < r && off[i + 1] - off[i] >= min_len;
    }
    for (int t = 0; t < 3; ++t) {
      const uint32_t m = t == 0 ? 0u : (t == 1 ? mask1 : mask2);
      if (!((tables >> t) & 1u) || (t > 0 && m == 0)) continue;  // uniform
      unsigned long long* tab = keys + (size_t)t * H;
      unsigned long long key[kInsertItems], prev[kInsertItems];
      uint32_t h[kInsertItems];
      bool go[kInsertItems];
#pragma unroll
      for (int j = 0; j < kInsertItems; ++j) {
        const int64_t i = i0 + j * kBlock + threadIdx.x;
        key[j] = ins[j] ? row_key(rows, i, d, piv[i].x, m) : kEmptyKey;
        // neighbouring rows often share a key: the lane before inserts it
        const unsigned long long before = shfl_up_u64(key[j]);
        go[j] = ins[j] && !(lane > 0 && before == key[j]);
        h[j] = key_hash(key[j]) & (H - 1);
      }
#pragma unroll
      for (int j = 0; j < kInsertItems; ++j) prev[j] = go[j] ? tab[h[j]] : key[j];
      uint32_t fresh = 0;
#pragma unroll
      for (int j = 0; j < kInsertItems; ++j) {
        if (!go[j]) continue;
        uint32_t hj = h[j];
        unsigned long long pv = prev[j];
        while (true) {  // H exceeds the number of rows, so a free slot exists
          // a slot only ever goes from empty to a key, so a plain read that
          // shows a key is final; an empty one is settled by the CAS
          if (pv == kEmptyKey) {
            pv = atomicCAS(&tab[hj], kEmptyKey, key[j]);
            if (pv == kEmptyKey) fresh |= 1u << j;
          }
          if (pv == kEmptyKey || pv == key[j]) break;
          hj = (hj + 1) & (H - 1);
          pv = tab[hj];
        }
      }
      // one atomic per wavefront for the new keys it inserted
      unsigned long long n_new = 0;
#pragma unroll
      for (int j = 0; j < kInsertItems; ++j) n_new += __popcll(__ballot((fresh >> j) & 1u));
      if (lane == 0 && n_new) atomicAdd(&distinct[t], n_new);
    }
  }
}

// Table 1: rep[slot] = the smallest row with that key (rep holds INT32_MAX on
// entry).
__global__ __launch_bounds__(kBlock) void k_filter_rep(const int32_t* __restrict__ rows,
                                                       int32_t r, int32_t d,
                                                       const int2* __restrict__ piv,
                                                       const int64_t* __restrict__ off,
                                                       int32_t min_len, uint32_t rmask,
                                                       const unsigned long long* __restrict__ keys,
                                                       uint32_t H, int32_t* __restrict__ rep) {
  // kInsertItems rows per thread and step, first probes loaded together
  for (int64_t i0 = (int64_t)blockIdx.x * kBlock * kInsertItems; i0 < r;
       i0 += (int64_t)gridDim.x * kBlock * kInsertItems) {
    unsigned long long key[kInsertItems], seen[kInsertItems];
    uint32_t h[kInsertItems];
    uint32_t act = 0;
#pragma unroll
    for (int j = 0; j < kInsertItems; ++j) {
      const int64_t i = i0 + j * kBlock + threadIdx.x;
      key[j] = 0;
      h[j] = 0;
      if (i < r && off[i + 1] - off[i] >= min_len) {
        act |= 1u << j;
        key[j] = row_key(rows, i, d, piv[i].x, rmask);
        h[j] = key_hash(key[j]) & (H - 1);
      }
    }
#pragma unroll
    for (int j = 0; j < kInsertItems; ++j) seen[j] = ((act >> j) & 1u) ? keys[h[j]] : 0ull;
#pragma unroll
    for (int j = 0; j < kInsertItems; ++j) {
      if (!((act >> j) & 1u)) continue;
      while (seen[j] != key[j]) {  // the key was inserted, so the probe ends at it
        h[j] = (h[j] + 1) & (H - 1);
        seen[j] = keys[h[j]];
      }
      const int32_t i = (int32_t)(i0 + j * kBlock + threadIdx.x);
      int32_t* slot = &rep[h[j]];
      if (*slot > i) atomicMin(slot, i);  // rep only decreases
    }
  }
}

// Dense ids and pool regions for the occupied slots of one table (keys[H]):
// counters[0] = groups, counters[1] = pool entries reserved (sum of raw list
// lengths).  Pivot-list groups (rep == NULL) keep their key in slot_key;
// groups by related images keep their representative row in slot_rep.
__global__ __launch_bounds__(kBlock) void k_filter_assign(DevGraph g,
                                                          const int32_t* __restrict__ rows,
                                                          int32_t d,
                                                          const int2* __restrict__ piv,
                                                          const unsigned long long* __restrict__ keys,
                                                          uint32_t H,
                                                          const int32_t* __restrict__ rep,
                                                          int32_t* __restrict__ dense,
                                                          unsigned long long* __restrict__ slot_key,
                                                          int32_t* __restrict__ slot_rep,
                                                          int64_t* __restrict__ slot_region,
                                                          unsigned long long* __restrict__ counters) {
  // kAssignTile slots per block and step (thread t owns slots t, t + kBlock,
  // ...); group ids and pool offsets are ranked within the block and
  // reserved with one atomic per counter and step.
  __shared__ unsigned long long s_scan[kWaves + 1];
  __shared__ unsigned long long s_base[2];
  for (int64_t h0 = (int64_t)blockIdx.x * kAssignTile; h0 < H;
       h0 += (int64_t)gridDim.x * kAssignTile) {
    // the slots' dependent loads go in phases (keys, representative rows,
    // pivots and images, list bounds), each phase's loads all in flight
    uint32_t occ = 0;
    int32_t L[kAssignItems];
    int32_t v[kAssignItems], code[kAssignItems];
    unsigned long long lmine = 0;
#pragma unroll
    for (int j = 0; j < kAssignItems; ++j) {
      const int64_t h = h0 + j * kBlock + threadIdx.x;
      const unsigned long long key = h < H ? keys[h] : kEmptyKey;
      occ |= (uint32_t)(key != kEmptyKey) << j;
      v[j] = (int32_t)(key & 0xffffffffull);
      code[j] = (int32_t)(((key >> 33) << 2) | ((key >> 32) & 1ull));
    }
    if (rep) {
#pragma unroll
      for (int j = 0; j < kAssignItems; ++j)
        v[j] = ((occ >> j) & 1u) ? rep[h0 + j * kBlock + threadIdx.x] : 0;  // the row
#pragma unroll
      for (int j = 0; j < kAssignItems; ++j) code[j] = ((occ >> j) & 1u) ? piv[v[j]].x : 0;
#pragma unroll
      for (int j = 0; j < kAssignItems; ++j)
        v[j] = ((occ >> j) & 1u) ? rows[(int64_t)v[j] * d + (code[j] >> 2)] : 0;
    }
#pragma unroll
    for (int j = 0; j < kAssignItems; ++j) {
      L[j] = 0;
      if ((occ >> j) & 1u) {
        const int32_t* o = (code[j] & 1) ? g.out_off : g.in_off;
        L[j] = o[v[j] + 1] - o[v[j]];
        lmine += (unsigned long long)L[j];
      }
    }
    unsigned long long nocc, nlen;
    const unsigned long long ex_s =
        block_exclusive_scan<unsigned long long>((unsigned long long)__popc(occ), s_scan, &nocc);
    const unsigned long long ex_p = block_exclusive_scan<unsigned long long>(lmine, s_scan, &nlen);
    if (threadIdx.x == 0) {
      s_base[0] = nocc ? atomicAdd(&counters[0], nocc) : 0ull;
      s_base[1] = nlen ? atomicAdd(&counters[1], nlen) : 0ull;
    }
    __syncthreads();
    unsigned long long sidx = s_base[0] + ex_s, region = s_base[1] + ex_p;
#pragma unroll
    for (int j = 0; j < kAssignItems; ++j) {
      if (!((occ >> j) & 1u)) continue;
      const int64_t h = h0 + j * kBlock + threadIdx.x;
      dense[h] = (int32_t)sidx;
      if (rep)
        slot_rep[sidx] = rep[h];
      else
        slot_key[sidx] = keys[h];
      slot_region[sidx] = (int64_t)region;
      ++sidx;
      region += (unsigned long long)L[j];
    }
    __syncthreads();  // s_base is rewritten by the next step
  }
}

// Pieces per group: the group's raw list length (the representative row's
// pivot list, or the list named by a table-0 key) split into runs of plen
// entries, into len[s] with per-block sums in bsum (same tiling as
// k_row_pivot), ready for launch_scan_lengths.
__global__ __launch_bounds__(kBlock) void k_filter_pieces(DevGraph g,
                                                          const int32_t* __restrict__ rows,
                                                          int32_t d,
                                                          const int2* __restrict__ piv,
                                                          int32_t nslots,
                                                          const unsigned long long* __restrict__ slot_key,
                                                          const int32_t* __restrict__ slot_rep,
                                                          int32_t plen, int64_t* __restrict__ len,
                                                          int64_t* __restrict__ bsum) {
  __shared__ int64_t s_scan[kWaves + 1];
  int64_t sum = 0;
#pragma unroll
  for (int it = 0; it < kPivotItems; ++it) {
    const int64_t s = (int64_t)blockIdx.x * kPivotTile + it * kBlock + threadIdx.x;
    if (s < nslots) {
      int32_t v, code;
      if (slot_rep) {
        const int64_t i = slot_rep[s];
        code = piv[i].x;
        v = rows[i * d + (code >> 2)];
      } else {
        const unsigned long long key = slot_key[s];
        v = (int32_t)(key & 0xffffffffull);
        code = (int32_t)(((key >> 33) << 2) | ((key >> 32) & 1ull));
      }
      const int64_t L = (code & 1) ? g.out_off[v + 1] - g.out_off[v] : g.in_off[v + 1] - g.in_off[v];
      const int64_t n = (L + plen - 1) / plen;
      len[s] = n;
      sum += n;
    }
  }
  const int64_t tot = block_sum<int64_t>(sum, s_scan);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// One wavefront per piece of a group (four per block; pbase: the exclusive
// prefix sums of the pieces per group, pbase[nslots] their total; wavefronts
// at or past the total exit): order-preserving compaction of the candidates of
// the piece's part of the representative row's pivot list that pass the
// vertex validator of position a, the pivot-arc predicate and every other
// condition between a and the positions in rmask (rmask == 0: the pivot
// position alone).  A piece is taken kFilterWaveTile entries at a time (entry
// base + 64 * it + lane in item it of a lane, so loads and stores are
// coalesced); every checked list is cut once per tile to the tile's id range,
// staged in the wavefront's LDS slice when short enough and searched there,
// else searched in the cut range.  Pieces are mostly short lists, so nothing
// waits on the other wavefronts of the block.  A one-piece group writes its
// list to pool + slot_region[s] and its length to fcount[s]; a piece of a
// longer group writes to tmp at the piece's own offset in the group's region,
// for k_filter_merge.  Every piece leaves its count in pcnt; pslot[piece]
// names its group and pdesc[piece] its list range, pivot code and row
// (k_filter_map).
constexpr int kFilterWaveItems = 4;
constexpr int kFilterWaveTile = 64 * kFilterWaveItems;

// Membership of the lanes' candidates c[] (those with their bit in keep) in
// the ascending run cl[lo, hi), cut to [cmin, cmax] and staged in wl when it
// fits.  Returns the bits whose candidate passes: present (and, with need,
// passing the arc predicate at the found position) when req, absent else.
__device__ __forceinline__ uint32_t filter_check(const DevGraph& g, const DevPlan* __restrict__ P,
                                                 int32_t a, int32_t q, bool in_dir, bool req,
                                                 int32_t lo, int32_t hi, int32_t cmin,
                                                 int32_t cmax, const int32_t (&c)[kFilterWaveItems],
                                                 uint32_t keep, int32_t* wl, int lane) {
  const int32_t* __restrict__ cl = in_dir ? g.in_nbrs : g.out_nbrs;
  if (hi - lo > kWaveList) {
    lo = wave_bound<int32_t>(cl, lo, hi, cmin, false);
    hi = wave_bound<int32_t>(cl, lo, hi, cmax, true);
  }
  const int32_t len = hi - lo;
  const bool staged = len <= kWaveList;
  if (staged) {
    wave_sync();  // earlier readers of wl are done
    for (int32_t t = lane; t < len; t += 64) wl[t] = cl[lo + t];
    wave_sync();
  }
  const bool need = req && (in_dir ? P->amask[a][q] : P->amask[q][a]) != 0;
  int32_t at[kFilterWaveItems];
  if (staged) {
#pragma unroll
    for (int it = 0; it < kFilterWaveItems; ++it) {
      const int32_t x = ((keep >> it) & 1u) ? lds_find(wl, len, c[it]) : -1;
      at[it] = x >= 0 ? lo + x : -1;
    }
  } else {
    // the items' searches of the one cut list advance in step
    int32_t l[kFilterWaveItems], h[kFilterWaveItems];
#pragma unroll
    for (int it = 0; it < kFilterWaveItems; ++it) {
      l[it] = lo;
      h[it] = ((keep >> it) & 1u) ? hi : lo;
    }
    for (;;) {
      int32_t mid[kFilterWaveItems], v[kFilterWaveItems];
      uint32_t go = 0;
#pragma unroll
      for (int it = 0; it < kFilterWaveItems; ++it) {
        const bool gi = l[it] < h[it];
        mid[it] = gi ? l[it] + ((h[it] - l[it]) >> 1) : 0;
        go |= (uint32_t)gi << it;
      }
      if (!go) break;
#pragma unroll
      for (int it = 0; it < kFilterWaveItems; ++it) v[it] = ((go >> it) & 1u) ? cl[mid[it]] : 0;
#pragma unroll
      for (int it = 0; it < kFilterWaveItems; ++it) {
        if (!((go >> it) & 1u)) continue;
        if (v[it] < c[it])
          l[it] = mid[it] + 1;
        else
          h[it] = mid[it];
      }
    }
#pragma unroll
    for (int it = 0; it < kFilterWaveItems; ++it)
      at[it] = ((keep >> it) & 1u) && l[it] < hi && cl[l[it]] == c[it] ? l[it] : -1;
  }
#pragma unroll
  for (int it = 0; it < kFilterWaveItems; ++it) {
    if (!((keep >> it) & 1u)) continue;
    const int32_t pos = at[it];
    bool ok;
    if (!req)
      ok = pos < 0;
    else if (!need)
      ok = pos >= 0;
    else
      ok = pos >= 0 && (in_dir ? arc_ok_in(g, P, a, q, pos) : arc_ok(g, P, q, a, pos));
    if (!ok) keep &= ~(1u << it);
  }
  return keep;
}

__global__ __launch_bounds__(kBlock) void k_filter_lists(DevGraph g, const DevPlan* __restrict__ P,
                                                         const uint32_t* __restrict__ abits,
                                                         int32_t a, const int32_t* __restrict__ rows,
                                                         uint32_t rmask, int32_t nslots,
                                                         const int64_t* __restrict__ pbase,
                                                         int32_t plen,
                                                         const int64_t* __restrict__ slot_region,
                                                         int32_t* __restrict__ pool,
                                                         int32_t* __restrict__ fcount,
                                                         int32_t* __restrict__ tmp,
                                                         int32_t* __restrict__ pcnt,
                                                         const int32_t* __restrict__ pslot,
                                                         const int4* __restrict__ pdesc) {
  __shared__ int32_t s_f[kWaves][kMaxK];
  __shared__ int32_t s_pool[kTilePool];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t piece = (int64_t)blockIdx.x * kWaves + wave;
  // the group, its list range, pivot code and row (or pivot vertex) are read
  // beside the total and used only below it
  const int64_t total = pbase[nslots];
  if (piece >= total) return;  // the whole wavefront: no block barrier follows
  const int32_t s = pslot[piece];
  const int4 pd = pdesc[piece];
  const int32_t d = a;
  const int32_t code = pd.z;
  const int64_t i = rmask ? pd.w : 0;
  const int32_t b = code >> 2;
  const bool out_dir = (code & 1) != 0;
  const uint32_t fw = P->fwd[a], bw = P->bwd[a];
  const bool iso = P->mode == 0;
  int32_t* f = s_f[wave];
  int32_t* wl = s_pool + wave * kWaveList;
  if (rmask) {
    if (lane < d) f[lane] = rows[i * d + lane];
  } else if (lane == 0) {
    f[b] = pd.w;
  }
  wave_sync();
  // relations checked here: every condition with a position in rmask (with
  // the pivot position alone for pivot-list groups) but the pivot arc itself
  const uint32_t cmask = rmask ? rmask : (1u << b);
  const int32_t lo = pd.x, hi = pd.y;
  const int32_t* __restrict__ lst = out_dir ? g.out_nbrs : g.in_nbrs;
  const int64_t p0 = pbase[s];
  const int64_t npieces = pbase[s + 1] - p0;
  int32_t* dst = npieces == 1 ? pool + slot_region[s] : tmp + slot_region[s] + (piece - p0) * plen;
  int32_t run = 0;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int32_t base = lo; base < hi; base += kFilterWaveTile) {
    const int32_t end = base + kFilterWaveTile < hi ? base + kFilterWaveTile : hi;
    int32_t c[kFilterWaveItems];
    uint32_t keep = 0;
#pragma unroll
    for (int it = 0; it < kFilterWaveItems; ++it) {
      const int32_t x = base + 64 * it + lane;
      c[it] = x < end ? lst[x] : 0;
    }
#pragma unroll
    for (int it = 0; it < kFilterWaveItems; ++it) {
      const int32_t x = base + 64 * it + lane;
      if (x < end) {
        const int32_t cc = c[it];
        bool ok = ((abits[cc >> 5] >> (cc & 31)) & 1u) != 0;
        if (ok) ok = out_dir ? arc_ok(g, P, b, a, x) : arc_ok_in(g, P, a, b, x);
        keep |= (uint32_t)ok << it;
      }
    }
    const int32_t cmin = lst[base], cmax = lst[end - 1];
    for (int q = 0; q < d; ++q) {
      if (!((cmask >> q) & 1u)) continue;
      if (!__any(keep != 0)) break;  // wave-uniform
      const int32_t fq = f[q];
      const bool arc_in = (fw >> q) & 1u;   // pattern arc q -> a: f(q) -> c in out(f(q))
      const bool arc_out = (bw >> q) & 1u;  // pattern arc a -> q: c -> f(q) in in(f(q))
      if (arc_in ? !(q == b && out_dir) : iso)
        keep = filter_check(g, P, a, q, false, arc_in, g.out_off[fq], g.out_off[fq + 1], cmin,
                            cmax, c, keep, wl, lane);
      if (arc_out ? !(q == b && !out_dir) : iso)
        keep = filter_check(g, P, a, q, true, arc_out, g.in_off[fq], g.in_off[fq + 1], cmin,
                            cmax, c, keep, wl, lane);
    }
    // list order is item order, then lane order
#pragma unroll
    for (int it = 0; it < kFilterWaveItems; ++it) {
      const uint64_t m = __ballot((keep >> it) & 1u);
      if ((keep >> it) & 1u) dst[run + __popcll(m & below)] = c[it];
      run += __popcll(m);
    }
  }
  if (lane == 0) {
    if (npieces == 1) fcount[s] = run;
    pcnt[piece] = run;
  }
}

// For every group s and each of its pieces j = pbase[s] .. pbase[s + 1]:
// pslot[j] = s and pdesc[j] = {first list entry, end, pivot code,
// representative row (rmask != 0) or pivot vertex}, so that a block of
// k_filter_lists starts loading its piece after one dependent read.
__global__ __launch_bounds__(kBlock) void k_filter_map(DevGraph g,
                                                       const int32_t* __restrict__ rows,
                                                       int32_t d,
                                                       const int2* __restrict__ piv,
                                                       int32_t nslots,
                                                       const unsigned long long* __restrict__ slot_key,
                                                       const int32_t* __restrict__ slot_rep,
                                                       int32_t plen,
                                                       const int64_t* __restrict__ pbase,
                                                       int32_t* __restrict__ pslot,
                                                       int4* __restrict__ pdesc) {
  for (int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x; s < nslots;
       s += (int64_t)gridDim.x * kBlock) {
    int32_t v, code, who;
    if (slot_rep) {
      who = slot_rep[s];
      code = piv[who].x;
      v = rows[(int64_t)who * d + (code >> 2)];
    } else {
      const unsigned long long key = slot_key[s];
      v = (int32_t)(key & 0xffffffffull);
      code = (int32_t)(((key >> 33) << 2) | ((key >> 32) & 1ull));
      who = v;
    }
    const int32_t v0 = (code & 1) ? g.out_off[v] : g.in_off[v];
    const int32_t v1 = (code & 1) ? g.out_off[v + 1] : g.in_off[v + 1];
    int32_t lo = v0;
    for (int64_t j = pbase[s]; j < pbase[s + 1]; ++j) {
      const int32_t hi = (int64_t)v1 - lo > plen ? lo + plen : v1;
      pslot[j] = (int32_t)s;
      pdesc[j] = make_int4(lo, hi, code, who);
      lo = hi;
    }
  }
}

// Pieces of groups with two or more: each block takes kMergePieces pieces;
// a thread per piece finds where its survivors go in the group's region (behind
// those of the pieces before it; the last piece writes the group's length to
// fcount), then the whole block moves all those survivors from tmp to pool.
__global__ __launch_bounds__(kBlock) void k_filter_merge(int32_t nslots,
                                                         const int64_t* __restrict__ pbase,
                                                         const int64_t* __restrict__ slot_region,
                                                         const int32_t* __restrict__ tmp,
                                                         const int32_t* __restrict__ pcnt,
                                                         const int32_t* __restrict__ pslot,
                                                         int32_t plen, int32_t* __restrict__ pool,
                                                         int32_t* __restrict__ fcount) {
  __shared__ int32_t s_scan[kWaves + 1];
  __shared__ int32_t s_off[kMergePieces];
  __shared__ int64_t s_src[kMergePieces], s_dst[kMergePieces];
  const int64_t total = pbase[nslots];
  const int64_t blk = (int64_t)blockIdx.x * kMergePieces + threadIdx.x;
  int32_t n = 0;
  int64_t src = 0, dst = 0;
  if (threadIdx.x < kMergePieces && blk < total) {
    const int32_t s = pslot[blk];
    const int64_t p0 = pbase[s], np = pbase[s + 1] - p0;
    if (np > 1) {
      const int64_t piece = blk - p0;
      int64_t pre = 0;
      for (int64_t q = p0; q < blk; ++q) pre += pcnt[q];
      n = pcnt[blk];
      src = slot_region[s] + piece * plen;
      dst = slot_region[s] + pre;
      if (piece == np - 1) fcount[s] = (int32_t)(pre + n);
    }
  }
  int32_t tot;
  const int32_t ex = block_exclusive_scan<int32_t>(n, s_scan, &tot);
  if (threadIdx.x < kMergePieces) {
    s_off[threadIdx.x] = ex;
    s_src[threadIdx.x] = src;
    s_dst[threadIdx.x] = dst;
  }
  __syncthreads();
  // entry of element e: the last piece whose offset is <= e (empty pieces
  // share the offset of the next non-empty one and come before it)
  for (int32_t e0 = threadIdx.x; e0 < tot; e0 += 4 * kBlock) {
    int32_t val[4];
    int64_t to[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t e = e0 + u * kBlock;
      if (e < tot) {
        int32_t l = 0, h = kMergePieces;
        while (h - l > 1) {
          const int32_t mid = (l + h) >> 1;
          if (s_off[mid] <= e) l = mid; else h = mid;
        }
        const int32_t k = e - s_off[l];
        val[u] = tmp[s_src[l] + k];
        to[u] = s_dst[l] + k;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (e0 + u * kBlock < tot) pool[to[u]] = val[u];
  }
}

// Redirect long rows to their filtered list: new lengths go to len[0..r) and
// their per-block sums to bsum (same tiling as k_row_pivot), ready for
// launch_scan_lengths.  off holds the old prefix sums.
__global__ __launch_bounds__(kBlock) void k_filter_apply(const int32_t* __restrict__ rows,
                                                         int32_t r, int32_t d,
                                                         int2* __restrict__ piv,
                                                         const int64_t* __restrict__ off,
                                                         int64_t* __restrict__ len,
                                                         int32_t min_len, uint32_t rmask,
                                                         const unsigned long long* __restrict__ keys,
                                                         uint32_t H,
                                                         const int32_t* __restrict__ dense,
                                                         const int32_t* __restrict__ slot_rep,
                                                         const int64_t* __restrict__ slot_region,
                                                         const int32_t* __restrict__ fcount,
                                                         int64_t* __restrict__ bsum) {
  // The items' dependent loads go in phases (lengths, keys and first probes,
  // probe resolution, group ids, group data), so a thread has kPivotItems of
  // each in flight.
  __shared__ int64_t s_scan[kWaves + 1];
  int64_t L[kPivotItems];
  int2 pv[kPivotItems];
  unsigned long long key[kPivotItems], seen[kPivotItems];
  uint32_t h[kPivotItems];
  uint32_t grp = 0;  // bit it: item it has a row whose list is long enough
#pragma unroll
  for (int it = 0; it < kPivotItems; ++it) {
    const int64_t i = (int64_t)blockIdx.x * kPivotTile + it * kBlock + threadIdx.x;
    L[it] = i < r ? off[i + 1] - off[i] : 0;
    if (i < r && L[it] >= min_len) grp |= 1u << it;
  }
#pragma unroll
  for (int it = 0; it < kPivotItems; ++it) {
    const int64_t i = (int64_t)blockIdx.x * kPivotTile + it * kBlock + threadIdx.x;
    key[it] = 0;
    h[it] = 0;
    if ((grp >> it) & 1u) {
      pv[it] = piv[i];
      key[it] = row_key(rows, i, d, pv[it].x, rmask);
      h[it] = key_hash(key[it]) & (H - 1);
    }
  }
#pragma unroll
  for (int it = 0; it < kPivotItems; ++it) seen[it] = ((grp >> it) & 1u) ? keys[h[it]] : 0ull;
  int32_t sidx[kPivotItems];
#pragma unroll
  for (int it = 0; it < kPivotItems; ++it) {
    if (!((grp >> it) & 1u)) continue;
    // the key was inserted, so the probe ends at it
    while (seen[it] != key[it]) {
      h[it] = (h[it] + 1) & (H - 1);
      seen[it] = keys[h[it]];
    }
  }
#pragma unroll
  for (int it = 0; it < kPivotItems; ++it) sidx[it] = ((grp >> it) & 1u) ? dense[h[it]] : 0;
  uint32_t same = grp;
  if (rmask != 0) {
    int64_t rep[kPivotItems];
#pragma unroll
    for (int it = 0; it < kPivotItems; ++it) rep[it] = ((grp >> it) & 1u) ? slot_rep[sidx[it]] : 0;
#pragma unroll
    for (int it = 0; it < kPivotItems; ++it) {
      if (!((grp >> it) & 1u)) continue;
      const int64_t i = (int64_t)blockIdx.x * kPivotTile + it * kBlock + threadIdx.x;
      bool eq = true;
      for (int q = 0; q < d; ++q)
        if ((rmask >> q) & 1u) eq = eq && rows[i * d + q] == rows[rep[it] * d + q];
      if (!eq) same &= ~(1u << it);
    }
  }
  int64_t sum = 0;
#pragma unroll
  for (int it = 0; it < kPivotItems; ++it) {
    const int64_t i = (int64_t)blockIdx.x * kPivotTile + it * kBlock + threadIdx.x;
    if (i >= r) continue;
    if ((same >> it) & 1u) {
      piv[i] = make_int2(pv[it].x | 2, (int32_t)slot_region[sidx[it]]);
      L[it] = fcount[sidx[it]];
    }
    len[i] = L[it];
    sum += L[it];
  }
  const int64_t tot = block_sum<int64_t>(sum, s_scan);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_reduce_counts(const unsigned long long* __restrict__ partials,
                                                          int32_t nparts,
                                                          unsigned long long* __restrict__ total,
                                                          uint32_t* __restrict__ overflow) {
  __shared__ unsigned long long s_v[kBlock];
  __shared__ uint32_t s_o[kBlock];
  unsigned long long s = 0;
  uint32_t ovf = 0;
  for (int32_t i = threadIdx.x; i < nparts; i += kBlock) {
    const unsigned long long y = s + partials[i];
    ovf |= y < s;
    s = y;
  }
  s_v[threadIdx.x] = s;
  s_o[threadIdx.x] = ovf;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const unsigned long long x = s_v[threadIdx.x], y = s_v[threadIdx.x + w];
      s_v[threadIdx.x] = x + y;
      s_o[threadIdx.x] |= s_o[threadIdx.x + w] | (uint32_t)(x + y < x);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const unsigned long long t0 = *total;
    const unsigned long long t1 = t0 + s_v[0];
    *total = t1;
    if (s_o[0] || t1 < t0) *overflow = 1u;
  }
}

// ------------------------------------------------------------ arc-predicate index
//
// Adjacency restricted to the arcs that pass one attribute predicate (every
// column c in cmask within [lo[c], hi[c]]), built for the out- and the in-CSR
// in the same launches (blockIdx.y is the side).  A tile of kArcTile arcs per
// block, one 64-bit word of pass bits per 64 arcs:
//   mask:    bits and per-tile counts (reads the predicate columns once);
//   scan:    exclusive scan of the tile counts (one block per side);
//   compact: word prefixes (kept for the offsets), then every passing arc's
//            target and columns to its rank among the passing arcs;
//   offsets: off'[v] = the passing arcs before off[v], from the word prefix
//            and a popcount.
// Rows stay sorted.  The mask and prefix arrays hold arc_index_words(m)
// entries per side; the last is one past every tile (zero bits, prefix =
// the total), so off[n] = m maps to the total whatever m is.
struct ArcPred {
  int32_t lo[kMaxCols], hi[kMaxCols];
  uint32_t cmask;
};

__device__ __forceinline__ bool arc_pred_ok(const int32_t* const* cols, const ArcPred& P,
                                            int64_t e) {
  bool ok = true;
#pragma unroll
  for (int c = 0; c < kMaxCols; ++c)
    if ((P.cmask >> c) & 1u) {
      const int32_t x = cols[c][e];
      ok = ok && x >= P.lo[c] && x <= P.hi[c];
    }
  return ok;
}

constexpr int kArcTileWords = kBlock;  // one word per thread
constexpr int64_t kArcTile = (int64_t)kArcTileWords * 64;

// m > 0.  Loads are unconditional (the index clamped to the last arc) and
// issued in batches, so a wave keeps many in flight.
__global__ __launch_bounds__(kBlock) void k_arc_mask(ArcIndexSides S, ArcPred P, int64_t m) {
  const ArcIndexSide& sd = S.s[blockIdx.y];
  __shared__ int64_t s_scan[kWaves + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // wave w fills words w*64 .. w*64+63 of the tile; lane j keeps word j
  const int64_t word0 = (int64_t)blockIdx.x * kArcTileWords + wave * 64;
  const int64_t e0 = word0 * 64 + lane;  // this lane's arc in word j: e0 + 64 j
  uint64_t okm = ~0ull;                  // bit j: that arc passes every column so far
  for (int c = 0; c < kMaxCols; ++c) {
    if (!((P.cmask >> c) & 1u)) continue;
    const int32_t* __restrict__ col = sd.cols[c];
    const int32_t lo = P.lo[c], hi = P.hi[c];
#pragma unroll 1
    for (int j0 = 0; j0 < 64; j0 += 16) {
      int32_t x[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) x[i] = col[min(e0 + 64 * (j0 + i), m - 1)];
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (x[i] < lo || x[i] > hi) okm &= ~(1ull << (j0 + i));
    }
  }
  uint64_t mine = 0;
  int64_t cnt = 0;
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    const uint64_t bits = __ballot(((okm >> j) & 1ull) && e0 + 64 * j < m);
    mine = lane == j ? bits : mine;
    cnt += __popcll(bits);
  }
  sd.mask[word0 + lane] = mine;
  const int64_t tot = block_sum<int64_t>(lane == 0 ? cnt : 0, s_scan);
  if (threadIdx.x == 0) {
    sd.bsum[blockIdx.x] = tot;
    if (blockIdx.x == 0) sd.mask[(int64_t)gridDim.x * kArcTileWords] = 0;
  }
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int j) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(x >> 32), j) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
}

// Copies 8 words' worth of one array (arcs e0 + 64 j, j = j0 .. j0 + 7) to the
// ranks in at (-1: the arc does not pass).
__device__ __forceinline__ void arc_copy8(const int32_t* __restrict__ src,
                                          int32_t* __restrict__ dst, int64_t e0, int j0,
                                          int64_t m, const int64_t (&at)[8]) {
  int32_t x[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) x[i] = src[min(e0 + 64 * (j0 + i), m - 1)];
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (at[i] >= 0) dst[at[i]] = x[i];
}

__global__ __launch_bounds__(kBlock) void k_arc_compact(ArcIndexSides S, int32_t ncols,
                                                        int64_t m, int64_t cap) {
  const ArcIndexSide& sd = S.s[blockIdx.y];
  __shared__ int64_t s_scan[kWaves + 1];
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * kArcTileWords + threadIdx.x;
  const uint64_t bits = sd.mask[w];
  int64_t tot;
  const int64_t pre =
      block_exclusive_scan<int64_t>(__popcll(bits), s_scan, &tot) + sd.bsum[blockIdx.x];
  sd.wpre[w] = (int32_t)pre;
  if (blockIdx.x == 0 && threadIdx.x == 0)
    sd.wpre[(int64_t)gridDim.x * kArcTileWords] = (int32_t)sd.bsum[gridDim.x];
  // the wave's 64 words, eight at a time: lane l handles arc 64 * word + l
  const uint64_t below = (1ull << lane) - 1ull;
  const int64_t e0 = (w - lane) * 64 + lane;
  const int32_t pre32 = (int32_t)pre;
#pragma unroll 1
  for (int j0 = 0; j0 < 64; j0 += 8) {
    int64_t at[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint64_t b = readlane64(bits, j0 + i);
      const int64_t r = (int64_t)__builtin_amdgcn_readlane(pre32, j0 + i) + __popcll(b & below);
      // ranks at or past cap: a side whose arcs disagree with the sized total
      at[i] = ((b >> lane) & 1ull) && r < cap ? r : -1;
    }
    arc_copy8(sd.nbrs, sd.nbrs_out, e0, j0, m, at);
    for (int c = 0; c < ncols; ++c) arc_copy8(sd.cols[c], sd.cols_out[c], e0, j0, m, at);
  }
}

__global__ __launch_bounds__(kBlock) void k_arc_offsets(ArcIndexSides S, int32_t n) {
  const ArcIndexSide& sd = S.s[blockIdx.y];
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v <= n;
       v += (int64_t)gridDim.x * kBlock) {
    const int32_t o = sd.off[v];
    const int64_t w = o >> 6;
    sd.off_out[v] = sd.wpre[w] + __popcll(sd.mask[w] & ((1ull << (o & 63)) - 1ull));
  }
}

inline int grid_for(int64_t items, int64_t per_block, int max_grid) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > max_grid) b = max_grid;
  return (int)b;
}

constexpr int kMaxGridSimple = 8192;

}  // namespace

hipError_t launch_derive_rows(const int32_t* off, int32_t n, int32_t m, int32_t* row_of,
                              hipStream_t stream) {
  if (m <= 0) return hipSuccess;
  k_derive_rows<<<grid_for(m, kBlock, kMaxGridSimple), kBlock, 0, stream>>>(off, n, m, row_of);
  return hipGetLastError();
}

hipError_t launch_check_rows(const int32_t* off, const int32_t* nbrs, const int32_t* row_of,
                             int32_t n, int32_t m, uint32_t* err, hipStream_t stream) {
  if (m <= 0) return hipSuccess;
  k_check_rows<<<grid_for(m, kBlock, kMaxGridSimple), kBlock, 0, stream>>>(off, nbrs, row_of, n,
                                                                           m, err);
  return hipGetLastError();
}

hipError_t launch_transpose_ids(const int32_t* in_off, const int32_t* in_nbrs,
                                const int32_t* in_row, const int32_t* out_off,
                                const int32_t* out_nbrs, int32_t n, int32_t m, int32_t* in_eid,
                                uint32_t* err, hipStream_t stream) {
  if (m <= 0) return hipSuccess;
  k_transpose_ids<<<grid_for(m, kBlock, kMaxGridSimple), kBlock, 0, stream>>>(
      in_off, in_nbrs, in_row, out_off, out_nbrs, n, m, in_eid, err);
  return hipGetLastError();
}

hipError_t launch_reverse_ids(const int32_t* out_off, const int32_t* out_nbrs, const int32_t* src,
                              int32_t m, int32_t* rev_eid, hipStream_t stream) {
  if (m <= 0) return hipSuccess;
  k_reverse_ids<<<grid_for(m, kBlock, kMaxGridSimple), kBlock, 0, stream>>>(out_off, out_nbrs, src,
                                                                            m, rev_eid);
  return hipGetLastError();
}

int64_t edge_scan_blocks(int64_t arcs) {
  const int64_t t = (arcs + kScanTile - 1) / kScanTile;
  return t < 1 ? 1 : t;
}

hipError_t launch_columns_in_order(const int32_t* col, const int32_t* in_eid, int32_t m,
                                   int32_t* col_in, hipStream_t stream) {
  if (m <= 0) return hipSuccess;
  k_columns_in_order<<<grid_for(m, kBlock, kMaxGridSimple), kBlock, 0, stream>>>(col, in_eid, m,
                                                                                 col_in);
  return hipGetLastError();
}

hipError_t launch_vertex_validator(const DevGraph& g, const DevPlan* plan, uint32_t* vbits,
                                   int64_t words, hipStream_t stream) {
  if (g.n <= 0) return hipSuccess;
  k_vertex_validator<<<grid_for((g.n + kValidatorSpan - 1) / kValidatorSpan, kWaves,
                                kMaxGridSimple),
                       kBlock, 0, stream>>>(g, plan, vbits, words);
  return hipGetLastError();
}

hipError_t launch_edge_scan(const DevGraph& g, const DevPlan* plan, const uint32_t* bits0,
                            const uint32_t* bits1, int32_t e_begin, int32_t e_end, int out_mode,
                            int32_t* out, unsigned long long* cursor, unsigned long long out_cap,
                            unsigned long long* blk_count, int grid, hipStream_t stream) {
  if (e_end <= e_begin) return hipSuccess;
  switch (out_mode) {
    case 0:
      k_edge_scan<0, kScanItems><<<grid, kBlock, 0, stream>>>(g, plan, bits0, bits1, e_begin,
                                                              e_end, out, cursor, out_cap,
                                                              blk_count);
      break;
    case 1:
      k_edge_scan<1, kScanItems><<<grid, kBlock, 0, stream>>>(g, plan, bits0, bits1, e_begin,
                                                              e_end, out, cursor, out_cap,
                                                              blk_count);
      break;
    default:
      k_edge_scan<2, kScanItems><<<grid, kBlock, 0, stream>>>(g, plan, bits0, bits1, e_begin,
                                                              e_end, out, cursor, out_cap,
                                                              blk_count);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_rows2_compact(int64_t* blk_count, int32_t nb, int64_t* bsum,
                                hipStream_t stream) {
  const int nbs = (int)(((int64_t)nb + kPivotTile - 1) / kPivotTile);
  k_count_sums<<<nbs, kBlock, 0, stream>>>(blk_count, nb, bsum);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_scan_lengths(blk_count, nb, bsum, stream);
}

hipError_t launch_overlap_filter(const DevGraph& g, const int32_t* rows, int64_t n, int32_t need,
                                 int32_t* out, unsigned long long* cursor, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int grid = grid_for((n + 63) / 64, kWaves, kMaxGridSimple);
  k_overlap_filter<<<grid, kBlock, 0, stream>>>(g, reinterpret_cast<const int2*>(rows), n, need,
                                                reinterpret_cast<int2*>(out), cursor);
  return hipGetLastError();
}

hipError_t launch_lookahead_filter(const DevGraph& g, const DevPlan* plan, const uint32_t* vbits,
                                   int64_t words, const int32_t* rows, int64_t n, int32_t d,
                                   uint32_t fmask, int32_t* out, unsigned long long* cursor,
                                   hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  constexpr int kGroup = 64;  // lanes per row (16 was measured 1.5x slower on the connectome)
  const int grid = grid_for((n * kGroup + 63) / 64, kWaves, kMaxGridSimple);
  k_lookahead_filter<kGroup><<<grid, kBlock, 0, stream>>>(g, plan, vbits, words, rows, n, d,
                                                          fmask, out, cursor);
  return hipGetLastError();
}

hipError_t launch_rows2_gather(const int32_t* sparse, const int64_t* prefix, int32_t nb,
                               int32_t e_begin, int32_t e_end, int32_t* dense, int64_t s2,
                               hipStream_t stream) {
  if (s2 <= 0) return hipSuccess;
  (void)e_begin;
  (void)e_end;
  k_gather_rows2<<<nb, kBlock, 0, stream>>>(reinterpret_cast<const int2*>(sparse), prefix,
                                            (int64_t)kScanTile,
                                            reinterpret_cast<int2*>(dense));
  return hipGetLastError();
}

hipError_t launch_row_pivot(const DevGraph& g, const DevPlan* plan, int32_t d,
                            const int32_t* rows, int32_t r, int2* piv, int64_t* off,
                            int64_t* bsum, hipStream_t stream) {
  if (r <= 0) return hipSuccess;
  const int nb = (int)(((int64_t)r + kPivotTile - 1) / kPivotTile);
  k_row_pivot<<<nb, kBlock, 0, stream>>>(g, plan, d, rows, r, piv, off, bsum);
  return hipGetLastError();
}

int64_t arc_index_tiles(int64_t m) { return std::max<int64_t>(1, (m + kArcTile - 1) / kArcTile); }
int64_t arc_index_words(int64_t m) { return arc_index_tiles(m) * kArcTileWords + 1; }

hipError_t launch_arc_index_count(const ArcIndexSides& S, const int32_t* lo, const int32_t* hi,
                                  uint32_t cmask, int64_t m, int64_t* totals,
                                  hipStream_t stream) {
  ArcPred P{};
  for (int c = 0; c < kMaxCols; ++c) {
    P.lo[c] = lo[c];
    P.hi[c] = hi[c];
  }
  P.cmask = cmask;
  if (m <= 0) return hipErrorInvalidValue;
  const int nb = (int)arc_index_tiles(m);
  k_arc_mask<<<dim3(nb, 2), kBlock, 0, stream>>>(S, P, m);
  hipError_t e = hipGetLastError();
  for (int side = 0; side < 2 && e == hipSuccess; ++side) {
    // tile offsets; the side's total also goes to totals[side]
    k_scan_bsum<<<1, kBlock, 0, stream>>>(S.s[side].bsum, nb, totals, side);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_arc_index_fill(const ArcIndexSides& S, int32_t n, int32_t ncols, int64_t m,
                                 int64_t cap, hipStream_t stream) {
  if (m <= 0) return hipErrorInvalidValue;
  const int nb = (int)arc_index_tiles(m);
  k_arc_compact<<<dim3(nb, 2), kBlock, 0, stream>>>(S, ncols, m, cap);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_arc_offsets<<<dim3(grid_for((int64_t)n + 1, kBlock, kMaxGridSimple), 2), kBlock, 0, stream>>>(
      S, n);
  return hipGetLastError();
}

hipError_t launch_scan_lengths(int64_t* off, int32_t r, int64_t* bsum, hipStream_t stream) {
  if (r <= 0) return hipSuccess;
  const int nb = (int)(((int64_t)r + kPivotTile - 1) / kPivotTile);
  k_scan_bsum<<<1, kBlock, 0, stream>>>(bsum, nb, off, r);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_scan_apply<<<nb, kBlock, 0, stream>>>(off, r, bsum);
  return hipGetLastError();
}

hipError_t launch_expand(const DevGraph& g, const DevPlan* plan, const uint32_t* abits, int32_t d,
                         const int32_t* rows, const int64_t* off, const int2* piv,
                         const int32_t* fpool, int32_t r, int64_t w_begin, int64_t w_end,
                         const int64_t* toff, uint32_t done, int out_mode, int32_t* out,
                         unsigned long long* cursor, unsigned long long out_cap,
                         unsigned long long* partials, int grid, hipStream_t stream) {
  if (w_end <= w_begin || r <= 0) return hipSuccess;
#define HPM_EXPAND(O, L)                                                                    \
  k_expand<O, L><<<grid, kBlock, 0, stream>>>(g, plan, abits, d, rows, off, piv, fpool, r, \
                                              w_begin, w_end, toff, done, out, cursor,     \
                                              out_cap, partials)
  const bool lng = toff != nullptr;
  switch (out_mode) {
    case 0:
      if (lng) HPM_EXPAND(0, true); else HPM_EXPAND(0, false);
      break;
    case 1:
      if (lng) HPM_EXPAND(1, true); else HPM_EXPAND(1, false);
      break;
    default:
      if (lng) HPM_EXPAND(2, true); else HPM_EXPAND(2, false);
      break;
  }
#undef HPM_EXPAND
  return hipGetLastError();
}

hipError_t launch_count_rows(const DevGraph& g, const DevPlan* plan, const uint32_t* abits,
                             int32_t d, const int32_t* rows, const int64_t* off, const int2* piv,
                             const int32_t* fpool, int32_t r, uint32_t umask, int64_t* rest,
                             unsigned long long* partials, int grid, hipStream_t stream) {
  if (r <= 0) return hipSuccess;
  if (umask)
    k_count_rows<true><<<grid, kBlock, 0, stream>>>(g, plan, abits, d, rows, off, piv, fpool, r,
                                                    umask, rest, partials);
  else
    k_count_rows<false><<<grid, kBlock, 0, stream>>>(g, plan, abits, d, rows, off, piv, fpool, r,
                                                     umask, rest, partials);
  return hipGetLastError();
}

hipError_t launch_split_rows(const int64_t* off, int32_t r, int64_t* soff, int64_t* toff,
                             int64_t* sbsum, int64_t* tbsum, hipStream_t stream) {
  if (r <= 0) return hipSuccess;
  const int nb = (int)(((int64_t)r + kPivotTile - 1) / kPivotTile);
  k_split_rows<<<nb, kBlock, 0, stream>>>(off, r, soff, toff, sbsum, tbsum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan_lengths(soff, r, sbsum, stream);
  if (e != hipSuccess) return e;
  return launch_scan_lengths(toff, r, tbsum, stream);
}

hipError_t launch_filter_insert(const int32_t* rows, int32_t r, int32_t d, const int2* piv,
                                const int64_t* off, int32_t min_len, uint32_t mask1,
                                uint32_t mask2, uint32_t tables, unsigned long long* keys,
                                uint32_t H, unsigned long long* distinct, hipStream_t stream) {
  if (r <= 0) return hipSuccess;
  k_filter_insert<<<grid_for(r, (int64_t)kBlock * kInsertItems, kMaxGridSimple), kBlock, 0,
                    stream>>>(
      rows, r, d, piv, off, min_len, mask1, mask2, tables, keys, H, distinct);
  return hipGetLastError();
}

hipError_t launch_filter_groups(const DevGraph& g, const int32_t* rows, int32_t r, int32_t d,
                                const int2* piv, const int64_t* off, int32_t min_len,
                                uint32_t rmask, const unsigned long long* keys, uint32_t H,
                                int32_t* rep, int32_t* dense, unsigned long long* slot_key,
                                int32_t* slot_rep, int64_t* slot_region,
                                unsigned long long* counters, hipStream_t stream) {
  if (r <= 0) return hipSuccess;
  if (rmask) {
    k_filter_rep<<<grid_for(r, (int64_t)kBlock * kInsertItems, kMaxGridSimple), kBlock, 0, stream>>>(
        rows, r, d, piv, off, min_len, rmask, keys, H, rep);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  k_filter_assign<<<grid_for(H, kAssignTile, kMaxGridSimple), kBlock, 0, stream>>>(
      g, rows, d, piv, keys, H, rmask ? rep : nullptr, dense, slot_key, slot_rep, slot_region,
      counters);
  return hipGetLastError();
}

hipError_t launch_filter_pieces(const DevGraph& g, const int32_t* rows, int32_t d,
                                const int2* piv, int32_t nslots,
                                const unsigned long long* slot_key, const int32_t* slot_rep,
                                int32_t plen, int64_t* pbase, int64_t* bsum, int32_t* pslot,
                                int4* pdesc, hipStream_t stream) {
  if (nslots <= 0) return hipSuccess;
  const int nb = (int)(((int64_t)nslots + kPivotTile - 1) / kPivotTile);
  k_filter_pieces<<<nb, kBlock, 0, stream>>>(g, rows, d, piv, nslots, slot_key, slot_rep, plen,
                                             pbase, bsum);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_scan_lengths(pbase, nslots, bsum, stream);
  if (e != hipSuccess) return e;
  k_filter_map<<<grid_for(nslots, kBlock, kMaxGridSimple), kBlock, 0, stream>>>(
      g, rows, d, piv, nslots, slot_key, slot_rep, plen, pbase, pslot, pdesc);
  return hipGetLastError();
}

hipError_t launch_filter_lists(const DevGraph& g, const DevPlan* plan, const uint32_t* abits,
                               int32_t a, const int32_t* rows, uint32_t rmask, int32_t nslots,
                               const int64_t* pbase, int32_t plen, int32_t grid,
                               const int64_t* slot_region, int32_t* pool, int32_t* fcount,
                               int32_t* tmp, int32_t* pcnt, const int32_t* pslot,
                               const int4* pdesc, hipStream_t stream) {
  if (nslots <= 0 || grid <= 0) return hipSuccess;
  // one wavefront per piece
  k_filter_lists<<<(grid + kWaves - 1) / kWaves, kBlock, 0, stream>>>(
      g, plan, abits, a, rows, rmask, nslots, pbase, plen, slot_region, pool, fcount, tmp, pcnt,
      pslot, pdesc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || tmp == nullptr) return e;
  k_filter_merge<<<(grid + kMergePieces - 1) / kMergePieces, kBlock, 0, stream>>>(
      nslots, pbase, slot_region, tmp, pcnt, pslot, plen, pool, fcount);
  return hipGetLastError();
}

hipError_t launch_filter_apply(const int32_t* rows, int32_t r, int32_t d, int2* piv,
                               const int64_t* off, int64_t* len, int32_t min_len, uint32_t rmask,
                               const unsigned long long* keys, uint32_t H, const int32_t* dense,
                               const int32_t* slot_rep, const int64_t* slot_region,
                               const int32_t* fcount, int64_t* bsum, hipStream_t stream) {
  if (r <= 0) return hipSuccess;
  const int nb = (int)(((int64_t)r + kPivotTile - 1) / kPivotTile);
  k_filter_apply<<<nb, kBlock, 0, stream>>>(rows, r, d, piv, off, len, min_len, rmask, keys, H,
                                            dense, slot_rep, slot_region, fcount, bsum);
  return hipGetLastError();
}

hipError_t launch_reduce_counts(const unsigned long long* partials, int32_t nparts,
                                unsigned long long* total, uint32_t* overflow,
                                hipStream_t stream) {
  k_reduce_counts<<<1, kBlock, 0, stream>>>(partials, nparts, total, overflow);
  return hipGetLastError();
}

}  // namespace hpm
