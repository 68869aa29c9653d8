// hpm_kernels.hip -- device side of libhpm (gfx950, wave64).
//
// Kernels, in the order a match runs them:
//   k_vertex_validator  vertex validator for pattern positions 0 and 1
//                       (Sec. III-B, Alg. 2; position 1 gets the same test,
//                       which is the degree part of Alg. 3)
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

#include <climits>

namespace hpm {
namespace {

__device__ __forceinline__ bool vertex_ok(const DevGraph& g, const DevPlan* __restrict__ P, int p,
                                          int32_t v) {
  const uint32_t mask = P->vmask[p];
  if (mask == 0) return true;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < kMaxCols; ++c) {
    if (mask & (1u << c)) {
      const int32_t x = g.vcol[c][v];
      ok = ok && x >= P->vlo[p][c] && x <= P->vhi[p][c];
    }
  }
  return ok;
}

__device__ __forceinline__ bool arc_ok(const DevGraph& g, const DevPlan* __restrict__ P, int p,
                                       int q, int32_t e) {
  const uint32_t mask = P->amask[p][q];
  if (mask == 0) return true;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < kMaxCols; ++c) {
    if (mask & (1u << c)) {
      const int32_t x = g.ecol[c][e];
      ok = ok && x >= P->alo[p][q][c] && x <= P->ahi[p][q][c];
    }
  }
  return ok;
}

// Index of key in the ascending run a[lo, hi), or -1.
__device__ __forceinline__ int32_t find_in(const int32_t* __restrict__ a, int32_t lo, int32_t hi,
                                           int32_t key) {
  int32_t l = lo, h = hi;
  while (l < h) {
    const int32_t mid = l + ((h - l) >> 1);
    if (a[mid] < key)
      l = mid + 1;
    else
      h = mid;
  }
  return (l < hi && a[l] == key) ? l : -1;
}

// Block-wide exclusive scan of one value per thread; *total gets the sum.
// Uses lds[kWaves + 1]; ends with a barrier so lds may be reused.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T x, T* lds, T* total) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  T v = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  if (lane == 63) lds[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    T s = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
      const T t = lds[i];
      lds[i] = s;
      s += t;
    }
    lds[kWaves] = s;
  }
  __syncthreads();
  const T res = lds[wid] + v - x;
  *total = lds[kWaves];
  __syncthreads();
  return res;
}

template <typename T>
__device__ __forceinline__ T block_sum(T x, T* lds) {
  T tot;
  (void)block_exclusive_scan<T>(x, lds, &tot);
  return tot;
}

// Logical block id such that consecutive ids run on the same XCD (blocks are
// dispatched round-robin over the 8 XCDs), so neighbouring tiles -- which
// share rows and adjacency lists -- share an L2.  Requires gridDim.x % 8 == 0.
__device__ __forceinline__ int64_t xcd_block_id() {
  const int64_t b = blockIdx.x;
  const int64_t per = gridDim.x >> 3;
  return (b & 7) * per + (b >> 3);
}

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

// ------------------------------------------------------------ vertex validator

__global__ __launch_bounds__(kBlock) void k_vertex_validator(DevGraph g,
                                                             const DevPlan* __restrict__ P,
                                                             uint8_t* __restrict__ vflag) {
  const int32_t pin0 = P->pin[0], pout0 = P->pout[0];
  const int32_t pin1 = P->pin[1], pout1 = P->pout[1];
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < g.n;
       v += (int64_t)gridDim.x * kBlock) {
    const int32_t dout = g.out_off[v + 1] - g.out_off[v];
    const int32_t din = g.in_off[v + 1] - g.in_off[v];
    uint8_t f = 0;
    if (din >= pin0 && dout >= pout0 && vertex_ok(g, P, 0, (int32_t)v)) f |= 1;
    if (din >= pin1 && dout >= pout1 && vertex_ok(g, P, 1, (int32_t)v)) f |= 2;
    vflag[v] = f;
  }
}

// ------------------------------------------------------------ arc scan

template <int OUT>
__global__ __launch_bounds__(kBlock) void k_edge_scan(DevGraph g, const DevPlan* __restrict__ P,
                                                      const uint8_t* __restrict__ vflag,
                                                      int32_t e_begin, int32_t e_end,
                                                      int32_t* __restrict__ out,
                                                      unsigned long long* __restrict__ cursor,
                                                      unsigned long long out_cap) {
  __shared__ unsigned long long s_scan[kWaves + 1];
  __shared__ unsigned long long s_base;
  const int fwd = P->mve_forward;
  const int rev = P->rev_rule;
  const int ps = fwd ? 0 : 1;  // the scanned arc is the image of pattern arc (ps -> pd)
  const int pd = fwd ? 1 : 0;
  const int32_t o0 = P->orig[0], o1 = P->orig[1];
  const int64_t ntiles = ((int64_t)e_end - e_begin + kScanTile - 1) / kScanTile;
  for (int64_t t = xcd_block_id(); t < ntiles; t += gridDim.x) {
    const int64_t tb = e_begin + t * kScanTile;
    int32_t v0s[kScanItems], v1s[kScanItems];
    uint32_t keep = 0;
#pragma unroll
    for (int iv = 0; iv < kScanItems / 4; ++iv) {
      const int64_t e0 = tb + ((int64_t)iv * kBlock + threadIdx.x) * 4;
      int32_t xs[4], ys[4];
      if (e0 + 4 <= e_end) {
        const int4 a = *reinterpret_cast<const int4*>(g.src + e0);
        const int4 b = *reinterpret_cast<const int4*>(g.out_nbrs + e0);
        xs[0] = a.x; xs[1] = a.y; xs[2] = a.z; xs[3] = a.w;
        ys[0] = b.x; ys[1] = b.y; ys[2] = b.z; ys[3] = b.w;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool in = e0 + j < e_end;
          xs[j] = in ? g.src[e0 + j] : -1;
          ys[j] = in ? g.out_nbrs[e0 + j] : -1;
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int32_t x = xs[j], y = ys[j];
        const int32_t v0 = fwd ? x : y;
        const int32_t v1 = fwd ? y : x;
        v0s[iv * 4 + j] = v0;
        v1s[iv * 4 + j] = v1;
        bool ok = x >= 0;
        if (ok) ok = (vflag[v0] & 1) != 0;
        if (ok) ok = (vflag[v1] & 2) != 0;
        if (ok) ok = arc_ok(g, P, ps, pd, (int32_t)(e0 + j));
        if (ok && rev) {
          const int32_t pos = find_in(g.out_nbrs, g.out_off[y], g.out_off[y + 1], x);
          ok = (rev == 1) ? (pos >= 0 && arc_ok(g, P, 1, 0, pos)) : (pos < 0);
        }
        keep |= (uint32_t)ok << (iv * 4 + j);
      }
    }
    const unsigned long long cnt = __popc(keep);
    unsigned long long total;
    const unsigned long long excl = block_exclusive_scan<unsigned long long>(cnt, s_scan, &total);
    if (threadIdx.x == 0) s_base = total ? atomicAdd(cursor, total) : 0ull;
    __syncthreads();
    if (OUT != 1 && keep) {
      unsigned long long slot = s_base + excl;
#pragma unroll
      for (int i = 0; i < kScanItems; ++i) {
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
}

// ------------------------------------------------------------ extension

__global__ __launch_bounds__(kBlock) void k_row_pivot(DevGraph g, const DevPlan* __restrict__ P,
                                                      int32_t d, const int32_t* __restrict__ rows,
                                                      int32_t r, int32_t* __restrict__ piv,
                                                      int64_t* __restrict__ len,
                                                      int64_t* __restrict__ bsum) {
  __shared__ int64_t s_scan[kWaves + 1];
  const uint32_t fw = P->fwd[d], bw = P->bwd[d];
  int64_t sum = 0;
#pragma unroll
  for (int it = 0; it < kPivotItems; ++it) {
    const int64_t i = (int64_t)blockIdx.x * kPivotTile + it * kBlock + threadIdx.x;
    if (i < r) {
      int32_t best = INT32_MAX, code = 0;
      for (int b = 0; b < d; ++b) {
        if (((fw | bw) >> b) & 1u) {
          const int32_t fb = rows[i * d + b];
          if ((fw >> b) & 1u) {
            const int32_t L = g.out_off[fb + 1] - g.out_off[fb];
            if (L < best) { best = L; code = (b << 1) | 1; }
          }
          if ((bw >> b) & 1u) {
            const int32_t L = g.in_off[fb + 1] - g.in_off[fb];
            if (L < best) { best = L; code = b << 1; }
          }
        }
      }
      if (best == INT32_MAX) best = 0;  // cannot happen: every position has an earlier neighbour
      piv[i] = code;
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
  __shared__ int64_t s_scan[kWaves + 1];
  int64_t carry = 0;
  for (int32_t base = 0; base < nb; base += kBlock) {
    const int32_t i = base + threadIdx.x;
    const int64_t x = i < nb ? bsum[i] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan<int64_t>(x, s_scan, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    bsum[nb] = carry;
    off[r] = carry;
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

template <int OUT>
__global__ __launch_bounds__(kBlock) void k_expand(
    DevGraph g, const DevPlan* __restrict__ P, int32_t d, const int32_t* __restrict__ rows,
    const int64_t* __restrict__ off, const int32_t* __restrict__ piv, int32_t r, int64_t w_begin,
    int64_t w_end, int32_t* __restrict__ out, unsigned long long* __restrict__ cursor,
    unsigned long long out_cap, unsigned long long* __restrict__ partials) {
  __shared__ int64_t s_off[kExpandTile + 1];
  __shared__ int32_t s_rng[2];
  __shared__ unsigned long long s_scan[kWaves + 1];
  __shared__ unsigned long long s_base;
  const int32_t a = d;
  const uint32_t fw = P->fwd[a], bw = P->bwd[a];
  const bool iso = P->mode == 0;
  const int32_t pin_a = P->pin[a], pout_a = P->pout[a];
  const int32_t k = P->k;
  unsigned long long my_count = 0;
  const int64_t ntiles = (w_end - w_begin + kExpandTile - 1) / kExpandTile;
  for (int64_t t = xcd_block_id(); t < ntiles; t += gridDim.x) {
    const int64_t tb = w_begin + t * kExpandTile;
    const int64_t te = min(tb + (int64_t)kExpandTile, w_end);
    if (threadIdx.x < 2) {
      // last row i in [0, r) with off[i] <= key
      const int64_t key = threadIdx.x == 0 ? tb : te - 1;
      int32_t lo = 0, hi = r - 1;
      while (lo < hi) {
        const int32_t mid = lo + ((hi - lo + 1) >> 1);
        if (off[mid] <= key)
          lo = mid;
        else
          hi = mid - 1;
      }
      s_rng[threadIdx.x] = lo;
    }
    __syncthreads();
    const int32_t r_lo = s_rng[0], r_hi = s_rng[1];
    const int32_t nrow = r_hi - r_lo + 1;
    const bool use_lds = nrow <= kExpandTile;
    if (use_lds)
      for (int32_t i = threadIdx.x; i <= nrow; i += kBlock) s_off[i] = off[r_lo + i];
    __syncthreads();

    int32_t cand[kExpandItems], crow[kExpandItems];
    uint32_t keep = 0;
#pragma unroll
    for (int it = 0; it < kExpandItems; ++it) {
      const int64_t w = tb + it * kBlock + threadIdx.x;
      cand[it] = 0;
      crow[it] = 0;
      if (w >= te) continue;
      int32_t i;
      int64_t oi;
      if (use_lds) {
        int32_t lo = 0, hi = nrow - 1;
        while (lo < hi) {
          const int32_t mid = lo + ((hi - lo + 1) >> 1);
          if (s_off[mid] <= w)
            lo = mid;
          else
            hi = mid - 1;
        }
        i = r_lo + lo;
        oi = s_off[lo];
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
        oi = off[lo];
      }
      const int32_t j = (int32_t)(w - oi);
      const int32_t code = piv[i];
      const int32_t b = code >> 1;
      const bool via_out = (code & 1) != 0;
      const int32_t* row = rows + (int64_t)i * d;
      const int32_t fb = row[b];
      int32_t c, eid;
      if (via_out) {
        const int32_t base = g.out_off[fb];
        c = g.out_nbrs[base + j];
        eid = base + j;
      } else {
        const int32_t base = g.in_off[fb];
        c = g.in_nbrs[base + j];
        eid = g.in_eid[base + j];
      }
      bool ok = via_out ? arc_ok(g, P, b, a, eid) : arc_ok(g, P, a, b, eid);
      for (int q = 0; q < d && ok; ++q) ok = row[q] != c;  // injectivity
      if (ok) {
        const int32_t dout = g.out_off[c + 1] - g.out_off[c];
        const int32_t din = g.in_off[c + 1] - g.in_off[c];
        ok = din >= pin_a && dout >= pout_a && vertex_ok(g, P, a, c);
      }
      for (int q = 0; q < d && ok; ++q) {
        const int32_t fq = row[q];
        // pattern arc q -> a  <=>  target arc f(q) -> c  (=> only, for monomorphism)
        if ((fw >> q) & 1u) {
          if (!(q == b && via_out)) {
            const int32_t pos = find_in(g.out_nbrs, g.out_off[fq], g.out_off[fq + 1], c);
            ok = pos >= 0 && arc_ok(g, P, q, a, pos);
          }
        } else if (iso) {
          ok = find_in(g.out_nbrs, g.out_off[fq], g.out_off[fq + 1], c) < 0;
        }
        if (!ok) break;
        // pattern arc a -> q  <=>  target arc c -> f(q)
        if ((bw >> q) & 1u) {
          if (!(q == b && !via_out)) {
            const int32_t pos = find_in(g.in_nbrs, g.in_off[fq], g.in_off[fq + 1], c);
            ok = pos >= 0 && arc_ok(g, P, a, q, g.in_eid[pos]);
          }
        } else if (iso) {
          ok = find_in(g.in_nbrs, g.in_off[fq], g.in_off[fq + 1], c) < 0;
        }
      }
      cand[it] = c;
      crow[it] = i;
      keep |= (uint32_t)ok << it;
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
    __syncthreads();  // s_off, s_rng and s_base are rewritten by the next tile
  }
  if (OUT != 0) {
    const unsigned long long tot = block_sum<unsigned long long>(my_count, s_scan);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
  }
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

hipError_t launch_vertex_validator(const DevGraph& g, const DevPlan* plan, uint8_t* vflag,
                                   hipStream_t stream) {
  if (g.n <= 0) return hipSuccess;
  k_vertex_validator<<<grid_for(g.n, kBlock, kMaxGridSimple), kBlock, 0, stream>>>(g, plan,
                                                                                   vflag);
  return hipGetLastError();
}

hipError_t launch_edge_scan(const DevGraph& g, const DevPlan* plan, const uint8_t* vflag,
                            int32_t e_begin, int32_t e_end, int out_mode, int32_t* out,
                            unsigned long long* cursor, unsigned long long out_cap, int grid,
                            hipStream_t stream) {
  if (e_end <= e_begin) return hipSuccess;
  switch (out_mode) {
    case 0:
      k_edge_scan<0><<<grid, kBlock, 0, stream>>>(g, plan, vflag, e_begin, e_end, out, cursor,
                                                  out_cap);
      break;
    case 1:
      k_edge_scan<1><<<grid, kBlock, 0, stream>>>(g, plan, vflag, e_begin, e_end, out, cursor,
                                                  out_cap);
      break;
    default:
      k_edge_scan<2><<<grid, kBlock, 0, stream>>>(g, plan, vflag, e_begin, e_end, out, cursor,
                                                  out_cap);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_row_pivot(const DevGraph& g, const DevPlan* plan, int32_t d,
                            const int32_t* rows, int32_t r, int32_t* piv, int64_t* off,
                            int64_t* bsum, hipStream_t stream) {
  if (r <= 0) return hipSuccess;
  const int nb = (int)(((int64_t)r + kPivotTile - 1) / kPivotTile);
  k_row_pivot<<<nb, kBlock, 0, stream>>>(g, plan, d, rows, r, piv, off, bsum);
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

hipError_t launch_expand(const DevGraph& g, const DevPlan* plan, int32_t d, const int32_t* rows,
                         const int64_t* off, const int32_t* piv, int32_t r, int64_t w_begin,
                         int64_t w_end, int out_mode, int32_t* out, unsigned long long* cursor,
                         unsigned long long out_cap, unsigned long long* partials, int grid,
                         hipStream_t stream) {
  if (w_end <= w_begin || r <= 0) return hipSuccess;
  switch (out_mode) {
    case 0:
      k_expand<0><<<grid, kBlock, 0, stream>>>(g, plan, d, rows, off, piv, r, w_begin, w_end, out,
                                               cursor, out_cap, partials);
      break;
    case 1:
      k_expand<1><<<grid, kBlock, 0, stream>>>(g, plan, d, rows, off, piv, r, w_begin, w_end, out,
                                               cursor, out_cap, partials);
      break;
    default:
      k_expand<2><<<grid, kBlock, 0, stream>>>(g, plan, d, rows, off, piv, r, w_begin, w_end, out,
                                               cursor, out_cap, partials);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_reduce_counts(const unsigned long long* partials, int32_t nparts,
                                unsigned long long* total, uint32_t* overflow,
                                hipStream_t stream) {
  k_reduce_counts<<<1, kBlock, 0, stream>>>(partials, nparts, total, overflow);
  return hipGetLastError();
}

}  // namespace hpm
