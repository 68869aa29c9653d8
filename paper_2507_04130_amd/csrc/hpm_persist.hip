// hpm_persist.hip -- the batched form of the edge-centric search as one
// persistent launch draining a device work queue.
//
// Every pattern of a batch goes through the same steps as a single match --
// vertex validator (Sec. III-B, Alg. 2), arc scan against pattern arc (0,1)
// with state injection of the surviving arcs as depth-2 partial mappings
// (Sec. III-B Alg. 3, Sec. III-C Alg. 4), then extension one position at a
// time with full feasibility against every mapped position (Sec. II-A,
// Eq. (1)-(3)).  The validator bitmaps of all patterns come from one launch
// (k_batch_validate); everything after runs as tasks of one queue drained by
// one kernel of resident blocks (k_persist):
//
//   SCAN     (q, arc range)      survivors -> chunks of depth-2 rows
//   EXPAND   (q, d, row chunk, candidate range)
//                                rows of d positions -> chunks of d+1
//                                positions, or counts at the last position
//
// A block pops a task, runs it, pushes the tasks it creates (output chunks, or
// the rest of a chunk whose candidates exceed one task's share) and takes the
// next.  Nothing returns to the host between depths or patterns, so small
// patterns of a batch overlap freely with large ones.
//
// Coherence between blocks on different XCDs (each XCD has its own L2) uses
// agent-scope atomic loads and stores, which bypass the non-coherent L2, for
// everything one block writes and another reads during the launch: queue
// words, task descriptors and the partial-mapping rows.  Workgroup-scope
// fences (a wait for the block's own stores) order a block's row stores
// before the descriptor that publishes them; no agent-scope cache flush or
// invalidation is issued.
//
// Queue: a linear array of slots.  A producer reserves slots by compare-and-
// swap on `tail` (never past the capacity), stores the descriptors, and then
// each slot's ready flag; a consumer advances `head` by compare-and-swap only
// over a ready slot.  `pending` counts tasks queued or running: it is raised
// before a push is published and lowered after a task has pushed all its
// children, so it is zero only when all work is done.  A block leaves when
// `pending` is zero, or when it has found no task for `idle_ticks` of the
// wall clock (polling with growing sleeps), so every launch ends; the host
// launches again while work is left.  Every descriptor is checked against
// the batch's bounds before it is run.
//
// Memory: output rows go to a bump arena (256-byte aligned allocations).  A
// pattern whose chunk or task does not fit is marked and its remaining tasks
// are dropped; the host runs it again with the single-query path.
#include "hpm_internal.h"
#include "hpm_device.h"

namespace hpm {
namespace {

constexpr int kPMaxRows = 1024;    // rows of one EXPAND task (LDS offsets, pivots)
constexpr int kPRowInts = 4096;    // row entries of one task staged in LDS
constexpr int kPScanItems = 4;     // arcs per thread per scan tile
constexpr int kPScanTile = kBlock * kPScanItems;

typedef int32_t v4i __attribute__((ext_vector_type(4)));

// Agent-scope (cache-bypassing) loads and stores for data shared between
// blocks during the launch.
template <typename T>
__device__ __forceinline__ T ld_shared(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_shared(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Orders this thread's earlier memory operations before its later ones
// (waits for its stores), without cache maintenance.
__device__ __forceinline__ void order_release() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
}
__device__ __forceinline__ void order_acquire() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ void mark_failed(const PParams& P, int32_t q, uint32_t bit) {
  atomicOr(&P.pflags[q], bit);
}

// Reserve n slots; -1 when the queue would pass its capacity.
__device__ int64_t q_reserve(const PParams& P, int64_t n) {
  unsigned long long t = ld_shared(&P.st->tail);
  for (;;) {
    if ((int64_t)t + n > P.qcap) return -1;
    const unsigned long long seen = atomicCAS(&P.st->tail, t, t + (unsigned long long)n);
    if (seen == t) return (int64_t)t;
    t = seen;
  }
}

__device__ void store_task(PTask* s, const PTask& t) {
  st_shared(&s->type, t.type);
  st_shared(&s->q, t.q);
  st_shared(&s->d, t.d);
  st_shared(&s->nrows, t.nrows);
  st_shared(&s->a, t.a);
  st_shared(&s->b, t.b);
  st_shared(&s->w0, t.w0);
  st_shared(&s->w1, t.w1);
}

__device__ void load_task(const PTask* s, PTask* t) {
  t->ready = 1;
  t->type = ld_shared(&s->type);
  t->q = ld_shared(&s->q);
  t->d = ld_shared(&s->d);
  t->nrows = ld_shared(&s->nrows);
  t->a = ld_shared(&s->a);
  t->b = ld_shared(&s->b);
  t->w0 = ld_shared(&s->w0);
  t->w1 = ld_shared(&s->w1);
}

// Publish n descriptors (thread 0 of a block, after a block barrier that
// follows every store they refer to).  Returns false (and marks pattern q)
// when the queue is full.
__device__ bool q_push(const PParams& P, const PTask* tasks, int32_t n, int32_t q) {
  if (n == 0) return true;
  const int64_t t0 = q_reserve(P, n);
  if (t0 < 0) {
    atomicOr(&P.st->error, kPErrQueueFull);
    mark_failed(P, q, kPatFailed);
    return false;
  }
  __hip_atomic_fetch_add(&P.st->pending, (unsigned long long)n, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  for (int32_t i = 0; i < n; ++i) store_task(P.queue + t0 + i, tasks[i]);
  order_release();
  for (int32_t i = 0; i < n; ++i) st_shared(&P.queue[t0 + i].ready, 1);
  return true;
}

// Thread 0: take the next task into *out.  1 = task, 0 = all work done or no
// task for idle_ticks of the wall clock.
__device__ int q_pop(const PParams& P, PTask* out) {
  int32_t nap = 1;
  long long idle_since = -1;
  for (;;) {
    const unsigned long long h = ld_shared(&P.st->head);
    const unsigned long long t = ld_shared(&P.st->tail);
    if (h < t) {
      if (ld_shared(&P.queue[h].ready)) {
        if (atomicCAS(&P.st->head, h, h + 1) == h) {
          order_acquire();
          load_task(P.queue + h, out);
          return 1;
        }
        continue;
      }
    } else if (ld_shared(&P.st->pending) == 0ull) {
      return 0;
    }
    const long long now = wall_clock64();
    if (idle_since < 0) idle_since = now;
    if (now - idle_since > P.idle_ticks) {
      atomicOr(&P.st->error, kPErrIdleExit);
      return 0;
    }
    for (int32_t i = 0; i < nap; ++i) __builtin_amdgcn_s_sleep(1);
    if (nap < 32) nap <<= 1;
  }
}

// Bump allocation of `ints` int32 entries, rounded to 64 (256 bytes); -1 when
// the arena is exhausted.
__device__ int64_t arena_alloc(const PParams& P, int64_t ints) {
  const unsigned long long want = (unsigned long long)((ints + 63) & ~int64_t(63));
  const unsigned long long at = atomicAdd(&P.st->arena_top, want);
  if ((int64_t)(at + want) > P.arena_cap) return -1;
  return (int64_t)at;
}

struct PShared {
  PTask task;
  int32_t have;
  int32_t fail;
  // output chunk of the running task
  int64_t out_at;    // arena offset of the chunk (ints)
  int32_t out_cap;   // rows it holds
  int32_t out_fill;  // rows written
  unsigned long long scan[kWaves + 1];
  int64_t off[kPMaxRows + 1];
  int2 piv[kPMaxRows];
  int32_t rows[kPRowInts];
};

// Thread 0: publish the running task's output chunk (if it holds rows).
__device__ void flush_chunk(const PParams& P, PShared& S, int32_t q, int32_t width) {
  if (S.out_fill > 0 && !S.fail) {
    PTask t{};
    t.type = kTaskExpand;
    t.q = q;
    t.d = width;
    t.nrows = S.out_fill;
    t.a = S.out_at;
    t.w0 = 0;
    t.w1 = -1;
    if (!q_push(P, &t, 1, q)) S.fail = 1;
  }
  S.out_fill = 0;
  S.out_cap = 0;
}

// Block-wide: make room for `total` new rows of `width` entries; rows left
// to come in this task are at most `bound` (>= total).  Thread 0 publishes a
// full chunk and allocates the next; afterwards S.out_at / S.out_fill say
// where the block's rows go.  Returns false when the pattern has failed.
__device__ bool reserve_rows(const PParams& P, PShared& S, int32_t q, int32_t width,
                             int32_t total, int64_t bound) {
  if (threadIdx.x == 0 && !S.fail && total > 0 && S.out_fill + total > S.out_cap) {
    flush_chunk(P, S, q, width);
    if (!S.fail) {
      int64_t cap = bound < P.chunk_rows ? bound : P.chunk_rows;
      if (cap < total) cap = total;
      if (cap > kPMaxRows) cap = kPMaxRows;
      const int64_t at = arena_alloc(P, cap * width);
      if (at < 0) {
        atomicOr(&P.st->error, kPErrArenaFull);
        mark_failed(P, q, kPatFailed);
        S.fail = 1;
      } else {
        S.out_at = at;
        S.out_cap = (int32_t)cap;
        S.out_fill = 0;
      }
    }
  }
  __syncthreads();
  return !S.fail;
}

// ------------------------------------------------------------ validator

// Bitmaps of every position of every pattern (blockIdx.y = pattern): bit v of
// bitmap (q, p) set when v passes position p's vertex validator (predicates,
// in/out degree at least the pattern's).  64 consecutive vertices per
// wavefront step, two words per position.
__global__ __launch_bounds__(kBlock) void k_batch_validate(DevGraph g,
                                                           const DevPlan* __restrict__ plans,
                                                           uint32_t* __restrict__ bits,
                                                           const int64_t* __restrict__ bit_base,
                                                           int64_t words) {
  const int32_t q = blockIdx.y;
  const DevPlan* __restrict__ pl = plans + q;
  const int32_t k = pl->k;
  uint32_t* out = bits + bit_base[q];
  const int lane = threadIdx.x & 63;
  const int64_t vend = (int64_t)(g.n + 63) / 64 * 64;
  for (int64_t base = ((int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6)) * 64; base < vend;
       base += (int64_t)gridDim.x * kBlock) {
    const int64_t v = base + lane;
    const bool in = v < g.n;
    int32_t din = 0, dout = 0;
    if (in) {
      dout = g.out_off[v + 1] - g.out_off[v];
      din = g.in_off[v + 1] - g.in_off[v];
    }
    for (int p = 0; p < k; ++p) {
      const bool ok = in && din >= pl->pin[p] && dout >= pl->pout[p] &&
                      vertex_ok(g, pl, p, (int32_t)v);
      const uint64_t m = __ballot(ok);
      if (lane < 2) out[p * words + (base >> 5) + lane] = (uint32_t)(m >> (32 * lane));
    }
  }
}

// ------------------------------------------------------------ SCAN

__device__ void run_scan(const PParams& P, PShared& S, const PTask& t) {
  const int32_t q = t.q;
  const DevPlan* __restrict__ pl = P.plans + q;
  const DevGraph& g = P.g;
  const int32_t k = pl->k;
  const int fwd = pl->mve_forward;
  const int rev = pl->rev_rule;
  const int ps = fwd ? 0 : 1;
  const int pd = fwd ? 1 : 0;
  const uint32_t* bits0 = P.bits + P.bit_base[q];
  const uint32_t* bits1 = bits0 + P.words;
  const uint32_t* tbits = fwd ? bits0 : bits1;  // flags of the tail x
  const uint32_t* hbits = fwd ? bits1 : bits0;  // flags of the head y
  const uint32_t emask = pl->amask[ps][pd];
  unsigned long long count = 0;
  for (int64_t tb = t.a; tb < t.b; tb += kPScanTile) {
    const int64_t e0 = tb + (int64_t)threadIdx.x * kPScanItems;
    int32_t xs[kPScanItems], ys[kPScanItems];
    uint32_t keep = 0;
    if (e0 + kPScanItems <= t.b) {
      const v4i a = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(g.src + e0));
      const v4i b = __builtin_nontemporal_load(reinterpret_cast<const v4i*>(g.out_nbrs + e0));
      xs[0] = a.x; xs[1] = a.y; xs[2] = a.z; xs[3] = a.w;
      ys[0] = b.x; ys[1] = b.y; ys[2] = b.z; ys[3] = b.w;
      keep = 0xfu;
    } else {
#pragma unroll
      for (int j = 0; j < kPScanItems; ++j) {
        const bool in = e0 + j < t.b;
        xs[j] = in ? g.src[e0 + j] : 0;
        ys[j] = in ? g.out_nbrs[e0 + j] : 0;
        keep |= (uint32_t)in << j;
      }
    }
#pragma unroll
    for (int j = 0; j < kPScanItems; ++j)
      if (((keep >> j) & 1u) && !test_bit(tbits, xs[j])) keep &= ~(1u << j);
#pragma unroll
    for (int j = 0; j < kPScanItems; ++j)
      if (((keep >> j) & 1u) && !test_bit(hbits, ys[j])) keep &= ~(1u << j);
    if (emask) {
#pragma unroll
      for (int j = 0; j < kPScanItems; ++j)
        if (((keep >> j) & 1u) && !arc_ok(g, pl, ps, pd, (int32_t)(e0 + j))) keep &= ~(1u << j);
    }
    if (rev) {
#pragma unroll
      for (int j = 0; j < kPScanItems; ++j) {
        if (!((keep >> j) & 1u)) continue;
        const int32_t r = g.rev_eid[e0 + j];
        const bool ok = (rev == 1) ? (r >= 0 && arc_ok(g, pl, 1, 0, r)) : (r < 0);
        if (!ok) keep &= ~(1u << j);
      }
    }
    const int32_t cnt = __popc(keep);
    if (k == 2) {
      count += cnt;
      continue;
    }
    unsigned long long total;
    const unsigned long long excl =
        block_exclusive_scan<unsigned long long>((unsigned long long)cnt, S.scan, &total);
    if (total == 0) continue;
    if (!reserve_rows(P, S, q, 2, (int32_t)total, t.b - tb)) return;
    int32_t* out = P.arena + S.out_at + (int64_t)(S.out_fill + (int32_t)excl) * 2;
#pragma unroll
    for (int j = 0; j < kPScanItems; ++j) {
      if ((keep >> j) & 1u) {
        st_shared(out, fwd ? xs[j] : ys[j]);
        st_shared(out + 1, fwd ? ys[j] : xs[j]);
        out += 2;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) S.out_fill += (int32_t)total;
  }
  if (k == 2) {
    const unsigned long long tot = block_sum<unsigned long long>(count, S.scan);
    if (threadIdx.x == 0 && tot) {
      const unsigned long long old = atomicAdd(&P.counts[q], tot);
      if (old + tot < old) mark_failed(P, q, kPatOverflow);
    }
    return;
  }
  __syncthreads();
  if (threadIdx.x == 0) flush_chunk(P, S, q, 2);
}

// ------------------------------------------------------------ EXPAND

// Is there an arc u -> v?  Out-CSR id of the arc (or, when found through
// v's in-list, its in-CSR position with *via_in set), -1 if none.  strategy
// kStratShorter searches the shorter of out(u) and in(v); kStratMapped always
// searches the list of the mapped vertex (out(u) when u_mapped, else in(v)),
// which the row's candidates share.
__device__ __forceinline__ int32_t arc_lookup(const DevGraph& g, int32_t u, int32_t v,
                                              bool u_mapped, int strategy, bool* via_in) {
  bool use_in;
  if (strategy == kStratShorter)
    use_in = (g.in_off[v + 1] - g.in_off[v]) < (g.out_off[u + 1] - g.out_off[u]);
  else
    use_in = !u_mapped;
  *via_in = use_in;
  return use_in ? find_in(g.in_nbrs, g.in_off[v], g.in_off[v + 1], u)
                : find_in(g.out_nbrs, g.out_off[u], g.out_off[u + 1], v);
}

template <int ITEMS>
__device__ void run_expand(const PParams& P, PShared& S, const PTask& t) {
  const int32_t q = t.q;
  const DevPlan* __restrict__ pl = P.plans + q;
  const DevGraph& g = P.g;
  const int32_t k = pl->k;
  const int32_t d = t.d;       // positions mapped; position a = d is filled
  const int32_t a = d;
  const int32_t nrows = t.nrows;
  const int32_t* grows = P.arena + t.a;
  const uint32_t fw = pl->fwd[a], bw = pl->bwd[a];
  const bool iso = pl->mode == 0;
  const bool last = a == k - 1;
  const uint32_t* abits = P.bits + P.bit_base[q] + (int64_t)a * P.words;
  const bool rows_lds = nrows * d <= kPRowInts;
  constexpr int kTile = kBlock * ITEMS;
  auto row_at = [&](int32_t i, int x) -> int32_t {
    return rows_lds ? S.rows[i * d + x] : ld_shared(grows + (int64_t)i * d + x);
  };

  if (rows_lds)
    for (int32_t i = threadIdx.x; i < nrows * d; i += kBlock) S.rows[i] = ld_shared(grows + i);
  __syncthreads();
  // candidate source per row: the shortest list among the mapped neighbours
  // of position a (out(f(b)) for a pattern arc b -> a, in(f(b)) for a -> b)
  for (int32_t i = threadIdx.x; i < nrows; i += kBlock) {
    int32_t best = INT32_MAX, code = 0, base = 0;
    for (int b = 0; b < d; ++b) {
      if (!(((fw | bw) >> b) & 1u)) continue;
      const int32_t fb = row_at(i, b);
      if ((fw >> b) & 1u) {
        const int32_t lo = g.out_off[fb], L = g.out_off[fb + 1] - lo;
        if (L < best) { best = L; code = (b << 1) | 1; base = lo; }
      }
      if ((bw >> b) & 1u) {
        const int32_t lo = g.in_off[fb], L = g.in_off[fb + 1] - lo;
        if (L < best) { best = L; code = b << 1; base = lo; }
      }
    }
    S.piv[i] = make_int2(code, base);
    S.off[i + 1] = best == INT32_MAX ? 0 : best;
  }
  __syncthreads();
  // inclusive prefix sums of the list lengths into off[1..nrows]
  {
    unsigned long long carry = 0;
    for (int32_t base = 0; base < nrows; base += kBlock) {
      const int32_t i = base + threadIdx.x;
      const unsigned long long x = i < nrows ? (unsigned long long)S.off[i + 1] : 0ull;
      unsigned long long tot;
      const unsigned long long ex = block_exclusive_scan<unsigned long long>(x, S.scan, &tot);
      if (i < nrows) S.off[i + 1] = (int64_t)(carry + ex + x);
      carry += tot;
    }
    if (threadIdx.x == 0) S.off[0] = 0;
  }
  __syncthreads();
  const int64_t W = S.off[nrows];
  int64_t w0 = t.w0, w1 = t.w1;
  if (w1 < 0) {
    w0 = 0;
    w1 = W;
    if (W > P.task_work) {
      // the rest of this chunk's candidates become tasks of their own
      w1 = P.task_work;
      if (threadIdx.x == 0) {
        int64_t w = P.task_work;
        while (w < W && !S.fail) {
          int32_t n = 0;
          PTask buf[8];
          for (; n < 8 && w < W; ++n, w += P.task_work) {
            PTask s = t;
            s.w0 = w;
            s.w1 = w + P.task_work < W ? w + P.task_work : W;
            buf[n] = s;
          }
          if (!q_push(P, buf, n, q)) S.fail = 1;
        }
      }
    }
  }
  if (w0 < 0) w0 = 0;
  if (w1 > W) w1 = W;
  unsigned long long count = 0;
  for (int64_t tb = w0; tb < w1; tb += kTile) {
    int32_t cand[ITEMS], crow[ITEMS];
    uint32_t keep = 0;
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const int64_t w = tb + it * kBlock + threadIdx.x;
      int32_t i = 0, c = 0;
      bool ok = w < w1;
      if (ok) {
        int32_t lo = 0, hi = nrows - 1;  // last row with off[row] <= w
        while (lo < hi) {
          const int32_t mid = (lo + hi + 1) >> 1;
          if (S.off[mid] <= w)
            lo = mid;
          else
            hi = mid - 1;
        }
        i = lo;
        const int2 pv = S.piv[i];
        const int32_t b = pv.x >> 1;
        const bool via_out = (pv.x & 1) != 0;
        const int32_t pos = pv.y + (int32_t)(w - S.off[i]);
        c = via_out ? g.out_nbrs[pos] : g.in_nbrs[pos];
        ok = test_bit(abits, c);
        // the pivot arc's predicate
        if (ok) {
          if (via_out)
            ok = arc_ok(g, pl, b, a, pos);
          else
            ok = arc_ok_in(g, pl, a, b, pos);
        }
        for (int x = 0; x < d && ok; ++x) ok = row_at(i, x) != c;  // injectivity
        for (int x = 0; x < d && ok; ++x) {
          const int32_t fx = row_at(i, x);
          const bool arc_in = (fw >> x) & 1u;   // pattern arc x -> a
          const bool arc_out = (bw >> x) & 1u;  // pattern arc a -> x
          if ((arc_in && !(x == b && via_out)) || (!arc_in && iso)) {
            bool vin;
            const int32_t e = arc_lookup(g, fx, c, true, P.strategy, &vin);
            if (arc_in)
              ok = e >= 0 && (vin ? arc_ok_in(g, pl, x, a, e) : arc_ok(g, pl, x, a, e));
            else
              ok = e < 0;
          }
          if (ok && ((arc_out && !(x == b && !via_out)) || (!arc_out && iso))) {
            bool vin;
            const int32_t e = arc_lookup(g, c, fx, false, P.strategy, &vin);
            if (arc_out)
              ok = e >= 0 && (vin ? arc_ok_in(g, pl, a, x, e) : arc_ok(g, pl, a, x, e));
            else
              ok = e < 0;
          }
        }
      }
      cand[it] = c;
      crow[it] = i;
      keep |= (uint32_t)ok << it;
    }
    const int32_t cnt = __popc(keep);
    if (last) {
      count += cnt;
      continue;
    }
    unsigned long long total;
    const unsigned long long excl =
        block_exclusive_scan<unsigned long long>((unsigned long long)cnt, S.scan, &total);
    if (total == 0) continue;
    if (!reserve_rows(P, S, q, d + 1, (int32_t)total, w1 - tb)) return;
    int32_t* out = P.arena + S.out_at + (int64_t)(S.out_fill + (int32_t)excl) * (d + 1);
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      if ((keep >> it) & 1u) {
        for (int x = 0; x < d; ++x) st_shared(out + x, row_at(crow[it], x));
        st_shared(out + d, cand[it]);
        out += d + 1;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) S.out_fill += (int32_t)total;
  }
  if (last) {
    const unsigned long long tot = block_sum<unsigned long long>(count, S.scan);
    if (threadIdx.x == 0 && tot) {
      const unsigned long long old = atomicAdd(&P.counts[q], tot);
      if (old + tot < old) mark_failed(P, q, kPatOverflow);
    }
    return;
  }
  __syncthreads();
  if (threadIdx.x == 0) flush_chunk(P, S, q, d + 1);
}

// A descriptor inside the batch's bounds (anything else is never run).
__device__ bool task_ok(const PParams& P, const PTask& t) {
  if (t.q < 0 || t.q >= P.n_pat) return false;
  if (t.type == kTaskScan) return t.a >= 0 && t.a < t.b && t.b <= P.g.m;
  if (t.type != kTaskExpand) return false;
  const int32_t k = P.plans[t.q].k;
  return t.d >= 2 && t.d < k && t.nrows >= 1 && t.nrows <= kPMaxRows && t.a >= 0 &&
         t.a + (int64_t)t.nrows * t.d <= P.arena_cap && (t.w1 < 0 || t.w0 <= t.w1);
}

template <int ITEMS>
__global__ __launch_bounds__(kBlock) void k_persist(PParams P) {
  __shared__ PShared S;
  for (;;) {
    if (threadIdx.x == 0) {
      S.have = q_pop(P, &S.task);
      S.fail = 0;
      S.out_fill = 0;
      S.out_cap = 0;
    }
    __syncthreads();
    if (S.have <= 0) break;
    const PTask t = S.task;
    bool run = task_ok(P, t);
    if (!run && threadIdx.x == 0) {
      atomicOr(&P.st->error, kPErrBadTask);
      if (t.q >= 0 && t.q < P.n_pat) mark_failed(P, t.q, kPatFailed);
    }
    if (run) run = (ld_shared(&P.pflags[t.q]) & kPatFailed) == 0;
    if (run) {
      if (t.type == kTaskScan)
        run_scan(P, S, t);
      else
        run_expand<ITEMS>(P, S, t);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      atomicAdd(&P.st->tasks[t.type & 3], 1ull);
      // children are published; this task is done
      __hip_atomic_fetch_add(&P.st->pending, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace

hipError_t launch_batch_validate(const DevGraph& g, const DevPlan* plans, uint32_t* bits,
                                 const int64_t* bit_base, int64_t words, int32_t n_pat,
                                 hipStream_t stream) {
  const int64_t spans = ((int64_t)g.n + 63) / 64;
  int64_t bx = (spans + kWaves - 1) / kWaves;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(k_batch_validate, dim3((unsigned)bx, (unsigned)n_pat), dim3(kBlock), 0,
                     stream, g, plans, bits, bit_base, words);
  return hipGetLastError();
}

int persist_blocks_per_cu(int items) {
  int nb = 0;
  hipError_t e;
  if (items == 1)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<1>, kBlock, 0);
  else if (items == 2)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<2>, kBlock, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist<4>, kBlock, 0);
  return e == hipSuccess ? nb : 0;
}

hipError_t launch_persist(const PParams& P, int items, int grid, hipStream_t stream) {
  if (items == 1)
    hipLaunchKernelGGL(k_persist<1>, dim3(grid), dim3(kBlock), 0, stream, P);
  else if (items == 2)
    hipLaunchKernelGGL(k_persist<2>, dim3(grid), dim3(kBlock), 0, stream, P);
  else
    hipLaunchKernelGGL(k_persist<4>, dim3(grid), dim3(kBlock), 0, stream, P);
  return hipGetLastError();
}

}  // namespace hpm
