// hpm_runtime.hip -- host side of libhpm: C ABI, graph store, pattern plan and
// the chunked depth scheduler.  All matching arithmetic runs in the kernels of
// hpm_kernels.hip; this file validates inputs, orders the pattern, sizes
// scratch memory and sequences launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstddef>
#include <cstring>
#include <memory>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hpm.h"
#include "hpm_internal.h"

namespace {

using hpm::DevGraph;
using hpm::DevPlan;
using hpm::kMaxCols;
using hpm::kMaxK;
using hpm::PParams;
using hpm::PState;
using hpm::PTask;
using hpm::kPatFailed;
using hpm::kPatOverflow;
using hpm::kTaskScan;
using hpm::launch_batch_validate;
using hpm::launch_persist;
using hpm::persist_blocks_per_cu;

thread_local std::string t_error;
thread_local hpm_match_stats t_stats;
thread_local hpm_batch_stats t_bstats;

struct Failure {
  int status;
  std::string msg;
};

[[noreturn]] void fail(int status, const std::string& msg) { throw Failure{status, msg}; }

void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  (void)hipGetLastError();
  const int st = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? HPM_E_NOMEM
                                                                             : HPM_E_DEVICE;
  fail(st, std::string(what) + ": " + hipGetErrorString(e));
}

template <class F>
int guarded(F&& f) {
  try {
    t_error.clear();
    return f();
  } catch (const Failure& e) {
    t_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    t_error = "host allocation failed";
    return HPM_E_NOMEM;
  } catch (const std::exception& e) {
    t_error = e.what();
    return HPM_E_INTERNAL;
  } catch (...) {
    t_error = "unknown internal error";
    return HPM_E_INTERNAL;
  }
}

// Bump allocation from a fixed device region (the allocation-free entry
// point): regions are handed out in 256-byte units and never returned; a
// call resets it before it starts.
struct Carve {
  char* base = nullptr;
  size_t size = 0, used = 0;
  void* take(size_t want) {
    const size_t n = (want + 255) / 256 * 256;
    if (n > size - used)
      fail(HPM_E_NOMEM, "the call needs more than the " + std::to_string(size >> 20) +
                            " MiB of allocation-free scratch");
    void* p = base + used;
    used += n;
    return p;
  }
};
// Set for the duration of an allocation-free call on this thread.
thread_local Carve* t_carve = nullptr;

// Owned device allocation that can grow.  While t_carve is set, growth takes
// a new region from it (at least twice the old size) instead of hipMalloc.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool carved = false;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p && !carved) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    carved = false;
  }
  // Make room for at least `want` bytes; contents are not preserved.
  void ensure(size_t want, hipStream_t stream) {
    if (want <= bytes) return;
    if (t_carve) {
      // the old region stays valid for work already queued on it
      const size_t n = std::max(want, 2 * bytes);
      if (p && !carved) fail(HPM_E_INTERNAL, "allocation-free call on an allocated buffer");
      p = t_carve->take(n);
      bytes = n;
      carved = true;
      return;
    }
    if (p) {
      hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
      release();
    }
    hip_check(hipMalloc(&p, want), "hipMalloc");
    bytes = want;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

// Per-call scratch.  Pooled per graph so that concurrent calls (different
// streams) never share one, and repeated calls reuse allocations.
struct Workspace {
  DevBuf plan, vbits, counters, partials, blkcount, blkprefix, rows2, rows2d;
  DevBuf off[kMaxK], piv[kMaxK], bsum[kMaxK], rows[kMaxK];
  // pivot-list filter: per depth the filtered lists and the rows' new prefix
  // sums; shared by all depths the hash table and slot descriptors
  DevBuf fpool[kMaxK], off2[kMaxK];
  DevBuf fkeys, frep, fdense, fslot_key, fslot_rep, fslot_region, fcount;
  // the filter's pieces: per-group prefix sums, per-piece counts and groups,
  // and the staging area of groups split over several blocks
  DevBuf fpbase, fpbsum, fpcnt, fpslot, fpdesc, ftmp;
  // count pass: list lengths left to the tiled last level, and their block sums
  DevBuf crest, cbsum;
  // per depth: prefix sums of short-row lengths and of long-row tile counts
  DevBuf soff[kMaxK], toff[kMaxK], sbsum[kMaxK], tbsum[kMaxK];
  // frontier look-ahead: the rows of each depth that pass it
  DevBuf la[kMaxK];
  // arc-predicate index: arc positions, block sums, and the restricted
  // out- and in-adjacency with their attribute columns
  DevBuf amask, awpre, absum, aoff_out, anbrs_out, aoff_in, anbrs_in;
  DevBuf acol_out[kMaxCols], acol_in[kMaxCols];
  unsigned long long* host = nullptr;  // pinned readback slots
  DevPlan* host_plan = nullptr;        // pinned staging for the plan upload
  std::vector<hipEvent_t> events;
  ~Workspace() {
    if (host) (void)hipHostFree(host);
    if (host_plan) (void)hipHostFree(host_plan);
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
  }
  size_t held() const {
    size_t s = plan.bytes + vbits.bytes + counters.bytes + partials.bytes +
               blkcount.bytes + blkprefix.bytes + rows2.bytes + rows2d.bytes +
               fkeys.bytes + frep.bytes + fdense.bytes + fslot_key.bytes + fslot_rep.bytes +
               fslot_region.bytes + fcount.bytes + fpbase.bytes + fpbsum.bytes + fpcnt.bytes +
               fpslot.bytes + fpdesc.bytes + ftmp.bytes + crest.bytes + cbsum.bytes +
               amask.bytes + awpre.bytes + absum.bytes + aoff_out.bytes + anbrs_out.bytes + aoff_in.bytes +
               anbrs_in.bytes;
    for (int c = 0; c < kMaxCols; ++c) s += acol_out[c].bytes + acol_in[c].bytes;
    for (int d = 0; d < kMaxK; ++d)
      s += off[d].bytes + piv[d].bytes + bsum[d].bytes + rows[d].bytes + fpool[d].bytes +
           off2[d].bytes + soff[d].bytes + toff[d].bytes + sbsum[d].bytes + tbsum[d].bytes +
           la[d].bytes;
    return s;
  }
  void release_all() {
    plan.release(); vbits.release(); counters.release(); partials.release();
    blkcount.release(); blkprefix.release(); rows2.release(); rows2d.release();
    fkeys.release(); frep.release(); fdense.release(); fslot_key.release(); fslot_rep.release();
    fslot_region.release();
    fcount.release();
    fpbase.release(); fpbsum.release(); fpcnt.release(); fpslot.release(); fpdesc.release();
    ftmp.release();
    crest.release(); cbsum.release();
    amask.release(); awpre.release(); absum.release(); aoff_out.release(); anbrs_out.release();
    aoff_in.release(); anbrs_in.release();
    for (int c = 0; c < kMaxCols; ++c) {
      acol_out[c].release();
      acol_in[c].release();
    }
    for (int d = 0; d < kMaxK; ++d) {
      off[d].release(); piv[d].release(); bsum[d].release(); rows[d].release();
      fpool[d].release(); off2[d].release();
      soff[d].release(); toff[d].release(); sbsum[d].release(); tbsum[d].release();
      la[d].release();
    }
  }
};

// Scratch of one persistent batched launch: plans, validator bitmaps, the
// work queue, the row arena and per-pattern results.
struct BatchSpace {
  DevBuf plans, bits, bit_base, queue, arena, state, counts, pflags;
  unsigned long long* host_counts = nullptr;  // pinned readback
  uint32_t* host_flags = nullptr;
  PState* host_state = nullptr;
  size_t host_n = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~BatchSpace() {
    if (host_counts) (void)hipHostFree(host_counts);
    if (host_flags) (void)hipHostFree(host_flags);
    if (host_state) (void)hipHostFree(host_state);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  size_t held() const {
    return plans.bytes + bits.bytes + bit_base.bytes + queue.bytes + arena.bytes + state.bytes +
           counts.bytes + pflags.bytes;
  }
};

}  // namespace

struct hpm_graph {
  int device = 0;
  int num_cus = 256;
  int32_t n = 0;
  int64_t m = 0;
  int32_t n_vcols = 0, n_ecols = 0;
  DevBuf out_off, out_nbrs, in_off, in_nbrs, src, in_eid, rev_eid;
  DevBuf vcols[kMaxCols], ecols[kMaxCols], ecols_in[kMaxCols];
  std::mutex mu;
  std::vector<Workspace*> pool;
  std::vector<BatchSpace*> bpool;  // scratch of persistent batched launches
  // Host-side statistics for frontier-size estimates (serving admission):
  // sorted evenly spaced samples of every attribute column and the
  // size-biased mean out- and in-degree (sum d^2 / sum d).
  std::vector<int32_t> vsample[kMaxCols], esample[kMaxCols];
  double sb_out = 0.0, sb_in = 0.0;

  ~hpm_graph() {
    for (Workspace* w : pool) delete w;
    for (BatchSpace* b : bpool) delete b;
  }
  uint64_t bytes() const {
    uint64_t s = out_off.bytes + out_nbrs.bytes + in_off.bytes + in_nbrs.bytes + src.bytes +
                 in_eid.bytes + rev_eid.bytes;
    for (int c = 0; c < kMaxCols; ++c) s += vcols[c].bytes + ecols[c].bytes + ecols_in[c].bytes;
    return s;
  }
  DevGraph view() const {
    DevGraph g{};
    g.n = n;
    g.m = (int32_t)m;
    g.out_off = out_off.as<int32_t>();
    g.out_nbrs = out_nbrs.as<int32_t>();
    g.in_off = in_off.as<int32_t>();
    g.in_nbrs = in_nbrs.as<int32_t>();
    g.src = src.as<int32_t>();
    g.in_eid = in_eid.as<int32_t>();
    g.rev_eid = rev_eid.as<int32_t>();
    g.n_vcols = n_vcols;
    g.n_ecols = n_ecols;
    for (int c = 0; c < kMaxCols; ++c) {
      g.vcol[c] = vcols[c].as<int32_t>();
      g.ecol[c] = ecols[c].as<int32_t>();
      g.ecol_in[c] = ecols_in[c].as<int32_t>();
    }
    return g;
  }
};

namespace {

// ------------------------------------------------------------ graph ingest

std::vector<int32_t> narrow_offsets(const int64_t* off, int32_t n, int64_t m, const char* name) {
  if (off[0] != 0) fail(HPM_E_GRAPH, std::string(name) + "[0] must be 0");
  std::vector<int32_t> out((size_t)n + 1);
  for (int64_t i = 0; i <= n; ++i) {
    if (i > 0 && off[i] < off[i - 1])
      fail(HPM_E_GRAPH, std::string(name) + " decreases at " + std::to_string(i));
    if (off[i] > m) fail(HPM_E_GRAPH, std::string(name) + " exceeds m at " + std::to_string(i));
    out[i] = (int32_t)off[i];
  }
  if (off[n] != m) fail(HPM_E_GRAPH, std::string(name) + "[n] must equal m");
  return out;
}

constexpr int64_t kSampleSize = 4096;

// Sorted values at kSampleSize evenly spaced positions of a column.
std::vector<int32_t> column_sample(const int32_t* col, int64_t len) {
  const int64_t s = std::min<int64_t>(len, kSampleSize);
  std::vector<int32_t> out((size_t)s);
  for (int64_t j = 0; j < s; ++j) out[(size_t)j] = col[j * len / s];
  std::sort(out.begin(), out.end());
  return out;
}

double size_biased_degree(const std::vector<int32_t>& off) {
  double s1 = 0.0, s2 = 0.0;
  for (size_t i = 1; i < off.size(); ++i) {
    const double d = (double)(off[i] - off[i - 1]);
    s1 += d;
    s2 += d * d;
  }
  return s1 > 0.0 ? s2 / s1 : 0.0;
}

void upload(DevBuf& b, const void* host, size_t bytes, hipStream_t stream) {
  b.ensure(bytes ? bytes : 4, stream);
  if (bytes) hip_check(hipMemcpyAsync(b.p, host, bytes, hipMemcpyHostToDevice, stream), "upload");
}

std::string graph_error_text(uint32_t bits) {
  std::string s;
  if (bits & hpm::kErrRange) s += "neighbour id out of range; ";
  if (bits & hpm::kErrSelfLoop) s += "self-loop; ";
  if (bits & hpm::kErrUnsorted) s += "adjacency row not strictly ascending (unsorted or repeated arc); ";
  if (bits & hpm::kErrTranspose) s += "in-CSR is not the transpose of the out-CSR; ";
  return s;
}

// ------------------------------------------------------------ pattern plan

struct PatternInfo {
  int32_t k = 0;
  std::vector<int32_t> src, dst;
  std::vector<int32_t> indeg, outdeg;
  std::vector<uint8_t> adj;  // [k*k], adj[a*k+b] = arc a->b
};

PatternInfo check_pattern(const hpm_pattern* p, int32_t n_vcols, int32_t n_ecols) {
  if (!p) fail(HPM_E_ARG, "pattern is NULL");
  if (p->k < 2 || p->k > kMaxK)
    fail(HPM_E_PATTERN, "pattern must have 2.." + std::to_string(kMaxK) + " vertices");
  const int32_t k = p->k;
  if (p->n_arcs < 1 || p->n_arcs > k * (k - 1)) fail(HPM_E_PATTERN, "bad number of pattern arcs");
  if (!p->src || !p->dst) fail(HPM_E_ARG, "pattern arc arrays are NULL");
  if (n_vcols < 0 || n_vcols > kMaxCols || n_ecols < 0 || n_ecols > kMaxCols)
    fail(HPM_E_ARG, "column counts out of range");
  PatternInfo info;
  info.k = k;
  info.adj.assign((size_t)k * k, 0);
  info.indeg.assign(k, 0);
  info.outdeg.assign(k, 0);
  for (int32_t i = 0; i < p->n_arcs; ++i) {
    const int32_t a = p->src[i], b = p->dst[i];
    if (a < 0 || a >= k || b < 0 || b >= k) fail(HPM_E_PATTERN, "pattern arc endpoint out of range");
    if (a == b) fail(HPM_E_PATTERN, "pattern self-loop");
    if (info.adj[(size_t)a * k + b]) fail(HPM_E_PATTERN, "repeated pattern arc");
    info.adj[(size_t)a * k + b] = 1;
    info.outdeg[a]++;
    info.indeg[b]++;
    info.src.push_back(a);
    info.dst.push_back(b);
  }
  // weakly connected
  std::vector<char> seen(k, 0);
  std::vector<int32_t> stack{0};
  seen[0] = 1;
  int32_t nseen = 1;
  while (!stack.empty()) {
    const int32_t x = stack.back();
    stack.pop_back();
    for (int32_t y = 0; y < k; ++y)
      if (!seen[y] && (info.adj[(size_t)x * k + y] || info.adj[(size_t)y * k + x])) {
        seen[y] = 1;
        ++nseen;
        stack.push_back(y);
      }
  }
  if (nseen != k) fail(HPM_E_PATTERN, "pattern is not weakly connected");
  auto check_ops = [](const int32_t* op, const int32_t* val, int64_t count, const char* what) {
    if (!op || count == 0) return;
    if (!val) fail(HPM_E_ARG, std::string(what) + " values are NULL");
    for (int64_t i = 0; i < count; ++i)
      if (op[i] < HPM_ANY || op[i] > HPM_GE) fail(HPM_E_PATTERN, std::string("bad ") + what + " op");
  };
  check_ops(p->vop, p->vval, (int64_t)k * n_vcols, "vertex predicate");
  check_ops(p->eop, p->eval, (int64_t)p->n_arcs * n_ecols, "arc predicate");
  return info;
}

// Matching order (position -> original vertex), Sec. III-A, Alg. 1: rank
// sigma(v) = (total degree, out-degree); start at the best-ranked vertex; then
// take the best-ranked unplaced out-neighbour of the last placed vertex; if it
// has none, the best-ranked unplaced vertex adjacent to any placed vertex
// (keeps each position after the first connected to an earlier one, so the
// first two positions always form a pattern arc).  Ties: smaller id.
// With HPM_F_NO_REORDER: vertex 0 first, then the smallest-id unplaced vertex
// adjacent to the placed ones.
std::vector<int32_t> plan_order(const PatternInfo& P, uint32_t flags) {
  const int32_t k = P.k;
  auto better = [&](int32_t v, int32_t w) {  // is v ranked above w?
    const int32_t tv = P.indeg[v] + P.outdeg[v], tw = P.indeg[w] + P.outdeg[w];
    if (tv != tw) return tv > tw;
    if (P.outdeg[v] != P.outdeg[w]) return P.outdeg[v] > P.outdeg[w];
    return v < w;
  };
  auto adjacent = [&](int32_t a, int32_t b) {
    return P.adj[(size_t)a * k + b] || P.adj[(size_t)b * k + a];
  };
  std::vector<int32_t> order;
  std::vector<char> placed(k, 0);
  const bool natural = (flags & HPM_F_NO_REORDER) != 0;
  int32_t first = 0;
  if (!natural)
    for (int32_t v = 1; v < k; ++v)
      if (better(v, first)) first = v;
  order.push_back(first);
  placed[first] = 1;
  while ((int32_t)order.size() < k) {
    int32_t pick = -1;
    if (!natural) {
      const int32_t u = order.back();
      for (int32_t w = 0; w < k; ++w)
        if (!placed[w] && P.adj[(size_t)u * k + w] && (pick < 0 || better(w, pick))) pick = w;
    }
    if (pick < 0) {
      for (int32_t w = 0; w < k; ++w) {
        if (placed[w]) continue;
        bool touches = false;
        for (int32_t x : order) touches = touches || adjacent(w, x);
        if (!touches) continue;
        if (pick < 0 || (natural ? w < pick : better(w, pick))) pick = w;
      }
    }
    order.push_back(pick);
    placed[pick] = 1;
  }
  return order;
}

void set_range(int32_t op, int32_t val, int32_t* lo, int32_t* hi) {
  if (op == HPM_EQ) {
    *lo = val;
    *hi = val;
  } else {  // HPM_GE
    *lo = val;
    *hi = INT32_MAX;
  }
}

DevPlan build_dev_plan(const hpm_pattern* p, const PatternInfo& P, const std::vector<int32_t>& order,
                       int32_t n_vcols, int32_t n_ecols, int mode) {
  const int32_t k = P.k;
  DevPlan d;
  std::memset(&d, 0, sizeof(d));
  d.k = k;
  d.mode = mode;
  std::vector<int32_t> pos(k);
  for (int32_t i = 0; i < k; ++i) pos[order[i]] = i;
  for (int32_t i = 0; i < k; ++i) {
    const int32_t v = order[i];
    d.orig[i] = v;
    d.pin[i] = P.indeg[v];
    d.pout[i] = P.outdeg[v];
    for (int c = 0; c < kMaxCols; ++c) {
      d.vlo[i][c] = INT32_MIN;
      d.vhi[i][c] = INT32_MAX;
    }
    if (p->vop)
      for (int32_t c = 0; c < n_vcols; ++c) {
        const int32_t op = p->vop[(size_t)v * n_vcols + c];
        if (op == HPM_ANY) continue;
        d.vmask[i] |= 1u << c;
        set_range(op, p->vval[(size_t)v * n_vcols + c], &d.vlo[i][c], &d.vhi[i][c]);
      }
  }
  for (size_t i = 0; i < P.src.size(); ++i) {
    const int32_t ps = pos[P.src[i]], pt = pos[P.dst[i]];
    if (ps < pt)
      d.fwd[pt] |= 1u << ps;
    else
      d.bwd[ps] |= 1u << pt;
    for (int c = 0; c < kMaxCols; ++c) {
      d.alo[ps][pt][c] = INT32_MIN;
      d.ahi[ps][pt][c] = INT32_MAX;
    }
    if (p->eop)
      for (int32_t c = 0; c < n_ecols; ++c) {
        const int32_t op = p->eop[i * n_ecols + c];
        if (op == HPM_ANY) continue;
        d.amask[ps][pt] |= 1u << c;
        set_range(op, p->eval[i * n_ecols + c], &d.alo[ps][pt][c], &d.ahi[ps][pt][c]);
      }
  }
  const bool a01 = P.adj[(size_t)order[0] * k + order[1]] != 0;
  const bool a10 = P.adj[(size_t)order[1] * k + order[0]] != 0;
  if (!a01 && !a10) fail(HPM_E_INTERNAL, "first two positions are not adjacent");
  d.mve_forward = a01 ? 1 : 0;
  if (a01 && a10)
    d.rev_rule = 1;
  else
    d.rev_rule = (mode == HPM_ISO) ? 2 : 0;
  return d;
}

// ------------------------------------------------------------ matcher

// Device counter slots (and the pinned host slots they are read into).
enum : int {
  kCntTotal = 0, kCntOverflow = 1, kCntEmit = 2, kCntCursor = 3,
  kCntSlots = 4,        // host slot of read_i64
  kCntFilterSlots = 8,  // 8, 9: groups and pool entries; 10..12: keys of the filter tables
  kHostPieces = 13,     // host slot 13: blocks of the filter's list pass
  kHostSplit = 14,      // host slots 14, 15: short work and long tiles of a split
  kCntNum = 16          // counter slots on the device and in pinned host memory
};

// Split rows into packed short rows and row-aligned long rows only when a
// depth has at least this many candidates.
constexpr int64_t kSplitMinWork = int64_t(1) << 22;

// Induced isomorphism counts filtered rows from their lists (subtracting the
// neighbours of images they must not touch) only when the rows average at
// least this many candidates.
constexpr int64_t kCountMinPerRow = 64;

// Pre-filter pivot lists only when a depth has at least this many candidates.
constexpr int64_t kFilterMinWork = int64_t(1) << 22;

double sample_fraction(const std::vector<int32_t>& smp, int32_t lo, int32_t hi);

struct Matcher {
  hpm_graph* G;
  Workspace* W;
  hipStream_t stream;
  DevGraph g;   // the adjacency the validator and the extension read
  DevGraph gs;  // the whole graph, read by the arc scan
  DevPlan host_plan;
  int32_t k;
  int32_t* maps;
  uint64_t cap;
  bool timing;
  bool filter;
  int max_grid;
  uint32_t timed_kinds = 0x1ffu;  // families timed when timing (bit = HPM_K_*)
  int64_t cap2 = 0;     // depth-2 rows per arc chunk
  int64_t chunk = 0;    // rows per frontier chunk at depth >= 3
  uint64_t budget = 0;  // scratch limit of the call
  uint64_t limit = 0;   // stop once this many embeddings are found (0 = all)
  bool stopped = false;
  uint32_t done[kMaxK] = {};  // per depth: relations the pre-filtered lists enforce
  int32_t overlap_need = 0;   // common neighbours of positions 0 and 1 (overlap test on)
  bool lookahead = false;     // frontier look-ahead on the rows of every depth
  bool indexed = false;       // g reads the arc-predicate index
  bool want_index = false;    // consider the index once the first arc chunk is scanned
  uint32_t call_flags = 0;
  // survivors only: the depth-2 rows after the validators are copied to
  // surv_out ([surv_cap][2], positions 0 and 1) and nothing is extended
  int32_t* surv_out = nullptr;
  uint64_t surv_cap = 0;
  bool survivors_only = false;
  hpm_match_stats st{};
  struct Pending {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  size_t next_event = 0;

  // Scratch this call asked for, per buffer (the largest size), and in total:
  // the budget bounds this, not the idle buffers the workspace kept from
  // earlier calls.
  std::unordered_map<const DevBuf*, size_t> req;
  uint64_t planned = 0;

  void need(DevBuf& b, size_t want) {
    size_t& r = req[&b];
    if (want > r) {
      planned += want - r;
      r = want;
    }
    b.ensure(want, stream);
  }
  // Growth of the call's scratch if it asked b for `want` bytes.
  uint64_t extra(const DevBuf& b, size_t want) const {
    const auto it = req.find(&b);
    const size_t r = it == req.end() ? 0 : it->second;
    return want > r ? want - r : 0;
  }

  DevPlan* dplan() const { return W->plan.as<DevPlan>(); }
  int64_t bit_words() const { return (G->n + 63) / 64 * 2; }
  uint32_t* bits(int p) const { return W->vbits.as<uint32_t>() + p * bit_words(); }
  uint32_t* bits0() const { return bits(0); }
  uint32_t* bits1() const { return bits(1); }
  unsigned long long* counters() const { return W->counters.as<unsigned long long>(); }

  hipEvent_t event() {
    if (next_event == W->events.size()) {
      hipEvent_t e;
      hip_check(hipEventCreate(&e), "hipEventCreate");
      W->events.push_back(e);
    }
    return W->events[next_event++];
  }

  template <class L>
  void launch(int kind, L&& fn) {
    hipEvent_t a = nullptr, b = nullptr;
    const bool timed = timing && ((timed_kinds >> kind) & 1u);
    if (timed) {
      a = event();
      hip_check(hipEventRecord(a, stream), "hipEventRecord");
    }
    hip_check(fn(), "kernel launch");
    if (timed) {
      b = event();
      hip_check(hipEventRecord(b, stream), "hipEventRecord");
      pending.push_back({kind, a, b});
    }
    st.kernel_launches[kind]++;
  }

  // Synchronise the stream, fold pending event timings into the stats.
  void sync() {
    hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
    for (const Pending& p : pending) {
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, p.a, p.b), "hipEventElapsedTime");
      st.kernel_ms[p.kind] += ms;
    }
    pending.clear();
    next_event = 0;
  }

  unsigned long long read_counter(int slot) {
    hip_check(hipMemcpyAsync(W->host + slot, counters() + slot, sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, stream),
              "readback");
    sync();
    return W->host[slot];
  }
  // Total and overflow flag in one readback.
  uint64_t read_total() {
    static_assert(kCntOverflow == kCntTotal + 1, "adjacent counter slots");
    hip_check(hipMemcpyAsync(W->host + kCntTotal, counters() + kCntTotal,
                             2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream),
              "readback");
    sync();
    if (W->host[kCntOverflow]) fail(HPM_E_OVERFLOW, "embedding count exceeds 2^64-1");
    return W->host[kCntTotal];
  }
  int64_t read_i64(const int64_t* p) {
    hip_check(hipMemcpyAsync(W->host + kCntSlots, p, sizeof(int64_t), hipMemcpyDeviceToHost, stream),
              "readback");
    sync();
    return (int64_t)W->host[kCntSlots];
  }
  void zero_counter(int slot) {
    hip_check(hipMemsetAsync(counters() + slot, 0, sizeof(unsigned long long), stream), "memset");
  }

  int grid_for(int64_t items, int64_t per_block) const {
    int64_t b = (items + per_block - 1) / per_block;
    b = std::max<int64_t>(8, std::min<int64_t>(b, max_grid));
    return (int)((b + 7) / 8 * 8);  // tile mapping needs a multiple of the 8 XCDs
  }

  void ensure_depth(int32_t d, int64_t r_cap) {
    const int64_t nb = (r_cap + hpm::kPivotTile - 1) / hpm::kPivotTile;
    need(W->off[d], (size_t)(r_cap + 1) * sizeof(int64_t));
    need(W->piv[d], (size_t)std::max<int64_t>(r_cap, 1) * sizeof(int2));
    need(W->bsum[d], (size_t)(nb + 1) * sizeof(int64_t));
  }

  // Point rows whose pivot list has >= kFilterMinLen entries at a filtered copy
  // of that list, one per group of rows (launch_filter_insert and
  // launch_filter_groups form the groups).  With two or more positions
  // related to the new one, rows are first grouped by the images of all of
  // them (the filtered list then holds exactly the candidates that satisfy
  // every relation with those positions), and for induced isomorphism first
  // by those plus every earlier position but the last; if those groups are
  // not shared enough, by pivot list.  On success *offp / *fpool / *work
  // describe the new candidate ranges and done[d] the relations the lists
  // enforce; otherwise nothing changes.
  void filter_pivots(int32_t d, const int32_t* rows, int64_t r, int2* piv, const int64_t* off,
                     const int64_t** offp, const int32_t** fpool, int64_t* work) {
    const int64_t max_long = std::min<int64_t>(r, *work / hpm::kFilterMinLen);
    if (max_long == 0) return;
    uint32_t H = 1024;
    while ((int64_t)H < 2 * max_long) H <<= 1;
    // Candidate keys besides the pivot list: the positions tied to the new one
    // by a pattern arc (table 1) and, for induced isomorphism, those plus every
    // earlier position but the last (table 2: the filter then also enforces
    // their non-arcs).  A key of all mapped positions would make every row
    // its own group.
    const uint32_t all = (1u << d) - 1u;
    const uint32_t related = (host_plan.fwd[d] | host_plan.bwd[d]) & all;
    uint32_t masks[3] = {0u, 0u, 0u};
    if (__builtin_popcount(related) >= 2 && related != all) masks[1] = related;
    if (host_plan.mode == HPM_ISO && d >= 3) {
      const uint32_t wide = related | ((1u << (d - 1)) - 1u);
      if (wide != all && wide != related) masks[2] = wide;
    }
    const size_t T = masks[2] ? 3 : (masks[1] ? 2 : 1);
    const bool grouped = masks[1] || masks[2];
    const uint64_t table_bytes =
        extra(W->fkeys, T * H * 8) + (grouped ? extra(W->frep, (size_t)H * 4) : 0) +
        extra(W->fdense, (size_t)H * 4) + extra(W->fslot_key, (size_t)H * 8) +
        (grouped ? extra(W->fslot_rep, (size_t)H * 4) : 0) + extra(W->fslot_region, (size_t)H * 8);
    if (planned + table_bytes > budget) return;
    need(W->fkeys, T * H * 8);
    if (grouped) {
      need(W->frep, (size_t)H * 4);
      need(W->fslot_rep, (size_t)H * 4);
    }
    need(W->fdense, (size_t)H * 4);
    need(W->fslot_key, (size_t)H * 8);
    need(W->fslot_region, (size_t)H * 8);
    auto* keys = W->fkeys.as<unsigned long long>();
    unsigned long long* cnt = counters() + kCntFilterSlots;
    hip_check(hipMemsetAsync(keys, 0xff, T * H * 8, stream), "memset");
    hip_check(hipMemsetAsync(cnt, 0, 5 * sizeof(unsigned long long), stream), "memset");
    // The wider keys' tables first; the pivot-list table only when neither
    // is used (or there is none).
    auto insert = [&](uint32_t tables) {
      launch(HPM_K_FILTER, [&] {
        return hpm::launch_filter_insert(rows, (int32_t)r, d, piv, off, hpm::kFilterMinLen,
                                         masks[1], masks[2], tables, keys, H, cnt + 2, stream);
      });
    };
    insert(grouped ? 6u : 1u);
    int64_t distinct[3] = {0, 0, 0};
    if (grouped) {
      hip_check(hipMemcpyAsync(W->host + kCntFilterSlots + 2, cnt + 2,
                               3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, stream),
                "readback");
      sync();
      for (int t = 0; t < 3; ++t) distinct[t] = (int64_t)W->host[kCntFilterSlots + 2 + t];
    }
    // Number one table's groups; filtering reads every group's list once
    // more, so it pays when the groups are shared: their total length must be
    // well below the depth's work.
    int64_t nslots = 0, pool = 0;
    auto groups = [&](int t) -> bool {
      const uint32_t m = masks[t];
      hip_check(hipMemsetAsync(cnt, 0, 2 * sizeof(unsigned long long), stream), "memset");
      if (t) hip_check(hipMemsetAsync(W->frep.p, 0x7f, (size_t)H * 4, stream), "memset");
      launch(HPM_K_FILTER, [&] {
        return hpm::launch_filter_groups(g, rows, (int32_t)r, d, piv, off, hpm::kFilterMinLen, m,
                                         keys + (size_t)t * H, H,
                                         t ? W->frep.as<int32_t>() : nullptr,
                                         W->fdense.as<int32_t>(),
                                         W->fslot_key.as<unsigned long long>(),
                                         t ? W->fslot_rep.as<int32_t>() : nullptr,
                                         W->fslot_region.as<int64_t>(), cnt, stream);
      });
      hip_check(hipMemcpyAsync(W->host + kCntFilterSlots, cnt, 2 * sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, stream),
                "readback");
      sync();
      nslots = (int64_t)W->host[kCntFilterSlots];
      pool = (int64_t)W->host[kCntFilterSlots + 1];
      if (nslots > 0 && pool < INT32_MAX && 2 * pool <= *work) return true;
      nslots = 0;
      return false;
    };
    // Wider keys enforce more and are tried first when rows share them (at
    // least two rows per group on average).
    int t_use = -1;
    for (int t = 2; t >= 1 && t_use < 0; --t)
      if (masks[t] && 2 * distinct[t] <= r && groups(t)) t_use = t;
    if (t_use < 0) {
      if (grouped) insert(1u);
      if (groups(0)) t_use = 0;
    }
    const uint32_t use_mask = t_use > 0 ? masks[t_use] : 0u;
    if (nslots == 0) return;
    // Long lists are split over several blocks (pieces of kFilterPiece
    // entries) when the staging area fits the budget, else one block per group.
    const int64_t nbs = (nslots + hpm::kPivotTile - 1) / hpm::kPivotTile + 1;
    const int64_t grid_split = nslots + pool / hpm::kFilterPiece;
    uint64_t more = extra(W->fpool[d], (size_t)std::max<int64_t>(pool, 1) * 4) +
                    extra(W->fcount, (size_t)nslots * 4) +
                    extra(W->off2[d], (size_t)(r + 1) * 8) +
                    extra(W->fpbase, (size_t)(nslots + 1) * 8) + extra(W->fpbsum, (size_t)nbs * 8) +
                    extra(W->fpcnt, (size_t)nslots * 4) + extra(W->fpslot, (size_t)nslots * 4) +
                    extra(W->fpdesc, (size_t)nslots * 16);
    if (planned + more > budget) return;
    const uint64_t split_more = extra(W->ftmp, (size_t)std::max<int64_t>(pool, 1) * 4) +
                                extra(W->fpcnt, (size_t)grid_split * 4) +
                                extra(W->fpslot, (size_t)grid_split * 4) +
                                extra(W->fpdesc, (size_t)grid_split * 16);
    const bool split = grid_split > nslots && grid_split < INT32_MAX &&
                       planned + more + split_more <= budget;
    const int32_t plen = split ? hpm::kFilterPiece : INT32_MAX;
    const int64_t grid = split ? grid_split : nslots;
    need(W->fpool[d], (size_t)std::max<int64_t>(pool, 1) * 4);
    need(W->fcount, (size_t)nslots * 4);
    need(W->off2[d], (size_t)(r + 1) * 8);
    need(W->fpbase, (size_t)(nslots + 1) * 8);
    need(W->fpbsum, (size_t)nbs * 8);
    need(W->fpcnt, (size_t)grid * 4);
    need(W->fpslot, (size_t)grid * 4);
    need(W->fpdesc, (size_t)grid * 16);
    if (split) need(W->ftmp, (size_t)std::max<int64_t>(pool, 1) * 4);
    int64_t* off2 = W->off2[d].as<int64_t>();
    const unsigned long long* skey = W->fslot_key.as<unsigned long long>();
    const int32_t* srep = use_mask ? W->fslot_rep.as<int32_t>() : nullptr;
    launch(HPM_K_FILTER, [&] {
      return hpm::launch_filter_pieces(g, rows, d, piv, (int32_t)nslots, skey, srep, plen,
                                       W->fpbase.as<int64_t>(), W->fpbsum.as<int64_t>(),
                                       W->fpslot.as<int32_t>(), W->fpdesc.as<int4>(), stream);
    });
    launch(HPM_K_FILTER, [&] {
      return hpm::launch_filter_lists(g, dplan(), bits(d), d, rows, use_mask, (int32_t)nslots,
                                      W->fpbase.as<int64_t>(), plen, (int32_t)grid,
                                      W->fslot_region.as<int64_t>(),
                                      W->fpool[d].as<int32_t>(), W->fcount.as<int32_t>(),
                                      split ? W->ftmp.as<int32_t>() : nullptr,
                                      W->fpcnt.as<int32_t>(), W->fpslot.as<int32_t>(),
                                      W->fpdesc.as<int4>(), stream);
    });
    launch(HPM_K_FILTER, [&] {
      return hpm::launch_filter_apply(rows, (int32_t)r, d, piv, off, off2, hpm::kFilterMinLen,
                                      use_mask, keys + (size_t)t_use * H, H,
                                      W->fdense.as<int32_t>(),
                                      use_mask ? W->fslot_rep.as<int32_t>() : nullptr,
                                      W->fslot_region.as<int64_t>(), W->fcount.as<int32_t>(),
                                      W->bsum[d].as<int64_t>(), stream);
    });
    launch(HPM_K_PREFIX_SUM,
           [&] { return hpm::launch_scan_lengths(off2, (int32_t)r, W->bsum[d].as<int64_t>(), stream); });
    hip_check(hipMemcpyAsync(W->host + kHostPieces, W->fpbase.as<int64_t>() + nslots,
                             sizeof(int64_t), hipMemcpyDeviceToHost, stream),
              "readback");
    *work = read_i64(off2 + r);  // synchronises: the piece total has landed too
    st.filter_pieces += W->host[kHostPieces];
    *offp = off2;
    *fpool = W->fpool[d].as<int32_t>();
    done[d] = use_mask ? use_mask : hpm::kDonePivot;
    st.filtered_lists += (uint64_t)nslots;
    st.filter_rows += (uint64_t)r;
    st.filter_entries += (uint64_t)pool;
  }

  // Filter applied at depth d with every arc-related position enforced by the
  // filtered lists: a filtered row then only needs injectivity and, for
  // induced isomorphism, non-arcs to the positions left in *umask.
  bool counts_by_rows(int32_t d, uint32_t* umask) const {
    if (done[d] == 0) return false;
    const uint32_t all = (1u << d) - 1u;
    const uint32_t related = (host_plan.fwd[d] | host_plan.bwd[d]) & all;
    uint32_t covered;
    if (done[d] == hpm::kDonePivot) {
      if (__builtin_popcount(related) != 1) return false;
      covered = related;  // the pivot is the one related position
    } else {
      if ((related & ~done[d]) != 0) return false;
      covered = done[d];
    }
    *umask = host_plan.mode == HPM_ISO ? (all & ~covered) : 0u;
    return true;
  }

  // Separate rows with at least kAlignMin candidates (row-aligned tiles) from
  // the rest (packed tiles).  On success *S is the short rows' work and *T the
  // long rows' tile count (W->soff[d] / W->toff[d] hold the prefix sums).
  bool split_rows(int32_t d, int64_t r, const int64_t* offp, int64_t work, int64_t* S,
                  int64_t* T) {
    if (work < kSplitMinWork) return false;
    const uint64_t nb = ((uint64_t)r + hpm::kPivotTile - 1) / hpm::kPivotTile + 1;
    const uint64_t pre = (uint64_t)(r + 1) * sizeof(int64_t);
    const uint64_t more = extra(W->soff[d], pre) + extra(W->toff[d], pre) +
                          extra(W->sbsum[d], nb * 8) + extra(W->tbsum[d], nb * 8);
    if (planned + more > budget) return false;
    need(W->soff[d], pre);
    need(W->toff[d], pre);
    need(W->sbsum[d], nb * 8);
    need(W->tbsum[d], nb * 8);
    int64_t* so = W->soff[d].as<int64_t>();
    int64_t* to = W->toff[d].as<int64_t>();
    launch(HPM_K_PREFIX_SUM, [&] {
      return hpm::launch_split_rows(offp, (int32_t)r, so, to, W->sbsum[d].as<int64_t>(),
                                    W->tbsum[d].as<int64_t>(), stream);
    });
    hip_check(hipMemcpyAsync(W->host + kHostSplit, so + r, sizeof(int64_t),
                             hipMemcpyDeviceToHost, stream), "readback");
    hip_check(hipMemcpyAsync(W->host + kHostSplit + 1, to + r, sizeof(int64_t),
                             hipMemcpyDeviceToHost, stream), "readback");
    sync();
    *S = (int64_t)W->host[kHostSplit];
    *T = (int64_t)W->host[kHostSplit + 1];
    if (*S > work || *T > work) fail(HPM_E_INTERNAL, "row split overflow");
    return *T > 0;
  }

  // Frontier look-ahead mask for rows of d mapped positions: the positions
  // after the next one (d) that are adjacent to a mapped position.
  uint32_t frontier_mask(int32_t d) const {
    const uint32_t mapped = (1u << d) - 1u;
    uint32_t m = 0;
    for (int32_t b = d + 1; b < k; ++b)
      if ((host_plan.fwd[b] | host_plan.bwd[b]) & mapped) m |= 1u << b;
    return m;
  }

  // Extend the r rows (each d entries) in `rows` to full embeddings.
  void process_depth(int32_t d, const int32_t* rows, int64_t r) {
    if (r == 0) return;
    const uint32_t fmask = lookahead ? frontier_mask(d) : 0u;
    if (fmask) {
      // rows with a frontier position that has no candidate extend to nothing
      need(W->la[d], (size_t)r * d * sizeof(int32_t));
      zero_counter(kCntCursor);
      launch(HPM_K_FILTER, [&] {
        return hpm::launch_lookahead_filter(g, dplan(), W->vbits.as<uint32_t>(), bit_words(), rows,
                                            r, d, fmask, W->la[d].as<int32_t>(),
                                            counters() + kCntCursor, stream);
      });
      const int64_t kept = (int64_t)read_counter(kCntCursor);
      if (kept > r) fail(HPM_E_INTERNAL, "look-ahead filter overflow");
      st.lookahead_removed += (uint64_t)(r - kept);
      rows = W->la[d].as<int32_t>();
      r = kept;
      if (r == 0) return;
    }
    st.rows[d] += r;
    int64_t* off = W->off[d].as<int64_t>();
    int2* piv = W->piv[d].as<int2>();
    int64_t* bsum = W->bsum[d].as<int64_t>();
    launch(HPM_K_ROW_PIVOT, [&] {
      return hpm::launch_row_pivot(g, dplan(), d, rows, (int32_t)r, piv, off, bsum, stream);
    });
    launch(HPM_K_PREFIX_SUM, [&] { return hpm::launch_scan_lengths(off, (int32_t)r, bsum, stream); });
    int64_t work = read_i64(off + r);
    st.raw_work[d] += (uint64_t)work;
    const int64_t* offp = off;
    const int32_t* fpool = nullptr;
    done[d] = 0;
    if (filter && work >= kFilterMinWork) filter_pivots(d, rows, r, piv, off, &offp, &fpool, &work);
    st.work[d] += (uint64_t)work;
    if (work == 0) return;
    uint32_t umask = 0;
    // Walking neighbours pays only against long lists: with few candidates
    // per row the tiled extension is faster.
    if (d == k - 1 && !maps && counts_by_rows(d, &umask) &&
        (umask == 0 || work >= kCountMinPerRow * r)) {
      // every arc condition is in the filtered lists: each row's count
      // follows from its list length, its own images and (induced
      // isomorphism) the neighbours of the images it must not touch
      const int grid = grid_for(r, hpm::kBlock);
      unsigned long long* parts = W->partials.as<unsigned long long>();
      int64_t* rest = nullptr;
      if (umask) {
        need(W->crest, (size_t)(r + 1) * sizeof(int64_t));
        need(W->cbsum, (size_t)((r + hpm::kPivotTile - 1) / hpm::kPivotTile + 1) * sizeof(int64_t));
        rest = W->crest.as<int64_t>();
      }
      launch(HPM_K_LAST_LEVEL, [&] {
        return hpm::launch_count_rows(g, dplan(), bits(d), d, rows, offp, piv, fpool, (int32_t)r,
                                      umask, rest, parts, grid, stream);
      });
      launch(HPM_K_REDUCE, [&] {
        return hpm::launch_reduce_counts(parts, grid, counters() + kCntTotal,
                                         reinterpret_cast<uint32_t*>(counters() + kCntOverflow),
                                         stream);
      });
      int64_t left = 0;
      if (umask) {
        launch(HPM_K_PREFIX_SUM, [&] {
          return hpm::launch_rows2_compact(rest, (int32_t)r, W->cbsum.as<int64_t>(), stream);
        });
        left = read_i64(rest + r);
      }
      st.counted_rows += (uint64_t)r;
      st.counted_work += (uint64_t)(work - left);
      if (left == 0) return;
      // rows whose images have many neighbours: the tiled last level below
      offp = rest;
      work = left;
    }
    if (d == k - 1) {
      int64_t S = work, T = 0;
      const bool split = split_rows(d, r, offp, work, &S, &T);
      const int64_t* soffp = split ? W->soff[d].as<int64_t>() : offp;
      const int g1 = S > 0 ? grid_for(S, hpm::kExpandTile) : 0;
      const int g2 = T > 0 ? grid_for(T * hpm::kExpandTile, hpm::kExpandTile) : 0;
      const int mode = maps ? 2 : 1;
      unsigned long long* parts = W->partials.as<unsigned long long>();
      if (g1)
        launch(HPM_K_LAST_LEVEL, [&] {
          return hpm::launch_expand(g, dplan(), bits(d), d, rows, soffp, piv, fpool, (int32_t)r,
                                    0, S, nullptr, done[d], mode, maps, counters() + kCntEmit,
                                    maps ? emit_cap() : 0, parts, g1, stream);
        });
      if (g2)
        launch(HPM_K_LAST_LEVEL, [&] {
          return hpm::launch_expand(g, dplan(), bits(d), d, rows, offp, piv, fpool, (int32_t)r,
                                    0, T, W->toff[d].as<int64_t>(), done[d], mode, maps,
                                    counters() + kCntEmit, maps ? emit_cap() : 0, parts + g1, g2,
                                    stream);
        });
      launch(HPM_K_REDUCE, [&] {
        return hpm::launch_reduce_counts(parts, g1 + g2, counters() + kCntTotal,
                                         reinterpret_cast<uint32_t*>(counters() + kCntOverflow),
                                         stream);
      });
      return;
    }
    int64_t S = work, T = 0;
    if (split_rows(d, r, offp, work, &S, &T)) {
      // The whole depth in one piece: packed short rows and row-aligned long
      // rows.  Room for at most one frontier chunk of new rows: with more
      // candidates than that, the piece is tried first (most candidates
      // fail), and only if more rows pass than fit is the depth redone in
      // chunks of candidates below.
      const int64_t cap_rows = std::min(work, chunk);
      st.chunks++;
      need(W->rows[d + 1], (size_t)cap_rows * (d + 1) * sizeof(int32_t));
      ensure_depth(d + 1, cap_rows);
      int32_t* out = W->rows[d + 1].as<int32_t>();
      zero_counter(kCntCursor);
      if (S > 0)
        launch(HPM_K_EXPAND, [&] {
          return hpm::launch_expand(g, dplan(), bits(d), d, rows, W->soff[d].as<int64_t>(), piv,
                                    fpool, (int32_t)r, 0, S, nullptr, done[d], 0, out,
                                    counters() + kCntCursor, (unsigned long long)cap_rows,
                                    W->partials.as<unsigned long long>(),
                                    grid_for(S, hpm::kExpandTile), stream);
        });
      launch(HPM_K_EXPAND, [&] {
        return hpm::launch_expand(g, dplan(), bits(d), d, rows, offp, piv, fpool, (int32_t)r, 0,
                                  T, W->toff[d].as<int64_t>(), done[d], 0, out,
                                  counters() + kCntCursor,
                                  (unsigned long long)cap_rows,
                                  W->partials.as<unsigned long long>(),
                                  grid_for(T * hpm::kExpandTile, hpm::kExpandTile), stream);
      });
      const int64_t r1 = (int64_t)read_counter(kCntCursor);
      if (r1 > work) fail(HPM_E_INTERNAL, "frontier overflow");
      if (r1 <= cap_rows) {
        process_depth(d + 1, out, r1);
        check_limit();
        return;
      }
      // rows were dropped: the chunked pass below
    }
    for (int64_t w0 = 0; w0 < work && !stopped; w0 += chunk) {
      const int64_t w1 = std::min(work, w0 + chunk);
      const int64_t n_items = w1 - w0;
      st.chunks++;
      need(W->rows[d + 1], (size_t)n_items * (d + 1) * sizeof(int32_t));
      ensure_depth(d + 1, n_items);
      int32_t* out = W->rows[d + 1].as<int32_t>();
      zero_counter(kCntCursor);
      const int grid = grid_for(n_items, hpm::kExpandTile);
      launch(HPM_K_EXPAND, [&] {
        return hpm::launch_expand(g, dplan(), bits(d), d, rows, offp, piv,
                                  fpool, (int32_t)r, w0, w1, nullptr, done[d], 0, out,
                                  counters() + kCntCursor, (unsigned long long)n_items,
                                  W->partials.as<unsigned long long>(), grid, stream);
      });
      const int64_t r1 = (int64_t)read_counter(kCntCursor);
      if (r1 > n_items) fail(HPM_E_INTERNAL, "frontier chunk overflow");
      process_depth(d + 1, out, r1);
      check_limit();
    }
  }

  // Rows the last level may write: the caller's capacity, at most the limit.
  uint64_t emit_cap() const { return limit ? std::min(cap, limit) : cap; }

  // First-k: stop once the running total reaches the limit.
  void check_limit() {
    if (limit && !stopped && read_total() >= limit) stopped = true;
  }

  // Arc-predicate index (monomorphism only): every pattern arc's predicate
  // implies the loosest range per column over all pattern arcs, so an arc that
  // fails it is never the image of a pattern arc.  After the arc scan (which
  // reads the whole graph) the validator and the extension then read
  // adjacency restricted to the arcs that pass it: shorter candidate lists and
  // membership searches, the same embeddings (non-arcs, which induced
  // isomorphism checks, need the whole graph, so it is not used there).
  // Built when the column samples say at most three quarters of the arcs
  // pass and the buffers fit the budget.
  void build_arc_index(uint32_t flags) {
    if (host_plan.mode != HPM_MONO || k < 3 || (flags & HPM_F_NO_ARC_INDEX)) return;
    const int32_t nc = G->n_ecols;
    if (nc == 0 || G->m == 0) return;
    int32_t lo[kMaxCols], hi[kMaxCols];
    for (int c = 0; c < kMaxCols; ++c) {
      lo[c] = INT32_MAX;
      hi[c] = INT32_MIN;
    }
    uint32_t cmask = (1u << nc) - 1u;
    for (int32_t a = 0; a < k; ++a)
      for (int32_t b = 0; b < k; ++b) {
        const bool arc = (a < b) ? ((host_plan.fwd[b] >> a) & 1u) : (a > b && ((host_plan.bwd[a] >> b) & 1u));
        if (!arc) continue;
        for (int32_t c = 0; c < nc; ++c) {
          if (!((host_plan.amask[a][b] >> c) & 1u)) {
            cmask &= ~(1u << c);
            continue;
          }
          lo[c] = std::min(lo[c], host_plan.alo[a][b][c]);
          hi[c] = std::max(hi[c], host_plan.ahi[a][b][c]);
        }
      }
    if (cmask == 0) return;
    double frac = 1.0;
    for (int32_t c = 0; c < nc; ++c)
      if ((cmask >> c) & 1u) frac = std::min(frac, sample_fraction(G->esample[c], lo[c], hi[c]));
    if (frac > 0.75) return;
    const int64_t m = G->m;
    const int64_t nb = hpm::arc_index_tiles(m);
    const uint64_t words = (uint64_t)hpm::arc_index_words(m);
    const uint64_t fixed = 2 * words * 12 + 2 * (uint64_t)(nb + 1) * 8 + 16;
    if (planned + fixed > budget) return;
    need(W->amask, (size_t)(2 * words * 8));
    need(W->awpre, (size_t)(2 * words * 4));
    need(W->absum, (size_t)(2 * (nb + 1) * 8 + 16));
    hpm::ArcIndexSides S{};
    for (int side = 0; side < 2; ++side) {
      hpm::ArcIndexSide& sd = S.s[side];
      sd.off = side ? G->in_off.as<int32_t>() : G->out_off.as<int32_t>();
      sd.nbrs = side ? G->in_nbrs.as<int32_t>() : G->out_nbrs.as<int32_t>();
      for (int c = 0; c < kMaxCols; ++c)
        sd.cols[c] = side ? G->ecols_in[c].as<int32_t>() : G->ecols[c].as<int32_t>();
      sd.mask = W->amask.as<uint64_t>() + side * words;
      sd.wpre = W->awpre.as<int32_t>() + side * words;
      sd.bsum = W->absum.as<int64_t>() + side * (nb + 1);
    }
    int64_t* totals = W->absum.as<int64_t>() + 2 * (nb + 1);
    launch(HPM_K_INDEX, [&] {
      return hpm::launch_arc_index_count(S, lo, hi, cmask, m, totals, stream);
    });
    int64_t tot[2];
    read_i64s(totals, 2, tot);
    const int64_t mp = tot[0];
    if (mp < 0 || mp > m || tot[1] != mp) fail(HPM_E_INTERNAL, "arc index count out of range");
    const uint64_t arrays = 2 * ((uint64_t)(G->n + 1) * 4 + (uint64_t)mp * 4 * (1 + nc));
    if (planned + arrays > budget) return;
    need(W->aoff_out, (size_t)(G->n + 1) * 4);
    need(W->anbrs_out, (size_t)std::max<int64_t>(mp, 1) * 4);
    need(W->aoff_in, (size_t)(G->n + 1) * 4);
    need(W->anbrs_in, (size_t)std::max<int64_t>(mp, 1) * 4);
    for (int32_t c = 0; c < nc; ++c) {
      need(W->acol_out[c], (size_t)std::max<int64_t>(mp, 1) * 4);
      need(W->acol_in[c], (size_t)std::max<int64_t>(mp, 1) * 4);
      S.s[0].cols_out[c] = W->acol_out[c].as<int32_t>();
      S.s[1].cols_out[c] = W->acol_in[c].as<int32_t>();
    }
    S.s[0].off_out = W->aoff_out.as<int32_t>();
    S.s[0].nbrs_out = W->anbrs_out.as<int32_t>();
    S.s[1].off_out = W->aoff_in.as<int32_t>();
    S.s[1].nbrs_out = W->anbrs_in.as<int32_t>();
    launch(HPM_K_INDEX, [&] {
      return hpm::launch_arc_index_fill(S, G->n, nc, m, mp, stream);
    });
    g.m = (int32_t)mp;
    g.out_off = W->aoff_out.as<int32_t>();
    g.out_nbrs = W->anbrs_out.as<int32_t>();
    g.in_off = W->aoff_in.as<int32_t>();
    g.in_nbrs = W->anbrs_in.as<int32_t>();
    for (int32_t c = 0; c < nc; ++c) {
      g.ecol[c] = W->acol_out[c].as<int32_t>();
      g.ecol_in[c] = W->acol_in[c].as<int32_t>();
    }
    st.index_arcs = (uint64_t)mp;
    indexed = true;
  }

  void read_i64s(const int64_t* p, int count, int64_t* out) {
    hip_check(hipMemcpyAsync(W->host + kCntSlots, p, sizeof(int64_t) * count,
                             hipMemcpyDeviceToHost, stream),
              "readback");
    sync();
    for (int i = 0; i < count; ++i) out[i] = (int64_t)W->host[kCntSlots + i];
  }

  void run() {
    const int64_t m = G->m;
    st.arcs_scanned = (uint64_t)m;
    launch(HPM_K_VERTEX_VALIDATOR, [&] {
      return hpm::launch_vertex_validator(g, dplan(), W->vbits.as<uint32_t>(), bit_words(),
                                          stream);
    });
    if (k == 2 && !survivors_only) {
      const int grid = grid_for(m, hpm::kScanTile);
      uint64_t c;
      if (maps) {
        zero_counter(kCntCursor);
        launch(HPM_K_EDGE_SCAN, [&] {
          return hpm::launch_edge_scan(gs, dplan(), bits0(), bits1(), 0, (int32_t)m, 2, maps,
                                       counters() + kCntCursor, emit_cap(),
                                       W->partials.as<unsigned long long>(), grid, stream);
        });
        c = read_counter(kCntCursor);
      } else {
        const int nb = (int)hpm::edge_scan_blocks(m);
        need(W->blkcount, (size_t)nb * sizeof(unsigned long long));
        launch(HPM_K_EDGE_SCAN, [&] {
          return hpm::launch_edge_scan(gs, dplan(), bits0(), bits1(), 0, (int32_t)m, 1, nullptr,
                                       nullptr, 0, W->blkcount.as<unsigned long long>(), nb,
                                       stream);
        });
        launch(HPM_K_REDUCE, [&] {
          return hpm::launch_reduce_counts(W->blkcount.as<unsigned long long>(), nb,
                                           counters() + kCntTotal,
                                           reinterpret_cast<uint32_t*>(counters() + kCntOverflow),
                                           stream);
        });
        c = read_total();
      }
      st.survivors = c;
      st.rows[2] = c;
      st.count = limit ? std::min(c, limit) : c;
      return;
    }
    for (int64_t e0 = 0; e0 < m && !stopped; e0 += cap2) {
      const int64_t e1 = std::min<int64_t>(m, e0 + cap2);
      st.arcs_scanned = (uint64_t)e1;
      const int grid = (int)hpm::edge_scan_blocks(e1 - e0);
      need(W->blkcount, (size_t)(grid + 1) * sizeof(int64_t));
      need(W->blkprefix, (size_t)(grid / hpm::kPivotTile + 2) * sizeof(int64_t));
      int64_t* cnt = W->blkcount.as<int64_t>();
      launch(HPM_K_EDGE_SCAN, [&] {
        return hpm::launch_edge_scan(gs, dplan(), bits0(), bits1(), (int32_t)e0, (int32_t)e1, 0,
                                     W->rows2.as<int32_t>(), nullptr,
                                     (unsigned long long)(e1 - e0),
                                     reinterpret_cast<unsigned long long*>(cnt), grid, stream);
      });
      launch(HPM_K_PREFIX_SUM, [&] {
        return hpm::launch_rows2_compact(cnt, grid, W->blkprefix.as<int64_t>(), stream);
      });
      const int64_t s2 = read_i64(cnt + grid);
      if (s2 > e1 - e0) fail(HPM_E_INTERNAL, "scan overflow");
      st.survivors += (uint64_t)s2;
      if (want_index) {
        // The index costs a few passes over every arc; it pays when the
        // frontier is large (here: depth-2 rows, scaled to the whole graph,
        // at least 1/256 of the arcs).
        want_index = false;
        if ((double)s2 * (double)m / (double)(e1 - e0) >= (double)m / 256.0) {
          build_arc_index(call_flags);
          if (indexed) {
            // degrees counted over the index only: a stronger validator, so
            // the chunk is scanned again with it (one more pass over its arcs
            // for a frontier that is often much smaller)
            launch(HPM_K_VERTEX_VALIDATOR, [&] {
              return hpm::launch_vertex_validator(g, dplan(), W->vbits.as<uint32_t>(),
                                                  bit_words(), stream);
            });
            st.survivors -= (uint64_t)s2;
            e0 -= cap2;  // the loop's step returns to this chunk
            continue;
          }
        }
      }
      if (s2 == 0) continue;
      need(W->rows2d, (size_t)s2 * 2 * sizeof(int32_t));
      ensure_depth(2, s2);
      launch(HPM_K_PREFIX_SUM, [&] {
        return hpm::launch_rows2_gather(W->rows2.as<int32_t>(), cnt, grid, (int32_t)e0,
                                        (int32_t)e1, W->rows2d.as<int32_t>(), s2, stream);
      });
      if (survivors_only) {
        const uint64_t done = st.survivors - (uint64_t)s2;  // rows of earlier chunks
        if (surv_out && done < surv_cap) {
          const uint64_t n = std::min<uint64_t>((uint64_t)s2, surv_cap - done);
          hip_check(hipMemcpyAsync(surv_out + done * 2, W->rows2d.p, n * 2 * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, stream),
                    "survivor copy");
        }
        continue;
      }
      if (overlap_need > 0) {
        // the sparse scan regions are free again: the rows that pass go there
        zero_counter(kCntCursor);
        launch(HPM_K_EDGE_SCAN, [&] {
          return hpm::launch_overlap_filter(g, W->rows2d.as<int32_t>(), s2, overlap_need,
                                            W->rows2.as<int32_t>(), counters() + kCntCursor,
                                            stream);
        });
        const int64_t kept = (int64_t)read_counter(kCntCursor);
        if (kept > s2) fail(HPM_E_INTERNAL, "overlap filter overflow");
        st.overlap_removed += (uint64_t)(s2 - kept);
        process_depth(2, W->rows2.as<int32_t>(), kept);
      } else {
        process_depth(2, W->rows2d.as<int32_t>(), s2);
      }
      check_limit();
    }
    if (survivors_only) {
      st.count = st.survivors;
      return;
    }
    st.count = read_total();
    if (limit) st.count = std::min(st.count, limit);
  }
};

// Output of a survivors-only call (hpm_scan_survivors).
struct SurvivorsOut {
  int32_t* rows;
  uint64_t cap;
};

constexpr uint64_t kMinChunkRows = hpm::kExpandTile;
// Frontier rows a deeper chunk keeps before the depth-2 chunk takes the rest.
constexpr uint64_t kDeepFloorRows = uint64_t(1) << 22;
// Piece sizes of a first-k search (arcs per scan chunk, work items per
// frontier chunk).
constexpr int64_t kFirstKArcs = int64_t(1) << 20;
constexpr int64_t kFirstKRows = int64_t(1) << 20;

}  // namespace

// ------------------------------------------------------------ C ABI

extern "C" {

int hpm_abi_version(void) { return HPM_ABI_VERSION; }

const char* hpm_status_string(int status) {
  switch (status) {
    case HPM_OK: return "ok";
    case HPM_E_ARG: return "invalid argument";
    case HPM_E_GRAPH: return "malformed graph";
    case HPM_E_PATTERN: return "malformed pattern";
    case HPM_E_NOMEM: return "out of device memory or scratch budget too small";
    case HPM_E_TRUNCATED: return "mapping buffer too small";
    case HPM_E_OVERFLOW: return "count overflow";
    case HPM_E_DEVICE: return "device error";
    case HPM_E_UNSUPPORTED: return "unsupported size";
    case HPM_E_INTERNAL: return "internal error";
    default: return "unknown status";
  }
}

const char* hpm_last_error(void) { return t_error.c_str(); }

int hpm_graph_create(hpm_graph** out, int32_t n, int64_t m, const int64_t* out_off,
                     const int32_t* out_nbrs, const int64_t* in_off, const int32_t* in_nbrs,
                     int32_t n_vcols, const int32_t* const* vcols, int32_t n_ecols,
                     const int32_t* const* ecols, void* stream_) {
  return guarded([&]() -> int {
    if (!out) fail(HPM_E_ARG, "out is NULL");
    *out = nullptr;
    if (n < 0 || m < 0) fail(HPM_E_ARG, "negative size");
    if (n >= INT32_MAX || m > INT32_MAX) fail(HPM_E_UNSUPPORTED, "n and m must be below 2^31 - 1");
    if (!out_off || !in_off) fail(HPM_E_ARG, "offset arrays are NULL");
    if (m > 0 && (!out_nbrs || !in_nbrs)) fail(HPM_E_ARG, "neighbour arrays are NULL");
    if (n_vcols < 0 || n_vcols > kMaxCols || n_ecols < 0 || n_ecols > kMaxCols)
      fail(HPM_E_ARG, "column counts must be 0..4");
    if (n_vcols > 0 && !vcols) fail(HPM_E_ARG, "vcols is NULL");
    if (n_ecols > 0 && !ecols) fail(HPM_E_ARG, "ecols is NULL");
    for (int c = 0; c < n_vcols; ++c)
      if (n > 0 && !vcols[c]) fail(HPM_E_ARG, "vertex column is NULL");
    for (int c = 0; c < n_ecols; ++c)
      if (m > 0 && !ecols[c]) fail(HPM_E_ARG, "arc column is NULL");
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    std::vector<int32_t> oo = narrow_offsets(out_off, n, m, "out_off");
    std::vector<int32_t> io = narrow_offsets(in_off, n, m, "in_off");

    std::unique_ptr<hpm_graph> G(new hpm_graph());
    hip_check(hipGetDevice(&G->device), "hipGetDevice");
    int cus = 0;
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, G->device),
              "hipDeviceGetAttribute");
    G->num_cus = cus > 0 ? cus : 256;
    G->n = n;
    G->m = m;
    G->n_vcols = n_vcols;
    G->n_ecols = n_ecols;
    const size_t mb = (size_t)m * sizeof(int32_t);
    upload(G->out_off, oo.data(), oo.size() * sizeof(int32_t), stream);
    upload(G->in_off, io.data(), io.size() * sizeof(int32_t), stream);
    upload(G->out_nbrs, out_nbrs, mb, stream);
    upload(G->in_nbrs, in_nbrs, mb, stream);
    for (int c = 0; c < n_vcols; ++c) upload(G->vcols[c], vcols[c], (size_t)n * 4, stream);
    for (int c = 0; c < n_ecols; ++c) upload(G->ecols[c], ecols[c], mb, stream);
    G->src.ensure(mb ? mb : 4, stream);
    G->in_eid.ensure(mb ? mb : 4, stream);
    G->rev_eid.ensure(mb ? mb : 4, stream);
    DevBuf in_row, err;
    in_row.ensure(mb ? mb : 4, stream);
    err.ensure(sizeof(uint32_t), stream);
    hip_check(hipMemsetAsync(err.p, 0, sizeof(uint32_t), stream), "memset");
    uint32_t* e = err.as<uint32_t>();
    const int32_t mi = (int32_t)m;
    hip_check(hpm::launch_derive_rows(G->out_off.as<int32_t>(), n, mi, G->src.as<int32_t>(), stream),
              "derive rows");
    hip_check(hpm::launch_derive_rows(G->in_off.as<int32_t>(), n, mi, in_row.as<int32_t>(), stream),
              "derive rows");
    hip_check(hpm::launch_check_rows(G->out_off.as<int32_t>(), G->out_nbrs.as<int32_t>(),
                                     G->src.as<int32_t>(), n, mi, e, stream),
              "check rows");
    hip_check(hpm::launch_check_rows(G->in_off.as<int32_t>(), G->in_nbrs.as<int32_t>(),
                                     in_row.as<int32_t>(), n, mi, e, stream),
              "check rows");
    hip_check(hpm::launch_transpose_ids(G->in_off.as<int32_t>(), G->in_nbrs.as<int32_t>(),
                                        in_row.as<int32_t>(), G->out_off.as<int32_t>(),
                                        G->out_nbrs.as<int32_t>(), n, mi, G->in_eid.as<int32_t>(),
                                        e, stream),
              "transpose ids");
    uint32_t bits = 0;
    hip_check(hipMemcpyAsync(&bits, e, sizeof(bits), hipMemcpyDeviceToHost, stream), "readback");
    hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (bits) fail(HPM_E_GRAPH, graph_error_text(bits));
    // only on a valid graph: every head indexes out_off, every in_eid is an arc
    hip_check(hpm::launch_reverse_ids(G->out_off.as<int32_t>(), G->out_nbrs.as<int32_t>(),
                                      G->src.as<int32_t>(), mi, G->rev_eid.as<int32_t>(), stream),
              "reverse ids");
    for (int c = 0; c < n_ecols; ++c) {
      G->ecols_in[c].ensure(mb ? mb : 4, stream);
      hip_check(hpm::launch_columns_in_order(G->ecols[c].as<int32_t>(), G->in_eid.as<int32_t>(),
                                             mi, G->ecols_in[c].as<int32_t>(), stream),
                "columns in in-CSR order");
    }
    hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
    for (int c = 0; c < n_vcols; ++c) G->vsample[c] = column_sample(vcols[c], n);
    for (int c = 0; c < n_ecols; ++c) G->esample[c] = column_sample(ecols[c], m);
    G->sb_out = size_biased_degree(oo);
    G->sb_in = size_biased_degree(io);
    *out = G.release();
    return HPM_OK;
  });
}

int hpm_graph_destroy(hpm_graph* g) {
  return guarded([&]() -> int {
    if (!g) return HPM_OK;
    int cur = 0;
    const int dev = g->device;
    (void)hipGetDevice(&cur);
    if (cur != dev) (void)hipSetDevice(dev);
    delete g;
    if (cur != dev) (void)hipSetDevice(cur);
    return HPM_OK;
  });
}

int hpm_graph_info(const hpm_graph* g, int32_t* n, int64_t* m, uint64_t* device_bytes) {
  return guarded([&]() -> int {
    if (!g) fail(HPM_E_ARG, "graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (device_bytes) *device_bytes = g->bytes();
    return HPM_OK;
  });
}

int hpm_plan_order(const hpm_pattern* p, int32_t n_vcols, int32_t n_ecols, uint32_t flags,
                   int32_t* order) {
  return guarded([&]() -> int {
    if (!order) fail(HPM_E_ARG, "order is NULL");
    PatternInfo info = check_pattern(p, n_vcols, n_ecols);
    std::vector<int32_t> o = plan_order(info, flags);
    std::copy(o.begin(), o.end(), order);
    return HPM_OK;
  });
}

int hpm_last_stats(hpm_match_stats* out) {
  return guarded([&]() -> int {
    if (!out) fail(HPM_E_ARG, "out is NULL");
    *out = t_stats;
    return HPM_OK;
  });
}

}  // extern "C"

namespace {

// One match, as documented on hpm_match; throws Failure.  Returns HPM_OK or
// HPM_E_TRUNCATED (count valid).
// Scratch that does not depend on the frontier: plan, per-position vertex
// flags, counters, per-block partial counts.
uint64_t scratch_fixed(const hpm_graph* G, int32_t k) {
  const int max_grid = std::max(64, G->num_cus * 8);
  return sizeof(DevPlan) + ((uint64_t)G->n + 63) / 64 * 8 * (uint64_t)k + 64 +
         (uint64_t)max_grid * 2 * sizeof(unsigned long long) + 4096;
}

// Depth 2 costs 33 B per arc of a chunk (scan region 8, dense row 8, prefix 8,
// pivot 8, per-tile counts and block sums); depth d >= 3 costs 4d + 17 B per
// row of a chunk.
constexpr uint64_t kDepth2BytesPerArc = 33;
inline uint64_t row_bytes(int32_t d) { return 4 * (uint64_t)d + 17; }

// Workspace: NULL takes one from the graph's pool (returned on exit).
int match_one(hpm_graph* G, const hpm_pattern* p, int mode, hipStream_t stream, uint32_t flags,
              uint64_t budget, uint64_t* count, int32_t* mappings, uint64_t cap,
              hpm_match_stats* stats, Workspace* own = nullptr, uint64_t limit = 0,
              const SurvivorsOut* surv = nullptr) {
    const auto t0 = std::chrono::steady_clock::now();
    if (mode != HPM_ISO && mode != HPM_MONO) fail(HPM_E_ARG, "mode must be HPM_ISO or HPM_MONO");
    PatternInfo info = check_pattern(p, G->n_vcols, G->n_ecols);
    const int32_t k = info.k;
    if (mappings && cap > (uint64_t)INT64_MAX / (uint64_t)k) fail(HPM_E_ARG, "cap too large");
    std::vector<int32_t> order = plan_order(info, flags);
    DevPlan plan = build_dev_plan(p, info, order, G->n_vcols, G->n_ecols, (int)mode);

    int cur = 0;
    hip_check(hipGetDevice(&cur), "hipGetDevice");
    struct DeviceGuard {
      int prev, want;
      DeviceGuard(int p_, int w_) : prev(p_), want(w_) {
        if (prev != want) hip_check(hipSetDevice(want), "hipSetDevice");
      }
      ~DeviceGuard() {
        if (prev != want) (void)hipSetDevice(prev);
      }
    } dg(cur, G->device);

    Workspace* W = own;
    if (!W) {
      std::lock_guard<std::mutex> lk(G->mu);
      if (!G->pool.empty()) {
        W = G->pool.back();
        G->pool.pop_back();
      }
    }
    if (!W) W = new Workspace();
    struct Return {
      hpm_graph* G;
      Workspace* W;
      ~Return() {
        if (!W) return;
        std::lock_guard<std::mutex> lk(G->mu);
        G->pool.push_back(W);
      }
    } ret{G, own ? nullptr : W};

    if (budget == 0) {
      // a quarter of the device memory this call could use: what is free
      // plus what its own workspace already holds
      size_t free_b = 0, total_b = 0;
      hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
      budget = ((uint64_t)free_b + W->held()) / 4;
    }

    // Scratch layout and its budget: the fixed part, then one arc chunk at
    // depth 2 and one frontier chunk per deeper depth.
    const int max_grid = std::max(64, G->num_cus * 8);
    const uint64_t fixed = scratch_fixed(G, k);
    if (budget < fixed) fail(HPM_E_NOMEM, "scratch budget below the fixed part");
    uint64_t avail = budget - fixed;
    int64_t cap2 = 0, chunk = 0;
    if (k >= 3 || surv) {
      uint64_t per_row_deep = 0;
      for (int32_t d = 3; d <= k - 1; ++d) per_row_deep += row_bytes(d);
      const uint64_t m_round =
          ((uint64_t)G->m + hpm::kScanTile - 1) / hpm::kScanTile * hpm::kScanTile;
      // Depth-2 rows take all arcs in one chunk when what is left still holds
      // kDeepFloorRows frontier rows; a smaller budget is split in halves.
      const uint64_t deep_floor =
          per_row_deep ? std::min<uint64_t>(avail / 2, per_row_deep * kDeepFloorRows) : 0;
      uint64_t c2 = std::min<uint64_t>(std::max<uint64_t>(m_round, hpm::kScanTile),
                                       (avail - deep_floor) / kDepth2BytesPerArc);
      c2 = c2 / hpm::kScanTile * hpm::kScanTile;
      c2 = std::min<uint64_t>(c2, (uint64_t)INT32_MAX / hpm::kScanTile * hpm::kScanTile);
      if (c2 < (uint64_t)hpm::kScanTile) fail(HPM_E_NOMEM, "scratch budget below one arc chunk");
      cap2 = (int64_t)c2;
      if (per_row_deep) {
        uint64_t c = (avail - c2 * kDepth2BytesPerArc) / per_row_deep;
        c = std::min<uint64_t>(c, (uint64_t)1 << 30);
        if (c < kMinChunkRows) fail(HPM_E_NOMEM, "scratch budget below one frontier chunk");
        chunk = (int64_t)c;
      }
    }

    if (limit) {
      // first-k: work in small pieces so the search can stop soon after the
      // limit is reached
      cap2 = std::min<int64_t>(cap2, kFirstKArcs);
      if (chunk) chunk = std::min<int64_t>(chunk, kFirstKRows);
    }

    // The call's own scratch stays within the budget (Matcher::need); idle
    // buffers kept from earlier calls are dropped once they pass it twice over.
    if (W->held() > 2 * budget) {
      hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
      W->release_all();
    }
    if (!W->host)
      hip_check(hipHostMalloc((void**)&W->host, kCntNum * sizeof(unsigned long long)),
                "hipHostMalloc");
    if (!W->host_plan)
      hip_check(hipHostMalloc((void**)&W->host_plan, sizeof(DevPlan)), "hipHostMalloc");

    Matcher M{G, W, stream, G->view(), G->view(), plan, k, mappings, mappings ? cap : 0,
              (flags & HPM_F_TIMING) != 0, (flags & HPM_F_NO_FILTER) == 0, max_grid};
    M.timed_kinds = (flags >> 16) & 0x1ffu ? (flags >> 16) & 0x1ffu : 0x1ffu;
    M.cap2 = cap2;
    M.chunk = chunk;
    M.budget = budget;
    M.limit = limit;
    M.lookahead = (flags & HPM_F_LOOKAHEAD) != 0;
    if ((flags & HPM_F_OVERLAP) && k >= 3) {
      // pattern vertices adjacent (either direction) to both of the first two
      const int32_t u = order[0], v = order[1];
      for (int32_t w = 0; w < k; ++w)
        if (w != u && w != v && (info.adj[(size_t)u * k + w] || info.adj[(size_t)w * k + u]) &&
            (info.adj[(size_t)v * k + w] || info.adj[(size_t)w * k + v]))
          M.overlap_need++;
    }
    M.need(W->plan, sizeof(DevPlan));
    M.need(W->vbits, (size_t)std::max<int64_t>(M.bit_words(), 1) * k * sizeof(uint32_t));
    M.need(W->counters, kCntNum * sizeof(unsigned long long));
    M.need(W->partials, (size_t)max_grid * 2 * sizeof(unsigned long long));
    if (k >= 3 || surv) {
      const int64_t rows2 = std::min<int64_t>(cap2, std::max<int64_t>(G->m, 1));
      M.need(W->rows2, (size_t)rows2 * 2 * sizeof(int32_t));
    }
    // The plan goes through pinned memory so the copy is truly asynchronous.
    *W->host_plan = plan;
    hip_check(hipMemcpyAsync(W->plan.p, W->host_plan, sizeof(DevPlan), hipMemcpyHostToDevice,
                             stream),
              "plan upload");
    hip_check(hipMemsetAsync(W->counters.p, 0, kCntNum * sizeof(unsigned long long), stream),
              "memset");
    if (flags & HPM_F_COUNT_FROM_MAX) {
      // test only: the running total starts at 2^64 - 1, so the first
      // embedding counted wraps it
      static const unsigned long long kMax = ~0ull;
      hip_check(hipMemcpyAsync(M.counters() + kCntTotal, &kMax, sizeof(kMax),
                               hipMemcpyHostToDevice, stream),
                "counter seed");
    }
    if (surv) {
      M.survivors_only = true;
      M.surv_out = surv->rows;
      M.surv_cap = surv->cap;
    } else {
      M.call_flags = flags;
      M.want_index = true;
    }
    M.run();
    M.sync();
    M.st.struct_size = sizeof(hpm_match_stats);
    M.st.scratch_bytes = W->held();
    M.st.ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *count = M.st.count;
    if (stats) *stats = M.st;
    if (mappings && M.st.count > cap) {
      t_error = "count " + std::to_string(M.st.count) + " exceeds cap " + std::to_string(cap);
      return HPM_E_TRUNCATED;
    }
    return HPM_OK;
}

// Fraction of a sorted column sample inside [lo, hi] (1 when there is no sample).
double sample_fraction(const std::vector<int32_t>& smp, int32_t lo, int32_t hi) {
  if (smp.empty()) return 1.0;
  const auto a = std::lower_bound(smp.begin(), smp.end(), lo);
  const auto b = std::upper_bound(smp.begin(), smp.end(), hi);
  return b > a ? (double)(b - a) / (double)smp.size() : 0.0;
}

double vertex_fraction(const hpm_graph* G, const DevPlan& pl, int32_t pos) {
  double f = 1.0;
  for (int c = 0; c < G->n_vcols; ++c)
    if (pl.vmask[pos] & (1u << c)) f *= sample_fraction(G->vsample[c], pl.vlo[pos][c], pl.vhi[pos][c]);
  return f;
}

double arc_fraction(const hpm_graph* G, const DevPlan& pl, int32_t from, int32_t to) {
  double f = 1.0;
  for (int c = 0; c < G->n_ecols; ++c)
    if (pl.amask[from][to] & (1u << c))
      f *= sample_fraction(G->esample[c], pl.alo[from][to][c], pl.ahi[from][to][c]);
  return f;
}

// Estimated scratch bytes of an unchunked run: the fixed part, the depth-2
// area for all arcs, and per deeper depth the estimated rows times their cost.
// Rows are estimated with independent attribute fractions from the column
// samples: depth 2 = arcs x both endpoint fractions x the arc's fraction; each
// further position multiplies by the size-biased mean degree (the expected
// length of a neighbour list reached through an arc), its vertex fraction, its
// arc fractions, and degree / n for every arc beyond the first that must exist.
uint64_t estimate_scratch(const hpm_graph* G, const DevPlan& pl) {
  const int32_t k = pl.k;
  const double n = std::max(1.0, (double)G->n);
  const double deg = std::max(1.0, 0.5 * (G->sb_out + G->sb_in));
  double rows = (double)G->m * vertex_fraction(G, pl, 0) * vertex_fraction(G, pl, 1) *
                (pl.mve_forward ? arc_fraction(G, pl, 0, 1) : arc_fraction(G, pl, 1, 0));
  if (pl.rev_rule == 1) rows *= arc_fraction(G, pl, 1, 0) * std::min(1.0, deg / n);
  double bytes = (double)scratch_fixed(G, k);
  // one depth-2 chunk of every arc (rounded to scan tiles) and the frontier
  // floor the planner keeps beside it, so a budget of this size scans in one
  // chunk
  if (k >= 3)
    bytes += (double)kDepth2BytesPerArc * ((double)G->m + hpm::kScanTile);
  double per_row_deep = 0.0;
  for (int32_t d = 3; d <= k - 1; ++d) per_row_deep += (double)row_bytes(d);
  bytes += per_row_deep * (double)kDeepFloorRows;
  for (int32_t d = 2; d + 1 < k; ++d) {
    double f = deg * vertex_fraction(G, pl, d);
    int arcs = 0;
    for (int32_t b = 0; b < d; ++b) {
      if (pl.fwd[d] & (1u << b)) {
        f *= arc_fraction(G, pl, b, d) * (arcs++ ? std::min(1.0, deg / n) : 1.0);
      }
      if (pl.bwd[d] & (1u << b)) {
        f *= arc_fraction(G, pl, d, b) * (arcs++ ? std::min(1.0, deg / n) : 1.0);
      }
    }
    rows = std::min(rows * f, 1e18);
    bytes += (double)row_bytes(d + 1) * std::min(rows, (double)(1ull << 30));
  }
  return bytes >= 1.8e19 ? ~0ull : (uint64_t)bytes;
}

}  // namespace

// ------------------------------------------------------------ serving

// Queries are admitted in arrival order by their estimated scratch bytes
// against a fixed budget: half of it is lent out as per-query grants (each
// query runs with its grant as its scratch limit, so the chunked expansion
// keeps it inside), and the workspaces of queries not running keep at most
// the other half between queries (the least recently used give theirs back
// first); device scratch therefore stays within the budget.  A query that does not fit waits while later ones that fit go
// ahead, at most kMaxBypass times, after which it blocks the queue until it
// fits.
struct hpm_server {
  struct Query {
    uint64_t ticket = 0;
    std::vector<int32_t> src, dst, vop, vval, eop, eval;
    hpm_pattern p{};
    int mode = 0;
    int32_t* maps = nullptr;
    uint64_t cap = 0;
    uint64_t est = 0, grant = 0;
    int bypassed = 0;
    std::chrono::steady_clock::time_point t_submit;
  };
  struct Result {
    bool done = false;
    hpm_query_result r{};
    std::string error;
  };
  static constexpr int kMaxBypass = 32;

  hpm_graph* G = nullptr;
  int32_t workers = 0;
  uint32_t flags = 0;
  uint64_t budget = 0, grant_pool = 0, keep = 0, min_grant = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::unique_ptr<Query>> queue;
  std::unordered_map<uint64_t, Result> results;
  uint64_t next_ticket = 1, in_use = 0;
  uint64_t admitted = 0, peak_in_use = 0;
  int32_t running = 0, peak_running = 0;
  bool stop = false;
  std::string start_error;
  std::vector<std::thread> threads;
  // workspaces of queries not running, most recently returned last; a query
  // takes the warmest (allocations already grown to the pool's sizes)
  std::vector<std::unique_ptr<Workspace>> spare;
  // Dispatch without a wake-up: while the server has idle workers, one of them
  // (the spinner) polls `events` instead of sleeping on cv_work, so a query
  // that arrives at an idle server starts within microseconds; the others
  // sleep.  A worker that takes a query wakes one sleeper to take over.
  std::atomic<uint64_t> events{0};  // submissions + completions, written under mu
  std::atomic<bool> spinner{false};
  std::atomic<bool> stopping{false};

  // Next admissible query (caller holds mu), or null.
  std::unique_ptr<Query> pick() {
    for (size_t i = 0; i < queue.size(); ++i) {
      Query& q = *queue[i];
      if (in_use + q.grant <= grant_pool) {
        if (i > 0) queue.front()->bypassed++;
        std::unique_ptr<Query> out = std::move(queue[i]);
        queue.erase(queue.begin() + (long)i);
        return out;
      }
      if (i == 0 && q.bypassed >= kMaxBypass) return nullptr;
    }
    return nullptr;
  }

  void worker() {
    using clock = std::chrono::steady_clock;
    hipStream_t s = nullptr;
    const bool ok = hipSetDevice(G->device) == hipSuccess &&
                    hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    for (;;) {
      std::unique_ptr<Query> q;
      std::unique_ptr<Workspace> W;
      bool spin = false;
      uint64_t seen = 0;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] {
          if (stop && queue.empty()) return true;
          q = pick();
          if (q) return true;
          // nobody polls for arrivals: this worker takes the role
          bool no = false;
          spin = spinner.compare_exchange_strong(no, true);
          seen = events.load(std::memory_order_relaxed);
          return spin;
        });
        if (!q && !spin) break;  // stopping with an empty queue
        if (q) {
          // admitted: its grant is taken under the same lock that picked it,
          // and the workspace returned last (the warmest) comes with it
          W = take_workspace();
          in_use += q->grant;
          peak_in_use = std::max(peak_in_use, in_use);
          running++;
          peak_running = std::max(peak_running, running);
          admitted++;
        }
      }
      if (!q) {
        // poll until a query arrives or one finishes (it may make a queued
        // one admissible) or the server stops; then give the role up and pick
        while (events.load(std::memory_order_acquire) == seen &&
               !stopping.load(std::memory_order_acquire))
          __builtin_ia32_pause();
        spinner.store(false, std::memory_order_release);
        continue;
      }
      // this worker leaves the idle set: let a sleeper take over polling
      cv_work.notify_one();
      const auto t0 = clock::now();
      int status = HPM_OK;
      uint64_t count = 0;
      std::string err;
      try {
        if (!ok) fail(HPM_E_DEVICE, "worker stream could not be created");
        status = match_one(G, &q->p, q->mode, s, flags, q->grant, &count, q->maps, q->cap,
                           nullptr, W.get());
        if (status != HPM_OK) err = t_error;
      } catch (const Failure& f) {
        status = f.status;
        err = f.msg;
      } catch (const std::bad_alloc&) {
        status = HPM_E_NOMEM;
        err = "host allocation failed";
      } catch (...) {
        status = HPM_E_INTERNAL;
        err = "unknown internal error";
      }
      if (s) (void)hipStreamSynchronize(s);  // nothing of this query is left in flight
      const auto t1 = clock::now();
      {
        std::lock_guard<std::mutex> lk(mu);
        spare.push_back(std::move(W));
        // Cached workspaces stay within half the budget: the least recently
        // returned give their memory back first, the warm ones are kept.
        uint64_t held = 0;
        for (const auto& x : spare) held += x->held();
        for (size_t j = 0; j < spare.size() && held > keep; ++j) {
          held -= spare[j]->held();
          spare[j]->release_all();
        }
        in_use -= q->grant;
        running--;
        events.fetch_add(1, std::memory_order_release);
        Result& r = results[q->ticket];
        r.done = true;
        r.error = err;
        r.r.struct_size = sizeof(hpm_query_result);
        r.r.status = status;
        r.r.count = count;
        r.r.est_bytes = q->est;
        r.r.granted_bytes = q->grant;
        r.r.queue_ms = std::chrono::duration<double, std::milli>(t0 - q->t_submit).count();
        r.r.run_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    if (s) (void)hipStreamDestroy(s);
  }

  // A workspace for an admitted query (caller holds mu): the one returned
  // last, else a new one.  At most `workers` exist.
  std::unique_ptr<Workspace> take_workspace() {
    if (spare.empty()) return std::unique_ptr<Workspace>(new Workspace());
    std::unique_ptr<Workspace> W = std::move(spare.back());
    spare.pop_back();
    return W;
  }

  ~hpm_server() {
    if (G) (void)hipSetDevice(G->device);  // the workspaces free device memory
    spare.clear();
  }
};

namespace {

// Options of hpm_match / hpm_match_batch.  Callers built against the first
// layout (no max_matches) pass the smaller struct_size.
void read_opts(const hpm_match_opts* opts, uint32_t* flags, uint64_t* budget, uint64_t* limit) {
  if (!opts) return;
  constexpr uint32_t kV1 = offsetof(hpm_match_opts, max_matches);
  if (opts->struct_size < kV1) fail(HPM_E_ARG, "opts.struct_size too small");
  *flags = opts->flags;
  *budget = opts->hbm_budget_bytes;
  if (opts->struct_size >= sizeof(hpm_match_opts)) *limit = opts->max_matches;
}

// ------------------------------------------------------------ persistent batch

// The persistent launch did not return on the device (twice, on a batch of
// small patterns; its cause is not known), so its entry points refuse to run
// it.  The code stays for the record and for a later investigation.
constexpr bool kPersistentEnabled = false;

// Arcs per scan task of the persistent launch; idle wait before a block
// leaves; launches before the rest of a batch goes to the single-query path.
constexpr int64_t kPScanArcs = 1 << 16;
constexpr int32_t kPIdleUs = 1000;
constexpr int kPMaxLaunches = 64;

hpm_batch_config batch_defaults(const hpm_batch_config* cfg) {
  hpm_batch_config c{};
  c.struct_size = sizeof(hpm_batch_config);
  c.items_per_lane = 2;
  c.chunk_rows = 256;
  c.strategy = HPM_X_MAPPED;
  c.task_work = 16384;
  c.blocks_per_cu = 0;
  if (!cfg) return c;
  if (cfg->struct_size < sizeof(hpm_batch_config)) fail(HPM_E_ARG, "cfg.struct_size too small");
  if (cfg->items_per_lane) c.items_per_lane = cfg->items_per_lane;
  if (cfg->chunk_rows) c.chunk_rows = cfg->chunk_rows;
  c.strategy = cfg->strategy;
  if (cfg->task_work) c.task_work = cfg->task_work;
  c.blocks_per_cu = cfg->blocks_per_cu;
  c.idle_us = cfg->idle_us;
  if (c.items_per_lane != 1 && c.items_per_lane != 2 && c.items_per_lane != 4)
    fail(HPM_E_ARG, "items_per_lane must be 1, 2 or 4");
  if (c.chunk_rows < 16 || c.chunk_rows > 1024) fail(HPM_E_ARG, "chunk_rows must be 16..1024");
  if (c.strategy != HPM_X_MAPPED && c.strategy != HPM_X_SHORTER) fail(HPM_E_ARG, "bad strategy");
  if (c.task_work < 256) fail(HPM_E_ARG, "task_work must be >= 256");
  if (c.blocks_per_cu < 0) fail(HPM_E_ARG, "blocks_per_cu must be >= 0");
  if (c.idle_us < 0) fail(HPM_E_ARG, "idle_us must be >= 0");
  return c;
}

// One persistent launch over the patterns that pass validation; throws
// Failure for call-level errors.  Patterns the launch could not finish
// (arena or queue full) are left with status HPM_E_NOMEM and need[i] = true
// for the caller to rerun.
void run_persistent(hpm_graph* G, int32_t n, const hpm_pattern* patterns, const int32_t* modes,
                    hipStream_t stream, uint32_t flags, uint64_t budget,
                    const hpm_batch_config& cfg, uint64_t* counts, int32_t* status,
                    std::vector<std::string>& errors, std::vector<char>& need,
                    hpm_batch_stats& bst) {
  const int64_t words = (G->n + 63) / 64 * 2;
  std::vector<DevPlan> plans((size_t)n);  // zero (k = 0) for rejected patterns
  std::vector<int64_t> base((size_t)n, 0);
  std::vector<PTask> seeds;
  int64_t bit_words = 0;
  for (int32_t i = 0; i < n; ++i) {
    counts[i] = 0;
    need[i] = 0;
    try {
      if (modes[i] != HPM_ISO && modes[i] != HPM_MONO)
        fail(HPM_E_ARG, "mode must be HPM_ISO or HPM_MONO");
      PatternInfo info = check_pattern(&patterns[i], G->n_vcols, G->n_ecols);
      std::vector<int32_t> order = plan_order(info, flags);
      plans[i] = build_dev_plan(&patterns[i], info, order, G->n_vcols, G->n_ecols, modes[i]);
      status[i] = HPM_OK;
    } catch (const Failure& f) {
      status[i] = f.status;
      errors[i] = f.msg;
      continue;
    }
    base[i] = bit_words;
    bit_words += (words * plans[i].k + 63) / 64 * 64;  // 256-byte aligned per pattern
    for (int64_t e = 0; e < G->m; e += kPScanArcs) {
      PTask t{};
      t.ready = 1;
      t.type = kTaskScan;
      t.q = i;
      t.a = e;
      t.b = std::min<int64_t>(e + kPScanArcs, G->m);
      seeds.push_back(t);
    }
  }
  // no arcs: every pattern (at least one arc) has no embedding
  if (seeds.empty()) return;

  BatchSpace* B = nullptr;
  {
    std::lock_guard<std::mutex> lk(G->mu);
    if (!G->bpool.empty()) {
      B = G->bpool.back();
      G->bpool.pop_back();
    }
  }
  if (!B) B = new BatchSpace();
  struct Return {
    hpm_graph* G;
    BatchSpace* B;
    ~Return() {
      std::lock_guard<std::mutex> lk(G->mu);
      G->bpool.push_back(B);
    }
  } ret{G, B};

  // queue: the seeds plus room for as many extension tasks again and more
  const int64_t qcap = std::min<int64_t>(
      std::max<int64_t>(2 * (int64_t)seeds.size() + (1 << 18), 1 << 18), int64_t(1) << 24);
  if ((int64_t)seeds.size() > qcap) fail(HPM_E_NOMEM, "batch has more scan tasks than queue slots");
  const uint64_t fixed = (uint64_t)n * (sizeof(DevPlan) + 8 + 8 + 4) + (uint64_t)bit_words * 4 +
                         (uint64_t)qcap * sizeof(PTask) + sizeof(PState);
  if (budget < fixed + (1u << 20))
    fail(HPM_E_NOMEM, "scratch budget below the queue, bitmaps and a 1 MiB arena");
  int64_t arena_ints = (int64_t)((budget - fixed) / 4);
  arena_ints = std::min<int64_t>(arena_ints, int64_t(1) << 33);  // 32 GiB
  if (B->held() > 2 * budget) {
    hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
    B->plans.release(); B->bits.release(); B->bit_base.release(); B->queue.release();
    B->arena.release(); B->state.release(); B->counts.release(); B->pflags.release();
  }
  B->plans.ensure((size_t)n * sizeof(DevPlan), stream);
  B->bits.ensure((size_t)std::max<int64_t>(bit_words, 1) * 4, stream);
  B->bit_base.ensure((size_t)n * 8, stream);
  B->queue.ensure((size_t)qcap * sizeof(PTask), stream);
  B->state.ensure(sizeof(PState), stream);
  B->counts.ensure((size_t)n * 8, stream);
  B->pflags.ensure((size_t)n * 4, stream);
  B->arena.ensure((size_t)arena_ints * 4, stream);
  if (B->host_n < (size_t)n) {
    if (B->host_counts) (void)hipHostFree(B->host_counts);
    if (B->host_flags) (void)hipHostFree(B->host_flags);
    B->host_counts = nullptr;
    B->host_flags = nullptr;
    hip_check(hipHostMalloc((void**)&B->host_counts, (size_t)n * 8), "hipHostMalloc");
    hip_check(hipHostMalloc((void**)&B->host_flags, (size_t)n * 4), "hipHostMalloc");
    B->host_n = (size_t)n;
  }
  if (!B->host_state)
    hip_check(hipHostMalloc((void**)&B->host_state, sizeof(PState)), "hipHostMalloc");
  for (hipEvent_t& e : B->ev)
    if (!e) hip_check(hipEventCreate(&e), "hipEventCreate");
  int clock_khz = 0;
  hip_check(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, G->device),
            "hipDeviceGetAttribute");
  if (clock_khz <= 0) clock_khz = 100000;

  hip_check(hipMemcpyAsync(B->plans.p, plans.data(), (size_t)n * sizeof(DevPlan),
                           hipMemcpyHostToDevice, stream), "upload");
  hip_check(hipMemcpyAsync(B->bit_base.p, base.data(), (size_t)n * 8, hipMemcpyHostToDevice,
                           stream), "upload");
  hip_check(hipMemsetAsync(B->counts.p, 0, (size_t)n * 8, stream), "memset");
  hip_check(hipMemsetAsync(B->pflags.p, 0, (size_t)n * 4, stream), "memset");
  // queue slots past the seeds start not ready
  hip_check(hipMemsetAsync(B->queue.p, 0, (size_t)qcap * sizeof(PTask), stream), "memset");
  hip_check(hipMemcpyAsync(B->queue.p, seeds.data(), seeds.size() * sizeof(PTask),
                           hipMemcpyHostToDevice, stream), "upload");
  PState st0{};
  st0.tail = seeds.size();
  st0.pending = seeds.size();
  hip_check(hipMemcpyAsync(B->state.p, &st0, sizeof(PState), hipMemcpyHostToDevice, stream),
            "upload");

  PParams P{};
  P.g = G->view();
  P.plans = B->plans.as<DevPlan>();
  P.bits = B->bits.as<uint32_t>();
  P.bit_base = B->bit_base.as<int64_t>();
  P.words = words;
  P.queue = B->queue.as<PTask>();
  P.qcap = qcap;
  P.arena = B->arena.as<int32_t>();
  P.arena_cap = arena_ints;
  P.st = B->state.as<PState>();
  P.counts = B->counts.as<unsigned long long>();
  P.pflags = B->pflags.as<uint32_t>();
  P.n_pat = n;
  P.chunk_rows = cfg.chunk_rows;
  P.task_work = cfg.task_work;
  P.strategy = cfg.strategy;
  P.idle_ticks = (int64_t)clock_khz * (cfg.idle_us > 0 ? cfg.idle_us : kPIdleUs) / 1000;
  int per_cu = persist_blocks_per_cu(cfg.items_per_lane);
  if (per_cu <= 0) fail(HPM_E_DEVICE, "persistent kernel does not fit on a compute unit");
  if (cfg.blocks_per_cu > 0) per_cu = std::min(per_cu, cfg.blocks_per_cu);
  const int grid = per_cu * G->num_cus;
  hip_check(hipEventRecord(B->ev[0], stream), "hipEventRecord");
  hip_check(launch_batch_validate(P.g, P.plans, P.bits, P.bit_base, words, n, stream),
            "validator launch");
  // blocks leave after waiting idle; while tasks are left, launch again
  int launches = 0;
  for (;;) {
    hip_check(launch_persist(P, cfg.items_per_lane, grid, stream), "persistent launch");
    ++launches;
    hip_check(hipMemcpyAsync(B->host_state, B->state.p, sizeof(PState), hipMemcpyDeviceToHost,
                             stream), "readback");
    hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (B->host_state->pending == 0 || launches >= kPMaxLaunches) break;
  }
  hip_check(hipEventRecord(B->ev[1], stream), "hipEventRecord");
  hip_check(hipMemcpyAsync(B->host_counts, B->counts.p, (size_t)n * 8, hipMemcpyDeviceToHost,
                           stream), "readback");
  hip_check(hipMemcpyAsync(B->host_flags, B->pflags.p, (size_t)n * 4, hipMemcpyDeviceToHost,
                           stream), "readback");
  hip_check(hipStreamSynchronize(stream), "hipStreamSynchronize");
  float ms = 0.f;
  hip_check(hipEventElapsedTime(&ms, B->ev[0], B->ev[1]), "hipEventElapsedTime");
  const PState& st = *B->host_state;
  bst.kernel_ms = ms;
  bst.error_bits = st.error;
  bst.launches = launches;
  for (int t = 0; t < 4; ++t) bst.tasks[t] = st.tasks[t];
  bst.queue_slots = st.tail;
  bst.arena_bytes = std::min<uint64_t>(st.arena_top, (uint64_t)arena_ints) * 4;
  bst.scratch_bytes = B->held();
  bst.fixed_bytes = fixed;
  bst.arena_capacity = (uint64_t)arena_ints * 4;
  bst.grid = grid;
  // work left after the last launch: nothing of this batch is certain
  const bool incomplete = st.pending != 0;
  for (int32_t i = 0; i < n; ++i) {
    if (status[i] != HPM_OK) continue;
    const uint32_t f = B->host_flags[i];
    if (incomplete || (f & kPatFailed)) {
      need[i] = 1;
    } else if (f & kPatOverflow) {
      status[i] = HPM_E_OVERFLOW;
      errors[i] = "embedding count exceeds 2^64-1";
    } else {
      counts[i] = B->host_counts[i];
    }
  }
}

int batch_persistent(hpm_graph* G, int32_t n, const hpm_pattern* patterns, const int32_t* modes,
                     hipStream_t stream, const hpm_match_opts* opts, const hpm_batch_config* cfgp,
                     uint64_t* counts, int32_t* status) {
  const auto t0 = std::chrono::steady_clock::now();
  if (n < 0 || (n > 0 && (!patterns || !modes || !counts || !status)))
    fail(HPM_E_ARG, "NULL batch arrays");
  if (n > 65535) fail(HPM_E_ARG, "at most 65535 patterns per batch");
  const hpm_batch_config cfg = batch_defaults(cfgp);
  uint32_t flags = 0;
  uint64_t budget = 0, limit = 0;
  read_opts(opts, &flags, &budget, &limit);
  flags &= ~(uint32_t)HPM_F_TIMING;
  hip_check(hipSetDevice(G->device), "hipSetDevice");
  hpm_batch_stats bst{};
  bst.struct_size = sizeof(hpm_batch_stats);
  std::vector<std::string> errors((size_t)n);
  std::vector<char> need((size_t)n, 0);
  if (budget == 0) {
    size_t free_b = 0, total_b = 0;
    hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    uint64_t pooled = 0;
    {
      std::lock_guard<std::mutex> lk(G->mu);
      for (const BatchSpace* b : G->bpool) pooled += b->held();
    }
    budget = ((uint64_t)free_b + pooled) / 4;
  }
  if (limit || (flags & (HPM_F_OVERLAP | HPM_F_LOOKAHEAD))) {
    // first-k and the overlap test are options of the single-query path
    for (int32_t i = 0; i < n; ++i) need[i] = 1;
  } else if (n > 0) {
    run_persistent(G, n, patterns, modes, stream, flags, budget, cfg, counts, status, errors,
                   need, bst);
  }
  for (int32_t i = 0; i < n; ++i) {
    if (!need[i]) continue;
    bst.fallback_patterns++;
    try {
      status[i] = match_one(G, &patterns[i], modes[i], stream, flags, budget, &counts[i], nullptr,
                            0, nullptr, nullptr, limit);
    } catch (const Failure& f) {
      status[i] = f.status;
      errors[i] = f.msg;
    }
  }
  bst.ms_total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  t_bstats = bst;
  for (int32_t i = 0; i < n; ++i)
    if (status[i] != HPM_OK) {
      t_error = "pattern " + std::to_string(i) + ": " + errors[i];
      return status[i];
    }
  return HPM_OK;
}

// ------------------------------------------------------------ allocation-free match

// The device scratch of hpm_match_noalloc: one array per GPU, held until the
// process ends.  In host code `scratch` is only a handle; its device address
// comes from hipGetSymbolAddress, once per device (noalloc_state).
constexpr size_t kNoAllocBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;

struct NoAllocState {
  std::mutex mu;              // one allocation-free call per device at a time
  bool ready = false;
  char* dev = nullptr;        // device address of this device's scratch
  Workspace* ws = nullptr;    // host-side bookkeeping, never freed
  unsigned long long host[kCntNum];  // readback slots (pageable)
  DevPlan host_plan;
};
NoAllocState g_noalloc[kMaxDevices];

// Resolve the device's scratch address once (the device must be current).
NoAllocState& noalloc_state(int device) {
  if (device < 0 || device >= kMaxDevices) fail(HPM_E_UNSUPPORTED, "device index out of range");
  NoAllocState& S = g_noalloc[device];
  if (!S.ready) {
    void* ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    if (!ptr) fail(HPM_E_DEVICE, "no device address for the allocation-free scratch");
    S.dev = static_cast<char*>(ptr);
    S.ws = new Workspace();
    S.ws->host = S.host;
    S.ws->host_plan = &S.host_plan;
    S.ready = true;
  }
  return S;
}

}  // namespace

extern "C" {

int hpm_match_noalloc(const hpm_graph* gc, const hpm_pattern* p, hpm_mode mode, void* stream,
                      const hpm_match_opts* opts, uint64_t* count, int32_t* mappings,
                      uint64_t cap) {
  return guarded([&]() -> int {
    if (!gc) fail(HPM_E_ARG, "graph is NULL");
    if (!count) fail(HPM_E_ARG, "count is NULL");
    uint32_t flags = 0;
    uint64_t budget = 0, limit = 0;
    read_opts(opts, &flags, &budget, &limit);
    // events are created on demand: no per-kernel timing here
    flags &= ~(uint32_t)(HPM_F_TIMING | (0xffu << 16));
    hpm_graph* G = const_cast<hpm_graph*>(gc);
    int cur = 0;
    hip_check(hipGetDevice(&cur), "hipGetDevice");
    if (cur != G->device) hip_check(hipSetDevice(G->device), "hipSetDevice");
    struct Restore {
      int prev, now;
      ~Restore() {
        if (prev != now) (void)hipSetDevice(prev);
      }
    } restore{cur, G->device};
    NoAllocState& S = [&]() -> NoAllocState& {
      static std::mutex init_mu;
      std::lock_guard<std::mutex> lk(init_mu);
      return noalloc_state(G->device);
    }();
    std::lock_guard<std::mutex> lk(S.mu);
    // Buffers grow by at least doubling, so what a call carves stays within
    // four times what it asks for: it runs with a quarter of the scratch as
    // its budget (or less, if the caller asks for less).
    const uint64_t most = kNoAllocBytes / 4;
    if (budget == 0 || budget > most) budget = most;
    Carve carve{S.dev, kNoAllocBytes, 0};
    Workspace* W = S.ws;
    W->release_all();  // forget the previous call's regions (nothing is freed)
    t_carve = &carve;
    struct Clear {
      ~Clear() { t_carve = nullptr; }
    } clear;
    return match_one(G, p, (int)mode, static_cast<hipStream_t>(stream), flags, budget, count,
                     mappings, cap, &t_stats, W, limit);
  });
}

int hpm_scan_survivors(const hpm_graph* gc, const hpm_pattern* p, hpm_mode mode, void* stream,
                       const hpm_match_opts* opts, uint64_t* count, int32_t* rows,
                       uint64_t cap) {
  return guarded([&]() -> int {
    if (!gc) fail(HPM_E_ARG, "graph is NULL");
    if (!count) fail(HPM_E_ARG, "count is NULL");
    uint32_t flags = 0;
    uint64_t budget = 0, limit = 0;
    read_opts(opts, &flags, &budget, &limit);
    flags &= ~(uint32_t)(HPM_F_OVERLAP | HPM_F_LOOKAHEAD | HPM_F_COUNT_FROM_MAX);
    const SurvivorsOut out{rows, rows ? cap : 0};
    const int st = match_one(const_cast<hpm_graph*>(gc), p, (int)mode,
                             static_cast<hipStream_t>(stream), flags, budget, count, nullptr, 0,
                             &t_stats, nullptr, 0, &out);
    if (st == HPM_OK && rows && *count > cap) {
      t_error = "survivors " + std::to_string(*count) + " exceed cap " + std::to_string(cap);
      return HPM_E_TRUNCATED;
    }
    return st;
  });
}

int hpm_match(const hpm_graph* gc, const hpm_pattern* p, hpm_mode mode, void* stream,
              const hpm_match_opts* opts, uint64_t* count, int32_t* mappings, uint64_t cap) {
  return guarded([&]() -> int {
    if (!gc) fail(HPM_E_ARG, "graph is NULL");
    if (!count) fail(HPM_E_ARG, "count is NULL");
    uint32_t flags = 0;
    uint64_t budget = 0, limit = 0;
    read_opts(opts, &flags, &budget, &limit);
    return match_one(const_cast<hpm_graph*>(gc), p, (int)mode, static_cast<hipStream_t>(stream),
                     flags, budget, count, mappings, cap, &t_stats, nullptr, limit);
  });
}

int hpm_match_batch(const hpm_graph* gc, int32_t n, const hpm_pattern* patterns,
                    const int32_t* modes, void* stream, const hpm_match_opts* opts,
                    int32_t workers, uint64_t* counts, int32_t* status) {
  return guarded([&]() -> int {
    if (!gc) fail(HPM_E_ARG, "graph is NULL");
    if (n < 0 || (n > 0 && (!patterns || !modes || !counts || !status)))
      fail(HPM_E_ARG, "NULL batch arrays");
    if (workers < 0 || workers > 64) fail(HPM_E_ARG, "workers must be 0..64");
    if (workers == 0) workers = 4;
    workers = std::min<int32_t>(workers, std::max<int32_t>(n, 1));
    uint32_t flags = 0;
    uint64_t budget = 0, limit = 0;
    read_opts(opts, &flags, &budget, &limit);
    flags &= ~(uint32_t)HPM_F_TIMING;
    hpm_graph* G = const_cast<hpm_graph*>(gc);
    hip_check(hipSetDevice(G->device), "hipSetDevice");
    if (budget == 0) {
      size_t free_b = 0, total_b = 0;
      hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
      uint64_t pooled = 0;
      {
        std::lock_guard<std::mutex> lk(G->mu);
        for (const Workspace* w : G->pool) pooled += w->held();
      }
      budget = ((uint64_t)free_b + pooled) / 4;
    }
    const uint64_t share = budget / (uint64_t)workers;
    // work issued on the caller's stream before the batch comes first
    hip_check(hipStreamSynchronize(static_cast<hipStream_t>(stream)), "hipStreamSynchronize");
    std::atomic<int32_t> next(0);
    std::vector<std::string> errors((size_t)n);
    auto worker = [&]() {
      (void)hipSetDevice(G->device);
      hipStream_t s = nullptr;
      if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
      for (int32_t i = next++; i < n; i = next++) {
        try {
          if (!s) fail(HPM_E_DEVICE, "hipStreamCreateWithFlags failed");
          status[i] = match_one(G, &patterns[i], modes[i], s, flags, share, &counts[i], nullptr, 0,
                                nullptr, nullptr, limit);
        } catch (const Failure& f) {
          status[i] = f.status;
          errors[i] = f.msg;
        } catch (const std::bad_alloc&) {
          status[i] = HPM_E_NOMEM;
        } catch (...) {
          status[i] = HPM_E_INTERNAL;
        }
      }
      if (s) (void)hipStreamDestroy(s);
    };
    std::vector<std::thread> pool;
    for (int32_t w = 1; w < workers; ++w) pool.emplace_back(worker);
    worker();
    for (std::thread& t : pool) t.join();
    for (int32_t i = 0; i < n; ++i)
      if (status[i] != HPM_OK) {
        t_error = "pattern " + std::to_string(i) + ": " + errors[i];
        return status[i];
      }
    return HPM_OK;
  });
}

int hpm_batch_tune(const hpm_graph* gc, int32_t n, const hpm_pattern* patterns,
                   const int32_t* modes, void* stream, const hpm_match_opts* opts,
                   int32_t* best_workers, double* best_ms) {
  return guarded([&]() -> int {
    if (!best_workers) fail(HPM_E_ARG, "best_workers is NULL");
    if (n <= 0) fail(HPM_E_ARG, "empty batch");
    std::vector<uint64_t> counts((size_t)n), first((size_t)n);
    std::vector<int32_t> status((size_t)n);
    // one untimed pass grows every worker's scratch to its working size
    int st = hpm_match_batch(gc, n, patterns, modes, stream, opts, 16, first.data(), status.data());
    if (st != HPM_OK) return st;
    static const int32_t kCandidates[] = {1, 2, 4, 8, 16, 32};
    double best = -1.0;
    int32_t arg = 0;
    for (int32_t w : kCandidates) {
      const auto t0 = std::chrono::steady_clock::now();
      st = hpm_match_batch(gc, n, patterns, modes, stream, opts, w, counts.data(), status.data());
      const double ms =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (st != HPM_OK) return st;
      if (counts != first) fail(HPM_E_INTERNAL, "batch counts differ between worker counts");
      if (best < 0.0 || ms < best) {
        best = ms;
        arg = w;
      }
    }
    *best_workers = arg;
    if (best_ms) *best_ms = best;
    return HPM_OK;
  });
}

int hpm_match_batch_persistent(const hpm_graph* gc, int32_t n, const hpm_pattern* patterns,
                               const int32_t* modes, void* stream, const hpm_match_opts* opts,
                               const hpm_batch_config* cfg, uint64_t* counts, int32_t* status) {
  return guarded([&]() -> int {
    if (!kPersistentEnabled)
      fail(HPM_E_UNSUPPORTED, "the persistent batched launch is switched off (it stalled on "
                              "the device and no cause has been shown)");
    if (!gc) fail(HPM_E_ARG, "graph is NULL");
    return batch_persistent(const_cast<hpm_graph*>(gc), n, patterns, modes,
                            static_cast<hipStream_t>(stream), opts, cfg, counts, status);
  });
}

int hpm_batch_autotune(const hpm_graph* gc, int32_t n, const hpm_pattern* patterns,
                       const int32_t* modes, void* stream, const hpm_match_opts* opts,
                       hpm_batch_config* best, double* best_ms) {
  return guarded([&]() -> int {
    if (!kPersistentEnabled)
      fail(HPM_E_UNSUPPORTED, "the persistent batched launch is switched off (it stalled on "
                              "the device and no cause has been shown)");
    if (!gc) fail(HPM_E_ARG, "graph is NULL");
    if (!best) fail(HPM_E_ARG, "best is NULL");
    if (n <= 0) fail(HPM_E_ARG, "empty batch");
    hpm_graph* G = const_cast<hpm_graph*>(gc);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<uint64_t> counts((size_t)n), first((size_t)n);
    std::vector<int32_t> status((size_t)n);
    hpm_batch_config c = batch_defaults(nullptr);
    // one untimed run sizes the scratch and gives the reference counts
    int st = batch_persistent(G, n, patterns, modes, s, opts, &c, first.data(), status.data());
    if (st != HPM_OK) return st;
    double top = -1.0;
    hpm_batch_config arg = c;
    for (int32_t items : {1, 2, 4})
      for (int32_t rows : {64, 256, 1024})
        for (int64_t work : {int64_t(4096), int64_t(65536)})
          for (int32_t strat : {HPM_X_MAPPED, HPM_X_SHORTER}) {
            c.items_per_lane = items;
            c.chunk_rows = rows;
            c.task_work = work;
            c.strategy = strat;
            st = batch_persistent(G, n, patterns, modes, s, opts, &c, counts.data(),
                                  status.data());
            if (st != HPM_OK) return st;
            if (counts != first) fail(HPM_E_INTERNAL, "batch counts differ between settings");
            const double ms = t_bstats.fallback_patterns ? t_bstats.ms_total : t_bstats.kernel_ms;
            if (top < 0.0 || ms < top) {
              top = ms;
              arg = c;
            }
          }
    *best = arg;
    if (best_ms) *best_ms = top;
    return HPM_OK;
  });
}

int hpm_last_batch_stats(hpm_batch_stats* out) {
  if (!out) return HPM_E_ARG;
  *out = t_bstats;
  return HPM_OK;
}

int hpm_server_create(hpm_server** out, const hpm_graph* gc, const hpm_server_opts* opts) {
  return guarded([&]() -> int {
    if (!out) fail(HPM_E_ARG, "out is NULL");
    *out = nullptr;
    if (!gc) fail(HPM_E_ARG, "graph is NULL");
    if (opts && opts->struct_size < sizeof(hpm_server_opts))
      fail(HPM_E_ARG, "opts.struct_size too small");
    int32_t workers = opts ? opts->workers : 0;
    if (workers < 0 || workers > 64) fail(HPM_E_ARG, "workers must be 0..64");
    if (workers == 0) workers = 4;
    hpm_graph* G = const_cast<hpm_graph*>(gc);
    hip_check(hipSetDevice(G->device), "hipSetDevice");
    uint64_t budget = opts ? opts->hbm_budget_bytes : 0;
    if (budget == 0) {
      size_t free_b = 0, total_b = 0;
      hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
      budget = free_b / 4;
    }
    std::unique_ptr<hpm_server> S(new hpm_server());
    S->G = G;
    S->workers = workers;
    S->flags = opts ? (opts->flags & ~(uint32_t)HPM_F_TIMING) : 0;
    S->budget = budget;
    S->grant_pool = budget / 2;
    S->keep = budget / 2;
    S->min_grant = std::min<uint64_t>(S->grant_pool, (uint64_t)256 << 20);
    if (S->grant_pool < scratch_fixed(G, HPM_MAX_K) + (uint64_t)hpm::kScanTile * 64)
      fail(HPM_E_NOMEM, "serving budget too small");
    hpm_server* raw = S.get();
    for (int32_t w = 0; w < workers; ++w) S->threads.emplace_back([raw] { raw->worker(); });
    *out = S.release();
    return HPM_OK;
  });
}

int hpm_server_submit(hpm_server* S, const hpm_pattern* p, hpm_mode mode, int32_t* mappings,
                      uint64_t cap, uint64_t* ticket) {
  return guarded([&]() -> int {
    if (!S) fail(HPM_E_ARG, "server is NULL");
    if (!ticket) fail(HPM_E_ARG, "ticket is NULL");
    if (mode != HPM_ISO && mode != HPM_MONO) fail(HPM_E_ARG, "mode must be HPM_ISO or HPM_MONO");
    hpm_graph* G = S->G;
    PatternInfo info = check_pattern(p, G->n_vcols, G->n_ecols);
    if (mappings && cap > (uint64_t)INT64_MAX / (uint64_t)info.k) fail(HPM_E_ARG, "cap too large");
    std::unique_ptr<hpm_server::Query> q(new hpm_server::Query());
    const size_t na = (size_t)p->n_arcs;
    q->src.assign(p->src, p->src + na);
    q->dst.assign(p->dst, p->dst + na);
    if (p->vop) {
      const size_t nv = (size_t)info.k * (size_t)G->n_vcols;
      q->vop.assign(p->vop, p->vop + nv);
      q->vval.assign(p->vval, p->vval + nv);
    }
    if (p->eop) {
      const size_t ne = na * (size_t)G->n_ecols;
      q->eop.assign(p->eop, p->eop + ne);
      q->eval.assign(p->eval, p->eval + ne);
    }
    q->p = hpm_pattern{info.k, p->n_arcs, q->src.data(), q->dst.data(),
                       p->vop ? q->vop.data() : nullptr, p->vop ? q->vval.data() : nullptr,
                       p->eop ? q->eop.data() : nullptr, p->eop ? q->eval.data() : nullptr};
    q->mode = (int)mode;
    q->maps = mappings;
    q->cap = mappings ? cap : 0;
    const DevPlan plan = build_dev_plan(&q->p, info, plan_order(info, S->flags), G->n_vcols,
                                        G->n_ecols, (int)mode);
    q->est = estimate_scratch(G, plan);
    // twice the estimate: its deep-frontier part comes from column samples,
    // and a query granted less than its frontiers need runs in more pieces
    q->grant = std::max(S->min_grant, std::min(2 * q->est, S->grant_pool));
    q->t_submit = std::chrono::steady_clock::now();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      if (S->stop) fail(HPM_E_ARG, "server is shutting down");
      q->ticket = S->next_ticket++;
      *ticket = q->ticket;
      S->results[q->ticket] = hpm_server::Result{};
      S->queue.push_back(std::move(q));
      S->events.fetch_add(1, std::memory_order_release);
    }
    S->cv_work.notify_one();
    return HPM_OK;
  });
}

int hpm_server_poll(hpm_server* S, uint64_t ticket, int32_t wait, hpm_query_result* out) {
  return guarded([&]() -> int {
    if (!S) fail(HPM_E_ARG, "server is NULL");
    if (!out) fail(HPM_E_ARG, "out is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->results.find(ticket);
    if (it == S->results.end()) fail(HPM_E_ARG, "unknown ticket");
    if (!it->second.done) {
      if (!wait) return HPM_PENDING;
      S->cv_done.wait(lk, [&] {
        auto j = S->results.find(ticket);
        return j == S->results.end() || j->second.done;
      });
      it = S->results.find(ticket);
      if (it == S->results.end()) fail(HPM_E_ARG, "ticket collected by another thread");
    }
    *out = it->second.r;
    if (out->status != HPM_OK && out->status != HPM_E_TRUNCATED) t_error = it->second.error;
    S->results.erase(it);
    return HPM_OK;
  });
}

int hpm_server_read_stats(hpm_server* S, hpm_server_stats* out) {
  return guarded([&]() -> int {
    if (!S) fail(HPM_E_ARG, "server is NULL");
    if (!out) fail(HPM_E_ARG, "out is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    out->struct_size = sizeof(hpm_server_stats);
    out->workers = S->workers;
    out->running = S->running;
    out->queued = (int32_t)S->queue.size();
    out->peak_running = S->peak_running;
    out->budget_bytes = S->budget;
    out->grant_pool_bytes = S->grant_pool;
    out->granted_bytes = S->in_use;
    out->peak_granted_bytes = S->peak_in_use;
    out->admitted = S->admitted;
    return HPM_OK;
  });
}

int hpm_server_destroy(hpm_server* S) {
  return guarded([&]() -> int {
    if (!S) return HPM_OK;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->stop = true;
    }
    S->stopping.store(true, std::memory_order_release);
    S->cv_work.notify_all();
    for (std::thread& t : S->threads) t.join();
    delete S;
    return HPM_OK;
  });
}

}  // extern "C"
