// hpm_oracle.cpp -- TEST INFRASTRUCTURE ONLY.  Plain CPU reference matcher.
//
// This file is the oracle against which the HIP matcher is checked.  Only the
// test suite, the smoke check and the benchmark's CPU-baseline leg may load it;
// the product path never links, loads or calls it, and it shares no code,
// header or table with the library.
//
// What it computes is the plain definition of the problem (Sec. II-A):
// all injective maps f from pattern vertices to target vertices such that
//   * every pattern arc (a,b) maps onto a target arc (f(a),f(b))          Eq. (1), "=>"
//   * for induced isomorphism also every non-arc maps onto a non-arc      Eq. (1), "<="
//     (monomorphism drops this direction, Sec. II-A last paragraph)
//   * every vertex predicate holds on f(a)                                Eq. (2)
//   * every arc predicate holds on the image arc's attributes             Eq. (3)
// Predicates generalise the label equality of Eq. (2)-(3) to one of
// {ANY, EQ value, GE value} per attribute column, conjunctively.
//
// The search is the textbook one: start from the empty mapping, fix the
// pattern vertices in a breadth-first order over the undirected pattern, and
// take the candidates for each vertex from the adjacency of an already mapped
// neighbour (all target vertices when there is none).  Every candidate is
// checked against every mapped vertex, in both arc directions.  There is no
// degree reordering, no validator and no edge-centric start here: those are
// the accelerations the paper adds (Sec. III), and the paper's correctness and
// completeness theorems (Sec. III-C) say they reach this same set.
//
// Counted objects are embeddings (injective maps), so automorphic images are
// distinct results.  Self-loops are not expected in either graph.
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <omp.h>

#include <atomic>

namespace {

struct Graph {
  int32_t n;
  int64_t m;
  const int64_t* out_off;
  const int32_t* out_nbrs;
  const int64_t* in_off;
  const int32_t* in_nbrs;
  int32_t n_vcols;
  const int32_t* vcols;  // [n_vcols][n]
  int32_t n_ecols;
  const int32_t* ecols;  // [n_ecols][m], out-CSR arc order
};

struct Pattern {
  int32_t k, n_arcs;
  const int32_t *src, *dst;
  const int32_t *vop, *vval;  // [k][n_vcols]
  const int32_t *eop, *eval;  // [n_arcs][n_ecols]
};

enum { OP_ANY = 0, OP_EQ = 1, OP_GE = 2 };
enum { MODE_ISO = 0, MODE_MONO = 1 };

bool pred(int32_t op, int32_t val, int32_t x) {
  if (op == OP_ANY) return true;
  if (op == OP_EQ) return x == val;
  return x >= val;  // OP_GE
}

// Out-CSR position of arc u->v, or -1 when there is no such arc.
int64_t find_arc(const Graph& g, int32_t u, int32_t v) {
  const int32_t* lo = g.out_nbrs + g.out_off[u];
  const int32_t* hi = g.out_nbrs + g.out_off[u + 1];
  const int32_t* it = std::lower_bound(lo, hi, v);
  if (it != hi && *it == v) return it - g.out_nbrs;
  return -1;
}

struct Plan {
  int32_t k;
  std::vector<int32_t> order;     // order[d] = pattern vertex fixed at depth d
  std::vector<int32_t> anchor;    // earlier pattern vertex supplying candidates, or -1
  std::vector<int32_t> anchor_out;// 1: candidates are out(f(anchor)), 0: in(f(anchor))
  std::vector<int32_t> arc_id;    // [k*k]: pattern arc index of (a,b), or -1
};

Plan make_plan(const Pattern& p) {
  Plan pl;
  pl.k = p.k;
  pl.arc_id.assign((size_t)p.k * p.k, -1);
  for (int32_t i = 0; i < p.n_arcs; ++i) pl.arc_id[(size_t)p.src[i] * p.k + p.dst[i]] = i;
  // Breadth-first order over the undirected pattern, neighbours by increasing id;
  // a new component (if any) starts at its smallest unvisited vertex.
  std::vector<char> seen(p.k, 0);
  for (int32_t s = 0; s < p.k; ++s) {
    if (seen[s]) continue;
    seen[s] = 1;
    size_t head = pl.order.size();
    pl.order.push_back(s);
    while (head < pl.order.size()) {
      int32_t x = pl.order[head++];
      for (int32_t y = 0; y < p.k; ++y) {
        bool adj = pl.arc_id[(size_t)x * p.k + y] >= 0 || pl.arc_id[(size_t)y * p.k + x] >= 0;
        if (adj && !seen[y]) { seen[y] = 1; pl.order.push_back(y); }
      }
    }
  }
  pl.anchor.assign(p.k, -1);
  pl.anchor_out.assign(p.k, 0);
  for (int32_t d = 1; d < p.k; ++d) {
    int32_t a = pl.order[d];
    for (int32_t e = 0; e < d; ++e) {
      int32_t b = pl.order[e];
      if (pl.arc_id[(size_t)b * p.k + a] >= 0) { pl.anchor[d] = b; pl.anchor_out[d] = 1; break; }
      if (pl.arc_id[(size_t)a * p.k + b] >= 0) { pl.anchor[d] = b; pl.anchor_out[d] = 0; break; }
    }
  }
  return pl;
}

// SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014).
inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

inline uint64_t row_hash(const int32_t* row, int32_t k, uint64_t seed) {
  uint64_t h = mix64(seed ^ (uint64_t)k);
  for (int32_t i = 0; i < k; ++i)
    h = mix64(h ^ ((uint64_t)(uint32_t)row[i] + 0x9e3779b97f4a7c15ULL * (uint64_t)(i + 1)));
  return h;
}

const uint64_t kSeed1 = 0x243f6a8885a308d3ULL;
const uint64_t kSeed2 = 0x13198a2e03707344ULL;

struct Search {
  const Graph& g;
  const Pattern& p;
  const Plan& pl;
  int mode;
  bool keep_rows;
  std::vector<int32_t> f;       // f[pattern vertex] = target vertex (valid when mapped)
  uint64_t count = 0;
  uint64_t fp1 = 0, fp2 = 0;    // running fingerprint of the rows found
  // Optional bound on the search: every candidate image tested at any depth
  // (roots included) is one step; local tallies are flushed into *shared
  // every kFlush steps and the search stops once the shared total passes cap
  // (0 = unbounded).
  static constexpr uint64_t kFlush = 1 << 14;
  uint64_t cap = 0, tested = 0, unflushed = 0;
  std::atomic<uint64_t>* shared = nullptr;
  std::atomic<bool>* stop = nullptr;
  std::vector<int32_t> rows;    // flattened [count][k], original pattern order

  Search(const Graph& g_, const Pattern& p_, const Plan& pl_, int mode_, bool keep)
      : g(g_), p(p_), pl(pl_), mode(mode_), keep_rows(keep), f(p_.k, -1) {}

  bool vertex_ok(int32_t a, int32_t c) const {
    for (int32_t col = 0; col < g.n_vcols; ++col)
      if (!pred(p.vop[a * g.n_vcols + col], p.vval[a * g.n_vcols + col],
                g.vcols[(int64_t)col * g.n + c]))
        return false;
    return true;
  }

  bool arc_ok(int32_t arc, int64_t eid) const {
    for (int32_t col = 0; col < g.n_ecols; ++col)
      if (!pred(p.eop[arc * g.n_ecols + col], p.eval[arc * g.n_ecols + col],
                g.ecols[(int64_t)col * g.m + eid]))
        return false;
    return true;
  }

  // Pattern pair (a,b) at index ab = a*k+b against the target pair (u,v):
  // a pattern arc needs the target arc with its predicate; a pattern non-arc
  // needs a target non-arc under induced isomorphism and nothing otherwise.
  bool pair_ok(int32_t ab, int32_t u, int32_t v) const {
    int32_t arc = pl.arc_id[(size_t)ab];
    if (arc < 0 && mode != MODE_ISO) return true;
    int64_t eid = find_arc(g, u, v);
    if (arc >= 0) return eid >= 0 && arc_ok(arc, eid);
    return eid < 0;
  }

  // Is target vertex c a consistent image for pattern vertex a at depth d?
  bool feasible(int32_t d, int32_t a, int32_t c) const {
    for (int32_t e = 0; e < d; ++e)
      if (f[pl.order[e]] == c) return false;  // injectivity
    if (!vertex_ok(a, c)) return false;
    for (int32_t e = 0; e < d; ++e) {
      int32_t b = pl.order[e];
      int32_t fb = f[b];
      // direction b -> a, then a -> b; an absent pattern arc constrains the
      // target only under induced isomorphism, so monomorphism skips its lookup
      if (!pair_ok(b * p.k + a, fb, c) || !pair_ok(a * p.k + b, c, fb)) return false;
    }
    return true;
  }

  void extend(int32_t d) {
    if (d == p.k) {
      ++count;
      fp1 += row_hash(f.data(), p.k, kSeed1);
      fp2 += row_hash(f.data(), p.k, kSeed2);
      if (keep_rows) rows.insert(rows.end(), f.begin(), f.end());
      return;
    }
    int32_t a = pl.order[d];
    int32_t b = pl.anchor[d];
    if (b < 0) {
      for (int32_t c = 0; c < g.n; ++c) try_candidate(d, a, c);
      return;
    }
    int32_t fb = f[b];
    if (pl.anchor_out[d]) {
      for (int64_t i = g.out_off[fb]; i < g.out_off[fb + 1]; ++i) try_candidate(d, a, g.out_nbrs[i]);
    } else {
      for (int64_t i = g.in_off[fb]; i < g.in_off[fb + 1]; ++i) try_candidate(d, a, g.in_nbrs[i]);
    }
  }

  void try_candidate(int32_t d, int32_t a, int32_t c) {
    if (cap && stop->load(std::memory_order_relaxed)) return;
    tally();
    if (!feasible(d, a, c)) return;
    f[a] = c;
    extend(d + 1);
    f[a] = -1;
  }

  void tally() {
    ++tested;
    if (!cap || ++unflushed < kFlush) return;
    flush();
  }

  void flush() {
    if (shared->fetch_add(unflushed) + unflushed > cap) stop->store(true);
    unflushed = 0;
  }
};

void sort_rows_impl(int32_t* rows, uint64_t count, int32_t k) {
  std::vector<uint64_t> idx(count);
  for (uint64_t i = 0; i < count; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](uint64_t x, uint64_t y) {
    const int32_t* a = rows + x * k;
    const int32_t* b = rows + y * k;
    for (int32_t i = 0; i < k; ++i)
      if (a[i] != b[i]) return a[i] < b[i];
    return false;
  });
  std::vector<int32_t> tmp((size_t)count * k);
  for (uint64_t i = 0; i < count; ++i)
    std::memcpy(&tmp[i * k], rows + idx[i] * k, sizeof(int32_t) * k);
  if (!tmp.empty()) std::memcpy(rows, tmp.data(), sizeof(int32_t) * tmp.size());
}

}  // namespace

extern "C" {

// Result of one oracle run.  rows (if requested) is malloc'ed, [count][k] in
// original pattern-vertex order, sorted lexicographically; free with og_free.
typedef struct {
  uint64_t count;
  uint64_t fp1, fp2;   // order-independent fingerprint of the row set
  int32_t* rows;
} og_result;

// g_*: host CSR arrays as described on the Graph struct above.  root_mask: NULL
// (all roots) or uint8[n]; when given, only embeddings whose image of the first
// breadth-first vertex (pattern vertex 0 for a connected pattern) has a nonzero
// mask entry are enumerated.  max_tested: 0, or a bound on the number of
// candidate images (one target vertex for one pattern vertex, roots included)
// the search may test; the total tested is written to *tested when non-NULL.
// Returns 0; 1 when the bound was passed (count and rows are then not valid;
// the decision depends only on the total, not on thread timing); -1 on bad
// arguments.
int og_match(int32_t n, int64_t m, const int64_t* out_off, const int32_t* out_nbrs,
             const int64_t* in_off, const int32_t* in_nbrs, int32_t n_vcols, const int32_t* vcols,
             int32_t n_ecols, const int32_t* ecols, int32_t k, int32_t n_arcs, const int32_t* src,
             const int32_t* dst, const int32_t* vop, const int32_t* vval, const int32_t* eop,
             const int32_t* eval, int32_t mode, int32_t n_threads, const uint8_t* root_mask,
             int32_t keep_rows, uint64_t max_tested, uint64_t* tested, og_result* res) {
  if (!res || k < 1 || n < 0 || m < 0) return -1;
  std::atomic<uint64_t> shared_tested{0};
  std::atomic<bool> stop{false};
  Graph g{n, m, out_off, out_nbrs, in_off, in_nbrs, n_vcols, vcols, n_ecols, ecols};
  Pattern p{k, n_arcs, src, dst, vop, vval, eop, eval};
  Plan pl = make_plan(p);
  int32_t root = pl.order[0];
  if (n_threads <= 0) n_threads = omp_get_max_threads();
  std::vector<Search*> per(n_threads, nullptr);
  uint64_t total = 0, fp1 = 0, fp2 = 0, n_tested = 0;
#pragma omp parallel num_threads(n_threads) reduction(+ : total, fp1, fp2, n_tested)
  {
    int tid = omp_get_thread_num();
    Search* s = new Search(g, p, pl, mode, keep_rows != 0);
    s->cap = max_tested;
    s->shared = &shared_tested;
    s->stop = &stop;
    per[tid] = s;
#pragma omp for schedule(dynamic, 16)
    for (int32_t x = 0; x < n; ++x) {
      if (root_mask && !root_mask[x]) continue;
      s->try_candidate(0, root, x);
    }
    if (max_tested) s->flush();
    total += s->count;
    fp1 += s->fp1;
    fp2 += s->fp2;
    n_tested += s->tested;
  }
  if (tested) *tested = n_tested;
  if (max_tested && (stop.load() || n_tested > max_tested)) {
    for (Search* s : per) delete s;
    res->count = 0;
    res->fp1 = res->fp2 = 0;
    res->rows = nullptr;
    return 1;
  }
  res->count = total;
  res->fp1 = fp1;
  res->fp2 = fp2;
  res->rows = nullptr;
  if (keep_rows) {
    int32_t* rows = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)total * k + 1);
    size_t off = 0;
    for (Search* s : per) {
      if (!s || s->rows.empty()) continue;  // memcpy from an empty vector's NULL is undefined
      std::memcpy(rows + off, s->rows.data(), sizeof(int32_t) * s->rows.size());
      off += s->rows.size();
    }
    sort_rows_impl(rows, total, k);
    res->rows = rows;
  }
  for (Search* s : per) delete s;
  return 0;
}

// Membership test of given rows in the result set (the definition, Sec. II-A,
// Eq. (1)-(3), applied to one complete map at a time): row i (original pattern
// order) is an embedding when its images are pairwise distinct, every vertex
// predicate holds, every pattern arc (a,b) has the target arc (f(a),f(b)) with
// its predicate, and under induced isomorphism every other ordered pair maps to
// a non-arc.  ok[i] receives 1 or 0; returns the number of rows that pass, or
// -1 on bad arguments.
int64_t og_check_rows(int32_t n, int64_t m, const int64_t* out_off, const int32_t* out_nbrs,
                      const int64_t* in_off, const int32_t* in_nbrs, int32_t n_vcols,
                      const int32_t* vcols, int32_t n_ecols, const int32_t* ecols, int32_t k,
                      int32_t n_arcs, const int32_t* src, const int32_t* dst, const int32_t* vop,
                      const int32_t* vval, const int32_t* eop, const int32_t* eval, int32_t mode,
                      int32_t n_threads, const int32_t* rows, uint64_t count, uint8_t* ok) {
  if (k < 1 || n < 0 || m < 0 || (count && (!rows || !ok))) return -1;
  Graph g{n, m, out_off, out_nbrs, in_off, in_nbrs, n_vcols, vcols, n_ecols, ecols};
  Pattern p{k, n_arcs, src, dst, vop, vval, eop, eval};
  std::vector<int32_t> arc_id((size_t)k * k, -1);
  for (int32_t i = 0; i < n_arcs; ++i) arc_id[(size_t)src[i] * k + dst[i]] = i;
  if (n_threads <= 0) n_threads = omp_get_max_threads();
  int64_t good = 0;
#pragma omp parallel for num_threads(n_threads) schedule(static, 4096) reduction(+ : good)
  for (int64_t i = 0; i < (int64_t)count; ++i) {
    const int32_t* f = rows + (size_t)i * k;
    bool pass = true;
    for (int32_t a = 0; a < k && pass; ++a) {
      if (f[a] < 0 || f[a] >= n) pass = false;
      for (int32_t b = 0; b < a && pass; ++b)
        if (f[a] == f[b]) pass = false;
    }
    for (int32_t a = 0; a < k && pass; ++a)
      for (int32_t col = 0; col < n_vcols && pass; ++col)
        if (!pred(vop[a * n_vcols + col], vval[a * n_vcols + col],
                  vcols[(int64_t)col * n + f[a]]))
          pass = false;
    for (int32_t a = 0; a < k && pass; ++a)
      for (int32_t b = 0; b < k && pass; ++b) {
        if (a == b) continue;
        const int32_t arc = arc_id[(size_t)a * k + b];
        if (arc < 0 && mode != MODE_ISO) continue;
        const int64_t eid = find_arc(g, f[a], f[b]);
        if (arc < 0) {
          pass = eid < 0;
          continue;
        }
        if (eid < 0) {
          pass = false;
          continue;
        }
        for (int32_t col = 0; col < n_ecols && pass; ++col)
          if (!pred(eop[arc * n_ecols + col], eval[arc * n_ecols + col],
                    ecols[(int64_t)col * m + eid]))
            pass = false;
      }
    ok[i] = pass ? 1 : 0;
    good += pass ? 1 : 0;
  }
  (void)p;
  return good;
}

void og_free(void* p) { std::free(p); }

// Lexicographic in-place sort of [count][k] int32 rows.
void og_sort_rows(int32_t* rows, uint64_t count, int32_t k) { sort_rows_impl(rows, count, k); }

// Fingerprint of a row set: (sum of h1, sum of h2) mod 2^64, independent of row order.
void og_fingerprint(const int32_t* rows, uint64_t count, int32_t k, uint64_t* out2) {
  uint64_t a = 0, b = 0;
  for (uint64_t i = 0; i < count; ++i) {
    a += row_hash(rows + i * k, k, kSeed1);
    b += row_hash(rows + i * k, k, kSeed2);
  }
  out2[0] = a;
  out2[1] = b;
}

}  // extern "C"
