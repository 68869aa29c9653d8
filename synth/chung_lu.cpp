// chung_lu.cpp -- seeded directed Chung-Lu graph with reciprocity (input generator).
//
// Holds no matching logic: it only draws a random graph and lays it out as
// out- and in-CSR with attribute columns.  Every random number comes from a
// counter-based stream keyed by (seed, purpose, vertex or arc), so the output
// does not depend on the number of threads.
//
// Recipe:
//   1. out- and in-weights w_out[v], w_in[v] i.i.d. truncated Pareto
//      (density proportional to x^-gamma on [1, xmax], inverse CDF);
//   2. vertex u gets Poisson(B * w_out[u] / sum w_out) arc draws (B base draws
//      in expectation); each draw picks a head with probability proportional
//      to w_in (Walker/Vose alias table); self-loops and repeats are dropped;
//   3. arcs without a reverse are given one independently with probability p,
//      chosen so that the expected fraction of arcs whose reverse exists is
//      `recip`;
//   4. vertex label U{0..nlab-1}; arc weight 1 + floor(exp(mu + sigma Z)).
// B is set from the target arc count m and the measured repeat rate of a
// first pass, so the final arc count is close to (not exactly) m.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

inline uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
}

// xoshiro256** (Blackman & Vigna), seeded through splitmix64.
struct Rng {
  uint64_t s[4];
  explicit Rng(uint64_t key) {
    uint64_t x = key;
    for (int i = 0; i < 4; ++i) s[i] = splitmix64(x += 0x632be59bd9b4e019ULL);
  }
  static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
  uint64_t next() {
    const uint64_t r = rotl(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return r;
  }
  double uniform() { return (next() >> 11) * (1.0 / 9007199254740992.0); }  // [0,1)
  double normal() {                                                          // Box-Muller
    double u1 = uniform();
    while (u1 <= 0.0) u1 = uniform();
    const double u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

inline uint64_t stream_key(uint64_t seed, uint64_t purpose, uint64_t a, uint64_t b = 0) {
  return splitmix64(splitmix64(splitmix64(seed ^ (purpose * 0xd1342543de82ef95ULL)) ^ a) ^ b);
}

enum : uint64_t { kOutW = 1, kInW = 2, kArcs = 3, kRecip = 4, kLabel = 5, kWeight = 6 };

int64_t poisson(Rng& r, double lam) {
  if (lam <= 0.0) return 0;
  if (lam < 30.0) {  // Knuth's product of uniforms
    const double L = std::exp(-lam);
    int64_t k = 0;
    double p = 1.0;
    do {
      ++k;
      p *= r.uniform();
    } while (p > L);
    return k - 1;
  }
  const double x = std::floor(lam + std::sqrt(lam) * r.normal() + 0.5);  // normal approximation
  return x < 0 ? 0 : (int64_t)x;
}

struct Alias {
  std::vector<double> prob;
  std::vector<int32_t> alias;
  explicit Alias(const std::vector<double>& w) : prob(w.size()), alias(w.size()) {
    const size_t n = w.size();
    double sum = 0;
    for (double x : w) sum += x;
    std::vector<double> q(n);
    std::vector<int32_t> small, large;
    for (size_t i = 0; i < n; ++i) {
      q[i] = w[i] * n / sum;
      (q[i] < 1.0 ? small : large).push_back((int32_t)i);
    }
    while (!small.empty() && !large.empty()) {
      const int32_t s = small.back(), l = large.back();
      small.pop_back();
      prob[s] = q[s];
      alias[s] = l;
      q[l] = (q[l] + q[s]) - 1.0;
      if (q[l] < 1.0) {
        large.pop_back();
        small.push_back(l);
      }
    }
    for (int32_t l : large) { prob[l] = 1.0; alias[l] = l; }
    for (int32_t s : small) { prob[s] = 1.0; alias[s] = s; }
  }
  int32_t draw(Rng& r) const {
    const uint64_t x = r.next();
    const int32_t i = (int32_t)((x >> 32) * prob.size() >> 32);
    const double u = (x & 0xffffffffULL) * (1.0 / 4294967296.0);
    return u < prob[i] ? i : alias[i];
  }
};

// Row u of the base graph: sorted distinct heads, self-loops removed.
void base_row(uint64_t seed, int32_t u, int64_t draws, const Alias& in_alias,
              std::vector<int32_t>& row) {
  Rng r(stream_key(seed, kArcs, (uint64_t)u));
  row.clear();
  for (int64_t t = 0; t < draws; ++t) {
    const int32_t v = in_alias.draw(r);
    if (v != u) row.push_back(v);
  }
  std::sort(row.begin(), row.end());
  row.erase(std::unique(row.begin(), row.end()), row.end());
}

bool has_arc(const std::vector<int64_t>& off, const std::vector<int32_t>& nb, int32_t u,
             int32_t v) {
  return std::binary_search(nb.begin() + off[u], nb.begin() + off[u + 1], v);
}

// Transpose of a CSR (rows of the result sorted).
void transpose(int32_t n, const std::vector<int64_t>& off, const std::vector<int32_t>& nb,
               std::vector<int64_t>& toff, std::vector<int32_t>& tnb) {
  const int64_t m = off[n];
  std::vector<std::atomic<int64_t>> cnt(n);
  for (int32_t v = 0; v < n; ++v) cnt[v].store(0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) cnt[nb[e]].fetch_add(1, std::memory_order_relaxed);
  toff.assign((size_t)n + 1, 0);
  for (int32_t v = 0; v < n; ++v) toff[v + 1] = toff[v] + cnt[v].load(std::memory_order_relaxed);
  std::vector<std::atomic<int64_t>> pos(n);
  for (int32_t v = 0; v < n; ++v) pos[v].store(toff[v], std::memory_order_relaxed);
  tnb.assign((size_t)m, 0);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t u = 0; u < n; ++u)
    for (int64_t e = off[u]; e < off[u + 1]; ++e)
      tnb[pos[nb[e]].fetch_add(1, std::memory_order_relaxed)] = u;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t v = 0; v < n; ++v) std::sort(tnb.begin() + toff[v], tnb.begin() + toff[v + 1]);
}

}  // namespace

extern "C" {

// Generates the graph; the caller frees the returned arrays with cl_free.
// Returns the number of arcs, or -1 on bad arguments.
int64_t cl_generate(int32_t n, int64_t m_target, double gamma, double xmax, double recip,
                    int32_t nlab, double mu, double sigma, uint64_t seed, int32_t threads,
                    int64_t** out_off, int32_t** out_nbrs, int64_t** in_off, int32_t** in_nbrs,
                    int32_t** vlabel, int32_t** eweight) {
  if (n <= 1 || m_target <= 0 || gamma <= 1.0 || xmax < 1.0 || recip < 0 || recip >= 1)
    return -1;
  if (threads > 0) omp_set_num_threads(threads);
  const double al = gamma - 1.0, lo = std::pow(xmax, -al);
  std::vector<double> wo(n), wi(n);
#pragma omp parallel for schedule(static)
  for (int32_t v = 0; v < n; ++v) {
    Rng a(stream_key(seed, kOutW, (uint64_t)v)), b(stream_key(seed, kInW, (uint64_t)v));
    wo[v] = std::pow(1.0 - a.uniform() * (1.0 - lo), -1.0 / al);
    wi[v] = std::pow(1.0 - b.uniform() * (1.0 - lo), -1.0 / al);
  }
  double so = 0;
  for (double x : wo) so += x;
  const Alias in_alias(wi);

  // Base draws B: the reciprocity step adds about recip/(2-recip) of the base
  // count (natural reciprocity aside); calibrate the repeat rate on a pilot.
  const double grow = 1.0 + recip / (2.0 - recip);
  double B = (double)m_target / grow;
  std::vector<int64_t> draws(n), deg(n);
  std::vector<int64_t> off((size_t)n + 1, 0);
  for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel
    {
      std::vector<int32_t> row;
#pragma omp for schedule(dynamic, 1024)
      for (int32_t u = 0; u < n; ++u) {
        Rng r(stream_key(seed + pass, kArcs + 100, (uint64_t)u));
        draws[u] = poisson(r, B * wo[u] / so);
        base_row(seed + 1000003ULL * pass, u, draws[u], in_alias, row);
        deg[u] = (int64_t)row.size();
      }
    }
    int64_t M0 = 0, D = 0;
    for (int32_t u = 0; u < n; ++u) { M0 += deg[u]; D += draws[u]; }
    if (pass == 0) {
      const double keep = D ? (double)M0 / D : 1.0;  // fraction surviving dedup
      B = (double)m_target / grow / keep;
    }
  }
  const uint64_t rseed = seed + 1000003ULL;  // seed of the final pass
  for (int32_t u = 0; u < n; ++u) off[u + 1] = off[u] + deg[u];
  std::vector<int32_t> nb((size_t)off[n]);
#pragma omp parallel
  {
    std::vector<int32_t> row;
#pragma omp for schedule(dynamic, 1024)
    for (int32_t u = 0; u < n; ++u) {
      base_row(rseed, u, draws[u], in_alias, row);
      std::copy(row.begin(), row.end(), nb.begin() + off[u]);
    }
  }
  const int64_t M0 = off[n];

  // Reciprocity: arcs whose reverse is missing get one with probability p.
  int64_t R0 = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : R0)
  for (int32_t u = 0; u < n; ++u)
    for (int64_t e = off[u]; e < off[u + 1]; ++e) R0 += has_arc(off, nb, nb[e], u);
  const double A = std::max(0.0, (recip * M0 - R0) / (2.0 - recip));
  const double p = (M0 > R0) ? std::min(1.0, A / (double)(M0 - R0)) : 0.0;
  std::vector<uint8_t> add((size_t)M0, 0);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t u = 0; u < n; ++u)
    for (int64_t e = off[u]; e < off[u + 1]; ++e) {
      const int32_t v = nb[e];
      if (has_arc(off, nb, v, u)) continue;
      Rng r(stream_key(seed, kRecip, (uint64_t)u, (uint64_t)v));
      add[e] = r.uniform() < p;
    }
  // new arcs v -> u for add[u->v]: collect per head row v via the transpose
  std::vector<int64_t> toff;
  std::vector<int32_t> tnb;
  transpose(n, off, nb, toff, tnb);  // tnb row v: tails u of base arcs u -> v
  std::vector<int64_t> fdeg(n);
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t v = 0; v < n; ++v) {
    int64_t extra = 0;
    for (int64_t j = toff[v]; j < toff[v + 1]; ++j) {
      const int32_t u = tnb[j];
      const int64_t e = std::lower_bound(nb.begin() + off[u], nb.begin() + off[u + 1], v) -
                        nb.begin();
      extra += add[e];
    }
    fdeg[v] = (off[v + 1] - off[v]) + extra;
  }
  std::vector<int64_t>* foff = new std::vector<int64_t>((size_t)n + 1, 0);
  for (int32_t v = 0; v < n; ++v) (*foff)[v + 1] = (*foff)[v] + fdeg[v];
  const int64_t M = (*foff)[n];
  std::vector<int32_t> fnb((size_t)M);
#pragma omp parallel
  {
    std::vector<int32_t> row;
#pragma omp for schedule(dynamic, 4096)
    for (int32_t v = 0; v < n; ++v) {
      row.assign(nb.begin() + off[v], nb.begin() + off[v + 1]);
      for (int64_t j = toff[v]; j < toff[v + 1]; ++j) {
        const int32_t u = tnb[j];
        const int64_t e = std::lower_bound(nb.begin() + off[u], nb.begin() + off[u + 1], v) -
                          nb.begin();
        if (add[e]) row.push_back(u);
      }
      std::sort(row.begin(), row.end());
      std::copy(row.begin(), row.end(), fnb.begin() + (*foff)[v]);
    }
  }
  std::vector<int32_t>().swap(nb);
  std::vector<uint8_t>().swap(add);
  std::vector<int64_t> ioff;
  std::vector<int32_t> inb;
  transpose(n, *foff, fnb, ioff, inb);

  *out_off = (int64_t*)std::malloc(sizeof(int64_t) * ((size_t)n + 1));
  *in_off = (int64_t*)std::malloc(sizeof(int64_t) * ((size_t)n + 1));
  *out_nbrs = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)M + 4);
  *in_nbrs = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)M + 4);
  *vlabel = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)n);
  *eweight = (int32_t*)std::malloc(sizeof(int32_t) * (size_t)M + 4);
  std::memcpy(*out_off, foff->data(), sizeof(int64_t) * ((size_t)n + 1));
  std::memcpy(*in_off, ioff.data(), sizeof(int64_t) * ((size_t)n + 1));
  std::memcpy(*out_nbrs, fnb.data(), sizeof(int32_t) * (size_t)M);
  std::memcpy(*in_nbrs, inb.data(), sizeof(int32_t) * (size_t)M);
#pragma omp parallel for schedule(static)
  for (int32_t v = 0; v < n; ++v) {
    Rng r(stream_key(seed, kLabel, (uint64_t)v));
    (*vlabel)[v] = (int32_t)((r.next() >> 32) * (uint64_t)nlab >> 32);
  }
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t u = 0; u < n; ++u)
    for (int64_t e = (*foff)[u]; e < (*foff)[u + 1]; ++e) {
      Rng r(stream_key(seed, kWeight, (uint64_t)u, (uint64_t)fnb[e]));
      (*eweight)[e] = 1 + (int32_t)std::floor(std::exp(mu + sigma * r.normal()));
    }
  delete foff;
  return M;
}

void cl_free(void* p) { std::free(p); }

}  // extern "C"
