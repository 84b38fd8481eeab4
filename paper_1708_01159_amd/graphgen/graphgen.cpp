// Seeded synthetic graph generators and an undirected CSR builder (host only).
//
// This module prepares inputs; it contains none of the traversal's arithmetic.
// Every random draw comes from one counter-based generator: the SplitMix64
// finaliser (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014) applied to a Weyl sequence keyed by
// (seed, stream, index).  Draws are therefore independent of thread count and
// order, and a graph is a pure function of its parameters and seed.
//
// Generators (all produce undirected, loop-free, duplicate-free graphs stored
// as symmetric CSR with int64 row offsets and int32 ascending column ids):
//   * R-MAT (Chakrabarti, Zhan and Faloutsos, SDM 2004) with quadrant
//     probabilities A/B/C/D and an optional seeded vertex relabelling;
//   * an R x C four-neighbour grid with a given fraction of its edges deleted
//     uniformly without replacement;
//   * Chung-Lu with power-law expected degrees;
//   * Erdos-Renyi G(n, m) with m pairs drawn uniformly with replacement.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr uint64_t kGolden = 0x9e3779b97f4a7c15ULL;

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

inline uint64_t ctr_rand(uint64_t seed, uint64_t stream, uint64_t idx) {
  const uint64_t key = mix64(seed + kGolden * (stream + 1));
  return mix64(key + kGolden * (idx + 1));
}

// Uniform double in [0, 1) from the top 53 bits.
inline double u01(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

// Uniform integer in [0, bound) by 128-bit multiply-shift (Lemire).
inline uint64_t below(uint64_t x, uint64_t bound) {
  return (uint64_t)(((unsigned __int128)x * (unsigned __int128)bound) >> 64);
}

// Random streams: each generator draws from its own stream ids.
enum : uint64_t {
  S_RMAT = 1, S_PERM = 2, S_GRID_DEL = 3, S_CL_U = 4, S_CL_V = 5,
  S_ER_U = 6, S_ER_V = 7, S_SOURCES = 8,
};

struct Csr {
  int64_t n = 0;
  int64_t nnz = 0;
  std::vector<int64_t> offs;
  std::vector<int32_t> cols;
};

// Seeded permutation of [0, n) by Fisher-Yates, drawing from stream S_PERM.
std::vector<int32_t> seeded_permutation(int64_t n, uint64_t seed) {
  std::vector<int32_t> p((size_t)n);
  for (int64_t i = 0; i < n; ++i) p[(size_t)i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    const int64_t j = (int64_t)below(ctr_rand(seed, S_PERM, (uint64_t)i), (uint64_t)(i + 1));
    std::swap(p[(size_t)i], p[(size_t)j]);
  }
  return p;
}

// Builds the symmetric, loop-free, duplicate-free CSR of an undirected edge
// list.  With symmetrize == 0 the pairs are taken as directed arcs as given.
Csr build_csr(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
              int symmetrize, int drop_loops, int dedup) {
  Csr g;
  g.n = n;
  std::vector<std::atomic<int64_t>> cnt((size_t)n + 1);
  for (auto& c : cnt) c.store(0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    const int32_t u = src[i], v = dst[i];
    if (drop_loops && u == v) continue;
    cnt[(size_t)u].fetch_add(1, std::memory_order_relaxed);
    if (symmetrize) cnt[(size_t)v].fetch_add(1, std::memory_order_relaxed);
  }
  std::vector<int64_t> start((size_t)n + 1, 0);
  for (int64_t i = 0; i < n; ++i) start[(size_t)i + 1] = start[(size_t)i] + cnt[(size_t)i].load();
  const int64_t total = start[(size_t)n];
  std::vector<int32_t> tmp((size_t)total);
  for (int64_t i = 0; i < n; ++i) cnt[(size_t)i].store(start[(size_t)i], std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    const int32_t u = src[i], v = dst[i];
    if (drop_loops && u == v) continue;
    tmp[(size_t)cnt[(size_t)u].fetch_add(1, std::memory_order_relaxed)] = v;
    if (symmetrize) tmp[(size_t)cnt[(size_t)v].fetch_add(1, std::memory_order_relaxed)] = u;
  }
  // Sort every row (and drop repeats) so the result does not depend on the
  // order in which threads scattered the arcs.
  std::vector<int64_t> deg((size_t)n, 0);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t r = 0; r < n; ++r) {
    int32_t* b = tmp.data() + start[(size_t)r];
    int32_t* e = tmp.data() + start[(size_t)r + 1];
    std::sort(b, e);
    if (dedup) e = std::unique(b, e);
    deg[(size_t)r] = e - b;
  }
  g.offs.assign((size_t)n + 1, 0);
  for (int64_t i = 0; i < n; ++i) g.offs[(size_t)i + 1] = g.offs[(size_t)i] + deg[(size_t)i];
  g.nnz = g.offs[(size_t)n];
  g.cols.resize((size_t)g.nnz);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t r = 0; r < n; ++r)
    std::memcpy(g.cols.data() + g.offs[(size_t)r], tmp.data() + start[(size_t)r],
                (size_t)deg[(size_t)r] * sizeof(int32_t));
  return g;
}

Csr* finish(Csr&& g) {
  Csr* h = new (std::nothrow) Csr(std::move(g));
  return h;
}

}  // namespace

extern "C" {

typedef struct Csr gg_csr;

// R-MAT with 2^scale vertices and edgefactor * 2^scale generated pairs.
gg_csr* gg_rmat(int scale, int edgefactor, double A, double B, double C, uint64_t seed,
                int relabel) {
  if (scale < 1 || scale > 30 || edgefactor < 1) return nullptr;
  const int64_t n = (int64_t)1 << scale;
  const int64_t m = (int64_t)edgefactor * n;
  std::vector<int32_t> src((size_t)m), dst((size_t)m);
  const double ab = A + B, abc = A + B + C;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint32_t u = 0, v = 0;
    for (int b = 0; b < scale; ++b) {
      const double r = u01(ctr_rand(seed, S_RMAT, (uint64_t)e * (uint64_t)scale + (uint64_t)b));
      const uint32_t ru = r >= ab ? 1u : 0u;                       // lower half (C or D)
      const uint32_t rv = (r >= A && r < ab) || r >= abc ? 1u : 0u;  // right half (B or D)
      u = (u << 1) | ru;
      v = (v << 1) | rv;
    }
    src[(size_t)e] = (int32_t)u;
    dst[(size_t)e] = (int32_t)v;
  }
  if (relabel) {
    const std::vector<int32_t> p = seeded_permutation(n, seed);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
      src[(size_t)e] = p[(size_t)src[(size_t)e]];
      dst[(size_t)e] = p[(size_t)dst[(size_t)e]];
    }
  }
  return finish(build_csr(n, m, src.data(), dst.data(), 1, 1, 1));
}

// rows x cols four-neighbour grid; floor(delete_frac * m) of its m edges are
// deleted, chosen uniformly without replacement.  Vertex (r, c) has id r*cols+c.
gg_csr* gg_grid(int rows, int cols, double delete_frac, uint64_t seed) {
  if (rows < 1 || cols < 1 || delete_frac < 0.0 || delete_frac > 1.0) return nullptr;
  const int64_t n = (int64_t)rows * cols;
  const int64_t mh = (int64_t)rows * (cols - 1), mv = (int64_t)(rows - 1) * cols;
  const int64_t m = mh + mv;
  const int64_t k = (int64_t)std::floor(delete_frac * (double)m);
  std::vector<int64_t> idx((size_t)m);
  for (int64_t i = 0; i < m; ++i) idx[(size_t)i] = i;
  for (int64_t i = 0; i < k; ++i) {  // partial Fisher-Yates: idx[0..k) are deleted
    const int64_t j = i + (int64_t)below(ctr_rand(seed, S_GRID_DEL, (uint64_t)i), (uint64_t)(m - i));
    std::swap(idx[(size_t)i], idx[(size_t)j]);
  }
  const int64_t keep = m - k;
  std::vector<int32_t> src((size_t)keep), dst((size_t)keep);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < keep; ++t) {
    const int64_t e = idx[(size_t)(k + t)];
    int64_t a, b;
    if (e < mh) {
      const int64_t r = e / (cols - 1), c = e % (cols - 1);
      a = r * cols + c;
      b = a + 1;
    } else {
      const int64_t f = e - mh;
      const int64_t r = f / cols, c = f % cols;
      a = r * cols + c;
      b = a + cols;
    }
    src[(size_t)t] = (int32_t)a;
    dst[(size_t)t] = (int32_t)b;
  }
  return finish(build_csr(n, keep, src.data(), dst.data(), 1, 1, 1));
}

// Chung-Lu: expected degree of vertex i proportional to (i+1)^(-1/(gamma-1)),
// capped at sqrt(n * mean_deg) and rescaled (iteratively, with the cap held)
// so the weights average mean_deg.  n*mean_deg/2 endpoint pairs are drawn
// with probability proportional to the weights; loops and repeats are dropped.
gg_csr* gg_chung_lu(int64_t n, double gamma, double mean_deg, uint64_t seed, int relabel) {
  if (n < 2 || n > ((int64_t)1 << 31) - 1 || gamma <= 1.0 || mean_deg <= 0.0) return nullptr;
  std::vector<double> w((size_t)n);
  const double ex = -1.0 / (gamma - 1.0);
  for (int64_t i = 0; i < n; ++i) w[(size_t)i] = std::pow((double)(i + 1), ex);
  const double cap = std::sqrt((double)n * mean_deg);
  const double target = (double)n * mean_deg;
  double scale = 1.0;
  for (int it = 0; it < 64; ++it) {
    double capped = 0.0, free_sum = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double x = w[(size_t)i] * scale;
      if (x >= cap) capped += cap; else free_sum += w[(size_t)i];
    }
    const double ns = (target - capped) / free_sum;
    if (std::fabs(ns - scale) <= 1e-12 * scale) { scale = ns; break; }
    scale = ns;
  }
  std::vector<double> cdf((size_t)n);
  double acc = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    acc += std::min(w[(size_t)i] * scale, cap);
    cdf[(size_t)i] = acc;
  }
  const int64_t m = (int64_t)std::llround(target / 2.0);
  std::vector<int32_t> src((size_t)m), dst((size_t)m);
  auto draw = [&](uint64_t x) -> int32_t {
    const double r = u01(x) * acc;
    int64_t i = std::upper_bound(cdf.begin(), cdf.end(), r) - cdf.begin();
    if (i >= n) i = n - 1;
    return (int32_t)i;
  };
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    src[(size_t)e] = draw(ctr_rand(seed, S_CL_U, (uint64_t)e));
    dst[(size_t)e] = draw(ctr_rand(seed, S_CL_V, (uint64_t)e));
  }
  if (relabel) {
    const std::vector<int32_t> p = seeded_permutation(n, seed);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
      src[(size_t)e] = p[(size_t)src[(size_t)e]];
      dst[(size_t)e] = p[(size_t)dst[(size_t)e]];
    }
  }
  return finish(build_csr(n, m, src.data(), dst.data(), 1, 1, 1));
}

// Erdos-Renyi G(n, m): m pairs drawn uniformly with replacement; loops and
// repeated pairs are dropped, so the realised edge count is at most m.
gg_csr* gg_erdos_renyi(int64_t n, int64_t m, uint64_t seed) {
  if (n < 1 || n > ((int64_t)1 << 31) - 1 || m < 0) return nullptr;
  std::vector<int32_t> src((size_t)m), dst((size_t)m);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    src[(size_t)e] = (int32_t)below(ctr_rand(seed, S_ER_U, (uint64_t)e), (uint64_t)n);
    dst[(size_t)e] = (int32_t)below(ctr_rand(seed, S_ER_V, (uint64_t)e), (uint64_t)n);
  }
  return finish(build_csr(n, m, src.data(), dst.data(), 1, 1, 1));
}

// CSR from an explicit arc list (used for small hand-built graphs).
gg_csr* gg_from_edges(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                      int symmetrize, int drop_loops, int dedup) {
  if (n < 1 || m < 0 || (m > 0 && (!src || !dst))) return nullptr;
  for (int64_t i = 0; i < m; ++i)
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return nullptr;
  return finish(build_csr(n, m, src, dst, symmetrize, drop_loops, dedup));
}

int64_t gg_n(const gg_csr* g) { return g ? g->n : -1; }
int64_t gg_nnz(const gg_csr* g) { return g ? g->nnz : -1; }

void gg_copy(const gg_csr* g, int64_t* offs, int32_t* cols) {
  if (!g) return;
  if (offs) std::memcpy(offs, g->offs.data(), (size_t)(g->n + 1) * sizeof(int64_t));
  if (cols && g->nnz) std::memcpy(cols, g->cols.data(), (size_t)g->nnz * sizeof(int32_t));
}

void gg_free(gg_csr* g) { delete g; }

// k distinct sources drawn uniformly among vertices of degree > 0 (rejection
// sampling on stream S_SOURCES).  Returns the number written (< k only when
// fewer than k vertices have degree > 0).
int64_t gg_pick_sources(int64_t n, const int64_t* offs, int64_t k, uint64_t seed, int32_t* out) {
  if (n < 1 || !offs || k < 0 || !out) return -1;
  int64_t avail = 0;
  for (int64_t v = 0; v < n; ++v) avail += offs[v + 1] > offs[v];
  const int64_t want = std::min(k, avail);
  std::vector<uint8_t> taken((size_t)n, 0);
  int64_t got = 0;
  for (uint64_t i = 0; got < want; ++i) {
    const int64_t v = (int64_t)below(ctr_rand(seed, S_SOURCES, i), (uint64_t)n);
    if (offs[v + 1] == offs[v] || taken[(size_t)v]) continue;
    taken[(size_t)v] = 1;
    out[got++] = (int32_t)v;
  }
  return got;
}

// Raw counter-based draw, exposed so tests can check the generator's stream.
uint64_t gg_ctr_rand(uint64_t seed, uint64_t stream, uint64_t idx) {
  return ctr_rand(seed, stream, idx);
}

}  // extern "C"
