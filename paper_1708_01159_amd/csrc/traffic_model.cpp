// Host-side counts for the algorithmic-byte model of the roofline (a
// measurement helper for the benchmark, not part of the search): from a
// source's level array on a symmetric CSR graph, per depth d,
//   nf[d]     vertices at depth d            ef[d]    their degree sum
//   words[d]  64-vertex bitmap words holding a depth-d vertex
//   save[d]   over the vertices v at depth d+1: deg(v) - (position of the
//             first neighbour of v at depth d, counted from 1)
// A bottom-up level d probes, for every vertex still unvisited at d, its
// neighbours up to the first one in the frontier.  On a symmetric graph the
// neighbours of a vertex at depth L lie at depths L-1..L+1, so only the
// vertices found at d+1 stop early; every other unvisited vertex reads its
// whole row.  Hence probes(d) = (degree sum of the vertices unvisited at d)
// - save[d], with all of it computable in one pass over the rows.
#include <cstddef>
#include <cstdint>
#include <vector>

extern "C" int64_t tm_level_counts(int64_t n, const int64_t* offs, const int32_t* cols, const int32_t* level,
                                   int64_t cap, int64_t* nf, int64_t* ef, int64_t* words, int64_t* save) {
  int32_t dmax = -1;
  for (int64_t v = 0; v < n; ++v) dmax = level[v] > dmax ? level[v] : dmax;
  const int64_t D = (int64_t)dmax + 1;
  if (D > cap) return -1;
  for (int64_t d = 0; d < cap; ++d) nf[d] = ef[d] = words[d] = save[d] = 0;
  const int64_t nw = (n + 63) / 64;
#pragma omp parallel
  {
    std::vector<int64_t> lnf((std::size_t)D, 0), lef((std::size_t)D, 0), lwords((std::size_t)D, 0), lsave((std::size_t)D, 0);
#pragma omp for schedule(dynamic, 1024)
    for (int64_t w = 0; w < nw; ++w) {
      int32_t last = -2;  // depths seen in this word, deduplicated cheaply when repeated
      std::vector<int32_t> seen;
      for (int64_t v = w * 64; v < n && v < w * 64 + 64; ++v) {
        const int32_t L = level[v];
        if (L < 0) continue;
        const int64_t deg = offs[v + 1] - offs[v];
        lnf[(std::size_t)L] += 1;
        lef[(std::size_t)L] += deg;
        if (L != last) {
          bool dup = false;
          for (int32_t x : seen) dup = dup || x == L;
          if (!dup) {
            seen.push_back(L);
            lwords[(std::size_t)L] += 1;
          }
          last = L;
        }
        if (L >= 1) {
          int64_t pos = deg;  // no neighbour at depth L-1 cannot happen for L >= 1
          for (int64_t e = offs[v]; e < offs[v + 1]; ++e)
            if (level[cols[e]] == L - 1) {
              pos = e - offs[v] + 1;
              break;
            }
          lsave[(std::size_t)(L - 1)] += deg - pos;
        }
      }
    }
#pragma omp critical
    for (int64_t d = 0; d < D; ++d) {
      nf[d] += lnf[(std::size_t)d];
      ef[d] += lef[(std::size_t)d];
      words[d] += lwords[(std::size_t)d];
      save[d] += lsave[(std::size_t)d];
    }
  }
  return D;
}
