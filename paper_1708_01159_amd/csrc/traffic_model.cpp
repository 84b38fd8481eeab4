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

// Counts for a bottom-up level whose probes start from the dense head copy:
// every unvisited vertex with arcs reads its head record and probes its
// h(v) = min(4, deg) head neighbours -- ranked (the four of largest degree
// among its first 256 arcs, the library's choice on a skewed degree law) or
// else the row's first four arcs; when none of them is in the frontier and
// the row has at least four arcs, it reads the row bounds and probes the row
// from r0 (0 with a ranked head, 4 past the first arcs otherwise) up to the
// first frontier neighbour (to the row's end when there is none).  Per depth d:
//   fcost[d]  over the vertices at depth d: full(v) = h(v) + (deg >= 4 ? deg - r0 : 0),
//             the probes of a vertex that finds nothing
//   rowc[d]   vertices at depth d with deg >= 4 (a row read when nothing is found)
//   fsave[d]  over the vertices v at depth d+1: full(v) - found(v), found(v) =
//             h(v) on a head hit, else h(v) + (position of v's first neighbour
//             at depth d in the row, from 1) - r0
//   rsave[d]  vertices at depth d+1 with deg >= 4 found by their head (no row read)
// and in tot[0..1] the sums of full(v) and of [deg >= 4] over every vertex.
extern "C" int64_t tm_head_counts(int64_t n, const int64_t* offs, const int32_t* cols, const int32_t* level,
                                  int64_t cap, int64_t* fcost, int64_t* rowc, int64_t* fsave, int64_t* rsave,
                                  int64_t* tot, int32_t ranked) {
  const int64_t r0 = ranked ? 0 : 4;
  int32_t dmax = -1;
  for (int64_t v = 0; v < n; ++v) dmax = level[v] > dmax ? level[v] : dmax;
  const int64_t D = (int64_t)dmax + 1;
  if (D > cap) return -1;
  for (int64_t d = 0; d < cap; ++d) fcost[d] = rowc[d] = fsave[d] = rsave[d] = 0;
  int64_t tf = 0, tr = 0;
#pragma omp parallel reduction(+ : tf, tr)
  {
    std::vector<int64_t> lf((std::size_t)D, 0), lr((std::size_t)D, 0), lfs((std::size_t)D, 0), lrs((std::size_t)D, 0);
#pragma omp for schedule(dynamic, 4096)
    for (int64_t v = 0; v < n; ++v) {
      const int64_t deg = offs[v + 1] - offs[v];
      const int64_t h = deg < 4 ? deg : 4;
      const int64_t full = h + (deg >= 4 ? deg - r0 : 0);
      tf += full;
      tr += deg >= 4 ? 1 : 0;
      const int32_t L = level[v];
      if (L < 0) continue;
      lf[(std::size_t)L] += full;
      lr[(std::size_t)L] += deg >= 4 ? 1 : 0;
      if (L < 1) continue;
      // the ranked head: four largest degrees among the first 256 arcs, earlier arcs first on ties
      int32_t id[4] = {-1, -1, -1, -1};
      int64_t dg[4] = {-1, -1, -1, -1};
      const int64_t lim = deg < 256 ? deg : 256;
      for (int64_t k = 0; !ranked && k < h; ++k) id[k] = cols[offs[v] + k];
      for (int64_t e = 0; ranked && e < lim; ++e) {
        const int32_t u = cols[offs[v] + e];
        const int64_t du = offs[u + 1] - offs[u];
        if (du > dg[3]) {
          int k = 3;
          while (k > 0 && du > dg[k - 1]) {
            dg[k] = dg[k - 1];
            id[k] = id[k - 1];
            --k;
          }
          dg[k] = du;
          id[k] = u;
        }
      }
      bool hit = false;
      for (int k = 0; k < 4; ++k) hit = hit || (id[k] >= 0 && level[id[k]] == L - 1);
      int64_t found = h;
      if (!hit) {
        int64_t pos = deg;
        for (int64_t e = offs[v]; e < offs[v + 1]; ++e)
          if (level[cols[e]] == L - 1) {
            pos = e - offs[v] + 1;
            break;
          }
        found += deg >= 4 ? pos - r0 : 0;
      }
      lfs[(std::size_t)(L - 1)] += full - found;
      lrs[(std::size_t)(L - 1)] += (hit && deg >= 4) ? 1 : 0;
    }
#pragma omp critical
    for (int64_t d = 0; d < D; ++d) {
      fcost[d] += lf[(std::size_t)d];
      rowc[d] += lr[(std::size_t)d];
      fsave[d] += lfs[(std::size_t)d];
      rsave[d] += lrs[(std::size_t)d];
    }
  }
  tot[0] = tf;
  tot[1] = tr;
  return D;
}
