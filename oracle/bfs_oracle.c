/*
 * CPU correctness oracle for breadth-first search levels (test infrastructure).
 *
 * What it computes: for a source s of a graph G given as CSR, level[v] is the
 * hop distance from s to v, or -1 when v is not reachable.  The paper defines
 * the traversal as a level-synchronous BFS that starts with every depth at
 * infinity and the root at depth 0, and grows depth by one per level until no
 * new vertex is found (Section III-A, opening paragraphs and "Variants").
 * That result has a plain definition (shortest-path hop counts), so this file
 * is the textbook single-threaded FIFO-queue BFS, which reaches exactly that
 * definition: it shares no code with the GPU library.
 *
 * Outputs besides levels:
 *   parent[v]  the vertex from which v was first reached (parent[s] = s,
 *              -1 when unreached).  Parents are not unique in general;
 *   hist[d]    number of vertices at depth d (the frontier size of level d);
 *   ehist[d]   sum of the degrees of the vertices at depth d.
 *
 * Only tests, the smoke check and the bench's CPU-baseline leg use this file.
 */
#include <stdint.h>
#include <stdlib.h>

/* Returns the number of distinct depths (eccentricity of s plus one), or a
 * negative value on bad arguments / allocation failure.  hist and ehist may be
 * NULL; otherwise they must hold at least n entries. */
int64_t oracle_bfs(int64_t n, const int64_t *offs, const int32_t *cols, int64_t s,
                   int32_t *level, int32_t *parent, int64_t *hist, int64_t *ehist) {
  if (n < 1 || !offs || !level || !parent || s < 0 || s >= n) return -1;
  int32_t *queue = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!queue) return -2;
  for (int64_t v = 0; v < n; ++v) {
    level[v] = -1;
    parent[v] = -1;
  }
  int64_t head = 0, tail = 0;
  level[s] = 0;
  parent[s] = (int32_t)s;
  queue[tail++] = (int32_t)s;
  int32_t maxd = 0;
  while (head < tail) {
    const int32_t u = queue[head++];
    for (int64_t e = offs[u]; e < offs[u + 1]; ++e) {
      const int32_t v = cols[e];
      if (level[v] == -1) {
        level[v] = level[u] + 1;
        parent[v] = u;
        queue[tail++] = v;
        if (level[v] > maxd) maxd = level[v];
      }
    }
  }
  free(queue);
  if (hist) {
    for (int32_t d = 0; d <= maxd; ++d) hist[d] = 0;
  }
  if (ehist) {
    for (int32_t d = 0; d <= maxd; ++d) ehist[d] = 0;
  }
  for (int64_t v = 0; v < n; ++v) {
    if (level[v] < 0) continue;
    if (hist) hist[level[v]] += 1;
    if (ehist) ehist[level[v]] += offs[v + 1] - offs[v];
  }
  return (int64_t)maxd + 1;
}

/*
 * Weakly connected components (the second traversal on the switching
 * framework: the paper expects its per-iteration kernel choice to carry over
 * to other traversal algorithms, Section VI).  label[v] is the smallest
 * vertex id of the component that contains v, every arc u -> v joining u and
 * v whatever its direction.  That result has a plain definition, so this is
 * the textbook disjoint-set forest: one union per arc, with path halving,
 * the larger root linked under the smaller, so that every root is the
 * smallest id of its set.  Returns the number of components, or a negative
 * value on bad arguments / allocation failure.
 */
static int32_t cc_find(int32_t *up, int32_t x) {
  while (up[x] != x) {
    up[x] = up[up[x]];
    x = up[x];
  }
  return x;
}

int64_t oracle_components(int64_t n, const int64_t *offs, const int32_t *cols, int32_t *label) {
  if (n < 1 || !offs || !label) return -1;
  int32_t *up = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!up) return -2;
  for (int64_t v = 0; v < n; ++v) up[v] = (int32_t)v;
  for (int64_t u = 0; u < n; ++u) {
    for (int64_t e = offs[u]; e < offs[u + 1]; ++e) {
      int32_t a = cc_find(up, (int32_t)u), b = cc_find(up, cols[e]);
      if (a < b)
        up[b] = a;
      else if (b < a)
        up[a] = b;
    }
  }
  int64_t count = 0;
  for (int64_t v = 0; v < n; ++v) {
    label[v] = cc_find(up, (int32_t)v);
    if (label[v] == v) ++count;
  }
  free(up);
  return count;
}
